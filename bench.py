"""Benchmark of the Disentangled-4DGS render path on one MI355X.

Workload (the frames/s headline): 300,000 Gaussians (32-cluster mixture, SH degree 3)
rendered at 1352x1014 from 20 cameras on a 120-degree arc of radius 10, each at 300
evenly spaced times -- a camera-major sweep with the camera-stage cache on (the camera
stage runs once per camera; the time stage, binning, sort and blend once per frame).
One step = one camera's 300 frames.  Inputs are synthetic and resident in HBM before
timing starts.

Printed: one JSON line with frames/s (the sweep on four streams), the roofline of the
dominant kernel (the blend, timed by HIP events attached to its launches in a one-stream
pass over the same frames), the CPU oracle timed on a bounded sample of the same frames,
and side measurements: forward + backward at the same scene and resolution, the
fixed-camera multi-timestamp batch, and serving latency.

    python bench.py [--gpus 1] [--steps 20] [--warmup 10]
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

# HIP binds each stream to one of the process's hardware queues (GPU_MAX_HW_QUEUES, 4 by
# default).  With 4 queues the sweep's four streams, created after the one-stream kernel
# pass's, measured 21.4 k frames/s; with 8, 27.2 k (as with 4 when four other streams had
# been used first).  The benchmark allows 8 for its own process, before HIP initialises
# (a larger value in the environment is kept); config.hip_hw_queues reports it.
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or 4) < 8:
    os.environ["GPU_MAX_HW_QUEUES"] = "8"

FRAMES_PER_STEP = 300
# Blend roofline.  Algorithmic work per (pixel, splat) evaluation of Eq. 4, counted on
# the definition: exponent -1/2(a dx^2 + c dy^2) - b dx dy (11 flops), exp (1),
# alpha = amax G (1), T' = T (1 - alpha) (2), C += c alpha T (7)  ->  22 flops.  The
# evaluations are the oracle's exact count E (every pixel over its tile list up to its
# stop); the kernel skips many of them (splats whose alpha >= 1/255 box misses a
# wavefront's pixels), so this is an effective rate.
FLOPS_PER_EVAL = 22
# FP32 vector peak of MI355X: 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2 (packed) x 2.4 GHz.
ALU_PEAK_TFLOPS = 157.3
# The same without packed FP32 (the issue-slot bound of the code as compiled).
ALU_PEAK_NONPACKED_TFLOPS = 78.6
# 256 CU x 4 SIMD: a wave64 VALU instruction occupies a SIMD for 4 cycles at 2.4 GHz.
SIMDS, CLOCK_HZ, CYCLES_PER_VALU = 1024, 2.4e9, 4
# Blend adjoint, per evaluated (pixel, list entry) up to the pixel's last contributor:
# exponent 11, exp 1, alpha 1, T_i = T / (1 - alpha) 2, g.c 5, dL/dalpha 3, g.S 2,
# dL/dpower 2, offsets 2 + moments 5, colour gradients 3, the nine sums 9 -> 46 flops.
FLOPS_PER_BWD_EVAL = 46
HBM_PEAK_GBS = 8000.0
# Counter summaries (rocprofv3) of kernels, valid only while the sources they were taken
# with are unchanged (sources_sha256 in the summary).
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_SUMMARY = os.path.join(PROFILES, "k_blend_pmc_traffic_300k_1352x1014.txt")
BLEND_SOURCES = ("paper_2503_22159_amd/csrc/blend.hip", "paper_2503_22159_amd/csrc/internal.hpp",
                 "paper_2503_22159_amd/build.py")
SWEEP_SUMMARY = os.path.join(PROFILES, "sweep_valu_pmc_300k_1352x1014.txt")
SWEEP_SOURCES = ("paper_2503_22159_amd/csrc/project.hip", "paper_2503_22159_amd/csrc/emit.hpp",
                 "paper_2503_22159_amd/csrc/binsort.hip", "paper_2503_22159_amd/csrc/blend.hip",
                 "paper_2503_22159_amd/csrc/internal.hpp", "paper_2503_22159_amd/build.py")
BWD_SUMMARY = os.path.join(PROFILES, "backward_pmc_300k_1352x1014.txt")
BWD_SOURCES = ("paper_2503_22159_amd/csrc/backward.hip", "paper_2503_22159_amd/csrc/internal.hpp",
               "paper_2503_22159_amd/build.py")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10, help="untimed steps before each timed pass")
    ap.add_argument("--frames", type=int, default=FRAMES_PER_STEP, help="frames per step (times per camera)")
    ap.add_argument("--streams", type=int, default=4, help="HIP streams the sweep's frames alternate over")
    ap.add_argument("--tile-order", action="store_true",
                    help="launch the sweep's per-tile kernels longest list first (the kernel pass always does)")
    ap.add_argument("--unfused", action="store_true",
                    help="sweep through d4dgs_project + d4dgs_bin_sort instead of d4dgs_project_bin")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-bwd", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-times", action="store_true", help="skip the multi-timestamp batch measurement")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the side sweeps (camera cache off, one camera's 300 frames)")
    ap.add_argument("--no-steps", action="store_true",
                    help="skip the 8-view 800x800 (100k, SH1) and 4-view 2704x2028 (2M, SH3) forward+backward steps")
    ap.add_argument("--view-steps", default="c3,c5",
                    help="which of those steps to run: c3 (8 x 800x800, 100k SH1), c5 (4 x 2704x2028, 2M SH3)")
    ap.add_argument("--cpu-frames", type=int, default=100)
    ap.add_argument("--cpu-frames-1core", type=int, default=4, help="frames of the CPU sample timed on one core")
    ap.add_argument("--bwd-oracle-views", type=int, default=8,
                    help="views of the backward phase the oracle counts the adjoint's units on")
    ap.add_argument("--bwd-frames", type=int, default=40)
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="length of the 200 req/s serving stream")
    ap.add_argument("--serve-high-rates", default="2000,6000",
                    help="arrival rates (req/s, comma separated) of the heavier serving streams ('' : none)")
    ap.add_argument("--serve-high-seconds", type=float, default=10.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy a 256 MiB buffer three times (the reference kernel for scaling "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE to bytes)")
    return ap.parse_args()


def sources_sha256(sources=BLEND_SOURCES):
    import hashlib

    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def blend_sources_sha256():
    return sources_sha256(BLEND_SOURCES)


def counter_summary(path, sources):
    """The 'key: value' lines of a committed counter summary, or None when there is none or
    the kernels' sources have changed since the counters were taken."""
    try:
        with open(path) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith(" "))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    return kv if kv.get("sources_sha256") == sources_sha256(sources) else None


def _num(kv, key):
    try:
        return float(kv[key]) if kv is not None else None
    except (KeyError, ValueError):
        return None


def blend_traffic():
    """HBM bytes per blend launch from the committed counter summary (None if stale)."""
    return _num(counter_summary(TRAFFIC_SUMMARY, BLEND_SOURCES), "hbm_bytes_per_launch")


def issue_frac(valu_insts, seconds):
    """Share of the SIMDs' VALU issue slots that valu_insts wave instructions fill."""
    if valu_insts is None or not seconds:
        return None
    return valu_insts * CYCLES_PER_VALU / (SIMDS * CLOCK_HZ * seconds)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def copy_calibration():
    import torch

    n = 64 << 20  # 256 MiB of float32
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copy calibration: 3 copies of {4 * n} bytes", file=sys.stderr, flush=True)


def scene_order(render, ds_drawn):
    """The drawn scene stored in the library's spatial order (d4dgs_spatial_order +
    d4dgs_scene_permute); returns it and the step's time in ms (second of two runs)."""
    import torch

    render.spatially_ordered(ds_drawn)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ds, _ = render.spatially_ordered(ds_drawn)
    torch.cuda.synchronize()
    return ds, 1000.0 * (time.perf_counter() - t0)


def sweep(args, ds, cams, times, render, S, time_blends, tile_order, streams=None, cache=True):
    """The camera-major sweep: `args.warmup` untimed steps, then `args.steps` timed ones.
    Frames are independent, so consecutive frames go round-robin to S HIP streams
    (default priority), each with its own frame buffers: one frame's binning overlaps
    another's blend.  The streams share one camera-stage cache, so the camera stage runs
    once per camera (Alg. 1); a camera's first frame fills it after the other streams'
    frames of the previous camera, and their frames of the new camera wait for it
    (render.SharedCameraOrder).  With time_blends, every blend kernel is launched with a
    pair of HIP events (created and first recorded beforehand) that the launch sets to the
    kernel's own start and end; the benchmark does that on one stream, so that no other
    stream's kernels share the compute units meanwhile."""
    import torch

    W, H = cams[0].width, cams[0].height
    shared = render.CamCache(ds.n) if cache else False
    rends = [render.Renderer(ds, W, H, capacity=4 * ds.n, cache=shared, tile_order=tile_order) for _ in range(S)]
    streams = streams or [torch.cuda.Stream() for _ in range(S)]
    handles = [st.cuda_stream for st in streams]
    order = render.SharedCameraOrder(streams) if cache else None
    nfr = len(times)
    events = []
    if time_blends:
        events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(args.steps * nfr)]
        for i, (e0, e1) in enumerate(events):  # materialise the events outside the timed region
            e0.record(streams[i % S])
            e1.record(streams[i % S])

    fused = not getattr(args, "unfused", False)

    last = [None]

    def step(k, ev):
        cam = cams[k % len(cams)]
        miss = cam is not last[0]  # the cache misses on the first frame of a new camera
        last[0] = cam
        for i, t in enumerate(times):
            r = i % S
            rend, h = rends[r], handles[r]
            if order:
                order.before_miss(r) if (miss and i == 0) else order.before_hit(r)
            if fused:
                rend.project_bin(cam, t, h)
            else:
                rend.project(cam, t, h)
                rend.bin_sort(h)
            if order and miss and i == 0:
                order.after_miss(r)
            rend.blend(stream=h, events=ev[i] if ev else None)

    for k in range(args.warmup):
        step(len(cams) - 1 - k, None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k, events[k * nfr:(k + 1) * nfr])
    t_host = time.perf_counter() - t0
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert not any(r.overflowed() for r in rends), "instance capacity exceeded during the sweep"
    blend_ms = [a.elapsed_time(b) for a, b in events]
    return elapsed, (sum(blend_ms) / len(blend_ms) if blend_ms else None), t_host


def fwd_bwd(args, ds, cams, render, inputs):
    """Forward + backward at the same scene and resolution (training-style: no camera
    cache, every view's gradient added into one set of parameter gradients).  Views
    alternate over two streams with their own frame buffers, so one view's forward
    overlaps the previous view's backward; the backward passes, which all add into the
    same gradient arrays, are kept in order by events."""
    import numpy as np
    import torch

    W, H = cams[0].width, cams[0].height
    S = 2
    rends = [render.Renderer(ds, W, H, capacity=4 * ds.n, cache=False, keep_state=True) for _ in range(S)]
    streams = [torch.cuda.Stream() for _ in range(S)]
    grads = render.grads_like(ds)
    dL = torch.from_numpy(inputs.upstream_grad(7, W, H)).cuda()
    views = bwd_views(args, cams)
    bwd_done = [torch.cuda.Event() for _ in range(len(views) + 2)]

    def run(vs):
        prev = None
        for i, (cam, t) in enumerate(vs):
            r = i % S
            with torch.cuda.stream(streams[r]):
                rends[r].render(cam, t)
                if prev is not None:
                    streams[r].wait_event(prev)
                rends[r].backward(cam, t, dL, grads)
                ev = bwd_done[i]
                ev.record(streams[r])
                prev = ev

    run(views[:2])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(views)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    assert not any(r.overflowed() for r in rends)
    return {"frames_per_s": round(len(views) / el, 2), "ms_per_frame": round(1000 * el / len(views), 4),
            "frames": len(views), "camera_cache": False, "streams": S}


def bwd_views(args, cams):
    import numpy as np

    return [(cams[(3 * i) % len(cams)], np.float32((i % 10) / 9.0)) for i in range(args.bwd_frames)]


def bwd_kernel_pass(args, ds, cams, render, inputs):
    """The backward's two kernels timed on one stream (each alone on the GPU): every view
    rendered with its replay state, then d4dgs_render_bwd_timed, whose events mark the
    kernels' own start and end.  Returns their average durations in ms."""
    import torch

    W, H = cams[0].width, cams[0].height
    rend = render.Renderer(ds, W, H, capacity=4 * ds.n, cache=False, keep_state=True)
    grads = render.grads_like(ds)
    dL = torch.from_numpy(inputs.upstream_grad(7, W, H)).cuda()
    views = bwd_views(args, cams)
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in views]
    for ev in events:
        for e in ev:
            e.record()
    for cam, t in views[:2]:
        rend.render(cam, t)
        rend.backward(cam, t, dL, grads)
    torch.cuda.synchronize()
    for (cam, t), ev in zip(views, events):
        rend.render(cam, t)
        rend.backward(cam, t, dL, grads, events=ev)
    torch.cuda.synchronize()
    assert not rend.overflowed()
    bb = [ev[0].elapsed_time(ev[1]) for ev in events]
    pb = [ev[2].elapsed_time(ev[3]) for ev in events]
    return sum(bb) / len(bb), sum(pb) / len(pb)


def side_sweeps(args, ds, cams, times, render, ds_drawn):
    """The headline sweep with the camera-stage cache off (the camera stage then runs for
    every frame), one camera's 300 frames alone (camera 10: the analogue of a fixed test
    view's video), and the headline sweep on the scene in its drawn order (not spatially
    ordered), all on the sweep's streams."""
    import types

    S = max(1, args.streams)
    off = types.SimpleNamespace(warmup=2, steps=len(cams))
    el, _, _ = sweep(off, ds, cams, times, render, S, False, args.tile_order, cache=False)
    one = types.SimpleNamespace(warmup=2, steps=1)
    el1, _, _ = sweep(one, ds, [cams[10]], times, render, S, False, args.tile_order)
    eld, _, _ = sweep(off, ds_drawn, cams, times, render, S, False, args.tile_order)
    return {"cache_off_frames_per_s": round(len(cams) * len(times) / el, 2),
            "camera10_frames_per_s": round(len(times) / el1, 2),
            "drawn_order_frames_per_s": round(len(cams) * len(times) / eld, 2)}


def view_steps(inputs, render, which=("c3", "c5")):
    """Forward + backward steps of the two training-style workloads, on two streams as in
    the forward + backward phase (one view's forward overlaps the previous view's
    backward; the backward passes add into one set of gradients in order):
    8 views at 800x800 of 100k Gaussians (SH1), and 4 views at 2704x2028 of 2M Gaussians
    (SH3), with the step's peak device memory beyond the resident scene."""
    import numpy as np
    import torch

    out = {}
    for name in ("c3_8x800x800_100k", "c5_4x2704x2028_2M"):
        if name[:2] not in which:
            continue
        if name.startswith("c3"):
            sc, views, _ = inputs.fit_case()
        else:
            sc, views = inputs.large_scene(), inputs.large_views()
        ds = render.DeviceScene.from_inputs(sc)
        scene_bytes = sum(x.numel() * x.element_size() for x in ds.t.values())
        del sc
        W, H = views[0][0].width, views[0][0].height
        # instance capacity: 1.25 x the most any view needs (a sizing pass, untimed)
        probe = render.Renderer(ds, W, H, cache=False)
        most = 0
        for cam, t in views:
            probe.project_bin(cam, t)
            most = max(most, int(probe.st.num_inst.item()))
        assert not probe.overflowed()
        del probe
        cap = int(1.25 * most) + 1024
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        base = torch.cuda.memory_allocated()
        torch.cuda.reset_peak_memory_stats()
        rends = [render.Renderer(ds, W, H, capacity=cap, cache=False, keep_state=True) for _ in range(2)]
        streams = [torch.cuda.Stream() for _ in range(2)]
        grads = render.grads_like(ds)
        dL = torch.from_numpy(inputs.upstream_grad(11, W, H)).cuda()

        def step():
            prev = None
            for i, (cam, t) in enumerate(views):
                r = i % 2
                with torch.cuda.stream(streams[r]):
                    rends[r].render(cam, t)
                    if prev is not None:
                        streams[r].wait_event(prev)
                    rends[r].backward(cam, t, dL, grads)
                    prev = torch.cuda.Event()
                    prev.record(streams[r])

        step()
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            step()
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        assert not any(r.overflowed() for r in rends)
        out[name] = {"views": len(views), "ms_per_step": round(1e3 * el, 3),
                     "views_per_s": round(len(views) / el, 1),
                     "peak_step_bytes": int(torch.cuda.max_memory_allocated() - base),
                     "scene_bytes": int(scene_bytes)}
        del rends, grads, ds, dL
        torch.cuda.empty_cache()
    return out


def times_batch(args, ds, cams, render):
    """Fixed-viewpoint multi-timestamp rendering (d4dgs_render_times) at camera 10: wall
    time per call of T frames, and the marginal cost and device memory of one more frame
    (the paper's parallel-frame measurement)."""
    import numpy as np
    import torch

    W, H = cams[0].width, cams[0].height
    cam = cams[10]
    Ts, ms = [], []
    frame_bytes = None
    for T in (1, 2, 4, 8, 16, 32):
        tr = render.TimesRenderer(ds, W, H, T, capacity=4 * ds.n, cache=True)
        times = [np.float32((k + 0.5) / T) for k in range(T)]
        for _ in range(2):
            tr.render(cam, times)
        torch.cuda.synchronize()
        reps = max(4, 128 // T)
        t0 = time.perf_counter()
        for _ in range(reps):
            tr.render(cam, times)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        assert not tr.overflowed()
        Ts.append(T)
        ms.append(1000.0 * el / reps)
        if frame_bytes is None:
            f = tr.frames[0]
            frame_bytes = sum(x.numel() * x.element_size() for x in
                              (f.rec, f.count, f.offset, f.partial, f.keys, f.values, f.ranges, f.ws, tr.imgs[0]))
        del tr
    slope = float(np.polyfit(np.array(Ts, float), np.array(ms), 1)[0])
    return {"camera": 10, "T": Ts, "ms_per_call": [round(x, 4) for x in ms],
            "frames_per_s": [round(T / (m * 1e-3), 1) for T, m in zip(Ts, ms)],
            "ms_per_extra_frame": round(slope, 4), "device_bytes_per_frame": int(frame_bytes)}


def cpu_baseline(args, scene, cams, times):
    """The oracle (plain C + OpenMP, FP32 decisions / FP64 blend) on a bounded sample of
    the timed frames, on all host threads and on one; also returns the oracle's count of
    blend evaluations per frame and, over a sample of the backward phase's views, the
    units of the two adjoint kernels (evaluations up to each pixel's last contributor;
    drawn Gaussians and tile instances)."""
    import numpy as np

    import oracle

    oracle.build(force=False)
    n = args.cpu_frames
    # frame j: camera j mod 20 at time index 37 j mod 300 -- spread over the whole sweep
    sample = [(cams[j % len(cams)], times[(37 * j) % len(times)]) for j in range(n)]
    oracle.set_threads(0)
    evals = []
    t0 = time.perf_counter()
    for cam, t in sample:
        _, _, res = oracle.render(scene, cam, t)
        evals.append(res["n_eval"])
    el = time.perf_counter() - t0
    cores = oracle.num_threads()
    n1 = max(1, args.cpu_frames_1core)
    oracle.set_threads(1)
    t1 = time.perf_counter()
    for cam, t in sample[:n1]:
        oracle.render(scene, cam, t)
    el1 = time.perf_counter() - t1
    oracle.set_threads(0)
    base = {"value": round(n / el, 4), "unit": "frames/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} frames of the timed sweep (frame j: camera j mod {len(cams)}, time index "
                      f"37 j mod {len(times)}); project + bin + blend per frame, {el:.1f} s",
            "cpu": cpu_model(), "host_cpus": os.cpu_count(),
            "one_core": {"value": round(n1 / el1, 4), "unit": "frames/s", "cores": 1,
                         "sample": f"the first {n1} frames of the same sample, {el1:.1f} s"}}
    bw = {"evals": [], "drawn": [], "instances": []}
    for cam, t in bwd_views(args, cams)[:args.bwd_oracle_views]:
        proj, bins, res = oracle.render(scene, cam, t)
        bw["evals"].append(int(res["n_contrib"].astype(np.int64).sum()))
        bw["drawn"].append(int((proj["count"] > 0).sum()))
        bw["instances"].append(int(bins["I"]))
    bw = {k: sum(v) / len(v) for k, v in bw.items()}
    return base, sum(evals) / len(evals), bw


def blend_roofline(mean_evals, blend_ms):
    """The dominant kernel's roofline.  achieved: the algorithmic work of Eq. 4 (the
    oracle's evaluation count x 22 flops) over the blend's live-timed duration -- an
    effective rate, since the kernel skips the evaluations that cannot reach 1/255.
    executed: the VALU instructions the kernel issues per launch (committed SQ_INSTS_VALU
    summary, null once the blend's sources change) as a share of the SIMDs' issue slots
    over the same duration -- what the hardware does."""
    sec = blend_ms * 1e-3
    achieved = mean_evals * FLOPS_PER_EVAL / sec / 1e12
    kv = counter_summary(TRAFFIC_SUMMARY, BLEND_SOURCES)
    insts = _num(kv, "sq_insts_valu_per_launch")
    ifr = issue_frac(insts, sec)
    return {"bound": "alu", "kernel": "k_blend", "achieved": round(achieved, 3), "peak": ALU_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / ALU_PEAK_TFLOPS, 4), "traffic": blend_traffic(),
            "basis": "effective: oracle-counted (pixel, list entry) evaluations x 22 flops per live-timed launch",
            "evals_per_frame": int(mean_evals), "flops_per_eval": FLOPS_PER_EVAL,
            "peak_nonpacked": ALU_PEAK_NONPACKED_TFLOPS,
            "frac_nonpacked": round(achieved / ALU_PEAK_NONPACKED_TFLOPS, 4),
            "executed": {"valu_insts_per_launch": insts, "issue_frac": None if ifr is None else round(ifr, 4),
                         "source": os.path.relpath(TRAFFIC_SUMMARY, ROOT)}}


def sweep_issue(frames_per_s):
    """The whole frame against the chip's vector issue rate: the VALU wave instructions of
    one sweep frame, all five kernels (committed SQ_INSTS_VALU summary over 1200 frames of
    the 20-camera sweep; null once any of their sources change), times the measured frame
    rate, as a share of what 1,024 SIMDs issue at one wave64 instruction per 4 cycles.
    The four streams share the SIMDs, so a fraction near 1 means the sweep is bound by
    vector issue, not by memory or latency."""
    kv = counter_summary(SWEEP_SUMMARY, SWEEP_SOURCES)
    insts = _num(kv, "valu_insts_per_frame")
    ifr = None if insts is None else insts * frames_per_s * CYCLES_PER_VALU / (SIMDS * CLOCK_HZ)
    return {"bound": "valu issue", "valu_insts_per_frame": insts,
            "issue_floor_us_per_frame": None if insts is None else round(
                insts * CYCLES_PER_VALU / SIMDS / CLOCK_HZ * 1e6, 2),
            "issue_frac": None if ifr is None else round(ifr, 4),
            "source": os.path.relpath(SWEEP_SUMMARY, ROOT)}


def backward_rooflines(bw, bwd_ms, sh_degree):
    """Rooflines of the two adjoint kernels from the one-stream backward pass.
    k_blend_bwd (ALU): oracle-counted evaluations up to each pixel's last contributor x 46
    flops per live-timed launch, and its VALU issue share (committed SQ_INSTS_VALU).
    k_project_bwd (HBM): algorithmic bytes -- per drawn Gaussian its parameters read and its
    gradients read and written (3 x (16 + 3K) floats), per tile instance the 9 floats of
    its splat gradient -- per live-timed launch, against 8 TB/s; traffic from the
    committed FETCH_SIZE / WRITE_SIZE summary (null once the sources change)."""
    K = (sh_degree + 1) ** 2
    kv = counter_summary(BWD_SUMMARY, BWD_SOURCES)
    sb, sp = bwd_ms[0] * 1e-3, bwd_ms[1] * 1e-3
    ach = bw["evals"] * FLOPS_PER_BWD_EVAL / sb / 1e12
    insts = _num(kv, "k_blend_bwd_sq_insts_valu_per_launch")
    ifr = issue_frac(insts, sb)
    alg = bw["drawn"] * 3 * (16 + 3 * K) * 4 + bw["instances"] * 9 * 4
    gbs = alg / sp / 1e9
    return {"k_blend_bwd": {"bound": "alu", "achieved": round(ach, 3), "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                            "frac": round(ach / ALU_PEAK_TFLOPS, 4), "ms_avg": round(bwd_ms[0], 5),
                            "evals_per_launch": int(bw["evals"]), "flops_per_eval": FLOPS_PER_BWD_EVAL,
                            "executed": {"valu_insts_per_launch": insts,
                                         "issue_frac": None if ifr is None else round(ifr, 4)}},
            "k_project_bwd": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(gbs / HBM_PEAK_GBS, 4), "ms_avg": round(bwd_ms[1], 5),
                              "algorithmic_bytes": int(alg), "drawn_per_view": int(bw["drawn"]),
                              "instances_per_view": int(bw["instances"]),
                              "traffic": _num(kv, "k_project_bwd_hbm_bytes_per_launch")},
            "source": os.path.relpath(BWD_SUMMARY, ROOT)}


def progress(msg):
    """One line on stderr as each phase ends (stdout carries only the JSON line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


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
    if args.copy_calibration:
        copy_calibration()
    # the scene as drawn (Gaussians of all clusters interleaved), stored on the GPU in the
    # library's spatial order at load (untimed; its cost is reported)
    scene = inputs.clustered_scene(morton=False)
    ds_drawn = render.DeviceScene.from_inputs(scene)
    ds, order_ms = scene_order(render, ds_drawn)
    cams = inputs.arc_cameras()
    times = [np.float32(k / (args.frames - 1)) for k in range(args.frames)]
    W, H = cams[0].width, cams[0].height

    frames = args.steps * args.frames
    # the kernel pass: the sweep on one stream, every blend timed by HIP events attached to
    # its launch
    k_elapsed, blend_ms, _ = sweep(args, ds, cams, times, render, 1, True, True)
    progress(f"kernel pass done ({frames / k_elapsed:.0f} frames/s)")
    elapsed, _, t_host = sweep(args, ds, cams, times, render, max(1, args.streams), False, args.tile_order)
    progress(f"sweep done ({frames / elapsed:.0f} frames/s)")
    out = {
        "metric": "frames/sec @1352x1014, 300k Gaussians fwd/bwd; serving p50/p99 ms vs plain",
        "value": round(frames / elapsed, 2),
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
                               "camera-stage cache on", "frames_per_step": args.frames, "streams": args.streams,
                   "camera_cache": "one, shared by the streams (camera stage once per camera)",
                   "hip_hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4")),
                   "scene_order": "drawn order, reordered at load by d4dgs_spatial_order",
                   "tile_order": bool(args.tile_order),
                   "binning": "separate" if args.unfused else "fused",
                   "gaussians": scene.n, "width": W, "height": H},
        "scene_order_ms": round(order_ms, 3),
        "blend_ms_avg": round(blend_ms, 5),
        "kernel_pass": {"streams": 1, "tile_order": True, "frames": frames,
                        "frames_per_s": round(frames / k_elapsed, 2)},
        "host_enqueue_ms_per_frame": round(1000.0 * t_host / frames, 5),
    }
    bwd_ms = None
    if not args.no_bwd:
        out["fwd_bwd"] = fwd_bwd(args, ds, cams, render, inputs)
        bwd_ms = bwd_kernel_pass(args, ds, cams, render, inputs)
        out["fwd_bwd"]["bwd_kernel_pass"] = {"streams": 1, "views": args.bwd_frames,
                                             "k_blend_bwd_ms_avg": round(bwd_ms[0], 5),
                                             "k_project_bwd_ms_avg": round(bwd_ms[1], 5)}
        progress("forward + backward done")
    if not args.no_extras:
        out["sweep_extras"] = side_sweeps(args, ds, cams, times, render, ds_drawn)
        progress("side sweeps done")
    if not args.no_times:
        out["times_batch"] = times_batch(args, ds, cams, render)
        progress("multi-timestamp batches done")
    if not args.no_steps:
        out["view_steps"] = view_steps(inputs, render, args.view_steps.split(","))
        progress("view steps done")
    if not args.no_serve:
        try:
            from paper_2503_22159_amd import serve_bench

            rates = tuple(float(x) for x in args.serve_high_rates.split(",") if x.strip())
            out["serving"] = serve_bench.run(seconds=args.serve_seconds, high_rates=rates,
                                             high_seconds=args.serve_high_seconds)
            progress("serving done")
        except ImportError:
            out["serving"] = None
    if not args.no_cpu:
        base, mean_evals, bw = cpu_baseline(args, scene, cams, times)
        progress("CPU oracle done")
        out["cpu_baseline"] = base
        out["roofline"] = blend_roofline(mean_evals, blend_ms)
        out["roofline"]["sweep"] = sweep_issue(out["value"])
        if bwd_ms is not None:
            out["roofline"]["backward"] = backward_rooflines(bw, bwd_ms, scene.sh_degree)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
