"""Serving measurement: a Poisson stream of render requests against one resident scene.

The request stream follows the serving workload: 500k Gaussians (the clustered scene's distributions,
SH3) resident on the GPU; arrivals at 200 requests/s; each request a camera on the
radius-10 sphere, t ~ U[0, 1], resolution 640x480 / 1352x1014 / 1920x1080 with
probabilities 0.5 / 0.3 / 0.2; at most 64 requests on the GPU, admitted by an 8 GiB
scratch budget.  The stream is replayed open-loop (each request is submitted at its
arrival time regardless of completions) through

  * the continuous-batching server, and
  * the plain renderer: the same kernels, one request at a time on one stream.

Latency = completion - scheduled arrival (one monotonic clock).  A closed-loop burst of
requests (all submitted at once) measures the saturated throughput of both.
"""
from __future__ import annotations

import sys
import threading
import time

import numpy as np


def _replay(srv, reqs, outs, t0_ns):
    """Submit each request at its arrival time; a collector thread waits in order."""
    tickets = [None] * len(reqs)
    done = [None] * len(reqs)
    err = []

    def collect():
        try:
            for i in range(len(reqs)):
                while tickets[i] is None:
                    time.sleep(0.0002)
                done[i] = srv.wait(tickets[i], timeout_s=60.0)
        except Exception as e:  # surfaced below
            err.append(e)

    th = threading.Thread(target=collect)
    th.start()
    for i, (at, cam, t) in enumerate(reqs):
        target = t0_ns + int(at * 1e9)
        while True:
            d = target - time.monotonic_ns()
            if d <= 0:
                break
            time.sleep(min(d, 2_000_000) / 1e9 if d > 300_000 else 0)
        tickets[i] = srv.submit(cam, t, outs[i % len(outs)][(cam.width, cam.height)])
    th.join()
    if err:
        raise err[0]
    return done


def _summary(reqs, done, t0_ns):
    lat = np.array([(d["done_ns"] - (t0_ns + int(at * 1e9))) / 1e6 for (at, _, _), d in zip(reqs, done)])
    span = (max(d["done_ns"] for d in done) - t0_ns) / 1e9
    bs = np.array([d["batch_size"] for d in done])
    st = np.array([d["status"] for d in done])
    return {"p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_ms": round(float(lat.mean()), 3), "max_ms": round(float(lat.max()), 3),
            "frames_per_s": round(len(done) / span, 2), "requests": len(done),
            "mean_batch": round(float(bs.mean()), 2), "errors": int((st != 0).sum())}


def _burst(srv, reqs, outs):
    t0 = time.monotonic_ns()
    tks = [srv.submit(cam, t, outs[i % len(outs)][(cam.width, cam.height)]) for i, (_, cam, t) in enumerate(reqs)]
    done = [srv.wait(tk, timeout_s=60.0) for tk in tks]
    el = (max(d["done_ns"] for d in done) - t0) / 1e9
    return round(len(reqs) / el, 2)


def run(seconds=10.0, rate=200.0, n=500_000, burst=64, seed=1004):
    import torch

    from . import inputs, render
    from .serve import Server

    scene = inputs.serving_scene(n=n)
    ds = render.DeviceScene.from_inputs(scene)
    reqs = inputs.serving_requests(rate=rate, duration=seconds, seed=seed)
    ring = 128
    outs = [{(w, h): torch.empty((3, h, w), dtype=torch.float32, device="cuda") for (w, h) in inputs.RES_CHOICES}
            for _ in range(ring)]
    res = {"workload": f"500k Gaussians SH3 resident, Poisson {rate:g} req/s for {seconds:g} s "
                       f"({len(reqs)} requests), 640x480/1352x1014/1920x1080 @ 0.5/0.3/0.2, "
                       f"<=64 in flight, 8 GiB scratch"}
    with Server(ds, max_inflight=64, max_batch=16, budget_bytes=8 << 30, n_streams=4) as srv:
        _burst(srv, reqs[:16], outs)  # warm-up
        t0 = time.monotonic_ns() + 20_000_000
        done = _replay(srv, reqs, outs, t0)
        res["server"] = _summary(reqs, done, t0)
        res["server"]["burst_frames_per_s"] = _burst(srv, reqs[:burst], outs)
        res["server"]["arena_peak_bytes"] = srv.stats()["arena_peak_bytes"]
    print(f"serving: server replay done ({len(reqs)} requests)", file=sys.stderr, flush=True)
    with Server.plain(ds) as srv:
        _burst(srv, reqs[:16], outs)
        t0 = time.monotonic_ns() + 20_000_000
        done = _replay(srv, reqs, outs, t0)
        res["plain"] = _summary(reqs, done, t0)
        res["plain"]["burst_frames_per_s"] = _burst(srv, reqs[:burst], outs)
    torch.cuda.synchronize()
    return res
