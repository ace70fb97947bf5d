"""Serving measurement: a Poisson stream of render requests against one resident scene.

The request stream follows the serving workload: 500k Gaussians (the clustered scene's
distributions, SH3) resident on the GPU; arrivals at 200 requests/s for 60 s; each request
a camera on the radius-10 sphere, t ~ U[0, 1], resolution 640x480 / 1352x1014 / 1920x1080
with probabilities 0.5 / 0.3 / 0.2; at most 64 requests on the GPU, admitted by an 8 GiB
scratch budget.  The stream is replayed open-loop (each request is submitted at its
arrival time regardless of completions) through

  * the continuous-batching server (d4dgs_serve_*), and
  * the plain renderer: in arrival order, each request waits for its arrival time, then
    d4dgs_project_bin and d4dgs_render_fwd are called in the caller's thread on one
    stream and the thread waits for them to finish (one request at a time, FIFO).

The same two replay heavier streams (2,000 and 6,000 requests/s for 10 s by default; the
plain renderer's saturated rate is about 6,700 frames/s), where requests arrive while
others are on the GPU and batches form.  Latency = completion -
scheduled arrival (one monotonic clock).  A closed-loop burst of requests (all submitted
at once) measures the saturated throughput of both.
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
        _wait_until(t0_ns + int(at * 1e9))
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
    res = {"p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
           "mean_ms": round(float(lat.mean()), 3), "max_ms": round(float(lat.max()), 3),
           "frames_per_s": round(len(done) / span, 2), "requests": len(done),
           "mean_batch": round(float(bs.mean()), 2), "errors": int((st != 0).sum())}
    if all("submit_ns" in d for d in done):
        # where the time goes (p99 of each part): the submit call after the scheduled
        # arrival (the replaying thread's lateness), waiting for admission and launch, and
        # the request's own run until completion
        arr = np.array([t0_ns + int(at * 1e9) for at, _, _ in reqs], np.float64)
        sub = np.array([d["submit_ns"] for d in done], np.float64)
        sta = np.array([d["start_ns"] for d in done], np.float64)
        dn = np.array([d["done_ns"] for d in done], np.float64)
        res["p99_parts_ms"] = {"late_submit": round(float(np.percentile(sub - arr, 99)) / 1e6, 3),
                               "queued": round(float(np.percentile(sta - sub, 99)) / 1e6, 3),
                               "run": round(float(np.percentile(dn - sta, 99)) / 1e6, 3)}
    return res


def _burst(srv, reqs, outs):
    t0 = time.monotonic_ns()
    tks = [srv.submit(cam, t, outs[i % len(outs)][(cam.width, cam.height)]) for i, (_, cam, t) in enumerate(reqs)]
    done = [srv.wait(tk, timeout_s=60.0) for tk in tks]
    el = (max(d["done_ns"] for d in done) - t0) / 1e9
    return round(len(reqs) / el, 2)


def _wait_until(target_ns):
    while True:
        d = target_ns - time.monotonic_ns()
        if d <= 0:
            return
        time.sleep(min(d, 2_000_000) / 1e9 if d > 300_000 else 0)


def _plain_renderers(ds, render):
    """Fixed buffers per resolution of the stream (no camera cache: every request has its
    own camera)."""
    from . import inputs

    return {(w, h): render.Renderer(ds, w, h, capacity=4 * ds.n, cache=False) for (w, h) in inputs.RES_CHOICES}


def _replay_plain(rends, reqs, t0_ns):
    """Sequential plain renderer: returns each request's completion time (ns)."""
    import torch

    stream = torch.cuda.current_stream()
    ev = torch.cuda.Event()
    done_ns = []
    for at, cam, t in reqs:
        _wait_until(t0_ns + int(at * 1e9))
        rends[(cam.width, cam.height)].render(cam, t)
        ev.record(stream)
        while not ev.query():  # poll: a blocking wait adds the runtime's wake-up latency
            pass
        done_ns.append(time.monotonic_ns())
    return done_ns


def _plain_summary(reqs, done_ns, t0_ns, rends):
    done = [{"done_ns": d, "batch_size": 1, "status": 0} for d in done_ns]
    res = _summary(reqs, done, t0_ns)
    res["errors"] = sum(int(r.overflowed()) for r in rends.values())  # any capacity overflow
    return res


def _plain_burst(rends, reqs):
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _, cam, t in reqs:
        rends[(cam.width, cam.height)].render(cam, t)
    torch.cuda.synchronize()
    return round(len(reqs) / (time.perf_counter() - t0), 2)


def _serve_and_plain(ds, render, Server, reqs, outs, burst):
    res = {}
    with Server(ds, max_inflight=64, max_batch=16, budget_bytes=8 << 30, n_streams=4) as srv:
        _burst(srv, reqs[:16], outs)  # warm-up
        t0 = time.monotonic_ns() + 20_000_000
        done = _replay(srv, reqs, outs, t0)
        res["server"] = _summary(reqs, done, t0)
        res["server"]["burst_frames_per_s"] = _burst(srv, reqs[:burst], outs)
        st = srv.stats()
        res["server"]["arena_peak_bytes"] = st["arena_peak_bytes"]
        res["server"]["retried"] = st["retried"]  # overflowed requests rendered again
    print(f"serving: server replay done ({len(reqs)} requests)", file=sys.stderr, flush=True)
    rends = _plain_renderers(ds, render)
    _plain_burst(rends, reqs[:16])  # warm-up
    t0 = time.monotonic_ns() + 20_000_000
    done_ns = _replay_plain(rends, reqs, t0)
    res["plain"] = _plain_summary(reqs, done_ns, t0, rends)
    res["plain"]["burst_frames_per_s"] = _plain_burst(rends, reqs[:burst])
    print(f"serving: plain replay done ({len(reqs)} requests)", file=sys.stderr, flush=True)
    return res


def run(seconds=60.0, rate=200.0, n=500_000, burst=64, seed=1004, high_rates=(2000.0, 6000.0), high_seconds=10.0):
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
                       f"<=64 in flight, 8 GiB scratch",
           "plain_renderer": "direct d4dgs_project_bin + d4dgs_render_fwd calls in the caller's thread, "
                             "one request at a time"}
    res.update(_serve_and_plain(ds, render, Server, reqs, outs, burst))
    for k, hr in enumerate(high_rates if high_seconds else ()):
        hreqs = inputs.serving_requests(rate=hr, duration=high_seconds, seed=seed + 1 + k)
        res[f"load_{hr:g}_per_s"] = dict(
            workload=f"Poisson {hr:g} req/s for {high_seconds:g} s ({len(hreqs)} requests), same mix",
            **_serve_and_plain(ds, render, Server, hreqs, outs, burst))
    torch.cuda.synchronize()
    return res
