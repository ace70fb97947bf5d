"""The configuration the benchmark's headline frames/s times, tested as it runs there.

The sweep renders the 300k-Gaussian SH3 scene at 1352x1014 through the fused
d4dgs_project_bin, without the tile order and without replay state, frames round-robin
over four streams, each stream with its own buffers, all sharing one camera-stage cache
(so every frame after a camera's first is a cache hit), ordered across the streams by
render.SharedCameraOrder.  Every frame here is compared bit for bit with
the separate calls (d4dgs_project + d4dgs_bin_sort, tile order on, replay state kept),
which the forward parity tests check against the oracle, and one frame of the sweep is
compared with the oracle directly."""
import numpy as np
import pytest

import oracle
from _helpers import compare_images
from paper_2503_22159_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_22159_amd import render

    sc = inputs.clustered_scene()
    return sc, render.DeviceScene.from_inputs(sc), render


def test_four_stream_sweep_matches_separate_path_and_oracle(env):
    import torch

    sc, ds, R = env
    cams = inputs.arc_cameras()
    times = inputs.sweep_times()
    which = [(j, k) for j in (3, 10) for k in (0, 41, 97, 150, 233, 299)]
    frames = [(cams[j], times[k]) for j, k in which]
    W, H = cams[0].width, cams[0].height
    S = 4
    cache = R.CamCache(ds.n)
    rends = [R.Renderer(ds, W, H, capacity=4 * ds.n, cache=cache, tile_order=False) for _ in range(S)]
    assert all(not r.keep_state for r in rends)
    streams = [torch.cuda.Stream() for _ in range(S)]
    order = R.SharedCameraOrder(streams)
    outs = [torch.empty((3, H, W), dtype=torch.float32, device="cuda") for _ in frames]
    for i, (cam, t) in enumerate(frames):
        r = i % S
        miss = i == 0 or cam is not frames[i - 1][0]
        with torch.cuda.stream(streams[r]):
            h = streams[r].cuda_stream
            order.before_miss(r) if miss else order.before_hit(r)
            rends[r].project_bin(cam, t, h)
            if miss:
                order.after_miss(r)
            img = rends[r].blend(stream=h)
            outs[i].copy_(img)
    torch.cuda.synchronize()
    assert not any(r.overflowed() for r in rends)
    assert cache.c.misses == 2 and cache.c.hits == len(frames) - 2  # one miss per camera
    for i, (cam, t) in enumerate(frames):
        ref, _ = R.render_forward(ds, cam, t)
        assert torch.equal(outs[i], ref), f"frame {i}: camera {which[i][0]}, time index {which[i][1]}"
    cam, t = frames[7]
    _, bins, res = oracle.render(sc, cam, t)
    stats = compare_images(outs[7].cpu().numpy(), None, None, res)
    assert stats["n_flagged"] < 1000, stats
