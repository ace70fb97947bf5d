"""GPU tests of the fixed-viewpoint multi-timestamp render (d4dgs_render_times): every
frame equals the single-frame path at its t bit for bit (records, bins and image), and
one frame is checked against the oracle."""
import numpy as np
import pytest

import oracle
from _helpers import assert_bins_equal, assert_projection_equal, compare_images, decode_record, read_bins
from paper_2503_22159_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_22159_amd import render

    return render


def _single(R, ds, cam, t, bg, cap):
    import torch

    img, st = R.render_forward(ds, cam, t, bg, capacity=cap, keep_state=False)
    torch.cuda.synchronize()
    return img.cpu().numpy(), st


@pytest.mark.parametrize("cache", [True, False])
def test_times_equal_single_frames(R, cache):
    """20 frames (two projection launches of up to 16) at one camera; then the same call
    again (a camera-cache hit when the cache is on)."""
    import torch

    sc = inputs.clustered_scene(n=40_000)
    cam = inputs.arc_camera(7, width=337, height=253)
    ds = R.DeviceScene.from_inputs(sc)
    times = [np.float32(k / 19.0) for k in range(20)]
    bg = (0.1, 0.2, 0.3)
    cap = 4 * sc.n
    tr = R.TimesRenderer(ds, cam.width, cam.height, len(times), capacity=cap, cache=cache)
    for rep in range(2):
        imgs = [im.cpu().numpy() for im in tr.render(cam, times, bg)]
        torch.cuda.synchronize()
        assert not tr.overflowed()
        for i, t in enumerate(times):
            ref, st = _single(R, ds, cam, t, bg, cap)
            fr = tr.frames[i]
            assert np.array_equal(fr.count.cpu().numpy(), st.count.cpu().numpy()), (rep, i)
            act = st.count.cpu().numpy() > 0
            a = fr.rec.view(-1, 12).cpu().numpy()[act].view(np.uint32)
            b = st.rec.view(-1, 12).cpu().numpy()[act].view(np.uint32)
            assert np.array_equal(a, b), (rep, i)
            assert_bins_equal(read_bins(fr), read_bins(st))
            assert np.array_equal(imgs[i].view(np.uint32), ref.view(np.uint32)), (rep, i)
    if cache:
        assert tr.cache.c.misses == 1 and tr.cache.c.hits == 1


def test_times_frame_against_oracle(R):
    import torch

    sc = inputs.clustered_scene(n=40_000)
    cam = inputs.arc_camera(3, width=301, height=211)
    ds = R.DeviceScene.from_inputs(sc)
    times = [np.float32(0.0), np.float32(0.35), np.float32(1.0)]
    tr = R.TimesRenderer(ds, cam.width, cam.height, len(times), capacity=4 * sc.n)
    imgs = tr.render(cam, times)
    torch.cuda.synchronize()
    for i, t in enumerate(times):
        fr = tr.frames[i]
        orc_p = oracle.project(sc, cam, t, "f32")
        assert_projection_equal(decode_record(fr, sc.n), orc_p, near=(sc, cam, t))
        ob = oracle.bin(orc_p, cam)
        assert_bins_equal(read_bins(fr), ob)
        res = oracle.blend(orc_p, ob, cam)
        flagged = (res["flags"] & 7) > 0
        d = np.abs(imgs[i].cpu().numpy().astype(np.float64) - res["img"]).max(axis=0)
        assert d[~flagged].max() <= 1e-4, (i, d[~flagged].max())


def test_times_capacity_overflow_is_flagged(R):
    import torch

    sc, cam, t = inputs.small_case()
    ds = R.DeviceScene.from_inputs(sc)
    tr = R.TimesRenderer(ds, cam.width, cam.height, 2, capacity=16, cache=False)
    imgs = tr.render(cam, [t, t], bg=(0.5, 0.25, 0.125))
    torch.cuda.synchronize()
    assert tr.overflowed()
    for im in imgs:
        assert np.array_equal(im.cpu().numpy(), np.broadcast_to(np.float32([0.5, 0.25, 0.125])[:, None, None],
                                                                 im.shape))
