"""GPU tests of d4dgs_project_bin, the projection that also runs the binning's count
pass, against d4dgs_project + d4dgs_bin_sort (bit for bit: splat records, counts,
offsets, block offsets, sorted keys and values, ranges, image and replay state; the
tile order up to the order inside one length step, which is unspecified) and, on one
frame, against the oracle's binning.  Cases: spatially coherent blocks (grouped
counting), a scene stored in random order (every block's rectangle spans the image:
per-instance counting), camera-cache hits and misses, an instance overflow followed by
a frame that fits (the tile counters must come back to zero), an empty scene, separate
and fused calls alternating on one workspace, and a workspace whose counters were not
initialised (reported, nothing written outside the bins)."""
import numpy as np
import pytest

import oracle
from _helpers import assert_bins_equal, decode_record, read_bins
from paper_2503_22159_amd import inputs

pytestmark = pytest.mark.gpu

BG = (0.2, 0.1, 0.3)


@pytest.fixture(scope="module")
def R():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_22159_amd import render

    return render


def frame_arrays(r):
    """Everything a frame writes, as numpy arrays (bit patterns)."""
    import torch

    torch.cuda.synchronize()
    st = r.st
    n = st.n
    count = st.count[:n].cpu().numpy().view(np.uint32)
    rec = st.rec[:n * 12].cpu().numpy().view(np.uint32).reshape(n, 12)
    out = {"count": count, "rec": rec[count > 0], "num_inst": int(st.num_inst.item()),
           "status": int(st.status.item()), "ranges": st.ranges.cpu().numpy().view(np.uint32)}
    if out["status"] == 0:
        b = read_bins(st)
        out.update(keys=b["keys"], values=b["values"], offset=st.offset[:n].cpu().numpy().view(np.uint32),
                   partial=st.partial.cpu().numpy().view(np.uint32), order=st.order.cpu().numpy().view(np.uint32),
                   img=r.img.cpu().numpy().view(np.uint32), final_T=st.final_T.cpu().numpy().view(np.uint32),
                   n_contrib=st.n_contrib.cpu().numpy().view(np.uint32))
    return out


def order_keys(order, ranges, tx):
    """The tile order's sort key at each position: (row class, length step, longest
    first); inside a step the order is whatever the LDS atomics gave."""
    r = ranges.reshape(-1, 2)
    ln = (r[order, 1] - r[order, 0]).astype(np.int64)
    return ((order // tx) % 8) * 256 + (255 - np.minimum(ln >> 3, 255))


def assert_same(a, b, tx):
    assert a.keys() == b.keys()
    if "order" in a:
        assert np.array_equal(np.sort(a["order"]), np.sort(b["order"]))
        assert np.array_equal(order_keys(a["order"], a["ranges"], tx), order_keys(b["order"], b["ranges"], tx))
        a = {k: v for k, v in a.items() if k != "order"}
        b = {k: v for k, v in b.items() if k != "order"}
    for k in a:
        if isinstance(a[k], np.ndarray):
            assert a[k].shape == b[k].shape, k
            bad = np.nonzero(a[k] != b[k])
            assert bad[0].size == 0, (k, bad[0][:8])
        else:
            assert a[k] == b[k], (k, a[k], b[k])


def renderers(R, sc, width, height, capacity=None, cache=True):
    ds = R.DeviceScene.from_inputs(sc)
    fused = R.Renderer(ds, width, height, capacity=capacity, cache=cache, keep_state=True)
    sep = R.Renderer(ds, width, height, capacity=capacity, cache=cache, keep_state=True)
    return ds, fused, sep


def run_both(fused, sep, cam, t):
    fused.project_bin(cam, t)
    fused.blend(BG)
    sep.project(cam, t)
    sep.bin_sort()
    sep.blend(BG)
    a, b = frame_arrays(fused), frame_arrays(sep)
    assert_same(a, b, (cam.width + 15) // 16)
    return a


@pytest.mark.parametrize("cache", [True, False])
def test_fused_equals_separate_clustered_subset(R, cache):
    sc = inputs.clustered_scene(n=30_000)
    cams = [inputs.arc_camera(j, width=320, height=240) for j in (3, 7)]
    ds, fused, sep = renderers(R, sc, 320, 240, cache=cache)
    # camera-cache miss, hits at other times, another camera (miss), back (miss)
    for cam, t in ((cams[0], 0.2), (cams[0], 0.7), (cams[1], 0.5), (cams[0], 0.5)):
        a = run_both(fused, sep, cam, np.float32(t))
        assert a["num_inst"] > 0
    if cache:
        assert fused.cache.c.hits == sep.cache.c.hits == 1


def test_fused_matches_oracle_binning(R):
    sc = inputs.clustered_scene(n=30_000)
    cam = inputs.arc_camera(3, width=320, height=240)
    t = np.float32(0.4)
    ds, fused, sep = renderers(R, sc, 320, 240)
    a = run_both(fused, sep, cam, t)
    gp = decode_record(fused.st, sc.n)
    assert_bins_equal(read_bins(fused.st), oracle.bin(oracle.project(sc, cam, t, "f32"), cam))
    assert a["num_inst"] == int(gp["count"].sum())


def test_fused_random_order_counts_per_instance(R):
    """Gaussians stored in random order: every block of 256 spreads over the whole
    1352 x 1014 image (more than 2048 tiles), so every instance takes the per-instance
    counter and the atomic cursor."""
    sc = inputs.make_scene(77, 20_000, 1, clusters=32, cluster_box=(-5.0, 5.0), log_scale=(-4.5, 0.6),
                           morton=False)
    cam = inputs.arc_camera(10)
    ds, fused, sep = renderers(R, sc, cam.width, cam.height)
    for t in (0.3, 0.6):
        assert run_both(fused, sep, cam, np.float32(t))["num_inst"] > 0


def test_fused_full_size_frame(R):
    sc = inputs.clustered_scene()
    cams = inputs.arc_cameras()
    ds, fused, sep = renderers(R, sc, cams[0].width, cams[0].height)
    for j, t in ((10, 0.5), (10, 0.9), (0, 0.1)):
        assert run_both(fused, sep, cams[j], np.float32(t))["num_inst"] > 0


def test_huge_splats_match_oracle_binning(R):
    """Splats covering up to the whole 640 x 480 image: a wavefront's 64 Gaussians own up
    to 50k tile instances, which the count and scatter passes deal out in hundreds of
    rounds of 64 (each instance's owner carried across rounds), with temporally culled
    Gaussians (no instances) in between; every tile's list exceeds 512 keys (the radix
    sort).  Lists, keys and ranges are compared with the oracle's binning."""
    sc = inputs.make_scene(91, 4000, 1, clusters=8, cluster_box=(-3.0, 3.0), cluster_std=1.0, log_scale=(0.0, 0.8))
    cam = inputs.arc_camera(4, width=640, height=480)
    t = np.float32(0.45)
    orc = oracle.bin(oracle.project(sc, cam, t, "f32"), cam)
    assert orc["I"] > 2_000_000
    ds, fused, sep = renderers(R, sc, cam.width, cam.height, capacity=orc["I"] + 1024)
    a = run_both(fused, sep, cam, t)
    assert a["status"] == 0 and a["num_inst"] == orc["I"]
    assert_bins_equal(read_bins(fused.st), orc)


def test_fused_large_image_scans_in_rounds(R):
    """2704 x 2028 has 21,463 tiles: the tile scan adds the counts up first, then scans
    in three rounds of 8,192."""
    sc = inputs.clustered_scene(n=30_000)
    cam, t = inputs.large_views()[1]
    ds, fused, sep = renderers(R, sc, cam.width, cam.height)
    assert run_both(fused, sep, cam, t)["num_inst"] > 0


def test_fused_overflow_then_a_frame_that_fits(R):
    from paper_2503_22159_amd import binding as B

    sc, cam, t = inputs.small_case()
    near = cam
    far = inputs.look_at((0.0, 0.0, -14.0), width=128, height=128, fovx_deg=60.0)
    i_near = oracle.bin(oracle.project(sc, near, t), near)["I"]
    i_far = oracle.bin(oracle.project(sc, far, t), far)["I"]
    assert i_far < i_near - 1
    ds, fused, sep = renderers(R, sc, 128, 128, capacity=i_near - 1, cache=False)
    a = run_both(fused, sep, near, t)
    assert a["status"] == B.ERR_CAPACITY and a["num_inst"] == i_near
    # the overflowing frame left the tile counters zero: the next frame is exact
    fused.st.status.zero_()
    sep.st.status.zero_()
    a = run_both(fused, sep, far, t)
    assert a["status"] == 0 and a["num_inst"] == i_far


def test_fused_empty_scene(R):
    import torch

    sc, cam, t = inputs.small_case()
    ds, fused, sep = renderers(R, sc.subset(np.arange(0)), cam.width, cam.height)
    fused.project_bin(cam, t)
    img = fused.blend(BG)
    torch.cuda.synchronize()
    assert int(fused.st.num_inst.item()) == 0
    assert np.array_equal(img.cpu().numpy(), np.broadcast_to(np.float32(BG)[:, None, None], img.shape))


def test_fused_and_separate_calls_share_a_workspace(R):
    """d4dgs_bin_sort leaves the counters zero too, so the calls can alternate."""
    sc = inputs.clustered_scene(n=30_000)
    cam = inputs.arc_camera(5, width=320, height=240)
    ds, mixed, ref = renderers(R, sc, 320, 240, cache=False)
    for k, t in enumerate((0.1, 0.4, 0.8, 0.3)):
        if k % 2:
            mixed.project_bin(cam, np.float32(t))
        else:
            mixed.project(cam, np.float32(t))
            mixed.bin_sort()
        mixed.blend(BG)
        ref.project(cam, np.float32(t))
        ref.bin_sort()
        ref.blend(BG)
        assert_same(frame_arrays(mixed), frame_arrays(ref), (cam.width + 15) // 16)


def test_uninitialised_workspace_is_reported(R):
    """Counters that were not zero when the count pass started: the tile counts do not
    add up to the instance total, so the status word reports INVALID_ARG and every range
    is empty (the image is the background); d4dgs_workspace_init makes the workspace
    usable again."""
    import ctypes as C

    import torch

    from paper_2503_22159_amd import binding as B

    sc = inputs.clustered_scene(n=30_000)
    cam = inputs.arc_camera(3, width=320, height=240)
    t = np.float32(0.4)
    ds, fused, sep = renderers(R, sc, 320, 240, cache=False)
    for fill in (1, 255):
        fused.st.ws.fill_(fill)
        fused.st.status.zero_()
        fused.project_bin(cam, t)
        img = fused.blend(BG)
        torch.cuda.synchronize()
        assert int(fused.st.status.item()) == B.ERR_INVALID_ARG
        assert not np.any(np.diff(fused.st.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2), axis=1))
        assert np.array_equal(img.cpu().numpy(), np.broadcast_to(np.float32(BG)[:, None, None], img.shape))
    st = fused.st
    B.check(B.lib.d4dgs_workspace_init(C.c_void_p(st.ws.data_ptr()), st.ws.numel(), st.n, 320, 240, st.capacity,
                                       R._stream()))
    st.status.zero_()
    assert run_both(fused, sep, cam, t)["status"] == 0
