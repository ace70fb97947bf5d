"""GPU parity of the forward render path against the CPU oracle (through the C ABI).

Bars: bit-exact tile counts, rectangles, depth keys, 2D means and conics (the FP
contract), sorted keys/values/ranges; images within 1e-4 max-abs except at pixels the
oracle flags as holding a near-threshold evaluation (<= 2e-2 there, count reported)."""
import numpy as np
import pytest

import oracle
from _helpers import (assert_bins_equal, assert_projection_equal, compare_images, decode_record, read_bins)
from paper_2503_22159_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_22159_amd import render

    return render


def gpu_frame(R, scene, cam, t, bg=(0.0, 0.0, 0.0), cache=None, capacity=None):
    ds = R.DeviceScene.from_inputs(scene)
    img, st = R.render_forward(ds, cam, t, bg, capacity=capacity, cache=cache)
    import torch

    torch.cuda.synchronize()
    return ds, img.cpu().numpy(), st


def check_frame(R, scene, cam, t, bg=(0.0, 0.0, 0.0)):
    ds, img, st = gpu_frame(R, scene, cam, t, bg)
    gp = decode_record(st, scene.n)
    orc_p = oracle.project(scene, cam, t, "f32")
    assert_projection_equal(gp, orc_p, near=(scene, cam, t))
    gb = read_bins(st)
    # stage isolation: the oracle bins the GPU's own splat record
    assert_bins_equal(gb, oracle.bin(gp, cam))
    ob = oracle.bin(orc_p, cam)
    assert_bins_equal(gb, ob)
    res = oracle.blend(orc_p, ob, cam, bg)
    stats = compare_images(img, st.final_T.cpu().numpy(), st.n_contrib.cpu().numpy().view(np.uint32), res)
    return stats


def test_small_case_end_to_end(R):
    sc, cam, t = inputs.small_case()
    stats = check_frame(R, sc, cam, t)
    print("small_case", stats)


@pytest.mark.parametrize("t", [0.0, 0.37, 1.0])
def test_small_case_times_and_background(R, t):
    sc, cam, _ = inputs.small_case()
    check_frame(R, sc, cam, np.float32(t), bg=(0.2, 0.5, 0.9))


@pytest.mark.parametrize("wh", [(1, 1), (17, 33), (100, 75), (257, 129)])
def test_ragged_sizes(R, wh):
    sc, _, t = inputs.small_case()
    cam = inputs.look_at((0.0, 0.0, -6.0), width=wh[0], height=wh[1])
    check_frame(R, sc, cam, t, bg=(0.1, 0.1, 0.1))


def test_c2_scene_several_tiles_subset(R):
    """Config-2 distributions (SH3), 40k Gaussians, a 337x253 view: many tiles, ragged
    tail, oracle in seconds."""
    sc = inputs.clustered_scene(n=40_000)
    cam = inputs.arc_camera(7, width=337, height=253)
    for t in (np.float32(0.0), np.float32(0.5)):
        check_frame(R, sc, cam, t)


def test_c2_full_size_frame(R):
    """300k Gaussians at 1352x1014 (the benchmark's frame), camera 10 of the arc, t = 0.5."""
    sc = inputs.clustered_scene()
    cam = inputs.arc_cameras()[10]
    stats = check_frame(R, sc, cam, np.float32(0.5))
    print("c2 full", stats)


def dense_scene(n, copies):
    """n large splats over a 48x48 view (9 tiles), so that every Gaussian lands in every
    tile, plus `copies` exact copies of some of them (equal depths, which must come out
    ordered by Gaussian index): every bucket holds n + copies keys."""
    base = inputs.make_scene(50 + n, n, 0, box=(-0.3, 0.3), log_scale=(0.5, 0.1),
                             t_scale_range=(0.5, 1.0), vel_std=0.0)
    rng = np.random.default_rng(n)
    sc = base.subset(np.concatenate([np.arange(n), rng.choice(n, copies, replace=False)]))
    return sc, inputs.look_at((0.0, 0.0, -6.0), width=48, height=48)


@pytest.mark.parametrize("n", [150, 300, 1200, 3000])
def test_dense_tiles_every_sort_path(R, n):
    """Buckets of ~1.2 n keys take each per-tile sort: chunks of 64 ranked and merged (up to
    512 keys), radix sort beyond."""
    sc, cam = dense_scene(n, n // 5)
    check_frame(R, sc, cam, np.float32(0.5), bg=(0.1, 0.2, 0.3))


@pytest.mark.parametrize("s", [1, 2, 63, 64, 65, 127, 128, 129, 192, 193, 255, 256, 257, 511, 512, 513])
def test_sort_path_boundaries(R, s):
    """Buckets of exactly s keys, at and around the limits of each sort path (ranking up
    to 64 keys, 2, 4 and 8 merged chunks, radix sort beyond 512) and of a chunk (64)."""
    copies = s // 5
    sc, cam = dense_scene(s - copies, copies)
    proj = oracle.project(sc, cam, 0.5)
    assert int((proj["count"] > 0).sum()) == sc.n and bool((proj["count"] == 9).all())
    check_frame(R, sc, cam, np.float32(0.5), bg=(0.1, 0.2, 0.3))


def test_opaque_splats_take_the_clamp_path(R):
    """Every other Gaussian nearly opaque: their alpha reaches the 0.99 clamp, so they take
    the blend's general per-splat path (positive-exponent skip and clamp evaluated) and
    share batches with plain splats."""
    sc, cam, t = inputs.small_case()
    sc = sc.subset(np.arange(sc.n))
    sc.opacity[::2] = np.float32(0.9995)
    sc.t_scale[::2] = np.float32(0.5)
    check_frame(R, sc, cam, t, bg=(0.2, 0.2, 0.2))


def test_empty_and_all_culled(R):
    sc, cam, t = inputs.small_case()
    empty = sc.subset(np.arange(0))
    ds, img, st = gpu_frame(R, empty, cam, t, bg=(0.3, 0.2, 0.1))
    assert np.array_equal(img, np.broadcast_to(np.float32([0.3, 0.2, 0.1])[:, None, None], img.shape))
    # every Gaussian far from its temporal mean: nothing survives
    far = sc.subset(np.arange(sc.n))
    far.t_scale[:] = np.float32(1e-4)
    ds, img, st = gpu_frame(R, far, cam, np.float32(5.0), bg=(0.3, 0.2, 0.1))
    assert int(st.num_inst.item()) == 0
    assert np.array_equal(img, np.broadcast_to(np.float32([0.3, 0.2, 0.1])[:, None, None], img.shape))


def test_capacity_overflow_is_reported_and_retried(R):
    import ctypes as C

    from paper_2503_22159_amd import binding as B

    sc, cam, t = inputs.small_case()
    orc = oracle.bin(oracle.project(sc, cam, t), cam)
    # async path: status word set, no out-of-bounds writes
    ds = R.DeviceScene.from_inputs(sc)
    st = R.FrameState(sc.n, cam.width, cam.height, orc["I"] - 1)
    R.project(ds, cam, t, st)
    R.bin_sort(st)
    assert int(st.status.item()) == B.ERR_CAPACITY
    assert int(st.num_inst.item()) == orc["I"]
    # sync path returns CAPACITY
    st = R.FrameState(sc.n, cam.width, cam.height, orc["I"] - 1)
    R.project(ds, cam, t, st)
    sp, bn = st.splats(), st.bins()
    ni = C.c_int64(0)
    r = B.lib.d4dgs_bin_sort_sync(C.byref(sp), st.n, st.width, st.height, C.c_void_p(st.ws.data_ptr()),
                                  st.ws.numel(), C.byref(bn), C.byref(ni), R._stream())
    assert r == B.ERR_CAPACITY and ni.value == orc["I"]
    # exact capacity works; render_forward grows a too-small capacity and matches
    ds, img, st = gpu_frame(R, sc, cam, t, capacity=orc["I"])
    assert_bins_equal(read_bins(st), orc)
    ds, img2, st = gpu_frame(R, sc, cam, t, capacity=16)
    assert np.array_equal(img, img2)


def test_deterministic_and_cache_equivalent(R):
    import torch

    sc = inputs.clustered_scene(n=30_000)
    cam = inputs.arc_camera(3, width=320, height=240)
    ds = R.DeviceScene.from_inputs(sc)
    cache = R.CamCache(sc.n)
    outs = []
    for use_cache in (None, cache, cache):  # no cache, cache miss, cache hit
        img, st = R.render_forward(ds, cam, np.float32(0.25), cache=use_cache)
        torch.cuda.synchronize()
        outs.append((img.cpu().numpy(), read_bins(st)))
    assert cache.c.hits == 1 and cache.c.misses == 1
    for img, b in outs[1:]:
        assert np.array_equal(img, outs[0][0])
        assert_bins_equal(b, outs[0][1])
    # camera record of the cache is bit-exact with the oracle's camera stage
    n = sc.n
    rec = cache.buf[: 19 * n].view(19, n).cpu().numpy()
    orc = oracle.project(sc, cam, np.float32(0.25), "f32")
    ok = orc["count"] > 0
    for name, rows in (("p", slice(0, 3)), ("u", slice(3, 6)), ("covc", slice(6, 12)), ("m0", slice(12, 14)),
                       ("md", slice(14, 16))):
        assert np.array_equal(rec[rows][:, ok].view(np.uint32), orc[name][:, ok].view(np.uint32)), name


def test_invalid_arguments_rejected(R):
    import ctypes as C

    from paper_2503_22159_amd import binding as B

    sc, cam, t = inputs.small_case()
    ds = R.DeviceScene.from_inputs(sc)
    st = R.FrameState(sc.n, cam.width, cam.height, 10000)
    bad = B.camera_struct(cam)
    bad.znear = 0.0
    r = B.lib.d4dgs_project(C.byref(ds.struct()), C.byref(bad), 0.5, None, C.byref(st.splats()), R._stream())
    assert r == B.ERR_INVALID_ARG and "znear" in B.last_error()
    s = ds.struct()
    s.sh_degree = 4
    r = B.lib.d4dgs_project(C.byref(s), C.byref(B.camera_struct(cam)), 0.5, None, C.byref(st.splats()), R._stream())
    assert r == B.ERR_INVALID_ARG
    r = B.lib.d4dgs_bin_sort(C.byref(st.splats()), sc.n, cam.width, cam.height, C.c_void_p(st.ws.data_ptr()), 16,
                             C.byref(st.bins()), None, R._stream())
    assert r == B.ERR_OUT_OF_MEMORY


def test_timed_blend_matches_and_times_the_kernel(R):
    """d4dgs_render_fwd_timed writes what d4dgs_render_fwd writes and sets its events to
    the blend kernel's start and end (a positive duration); NULL events are rejected."""
    import ctypes as C

    import torch

    from paper_2503_22159_amd import binding as B

    sc = inputs.clustered_scene(n=30_000)
    cam = inputs.arc_camera(5, width=337, height=253)
    ds = R.DeviceScene.from_inputs(sc)
    rend = R.Renderer(ds, cam.width, cam.height, keep_state=True)
    rend.render(cam, np.float32(0.4), (0.1, 0.2, 0.3))
    torch.cuda.synchronize()
    ref = [rend.img.cpu().numpy(), rend.st.final_T.cpu().numpy(), rend.st.n_contrib.cpu().numpy()]
    for a in (rend.img, rend.st.final_T, rend.st.n_contrib):
        a.fill_(7)
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    ev[0].record()
    ev[1].record()
    rend.blend((0.1, 0.2, 0.3), events=ev)
    torch.cuda.synchronize()
    got = [rend.img.cpu().numpy(), rend.st.final_T.cpu().numpy(), rend.st.n_contrib.cpu().numpy()]
    for g, r in zip(got, ref):
        assert np.array_equal(g, r)
    ms = ev[0].elapsed_time(ev[1])
    assert 0.0 < ms < 100.0, ms
    r = B.lib.d4dgs_render_fwd_timed(C.byref(rend._sp), C.byref(rend._bn), cam.width, cam.height,
                                     C.byref(rend._bg((0.0, 0.0, 0.0))), rend._img, None, None, None, None,
                                     R._stream())
    assert r == B.ERR_INVALID_ARG and "event" in B.last_error()


def test_tile_order_is_longest_first_and_changes_nothing(R):
    """With a tile order the binning lists the tiles grouped by row mod 8 and, inside a
    group, longest list first (lengths in steps of 8); the per-tile kernels run in that
    order.  The sorted lists, the image, the replay state and the gradients are bitwise
    those of the row-order launch."""
    import torch

    sc = inputs.clustered_scene(n=40_000)
    cam = inputs.arc_camera(7, width=337, height=253)
    t = np.float32(0.5)
    ds = R.DeviceScene.from_inputs(sc)
    dL = torch.from_numpy(inputs.upstream_grad(5, cam.width, cam.height)).cuda()
    outs = []
    for use_order in (True, False):
        st = R.FrameState(sc.n, cam.width, cam.height, 400_000, tile_order=use_order)
        R.project(ds, cam, t, st)
        R.bin_sort(st)
        img = R.blend(st, (0.1, 0.2, 0.3), keep_state=True)
        g = R.render_backward(ds, cam, t, (0.1, 0.2, 0.3), st, dL)
        torch.cuda.synchronize()
        outs.append(([img.cpu().numpy(), st.final_T.cpu().numpy(), st.n_contrib.cpu().numpy()]
                     + [g[k].cpu().numpy() for k in sorted(g)], read_bins(st),
                     st.order.cpu().numpy().view(np.uint32) if use_order else None))
    for a, b in zip(outs[0][0], outs[1][0]):
        assert np.array_equal(a, b)
    assert_bins_equal(outs[0][1], outs[1][1])
    order, bins = outs[0][2], outs[0][1]
    tiles = bins["ranges"].shape[0]
    assert np.array_equal(np.sort(order), np.arange(tiles))
    cnt = bins["ranges"][:, 1].astype(np.int64) - bins["ranges"][:, 0]
    TX = (cam.width + 15) // 16
    cls = (order // TX) % 8
    assert np.all(np.diff(cls) >= 0)
    for x in range(8):
        seg = order[cls == x]
        assert np.all(np.diff(np.minimum(cnt[seg] >> 3, 255)) <= 0)
