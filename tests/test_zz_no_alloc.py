"""d4dgs_bin_sort_noalloc (the binning with its workspace in the library's static device
array) against d4dgs_bin_sort (a caller workspace), through the C ABI.

Each case projects once, then bins the same projection with both entry points (the
per-block sums that the binning consumes in place are restored in between) and compares
every output bit for bit: instance total, status word, keys, values, ranges, tile order
and per-Gaussian offsets.  The calls run in a row on one stream, each later case smaller
than the one before, so each reuses what the previous call left in the static array."""
import ctypes as C

import numpy as np
import pytest

from paper_2503_22159_amd import inputs

pytestmark = pytest.mark.gpu

OK, ERR_CAPACITY, ERR_OUT_OF_MEMORY = 0, 3, 2


@pytest.fixture(scope="module")
def env():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_22159_amd import binding, render

    return torch, binding, render


class Out:
    """Device buffers of one binning's outputs, pre-filled with a pattern."""

    def __init__(self, torch, B, n, tiles, cap):
        dev = "cuda"
        self.keys = torch.full((cap,), -1, dtype=torch.int64, device=dev)
        self.values = torch.full((cap,), -1, dtype=torch.int32, device=dev)
        self.ranges = torch.full((2 * tiles,), -1, dtype=torch.int32, device=dev)
        self.order = torch.full((tiles,), -1, dtype=torch.int32, device=dev)
        self.num = torch.full((1,), -1, dtype=torch.int64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        b = B.Bins()
        b.capacity = cap
        b.keys, b.values, b.ranges = self.keys.data_ptr(), self.values.data_ptr(), self.ranges.data_ptr()
        b.num_instances, b.order = self.num.data_ptr(), self.order.data_ptr()
        self.struct = b

    def host(self, offset):
        I = int(self.num.item())
        m = max(0, min(I, self.keys.numel()))
        return {"I": I, "status": int(self.status.item()), "keys": self.keys[:m].cpu().numpy(),
                "values": self.values[:m].cpu().numpy(), "ranges": self.ranges.cpu().numpy(),
                "order": np.sort(self.order.cpu().numpy()), "offset": offset.cpu().numpy()}


def bin_both(env, scene, cam, t, cap):
    torch, B, R = env
    ds = R.DeviceScene.from_inputs(scene)
    st = R.FrameState(ds.n, cam.width, cam.height, cap)
    R.project(ds, cam, t, st)
    tiles = cam.tiles
    partial = st.partial.clone()
    sp = st.splats()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    ref = Out(torch, B, ds.n, tiles, cap)
    print(f"noalloc case: n={ds.n} {cam.width}x{cam.height} capacity={cap}", flush=True)
    B.check(B.lib.d4dgs_bin_sort(C.byref(sp), ds.n, cam.width, cam.height, C.c_void_p(st.ws.data_ptr()),
                                 st.ws.numel(), C.byref(ref.struct), C.c_void_p(ref.status.data_ptr()), stream))
    a = ref.host(st.offset)
    st.partial.copy_(partial)
    st.offset.fill_(-7)
    new = Out(torch, B, ds.n, tiles, cap)
    B.check(B.lib.d4dgs_bin_sort_noalloc(C.byref(sp), ds.n, cam.width, cam.height, C.byref(new.struct),
                                         C.c_void_p(new.status.data_ptr()), stream))
    b = new.host(st.offset)
    torch.cuda.synchronize()
    return a, b


def assert_same(a, b):
    assert a["I"] == b["I"] and a["status"] == b["status"]
    for k in ("keys", "values", "ranges", "order", "offset"):
        assert np.array_equal(a[k], b[k]), k


def test_noalloc_matches_workspace_binning_on_calls_in_a_row(env):
    # 1: the benchmark's scene and frame size (300k Gaussians, 1352x1014)
    sc = inputs.clustered_scene()
    cams = inputs.arc_cameras()
    a, b = bin_both(env, sc, cams[10], np.float32(0.5), 4 * sc.n)
    assert a["status"] == OK and a["I"] > 100_000
    assert_same(a, b)
    # 2: smaller -- 2,000 Gaussians at 128x128
    sc2, cam2, t2 = inputs.small_case()
    a, b = bin_both(env, sc2, cam2, t2, 1 << 16)
    assert a["status"] == OK and 0 < a["I"] < 20_000
    assert_same(a, b)
    # 3: smaller capacity than the instances: both report the overflow alike
    a, b = bin_both(env, sc2, cam2, t2, 256)
    assert a["status"] == ERR_CAPACITY and a["I"] > 256
    assert_same(a, b)


def test_noalloc_rejects_sizes_beyond_the_static_scratch(env):
    torch, B, R = env
    bins = B.Bins()
    bins.capacity = (1 << 31) - 1  # 2^31 instances need 32 GiB of buckets
    sp = B.Splats()
    st = B.lib.d4dgs_bin_sort_noalloc(C.byref(sp), 1000, 1920, 1080, C.byref(bins), None, None)
    assert st == ERR_OUT_OF_MEMORY
    assert "static scratch" in B.last_error()
