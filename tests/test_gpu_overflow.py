"""Instance overflow: a frame whose tile instances exceed the bins' capacity renders only
the background, reports D4DGS_ERR_CAPACITY, and its adjoint adds nothing.

Before the frame, the offsets are set to 0 and the instance-gradient slots to 1.0, the
values a stale earlier frame could have left: if the adjoint summed any slot of such a
frame, gradients would be non-zero.  Both the separate calls (d4dgs_project +
d4dgs_bin_sort) and the fused d4dgs_project_bin are covered."""
import numpy as np
import pytest

from paper_2503_22159_amd import inputs

pytestmark = pytest.mark.gpu

ERR_CAPACITY = 3


@pytest.fixture(scope="module")
def R():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_22159_amd import render

    return render


def _stale(st, torch):
    st.offset.zero_()
    st.inst_grads = torch.ones(max(st.capacity, 1) * 12, dtype=torch.float32, device="cuda")


@pytest.mark.parametrize("fused", [False, True])
def test_overflowed_frame_has_zero_gradients(R, fused):
    import torch

    sc, cam, t = inputs.small_case()
    ds = R.DeviceScene.from_inputs(sc)
    bg = (0.25, 0.5, 0.75)
    cap = 64  # the small case has about 4,000 instances
    dL = torch.from_numpy(inputs.upstream_grad(3, cam.width, cam.height)).cuda()
    if fused:
        r = R.Renderer(ds, cam.width, cam.height, capacity=cap, cache=False, keep_state=True)
        _stale(r.st, torch)
        img = r.render(cam, t, bg)
        grads = R.grads_like(ds, split_stats=True)
        r.backward(cam, t, dL, grads, bg)
        st = r.st
    else:
        st = R.FrameState(ds.n, cam.width, cam.height, cap)
        _stale(st, torch)
        R.project(ds, cam, t, st)
        R.bin_sort(st)
        img = R.blend(st, bg, keep_state=True)
        grads = R.render_backward(ds, cam, t, bg, st, dL, grads=R.grads_like(ds, split_stats=True))
    torch.cuda.synchronize()
    assert int(st.status.item()) == ERR_CAPACITY
    assert int(st.num_inst.item()) > cap
    exp = torch.tensor(bg, dtype=torch.float32, device="cuda")[:, None, None].expand_as(img)
    assert torch.equal(img, exp)
    assert np.all(st.offset.cpu().numpy().view(np.uint32) == 0xFFFFFFFF)
    for k, g in grads.items():
        assert int(torch.count_nonzero(g).item()) == 0, k
