"""GPU parity of the time stage's alternative motion / covariance models
(D4DGS_MOTION_EXACT: the 2D mean is the exact projection of the moved mean;
D4DGS_MOTION_FROZEN_J: the Jacobian is taken at the camera stage's mean) against the
oracle run with the same model: the same bars as the default model (bit-exact records
and bins, images within 1e-4, gradients within 1e-3 relative)."""
import numpy as np
import pytest

import oracle
from _helpers import assert_bins_equal, assert_projection_equal, compare_images, decode_record, read_bins
from paper_2503_22159_amd import inputs
from test_gpu_backward import GROUPS, check_params, compare_group

pytestmark = pytest.mark.gpu
MODES = [1, 2]  # exact projection, frozen Jacobian


@pytest.fixture(scope="module")
def R():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_22159_amd import render

    return render


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("case", ["small_case", "clustered_subset"])
def test_forward_per_model(R, mode, case):
    import torch

    if case == "small_case":
        sc, cam, t = inputs.small_case()
    else:
        sc = inputs.clustered_scene(n=40_000)
        cam, t = inputs.arc_camera(9, width=337, height=253), np.float32(0.15)
    ds = R.DeviceScene.from_inputs(sc)
    img, st = R.render_forward(ds, cam, t, (0.1, 0.1, 0.1), motion=mode)
    torch.cuda.synchronize()
    with oracle.motion(mode):
        orc_p = oracle.project(sc, cam, t, "f32")
        ob = oracle.bin(orc_p, cam)
        res = oracle.blend(orc_p, ob, cam, (0.1, 0.1, 0.1))
    assert_projection_equal(decode_record(st, sc.n), orc_p)
    assert_bins_equal(read_bins(st), ob)
    compare_images(img.cpu().numpy(), st.final_T.cpu().numpy(), st.n_contrib.cpu().numpy().view(np.uint32), res)


@pytest.mark.parametrize("mode", MODES)
def test_gradients_per_model(R, mode):
    import torch

    sc, cam, t = inputs.small_case()
    ds = R.DeviceScene.from_inputs(sc)
    img, st = R.render_forward(ds, cam, t, motion=mode)
    with oracle.motion(mode):
        proj, bins, res = oracle.render(sc, cam, t)
        mask = res["flags"] > 0
        dL = inputs.upstream_grad(70 + mode, cam.width, cam.height) * (~mask)[None]
        gp_o, gs_o, _ = oracle.render_grad(sc, cam, t, dL.astype(np.float64))
    grads = R.render_backward(ds, cam, t, (0.0, 0.0, 0.0), st, torch.from_numpy(dL.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    errs = check_params({k: grads[k].cpu().numpy().astype(np.float64) for k in GROUPS}, gp_o)
    print("motion", mode, errs)


def test_flow_under_exact_projection(R):
    """The flow velocity is dm/dt of the exact projection; flow image and the gradients of
    image + flow upstream terms against the oracle."""
    import torch

    sc, cam, t = inputs.small_case()
    ds = R.DeviceScene.from_inputs(sc)
    img, flow, st = R.render_forward_flow(ds, cam, t, motion=1)
    torch.cuda.synchronize()
    with oracle.motion(1):
        proj, bins, res = oracle.render(sc, cam, t, flow=True)
        mask = res["flags"] > 0
        dL = inputs.upstream_grad(81, cam.width, cam.height) * (~mask)[None]
        dF = inputs.upstream_grad(82, cam.width, cam.height)[:2] * (~mask)[None]
        gp_o, gs_o, _ = oracle.render_grad(sc, cam, t, dL.astype(np.float64), dL_dflow=dF.astype(np.float64))
    act = proj["count"] > 0
    md_gpu = st.mdot.view(-1, 2).cpu().numpy().T
    np.testing.assert_allclose(md_gpu[:, act], proj["mdt"][:, act], rtol=2e-6, atol=2e-6)
    flagged = (res["flags"] & 7) > 0
    scale = max(1.0, float(np.abs(proj["mdt"][:, act]).max()))
    d = np.abs(flow.cpu().numpy().astype(np.float64) - res["flow"]).max(axis=0)
    assert d[~flagged].max() <= 1e-4 * scale
    grads = R.render_backward(ds, cam, t, (0.0, 0.0, 0.0), st, torch.from_numpy(dL.astype(np.float32)).cuda(),
                              dL_dflow=torch.from_numpy(dF.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    check_params({k: grads[k].cpu().numpy().astype(np.float64) for k in GROUPS}, gp_o)
