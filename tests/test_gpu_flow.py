"""GPU parity of the optical flow (Sec. 3.3), the flow-gradient guided consistency loss
(Eq. 16-17) and the adjoint with a flow upstream gradient, against the CPU oracle.

Bars: flow within 1e-4 x max |mdot| on pixels without a near-threshold evaluation; the
loss within 1e-4 relative and dL/dflow within 1e-4 of its largest magnitude on the same
(GPU-rendered) inputs; parameter gradients within 1e-3 relative, as for the colour."""
import numpy as np
import pytest

import oracle
from _helpers import compare_images, decode_record
from paper_2503_22159_amd import inputs
from test_gpu_backward import GROUPS, check_params, compare_group

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_22159_amd import render

    return render


def _flow_frame(R, sc, cam, t, bg=(0.0, 0.0, 0.0)):
    import torch

    ds = R.DeviceScene.from_inputs(sc)
    img, flow, st = R.render_forward_flow(ds, cam, t, bg)
    torch.cuda.synchronize()
    return ds, img, flow, st


@pytest.mark.parametrize("case", ["small_case", "clustered_subset"])
def test_flow_render_matches_oracle(R, case):
    if case == "small_case":
        sc, cam, t = inputs.small_case()
    else:
        sc = inputs.clustered_scene(n=40_000)
        cam, t = inputs.arc_camera(5, width=337, height=253), np.float32(0.6)
    ds, img, flow, st = _flow_frame(R, sc, cam, t, bg=(0.1, 0.2, 0.3))
    proj, bins, res = oracle.render(sc, cam, t, (0.1, 0.2, 0.3), flow=True)
    compare_images(img.cpu().numpy(), st.final_T.cpu().numpy(), st.n_contrib.cpu().numpy().view(np.uint32), res)
    act = proj["count"] > 0
    md_gpu = st.mdot.view(-1, 2).cpu().numpy().T
    np.testing.assert_allclose(md_gpu[:, act], proj["mdt"][:, act], rtol=1e-6, atol=1e-6)
    flagged = (res["flags"] & 7) > 0
    scale = max(1.0, float(np.abs(proj["mdt"][:, act]).max()))
    d = np.abs(flow.cpu().numpy().astype(np.float64) - res["flow"]).max(axis=0)
    assert d[~flagged].max() <= 1e-4 * scale, (d[~flagged].max(), scale)


def test_flow_loss_matches_oracle(R):
    import torch

    sc = inputs.clustered_scene(n=40_000)
    cam, t = inputs.arc_camera(12, width=301, height=199), np.float32(0.4)
    ds, img, flow, st = _flow_frame(R, sc, cam, t)
    for lam, eps in ((0.1, 1e-6), (2.0, 1e-2)):
        loss, dflow = R.flow_loss(img, flow, lam, eps)
        torch.cuda.synchronize()
        lo, do, info = oracle.flow_loss(img.cpu().numpy(), flow.cpu().numpy(), lam, eps)
        assert abs(float(loss.item()) - lo) <= 1e-4 * abs(lo), (float(loss.item()), lo)
        dg = dflow.cpu().numpy().astype(np.float64)
        assert np.abs(dg - do).max() <= 1e-4 * np.abs(do).max(), (np.abs(dg - do).max(), np.abs(do).max())


@pytest.mark.parametrize("wh", [(2, 2), (3, 3), (5, 4), (40, 3)])
def test_flow_loss_small_images(R, wh):
    import torch

    W, H = wh
    rng = np.random.default_rng(W * 10 + H)
    img = torch.from_numpy(rng.uniform(size=(3, H, W)).astype(np.float32)).cuda()
    flow = torch.from_numpy(rng.normal(size=(2, H, W)).astype(np.float32)).cuda()
    loss, dflow = R.flow_loss(img, flow, 0.5, 1e-4)
    torch.cuda.synchronize()
    lo, do, _ = oracle.flow_loss(img.cpu().numpy(), flow.cpu().numpy(), 0.5, 1e-4)
    assert abs(float(loss.item()) - lo) <= 1e-5 * max(1.0, abs(lo))
    np.testing.assert_allclose(dflow.cpu().numpy(), do, rtol=1e-4, atol=1e-6 * max(1.0, np.abs(do).max()))


def test_flow_loss_flat_image_is_not_an_edge(R):
    """A flat image (Sobel sums exactly zero) has no edges: L = lambda for a flow whose
    magnitude has a uniform Sobel gradient."""
    import torch

    H, W = 20, 30
    y, x = np.mgrid[0:H, 0:W].astype(np.float32)
    img = torch.full((3, H, W), 0.5, device="cuda")
    flow = torch.from_numpy(np.stack([2.0 * x, np.zeros_like(x)])).cuda()
    loss, _ = R.flow_loss(img, flow, 0.7, 0.0)
    torch.cuda.synchronize()
    assert abs(float(loss.item()) - 0.7) <= 1e-6


def test_flow_backward_matches_oracle(R):
    """Parameter gradients of sum(dL_dimg * img) + sum(dL_dflow * flow): GPU adjoint vs the
    oracle's (blend adjoint with flow channels + complex-step projection adjoint)."""
    import torch

    sc, cam, t = inputs.small_case()
    ds, img, flow, st = _flow_frame(R, sc, cam, t)
    proj, bins, res = oracle.render(sc, cam, t, flow=True)
    mask = res["flags"] > 0
    dL = inputs.upstream_grad(41, cam.width, cam.height) * (~mask)[None]
    dF = inputs.upstream_grad(42, cam.width, cam.height)[:2] * (~mask)[None]
    grads = R.render_backward(ds, cam, t, (0.0, 0.0, 0.0), st, torch.from_numpy(dL.astype(np.float32)).cuda(),
                              dL_dflow=torch.from_numpy(dF.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    gp_o, gs_o, _ = oracle.render_grad(sc, cam, t, dL.astype(np.float64), dL_dflow=dF.astype(np.float64))
    g = {k: grads[k].cpu().numpy().astype(np.float64) for k in GROUPS}
    errs = check_params(g, gp_o)
    print("flow grads rel err", errs)
    # instance slots: per-Gaussian sums of the flow (mdot) gradients
    n = sc.n
    rec = decode_record(st, n)
    ig = st.inst_grads.view(-1, 12).cpu().numpy().astype(np.float64)
    off = st.offset[:n].cpu().numpy().view(np.uint32).astype(np.int64)
    cnt = rec["count"].astype(np.int64)
    sums = np.zeros((n, 12))
    for gi in np.nonzero(cnt)[0]:
        sums[gi] = ig[off[gi]:off[gi] + cnt[gi]].sum(axis=0)
    compare_group("mdt", sums[:, 9:11].T, gs_o["mdt"])


def test_autograd_flow_loss_chain(R):
    """render_with_flow -> flow_gradient_loss -> backward equals the direct calls."""
    import torch

    sc = inputs.fit_case(n=10_000)[0]
    cam = inputs.look_at((0.0, 2.0, -9.0), width=160, height=120)
    t = np.float32(0.3)
    params = {k: torch.from_numpy(np.ascontiguousarray(getattr(sc, k))).cuda().requires_grad_(True)
              for k in R.FIELDS}
    img, flow = R.render_with_flow(*[params[k] for k in R.FIELDS], cam=cam, t=t, sh_degree=sc.sh_degree)
    loss = R.flow_gradient_loss(img, flow, 0.25, 1e-6) + img.square().mean()
    loss.backward()
    torch.cuda.synchronize()
    ds = R.DeviceScene.from_inputs(sc)
    img2, flow2, st = R.render_forward_flow(ds, cam, t)
    lf, dflow = R.flow_loss(img2, flow2, 0.25, 1e-6)
    dimg = 2.0 * img2 / img2.numel()
    g = R.render_backward(ds, cam, t, (0.0, 0.0, 0.0), st, dimg, dL_dflow=dflow)
    torch.cuda.synchronize()
    for k in R.FIELDS:
        a, b = params[k].grad.cpu().numpy(), g[k].cpu().numpy()
        np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-7 * max(1e-12, np.abs(b).max()))
