"""Pins of the oracle's optical flow and flow-gradient guided consistency loss (Sec. 3.3,
Eq. 16-17) against closed forms, special cases with known values and finite
differences.  CPU only."""
import math

import numpy as np
import pytest

from paper_2503_22159_amd import inputs
from test_oracle_pins import _fd_scene, _param_view, centre_cam, one_scene


# ------------------------------------------------------------------------------------ Sobel
def test_sobel_closed_forms(oracle_lib):
    """On the interior: ramp a x + b y + c -> (8a, 8b); x^2 -> (16 x, 0); x y -> (8 y, 8 x)
    (x = column, y = row, at the centre of the 3x3 window)."""
    H, W = 9, 12
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    gx, gy = oracle_lib.sobel(0.7 * x - 1.3 * y + 2.0)
    np.testing.assert_allclose(gx, 8 * 0.7, atol=1e-12)
    np.testing.assert_allclose(gy, -8 * 1.3, atol=1e-12)
    gx, gy = oracle_lib.sobel(x * x)
    np.testing.assert_allclose(gx, 16 * x[1:-1, 1:-1], atol=1e-12)
    np.testing.assert_allclose(gy, 0.0, atol=1e-12)
    gx, gy = oracle_lib.sobel(x * y)
    np.testing.assert_allclose(gx, 8 * y[1:-1, 1:-1], atol=1e-12)
    np.testing.assert_allclose(gy, 8 * x[1:-1, 1:-1], atol=1e-12)


# ------------------------------------------------------------------------------------- loss
def test_loss_zero_where_every_pixel_is_an_edge(oracle_lib):
    """An image whose gradient magnitude is the same at every interior pixel has
    normalised edge strength 1 everywhere: the loss and its gradient vanish."""
    H, W = 10, 13
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    img = np.stack([0.1 * x, -0.05 * x, 0.02 * x])
    rng = np.random.default_rng(0)
    loss, d, info = oracle_lib.flow_loss(img, rng.normal(size=(2, H, W)), 0.3, 1e-6)
    assert loss == pytest.approx(0.0, abs=1e-15)
    assert np.abs(d).max() < 1e-15


def test_loss_equals_lambda_for_uniform_flow_gradient_without_edges(oracle_lib):
    """Constant image (no edges) and u = c x, v = 0, eps = 0: M = c x has the same Sobel
    magnitude 8c everywhere, so every normalised term is 1 and L = lambda.  (0.5 keeps
    the Sobel sums of the flat image exactly 0.)"""
    H, W = 8, 11
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    img = np.full((3, H, W), 0.5)
    flow = np.stack([2.5 * x, np.zeros_like(x)])
    loss, _, info = oracle_lib.flow_loss(img, flow, 0.7, 0.0)
    assert loss == pytest.approx(0.7, rel=1e-12)
    assert info["max_gM"] == pytest.approx(8 * 2.5, rel=1e-12)


def test_normaliser_floor_keeps_noise_small(oracle_lib):
    """A flat image carrying rounding noise only (|grad I| ~ 1e-16) is not treated as an
    edge everywhere: the floor of the normaliser keeps its weight at 1."""
    H, W = 8, 11
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    img = np.full((3, H, W), 0.4)  # Sobel sums leave ~1e-16 of rounding
    flow = np.stack([2.5 * x, np.zeros_like(x)])
    loss, _, info = oracle_lib.flow_loss(img, flow, 0.7, 0.0)
    assert info["max_gI"] == 1e-6
    assert loss == pytest.approx(0.7, rel=1e-8)


def test_loss_invariant_to_flow_scale(oracle_lib):
    """With eps = 0 the normalisation makes L independent of the flow's units."""
    rng = np.random.default_rng(1)
    img = rng.uniform(size=(3, 9, 10))
    flow = rng.normal(size=(2, 9, 10))
    a = oracle_lib.flow_loss(img, flow, 1.0, 0.0)[0]
    b = oracle_lib.flow_loss(img, 37.0 * flow, 1.0, 0.0)[0]
    assert a == pytest.approx(b, rel=1e-12)


def test_loss_gradient_matches_finite_differences(oracle_lib):
    """dL/dflow against central differences of L with both normalisers held at their
    values at the expansion point (the reading under which the gradient is taken)."""
    rng = np.random.default_rng(2)
    H, W = 7, 9
    img = rng.uniform(size=(3, H, W))
    flow = rng.normal(size=(2, H, W))
    lam, eps = 0.5, 1e-3
    loss, d, info = oracle_lib.flow_loss(img, flow, lam, eps)
    norms = (info["max_gM"], info["max_gI"])
    h = 1e-6
    fd = np.zeros_like(flow)
    for idx in np.ndindex(flow.shape):
        fp = flow.copy()
        fm = flow.copy()
        fp[idx] += h
        fm[idx] -= h
        fd[idx] = (oracle_lib.flow_loss(img, fp, lam, eps, norms)[0] -
                   oracle_lib.flow_loss(img, fm, lam, eps, norms)[0]) / (2 * h)
    np.testing.assert_allclose(d, fd, rtol=1e-6, atol=1e-9 * np.abs(fd).max())


# ------------------------------------------------------------------------------------- flow
def _md_closed_form(cam, mean, vel):
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    p = R @ np.asarray(mean, np.float64) + np.asarray(cam.T, np.float64)
    u = R @ np.asarray(vel, np.float64)
    return np.array([cam.fx * u[0] / p[2], cam.fy * u[1] / p[2]])


def test_flow_single_and_stacked_gaussians_at_centre(oracle_lib):
    """At the pixel under a Gaussian's centre, G = 1: one Gaussian gives F = md alpha with
    md = f u_xy / p_z (u = R v); a second, nearer Gaussian at the same centre gives
    F = md1 a1 + md2 a2 (1 - a1)."""
    cam = centre_cam()
    v1, v2 = [0.3, -0.2, 0.1], [-0.4, 0.25, 0.0]
    t = np.float32(0.5)
    # velocities move the means: put both means at the origin at t by setting mu_t = t
    sc = one_scene([[0, 0, 0]], [[0.2, 0.1, 0.15]], [[1, 0, 0, 0]], [0.6], [0.5], [0.3], [v1], [[0.3, 0.5, 0.7]])
    proj, bins, res = oracle_lib.render(sc, cam, t, prec="f64", flow=True)
    a1 = proj["amax"][0]
    md1 = _md_closed_form(cam, [0, 0, 0], v1)
    np.testing.assert_allclose(res["flow"][:, 32, 32], md1 * a1, rtol=1e-6)
    sc2 = one_scene([[0, 0, 0], [0, 0, -1.0]], [[0.2, 0.1, 0.15], [0.1, 0.1, 0.1]], [[1, 0, 0, 0]] * 2,
                    [0.6, 0.5], [0.5, 0.5], [0.3, 0.3], [v1, v2], [[0.3, 0.5, 0.7], [0.1, 0.1, 0.1]])
    proj, bins, res = oracle_lib.render(sc2, cam, t, prec="f64", flow=True)
    near, far = (1, 0) if proj["depth"][1] < proj["depth"][0] else (0, 1)
    assert near == 1
    an, af = proj["amax"][near], proj["amax"][far]
    mdn = _md_closed_form(cam, [0, 0, -1.0], v2)
    expect = mdn * an + md1 * af * (1 - an)
    np.testing.assert_allclose(res["flow"][:, 32, 32], expect, rtol=1e-6)


def test_static_scene_has_zero_flow(oracle_lib):
    sc, cam, t = inputs.small_case()
    sc = sc.subset(np.arange(sc.n))
    sc.velocity[:] = 0.0
    _, _, res = oracle_lib.render(sc, cam, t, flow=True)
    assert np.abs(res["flow"]).max() == 0.0


def test_flow_adjoint_matches_finite_differences(oracle_lib):
    """Parameter gradients of sum(dL_dflow * flow) (blend adjoint with the flow channels
    + complex-step projection adjoint) against Richardson central differences."""
    sc, cam, t = _fd_scene(seed=7, n=40)
    base = {k: np.asarray(v, np.float64) for k, v in oracle_lib.scene_dict(sc).items()}
    dF = inputs.upstream_grad(31, cam.width, cam.height)[:2].astype(np.float64)
    zero = np.zeros((3, cam.height, cam.width))
    gp, gs, (proj, bins, res) = oracle_lib.render_grad(sc, cam, t, zero, prec="f64", arrays=base, dL_dflow=dF)
    contributing = np.unique(bins["values"])
    rng = np.random.default_rng(4)

    def L(arr):
        p, b, r = oracle_lib.render(sc, cam, t, prec="f64", arrays=arr, flow=True)
        # the decision hash of the same blend (skip / clamp / blend / stop per entry)
        dh = oracle_lib.blend(p, b, cam)["dhash"].tobytes()
        return float((dF * r["flow"]).sum()), b["values"].tobytes() + dh

    ref_vals = L(base)[1]
    checked = 0
    for name, dim in (("mean", 3), ("velocity", 3), ("scale", 3), ("opacity", 1), ("t_mean", 1)):
        got = tries = 0
        while got < 4 and tries < 40:
            tries += 1
            g = int(rng.choice(contributing))
            idx = int(rng.integers(dim))
            pos = _param_view(base, name, idx, g)
            vals, ok = {}, True
            for h in (1e-3, 5e-4):
                for sgn in (1, -1):
                    arr = {k: v.copy() for k, v in base.items()}
                    arr[name][pos] += sgn * h
                    val, vb = L(arr)
                    ok = ok and vb == ref_vals
                    vals[(h, sgn)] = val
            if not ok:
                continue
            d1 = (vals[(1e-3, 1)] - vals[(1e-3, -1)]) / 2e-3
            d2 = (vals[(5e-4, 1)] - vals[(5e-4, -1)]) / 1e-3
            fd = (4 * d2 - d1) / 3
            an = gp[name][pos]
            if abs(fd) < 1e-7 and abs(an) < 1e-7:
                continue
            assert abs(fd - an) <= 2e-3 * max(abs(fd), abs(an)), (name, idx, g, fd, an)
            got += 1
            checked += 1
    assert checked >= 12


def test_projection_adjoint_of_md_matches_fd(oracle_lib):
    """The md output of the projection (f u_xy / p_z) differentiated by complex step
    against central differences."""
    sc, cam, t = _fd_scene(seed=11, n=15, deg=0)
    base = {k: np.asarray(v, np.float64) for k, v in oracle_lib.scene_dict(sc).items()}
    proj = oracle_lib.project(sc, cam, t, "f64", base)
    rng = np.random.default_rng(5)
    z = lambda *shp: np.zeros(shp)
    gsplat = {"m": z(2, sc.n), "conic": z(3, sc.n), "amax": z(sc.n), "rgb": z(3, sc.n),
              "mdt": rng.normal(size=(2, sc.n))}
    active = (proj["count"] > 0).astype(np.int32)
    gp = oracle_lib.project_bwd(sc, cam, t, active, gsplat, base)
    act = active.astype(bool)
    for name, dim in (("mean", 3), ("velocity", 3)):
        for idx in range(dim):
            h = 1e-6
            ap = {k: v.copy() for k, v in base.items()}
            am = {k: v.copy() for k, v in base.items()}
            ap[name][idx] += h
            am[name][idx] -= h
            fd = ((gsplat["mdt"] * oracle_lib.project(sc, cam, t, "f64", ap)["mdt"]).sum(axis=0) -
                  (gsplat["mdt"] * oracle_lib.project(sc, cam, t, "f64", am)["mdt"]).sum(axis=0)) / (2 * h)
            np.testing.assert_allclose(gp[name][idx][act], fd[act], rtol=1e-6, atol=1e-9 * np.abs(fd).max())
