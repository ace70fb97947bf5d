"""Pins of the oracle's three motion / covariance models of the time stage (the readings of
Eq. 13-14): linear screen motion (Eq. 13 as printed, the default), exact projection of the
moved mean, and linear motion with the Jacobian frozen at the camera stage.  CPU only."""
import numpy as np
import pytest

from paper_2503_22159_amd import inputs
from test_oracle_pins import _fd_scene

LIN, EXACT, FROZEN = 0, 1, 2


def _scene_with_camera_velocity(cam, u_cam, seed=3, n=30):
    """Scene whose every velocity is R^T u_cam (camera-space velocity u_cam)."""
    sc, _, _ = _fd_scene(seed=seed, n=n, deg=0)
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    v = R.T @ np.asarray(u_cam, np.float64)
    sc = sc.subset(np.arange(sc.n))
    sc.velocity[:] = v.astype(np.float32)[:, None]
    return sc


def test_exact_equals_linear_without_depth_velocity(oracle_lib):
    cam = inputs.look_at((1.0, 0.5, -5.0), width=64, height=48)
    sc = _scene_with_camera_velocity(cam, [0.4, -0.3, 0.0])
    t = np.float32(0.8)
    with oracle_lib.motion(LIN):
        a = oracle_lib.render(sc, cam, t, prec="f64")
    with oracle_lib.motion(EXACT):
        b = oracle_lib.render(sc, cam, t, prec="f64")
    act = a[0]["count"] > 0
    # the float32 velocity leaves |u_z| ~ 1e-8 after the rotation
    np.testing.assert_allclose(b[0]["m"][:, act], a[0]["m"][:, act], rtol=1e-7, atol=1e-7)
    np.testing.assert_allclose(b[0]["mdt"][:, act], a[0]["mdt"][:, act], rtol=1e-7, atol=1e-7)
    np.testing.assert_allclose(b[2]["img"], a[2]["img"], atol=1e-6)


def test_exact_mean_is_pinhole_projection_of_moved_mean(oracle_lib):
    """m = pi(R (mu + tau v) + T) computed here directly, and mdt = dm/dt by differences."""
    cam = inputs.look_at((1.0, 0.5, -5.0), width=64, height=48)
    sc = _scene_with_camera_velocity(cam, [0.4, -0.3, 0.9])
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    T = np.asarray(cam.T, np.float64)

    def pinhole(t):
        tau = t - sc.t_mean.astype(np.float64)
        pw = sc.mean.astype(np.float64) + tau[None] * sc.velocity.astype(np.float64)
        pc = R @ pw + T[:, None]
        return np.stack([cam.fx * pc[0] / pc[2] + cam.cx, cam.fy * pc[1] / pc[2] + cam.cy])

    t = 0.6
    with oracle_lib.motion(EXACT):
        p = oracle_lib.project(sc, cam, t, "f64")
        h = 1e-5
        mp = oracle_lib.project(sc, cam, t + h, "f64")["m"]
        mm = oracle_lib.project(sc, cam, t - h, "f64")["m"]
    act = p["count"] > 0
    assert act.sum() > 5
    np.testing.assert_allclose(p["m"][:, act], pinhole(t)[:, act], rtol=1e-10, atol=1e-8)
    np.testing.assert_allclose(p["mdt"][:, act], ((mp - mm) / (2 * h))[:, act], rtol=1e-6, atol=1e-6)


def test_frozen_jacobian_equals_default_at_tau_zero(oracle_lib):
    sc, cam, _ = _fd_scene(seed=4, n=25, deg=1)
    sc = sc.subset(np.arange(sc.n))
    sc.t_mean[:] = np.float32(0.5)
    t = np.float32(0.5)
    with oracle_lib.motion(LIN):
        a = oracle_lib.project(sc, cam, t, "f64")
    with oracle_lib.motion(FROZEN):
        b = oracle_lib.project(sc, cam, t, "f64")
    for k in ("m", "conic", "amax", "rect", "count", "depth"):
        assert np.array_equal(a[k], b[k]), k


def test_frozen_jacobian_conic_does_not_change_with_time(oracle_lib):
    cam = inputs.look_at((1.0, 0.5, -5.0), width=64, height=48)
    sc = _scene_with_camera_velocity(cam, [0.2, 0.1, 0.8])
    sc.t_scale[:] = np.float32(5.0)  # keep every Gaussian alive over the interval
    with oracle_lib.motion(FROZEN):
        a = oracle_lib.project(sc, cam, 0.2, "f64")
        b = oracle_lib.project(sc, cam, 0.9, "f64")
    with oracle_lib.motion(LIN):
        c = oracle_lib.project(sc, cam, 0.9, "f64")
    act = (a["count"] > 0) & (b["count"] > 0)
    assert act.sum() > 5
    assert np.array_equal(a["conic"][:, act], b["conic"][:, act])
    assert not np.allclose(c["conic"][:, act], b["conic"][:, act])  # the default does move it


@pytest.mark.parametrize("mode", [EXACT, FROZEN])
def test_projection_adjoint_per_model_matches_fd(oracle_lib, mode):
    """Complex-step projection adjoint (incl. the flow velocity) vs central differences
    under each non-default model."""
    sc, cam, t = _fd_scene(seed=13, n=12, deg=1)
    base = {k: np.asarray(v, np.float64) for k, v in oracle_lib.scene_dict(sc).items()}
    rng = np.random.default_rng(mode)
    with oracle_lib.motion(mode):
        proj = oracle_lib.project(sc, cam, t, "f64", base)
        gsplat = {"m": rng.normal(size=(2, sc.n)), "conic": rng.normal(size=(3, sc.n)),
                  "amax": rng.normal(size=sc.n), "rgb": rng.normal(size=(3, sc.n)),
                  "mdt": rng.normal(size=(2, sc.n))}
        active = (proj["count"] > 0).astype(np.int32)
        gp = oracle_lib.project_bwd(sc, cam, t, active, gsplat, base)

        def contract(p):
            return sum(np.atleast_2d(gsplat[k] * p[k]).sum(axis=0) for k in ("m", "conic", "amax", "rgb", "mdt"))

        act = active.astype(bool)
        for name, dim in (("mean", 3), ("velocity", 3), ("scale", 3), ("quat", 4), ("t_mean", 1)):
            for idx in range(dim):
                h = 1e-6
                ap = {k: v.copy() for k, v in base.items()}
                am = {k: v.copy() for k, v in base.items()}
                if name == "t_mean":
                    ap[name] += h
                    am[name] -= h
                    an = gp[name]
                else:
                    ap[name][idx] += h
                    am[name][idx] -= h
                    an = gp[name][idx]
                fd = (contract(oracle_lib.project(sc, cam, t, "f64", ap)) -
                      contract(oracle_lib.project(sc, cam, t, "f64", am))) / (2 * h)
                np.testing.assert_allclose(an[act], fd[act], rtol=1e-5, atol=1e-6 * np.abs(fd).max() + 1e-9)
