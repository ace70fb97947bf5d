"""Pins of the oracle's tile rectangle and of the Jacobian's guard band.

Both decide integers (which tiles list a splat), and the GPU implements the same
conventions, so bit-exact GPU parity cannot catch a mistake in them: they are pinned here
against values computed another way.

- P2d, tile rectangle (the 3DGS screen extent the paper's rasteriser inherits,
  Sec. 3.2.2): a splat is listed in every 16x16 tile that meets the closed square
  [m - r, m + r]^2, r = ceil(3 sqrt(lambda_max)), lambda_max the larger eigenvalue of
  the dilated 2D covariance with the discriminant floored at 0.1.  Expected tiles are
  enumerated by brute force over the tile grid; r comes from the closed form of an
  isotropic footprint (lambda_max = sigma'^2 + sqrt(0.1)) or from numpy's eigenvalues
  of a covariance built with scipy's rotations and a numerically differentiated pixel
  map.  Centres sit on and next to tile edges, so a radius one pixel too large or too
  small moves a rectangle edge.
- P2e, guard band (Eq. 14-15): the Jacobian is taken at the camera-space mean with its
  lateral coordinates clamped to 1.3 x tan(fov / 2) of the depth.  Expected conics use
  the pixel map differentiated by central differences at the clamped point, for means
  beyond the band (both signs, both axes) and between 1.0 and 1.3 x tan(fov / 2).

The check_* functions raise AssertionError on a mismatch; tests/test_oracle_mutations.py
runs them against oracle builds with planted mistakes and expects them to fail.
"""
import math

import numpy as np
from scipy.spatial.transform import Rotation

from paper_2503_22159_amd import inputs
from test_oracle_pins import one_scene

TILE = 16


def tiles_meeting(lo, hi, ntiles):
    """Tiles k (0 <= k < ntiles) whose pixel span [16k, 16k + 16) meets [lo, hi]."""
    return [k for k in range(ntiles) if TILE * k <= hi and lo < TILE * (k + 1)]


def expected_rect(m, r, cam):
    TX = (cam.width + TILE - 1) // TILE
    TY = (cam.height + TILE - 1) // TILE
    xs = tiles_meeting(m[0] - r, m[0] + r, TX)
    ys = tiles_meeting(m[1] - r, m[1] + r, TY)
    if not xs or not ys:
        return None
    return [xs[0], ys[0], xs[-1] + 1, ys[-1] + 1]


def assert_rect(proj, g, rect, what):
    if rect is None:
        assert proj["count"][g] == 0, (what, proj["rect"][:, g])
        return
    got = [int(v) for v in proj["rect"][:, g]]
    assert got == rect, (what, got, rect)
    assert proj["count"][g] == (rect[2] - rect[0]) * (rect[3] - rect[1]), what


def _margin_to_int(x):
    return abs(x - round(x))


# ------------------------------------------------------------------------------------------ P2d
ISO_SCALES = (0.011, 0.05, 0.2, 0.3)


def isotropic_cases():
    """(scale, cx, cy) on a 160 x 160 image: the Gaussian sits at the world origin, 6 units
    in front of the camera, so its 2D mean is exactly (cx, cy).  Per scale: m - r on a
    tile edge in x and m + r on one in y, then the other way round (a larger radius moves
    x0 or y0, a smaller one x1 or y1), the mean itself on an edge, edges crossed by a
    quarter pixel, and means near the image border (rectangles clipped to the grid)."""
    cam = inputs.look_at((0.0, 0.0, -6.0), width=160, height=160)
    fx = float(cam.fx)
    cases = []
    for s in ISO_SCALES:
        sig2 = (fx * float(np.float32(s)) / 6.0) ** 2 + 0.3
        r = math.ceil(3.0 * math.sqrt(sig2 + math.sqrt(0.1)))
        cases += [(s, 48 + r, 96 - r), (s, 80 - r, 64 + r), (s, 64.0, 80.0),
                  (s, 32 + r + 0.25, 112 - r - 0.25), (s, 32 + r - 0.25, 112 - r + 0.25),
                  (s, 3.5, 157.0), (s, 150.5, 2.25)]
    return cases


def check_isotropic_rects(oracle):
    """P2d, isotropic: Sigma' = ((f s / z)^2 + 0.3) I (pin P2), so the discriminant is 0,
    lambda_max = sigma'^2 + sqrt(0.1) and r = ceil(3 sqrt(lambda_max))."""
    for s, cx, cy in isotropic_cases():
        cam = inputs.look_at((0.0, 0.0, -6.0), width=160, height=160, cx=cx, cy=cy)
        sig2 = (float(cam.fx) * float(np.float32(s)) / 6.0) ** 2 + 0.3
        lam = sig2 + math.sqrt(0.1)
        assert _margin_to_int(3.0 * math.sqrt(lam)) > 1e-3  # far from a rounding tie in FP32
        r = math.ceil(3.0 * math.sqrt(lam))
        sc = one_scene([[0, 0, 0]], [[s] * 3], [[1, 0, 0, 0]], [0.5], [0.5], [0.3], [[0, 0, 0]],
                       [[0.5, 0.5, 0.5]])
        proj = oracle.project(sc, cam, np.float32(0.5), "f32")
        assert float(proj["m"][0, 0]) == float(cam.cx) and float(proj["m"][1, 0]) == float(cam.cy)
        assert_rect(proj, 0, expected_rect((float(cam.cx), float(cam.cy)), r, cam), ("iso", s, cx, cy))


def _phi(P, cam):
    return np.array([cam.fx * P[0] / P[2] + cam.cx, cam.fy * P[1] / P[2] + cam.cy])


def _fd_jacobian(P, cam):
    J = np.zeros((2, 3))
    for k in range(3):
        h = 1e-6 * max(1.0, abs(P[k]))
        e = np.zeros(3)
        e[k] = h
        J[:, k] = (_phi(P + e, cam) - _phi(P - e, cam)) / (2 * h)
    return J


def _world_mean(cam, p_cam):
    """World-space mean (float32) whose camera-space position is p_cam."""
    R = cam.R.astype(np.float64).reshape(3, 3)
    return (R.T @ (np.asarray(p_cam, np.float64) - cam.T.astype(np.float64))).astype(np.float32)


def _expected_cov2d(cam, mu32, scale32, quat32, clamp=True):
    """Sigma' of a static Gaussian: scipy rotation for Sigma, the camera rotation, the
    pixel map differentiated at the (guard-band clamped) camera-space mean, + 0.3 I."""
    R = cam.R.astype(np.float64).reshape(3, 3)
    p = R @ mu32.astype(np.float64) + cam.T.astype(np.float64)
    q = quat32.astype(np.float64)
    Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()  # scipy: scalar last
    S = np.diag(scale32.astype(np.float64))
    Sig = Rq @ S @ S.T @ Rq.T
    pj = p.copy()
    if clamp:
        lim = (1.3 * float(cam.tan_fovx), 1.3 * float(cam.tan_fovy))
        for a in range(2):
            pj[a] = min(lim[a], max(-lim[a], p[a] / p[2])) * p[2]
    J = _fd_jacobian(pj, cam)
    return J @ R @ Sig @ R.T @ J.T + 0.3 * np.eye(2), p


def anisotropic_cases(seed=11, n=24):
    """Static anisotropic Gaussians inside the guard band (160 x 128 image, camera at
    (0, 0, -8)): the 2D mean of each is placed by the principal point so that m.x - r
    lies a quarter pixel right of a tile edge and m.y + r a quarter pixel right of one."""
    rng = np.random.default_rng(seed)
    base = inputs.look_at((0.0, 0.0, -8.0), width=160, height=128)
    out = []
    while len(out) < n:
        p_cam = np.array([rng.uniform(-1.5, 1.5), rng.uniform(-1.2, 1.2), rng.uniform(6.0, 10.0)])
        mu = _world_mean(base, p_cam)
        sc = np.exp(rng.normal(-2.0, 0.6, 3)).astype(np.float32)
        q = rng.normal(size=4).astype(np.float32)
        Sp, p = _expected_cov2d(base, mu, sc, q, clamp=False)
        a, b, c = Sp[0, 0], Sp[0, 1], Sp[1, 1]
        if (0.5 * (a - c)) ** 2 + b * b < 0.2:  # the 0.1 floor would decide lambda_max
            continue
        lam = float(np.linalg.eigvalsh(Sp).max())
        if _margin_to_int(3.0 * math.sqrt(lam)) < 1e-3:
            continue
        r = math.ceil(3.0 * math.sqrt(lam))
        # m = f p / z + c: choose c so that m.x - r = 16 kx + 1/4 and m.y + r = 16 ky + 1/4
        ox = float(base.fx) * p[0] / p[2]
        oy = float(base.fy) * p[1] / p[2]
        kx, ky = int(rng.integers(1, 5)), int(rng.integers(2, 6))
        cx = float(np.float32(TILE * kx + 0.25 + r - ox))
        cy = float(np.float32(TILE * ky + 0.25 - r - oy))
        out.append((mu, sc, q, cx, cy, r))
    return out


def check_anisotropic_rects(oracle):
    """P2d, anisotropic: r = ceil(3 sqrt(lambda_max)) with lambda_max from numpy's
    eigenvalues of the independently built Sigma'."""
    for i, (mu, sc, q, cx, cy, r) in enumerate(anisotropic_cases()):
        cam = inputs.look_at((0.0, 0.0, -8.0), width=160, height=128, cx=cx, cy=cy)
        scene = one_scene([mu], [sc], [q], [0.5], [0.5], [0.3], [[0, 0, 0]], [[0.5, 0.5, 0.5]])
        proj = oracle.project(scene, cam, np.float32(0.5), "f32")
        R = cam.R.astype(np.float64).reshape(3, 3)
        p = R @ mu.astype(np.float64) + cam.T.astype(np.float64)
        m = _phi(p, cam)
        assert np.allclose(proj["m"][:, 0], m, rtol=0, atol=1e-3), (i, proj["m"][:, 0], m)
        # the quarter pixel keeps every edge test away from the FP32 rounding of m
        assert_rect(proj, 0, expected_rect(m, r, cam), ("aniso", i))


# ------------------------------------------------------------------------------------------ P2e
def guard_band_cases():
    """(camera-space mean as multiples of (z tan_fovx, z tan_fovy), z).  Beyond the band
    in x, in y, in both, with either sign; and between 1.0 and 1.3 (no clamp)."""
    return [((1.6, 0.2), 5.0), ((-2.5, -0.1), 6.0), ((0.3, 1.9), 5.5), ((0.1, -1.45), 4.0),
            ((1.7, -2.2), 7.0), ((-1.4, 1.35), 6.5), ((1.15, -0.4), 5.0), ((-0.2, 1.2), 4.5),
            ((-1.18, -1.22), 6.0)]


def check_guard_band(oracle):
    """P2e: the conic is the inverse of J W Sigma W^T J^T + 0.3 I with J the pixel map's
    derivative at the clamped point; the mean itself is not clamped.  Large Gaussians
    whose mean lies beyond the image still reach into it: their rectangles are pinned
    too (r from numpy's eigenvalues)."""
    rng = np.random.default_rng(5)
    cam = inputs.look_at((0.0, 0.0, -6.0), width=160, height=128)
    mus, scs, qs, exp = [], [], [], []
    for (kx, ky), z in guard_band_cases():
        p_cam = np.array([kx * z * float(cam.tan_fovx), ky * z * float(cam.tan_fovy), z])
        mu = _world_mean(cam, p_cam)
        sc = np.exp(rng.normal(-0.6, 0.3, 3)).astype(np.float32)
        q = rng.normal(size=4).astype(np.float32)
        Sp, p = _expected_cov2d(cam, mu, sc, q, clamp=True)
        mus.append(mu)
        scs.append(sc)
        qs.append(q)
        exp.append((Sp, p))
    n = len(mus)
    scene = one_scene(mus, scs, qs, [0.5] * n, [0.5] * n, [0.3] * n, [[0, 0, 0]] * n, [[0.5, 0.5, 0.5]] * n)
    p64 = oracle.project(scene, cam, np.float32(0.5), "f64")
    p32 = oracle.project(scene, cam, np.float32(0.5), "f32")
    drawn = 0
    for g, (Sp, p) in enumerate(exp):
        Q = np.linalg.inv(Sp)
        np.testing.assert_allclose(p64["conic"][:, g], [Q[0, 0], Q[0, 1], Q[1, 1]], rtol=1e-7,
                                   atol=1e-9 * np.abs(Q).max(), err_msg=f"guard band case {g}")
        lam = float(np.linalg.eigvalsh(Sp).max())
        if _margin_to_int(3.0 * math.sqrt(lam)) < 1e-3:
            continue
        r = math.ceil(3.0 * math.sqrt(lam))
        rect = expected_rect(_phi(p, cam), r, cam)
        assert_rect(p32, g, rect, ("guard", g))
        drawn += rect is not None
    assert drawn >= 3  # some means beyond the image still reach into it


def test_p2d_isotropic_tile_rectangles(oracle_lib):
    check_isotropic_rects(oracle_lib)


def test_p2d_anisotropic_tile_rectangles(oracle_lib):
    check_anisotropic_rects(oracle_lib)


def test_p2e_guard_band_clamped_jacobian(oracle_lib):
    check_guard_band(oracle_lib)


def test_p2e_cases_straddle_the_band():
    """The cases exercise both sides of the clamp: beyond 1.3 on each axis and sign, and
    beyond 1.0 but inside 1.3 (a band scaled to 1.0 would clamp those)."""
    ks = [k for (kx, ky), _ in guard_band_cases() for k in (kx, ky)]
    assert any(k > 1.3 for k in ks) and any(k < -1.3 for k in ks)
    assert any(1.0 < abs(k) < 1.3 for k in ks)
    xs = [kx for (kx, _), _ in guard_band_cases()]
    ys = [ky for (_, ky), _ in guard_band_cases()]
    assert any(abs(k) > 1.3 for k in xs) and any(abs(k) > 1.3 for k in ys)
