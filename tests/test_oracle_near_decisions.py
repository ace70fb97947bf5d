"""Pins of the oracle's near-decision diagnostic (oracle.near_decisions).

The time stage takes integer decisions -- culls, the guard-band clamps, the radius
ceiling, the rectangle floors -- and the GPU must take each of them exactly as the
oracle does.  The diagnostic reports, in FP64, the Gaussians with a decision within
1e-5 (relative) of its threshold, the ones where FP32 arithmetic in another order could
go the other way.  Each pin places one Gaussian at a chosen distance from one threshold,
computed here from the threshold's definition, and checks that it is counted inside
the band and not counted outside it.
"""
import math

import numpy as np

import oracle
from test_oracle_pins import centre_cam, one_scene

KT = float(np.float32(11.0825272))  # 2 ln 255 in FP32, the temporal cull's constant


def gaussian(mean=(0.0, 0.0, 0.0), mut=0.5, st=0.1):
    return one_scene([list(mean)], [[0.05] * 3], [[1, 0, 0, 0]], [0.8], [mut], [st], [[0, 0, 0]], [[0.3, 0.5, 0.7]])


def near(sc, cam, t):
    return oracle.near_decisions(sc, cam, t)[0]


def test_temporal_cull_threshold():
    cam = centre_cam()
    sc = gaussian()
    mut, st = float(sc.t_mean[0]), float(sc.t_scale[0])
    for delta, counted in ((1e-7, True), (-1e-7, True), (3e-6, True), (1e-3, False), (-1e-3, False)):
        # tau^2 = KT st^2 (1 + delta): on the culled side for delta > 0
        t = mut + math.sqrt(KT * st * st * (1.0 + delta))
        assert (near(sc, cam, t) == 1) == counted, (delta,)


def radius(p):
    """r = ceil(3 sqrt(lambda_max)) of the first Gaussian, from its FP64 conic: the
    dilated covariance is the conic's inverse; lambda_max with the discriminant floored
    at 0.1 (the 3DGS screen extent)."""
    a, b, c = (float(v) for v in p["conic"][:, 0])
    det = a * c - b * b
    sa, sb, sc = c / det, -b / det, a / det
    mid = 0.5 * (sa + sc)
    lam = mid + math.sqrt(max(mid * mid - (sa * sc - sb * sb), 0.1))
    return math.ceil(3.0 * math.sqrt(lam))


def test_rectangle_floor_threshold():
    """(m.x - r) / 16 at a chosen distance from an integer: m.x = 16 k + r + eps.  A mean
    (x, 0, 0) at depth 6 projects to an m.x linear in x; the slope is measured, the
    radius read back at the placed position (the Jacobian depends on it) and the
    placement repeated until it is stable."""
    cam = centre_cam(128, 64)
    t = 0.5
    mx = lambda x: float(oracle.project(gaussian(mean=(x, 0.0, 0.0)), cam, t, "f64")["m"][0, 0])
    slope = (mx(0.01) - mx(-0.01)) / 0.02
    for eps, counted in ((1e-7, True), (-1e-7, True), (0.3, False), (-0.3, False)):
        x = 0.0
        for _ in range(4):
            p = oracle.project(gaussian(mean=(x, 0.0, 0.0)), cam, t, "f64")
            target = 16.0 * 3 + radius(p) + eps  # (m.x - r) / 16 = 3 + eps / 16
            x = x + (target - float(p["m"][0, 0])) / slope
        g = gaussian(mean=(x, 0.0, 0.0))
        p = oracle.project(g, cam, t, "f64")
        assert abs((float(p["m"][0, 0]) - radius(p)) / 16.0 - 3.0 - eps / 16.0) < 1e-6
        assert (near(g, cam, t) == 1) == counted, (eps,)


def test_headline_frame_reports_a_small_fraction():
    """On a config-2 frame the band holds a few hundred of 300k Gaussians: the diagnostic
    is selective."""
    from paper_2503_22159_amd import inputs

    sc = inputs.clustered_scene()
    cam = inputs.arc_cameras()[10]
    n, idx = oracle.near_decisions(sc, cam, 0.5)
    assert 0 < n < 0.01 * sc.n
    assert np.all(np.diff(idx) > 0)
