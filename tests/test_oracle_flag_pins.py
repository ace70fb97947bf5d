"""Pins of the oracle's near-threshold flags.

The GPU blend evaluates in FP32 and the oracle in FP64, so the discontinuous decisions of
Eq. 4 (the 1/255 alpha skip, the 1e-4 transmittance stop, the skip of a positive
exponent) may go different ways very close to their thresholds.  The oracle flags every
pixel holding such an evaluation, and the parity bar is looser there.  These pins place
one pixel at a chosen distance from each threshold, with the alpha or transmittance
computed here in closed form, and check that the pixel is flagged inside the margin and
not flagged (with the decision the threshold implies) outside it:

- alpha within 3e-5 relative of 1/255: bit 1;
- T' within 1e-9 absolute of 1e-4: bit 2;
- an exponent within 1e-5 of zero relative to its terms: bit 4.

The splats are given directly as projected 2D Gaussians (mean, conic, peak opacity,
colour) on one 16x16 tile; pixel (0, 0) samples at (0.5, 0.5).  The check_* functions
raise AssertionError on a mismatch; tests/test_oracle_mutations.py also runs them against
oracle builds with planted mistakes in the margins.
"""
import math

import numpy as np

import oracle
from paper_2503_22159_amd import inputs

CAM = inputs.look_at((0.0, 0.0, -6.0), width=16, height=16)
PX, PY = 0.5, 0.5


def blend(orc, means, conics, amax):
    n = len(amax)
    proj = {"n": n,
            "m": np.asarray(means, np.float64).T.copy(),
            "conic": np.asarray(conics, np.float64).T.copy(),
            "amax": np.asarray(amax, np.float64),
            "rgb": np.full((3, n), 0.5)}
    bins = {"values": np.arange(n, dtype=np.uint32), "ranges": np.array([[0, n]], np.uint32), "I": n}
    return orc.blend(proj, bins, CAM)


def pixel(res):
    return int(res["flags"][0, 0]), int(res["n_contrib"][0, 0])


# one splat half a pixel to the right of pixel (0, 0): power = -1/8 there
MEAN = (PX + 0.5, PY)
CONIC = (1.0, 0.0, 1.0)
G = math.exp(-0.125)


def check_alpha_band(orc):
    thr = 1.0 / 255.0
    for delta, flagged, blended in ((1e-5, True, True), (-1e-5, True, False), (2e-5, True, True),
                                    (1e-4, False, True), (-1e-4, False, False)):
        res = blend(orc, [MEAN], [CONIC], [thr * (1.0 + delta) / G])
        fl, nc = pixel(res)
        assert bool(fl & 1) == flagged, (delta, fl)
        assert nc == (1 if blended else 0), (delta, nc)


def check_t_band(orc):
    # alphas 0.95, 0.95, 1 - 0.04 (1 + eta): T' after the third = 1e-4 (1 + eta)
    for eta, flagged, contrib in ((2e-6, True, 3), (-2e-6, True, 2), (5e-6, True, 3),
                                  (1e-4, False, 3), (-1e-4, False, 2)):
        alphas = [0.95, 0.95, 1.0 - 0.04 * (1.0 + eta)]
        res = blend(orc, [MEAN] * 3, [CONIC] * 3, [a / G for a in alphas])
        fl, nc = pixel(res)
        assert bool(fl & 2) == flagged, (eta, fl)
        assert nc == contrib, (eta, nc)
        assert not fl & 1


def check_power_band(orc):
    # conic (1, 1, 1) (positive semidefinite); at d = (1, -1 + e) the exponent is
    # -(1 + (1 - e)^2) / 2 + (1 - e) = -e^2 / 2, its terms (1 + (1 - e)^2) / 2 + (1 - e)
    # ~ 2: relative size e^2 / 4
    for e, flagged in ((0.0, True), (1e-3, True), (2e-3, True), (1e-2, False), (5e-2, False)):
        mean = (PX - 1.0, PY + 1.0 - e)
        res = blend(orc, [mean], [(1.0, 1.0, 1.0)], [0.5])
        fl, _ = pixel(res)
        assert bool(fl & 4) == flagged, (e, fl)


def test_alpha_near_the_cutoff():
    check_alpha_band(oracle)


def test_transmittance_near_the_stop():
    check_t_band(oracle)


def test_exponent_near_zero():
    check_power_band(oracle)
