"""Planted mistakes in the oracle's tile rectangle, guard band and near-threshold flags must
fail their pins.

Each case copies the oracle's sources to a temporary directory, replaces one passage by a
plausible mistake, builds the copy with the oracle's own compiler flags, and runs the
pins of tests/test_oracle_rect_pins.py and tests/test_oracle_flag_pins.py against it: at
least one must raise.  The
unmodified copy must pass them (so a failure is the planted mistake's, not the build's).
CPU only.
"""
import os
import shutil

import pytest

import oracle
import test_oracle_flag_pins as flag_pins
import test_oracle_rect_pins as pins

ORACLE_DIR = os.path.dirname(os.path.abspath(oracle.__file__))

RADIUS = "DEC rad = CEILD(LIT(3.0) * SQRTD(lam1));"
FLOOR = "if (disc < LIT(0.1)) disc = LIT(0.1);"
X1 = "fx1 = FLOORD((mx + rad) / LIT(16.0)) + LIT(1.0);"
Y1 = "fy1 = FLOORD((my + rad) / LIT(16.0)) + LIT(1.0);"
BAND = "DEC limx = LIT(1.3) * cam->tan_fovx, limy = LIT(1.3) * cam->tan_fovy;"
CLAMP_X_LO = "if (RE(rx) < -limx) rx = -limx;"
CLAMP_Y_HI = "if (RE(ry) > limy) ry = limy;"
CLAMP_Y_LO = "if (RE(ry) < -limy) ry = -limy;"
ALPHA_FLAG = "if (dd <= OC_FLAG_ALPHA_REL * thr) fl |= 1;"
T_FLAG = "if (dd <= OC_FLAG_T_REL * (DEC)1e-4) fl |= 2;"
POWER_FLAG = "if (pw > -OC_FLAG_POWER_REL * scale && scale > 0) fl |= 4;"

# name -> (passage, replacement); the passage occurs exactly once in oracle_body.inc
MUTATIONS = {
    "radius 3 lambda": (RADIUS, "DEC rad = CEILD(LIT(3.0) * lam1);"),
    "radius 4 sqrt(lambda)": (RADIUS, "DEC rad = CEILD(LIT(4.0) * SQRTD(lam1));"),
    "radius + 1": (RADIUS, "DEC rad = CEILD(LIT(3.0) * SQRTD(lam1)) + LIT(1.0);"),
    "radius - 1": (RADIUS, "DEC rad = CEILD(LIT(3.0) * SQRTD(lam1)) - LIT(1.0);"),
    "radius 3 sqrt(lambda) unrounded": (RADIUS, "DEC rad = LIT(3.0) * SQRTD(lam1);"),
    "no discriminant floor": (FLOOR, ""),
    "x1 without + 1": (X1, "fx1 = FLOORD((mx + rad) / LIT(16.0));"),
    "y1 without + 1": (Y1, "fy1 = FLOORD((my + rad) / LIT(16.0));"),
    "x1 from the ceiling": (X1, "fx1 = CEILD((mx + rad) / LIT(16.0));"),
    "guard band unclamped": (BAND, "DEC limx = LIT(1e30) * cam->tan_fovx, limy = LIT(1e30) * cam->tan_fovy;"),
    "guard band 1.0": (BAND, "DEC limx = LIT(1.0) * cam->tan_fovx, limy = LIT(1.0) * cam->tan_fovy;"),
    "guard band 1.5": (BAND, "DEC limx = LIT(1.5) * cam->tan_fovx, limy = LIT(1.5) * cam->tan_fovy;"),
    "guard band from the other axis": (BAND, "DEC limx = LIT(1.3) * cam->tan_fovy, limy = LIT(1.3) * cam->tan_fovx;"),
    "guard band x only": (CLAMP_Y_HI + "\n    " + CLAMP_Y_LO, ""),
    "guard band lower x clamp to +limit": (CLAMP_X_LO, "if (RE(rx) < -limx) rx = limx;"),
    "alpha flag band 10x wider": (ALPHA_FLAG, "if (dd <= OC_FLAG_ALPHA_REL * (DEC)10.0 * thr) fl |= 1;"),
    "alpha flag band 10x narrower": (ALPHA_FLAG, "if (dd <= OC_FLAG_ALPHA_REL * (DEC)0.1 * thr) fl |= 1;"),
    "T flag band 5e-4 relative": (T_FLAG, "if (dd <= (DEC)5e-4 * (DEC)1e-4) fl |= 2;"),
    "T flag band absolute 1e-9 read as 1e-11": (T_FLAG, "if (dd <= (DEC)1e-11) fl |= 2;"),
    "T flag on T instead of T'": (T_FLAG, "if (RE(T) - (DEC)1e-4 <= OC_FLAG_T_REL * (DEC)1e-4 && (DEC)1e-4 - RE(T) <= OC_FLAG_T_REL * (DEC)1e-4) fl |= 2;"),
    "power flag only at exactly zero": (POWER_FLAG, "if (pw >= 0 && scale > 0) fl |= 4;"),
}


def _build(tmp_path, passage=None, replacement=None):
    src = tmp_path / "src"
    src.mkdir()
    for f in ("d4dgs_oracle.c", "oracle_body.inc"):
        shutil.copy(os.path.join(ORACLE_DIR, f), src / f)
    if passage is not None:
        body = (src / "oracle_body.inc").read_text()
        assert body.count(passage) == 1, passage
        (src / "oracle_body.inc").write_text(body.replace(passage, replacement))
    return oracle.compile_library(str(src), str(tmp_path / "liboracle_variant.so"))


def _pin_failures():
    failed = []
    for check in (pins.check_isotropic_rects, pins.check_anisotropic_rects, pins.check_guard_band,
                  flag_pins.check_alpha_band, flag_pins.check_t_band, flag_pins.check_power_band):
        try:
            check(oracle)
        except AssertionError:
            failed.append(check.__name__)
    return failed


def test_unmodified_copy_passes(tmp_path):
    with oracle.variant(_build(tmp_path)):
        assert _pin_failures() == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_fails_a_pin(tmp_path, name):
    passage, replacement = MUTATIONS[name]
    with oracle.variant(_build(tmp_path, passage, replacement)):
        failed = _pin_failures()
    assert failed, f"no pin caught the planted mistake '{name}'"
