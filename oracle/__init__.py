"""CPU oracle for the Disentangled 4D Gaussian Splatting render path.

TEST INFRASTRUCTURE ONLY.  Imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark -- never by the product package.  It wraps
liboracle.so (plain C, built from d4dgs_oracle.c by build()) through ctypes.

Functions follow the paper's pipeline (Alg. 1 and Sec. 3.2):
    project(scene, cam, t, prec)   camera stage + time stage, prec "f32" or "f64"
    bin(proj, cam)                 16x16 tile lists ordered by (tile, depth, index)
    blend(proj, bins, cam, bg)     Eq. 4 front to back, per pixel (FP64)
    blend_bruteforce(...)          the same blend, per-pixel lists built by brute force
    blend_bwd(...)                 exact adjoint of the blend (stored forward values)
    project_bwd(...)               projection adjoint by the complex-step method
    render(scene, cam, t, bg)      project(f32) -> bin -> blend
    render_grad(...)               gradients of sum(dL_dimg * image) w.r.t. parameters
    blend(..., flow=True)          also the optical flow of Sec. 3.3, F = sum md a T
    flow_loss(img, flow, lam, eps) the flow-gradient guided consistency loss (Eq. 16-17)
                                   and its gradient with respect to the flow

Precision: everything that decides an integer (culls, rectangles, depth keys) runs
in FP32 in the fixed operation order of the FP contract; blending and gradients run
in FP64 on the FP32 splat record.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "d4dgs_oracle.c")

PARAM_BLOCKS = (("mean", 3), ("scale", 3), ("quat", 4), ("opacity", 1), ("t_mean", 1),
                ("t_scale", 1), ("velocity", 3))


def build(force=True):
    """Compile liboracle.so with gcc (no fast-math, no FMA contraction, OpenMP)."""
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= max(
            os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "oracle_body.inc"))):
        return _LIB_PATH
    return compile_library(_HERE, _LIB_PATH)


def compile_library(src_dir, out_path):
    """Compile d4dgs_oracle.c (and the oracle_body.inc it includes) found in src_dir into
    out_path.  build() uses it on this directory; the mutation tests use it on edited
    copies of the two files."""
    tmp = out_path + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-shared", "-fPIC", "-Wall", "-Wno-unused-function", "-o", tmp,
           os.path.join(src_dir, "d4dgs_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True, cwd=src_dir)
    os.replace(tmp, out_path)
    return out_path


class _Scene(C.Structure):
    _fields_ = [("n", C.c_int32), ("sh_degree", C.c_int32)] + [
        (k, C.POINTER(C.c_double)) for k in
        ("mean", "scale", "quat", "opacity", "t_mean", "t_scale", "velocity", "sh")]


class _Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("tan_fovx", C.c_float), ("tan_fovy", C.c_float),
                ("znear", C.c_float), ("R", C.c_float * 9), ("T", C.c_float * 3),
                ("campos", C.c_float * 3)]


_lib = None


def _load(path):
    """ctypes handle of an oracle library with its argument types declared."""
    L = C.CDLL(path)
    P = C.c_void_p
    L.oc_version.restype = C.c_int
    for suf in ("f32", "f64"):
        f = getattr(L, "oc_project_" + suf)
        f.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.c_double] + [P] * 15
        f.restype = None
    L.oc_bin.argtypes = [C.c_int, C.c_int, C.c_int, P, P, P, P, P, P]
    L.oc_bin.restype = C.c_int64
    L.oc_blend.argtypes = [C.c_int, C.c_int, C.c_int] + [P] * 12
    L.oc_blend.restype = C.c_int64
    L.oc_blend_bruteforce.argtypes = [C.c_int, C.c_int, C.c_int] + [P] * 12
    L.oc_blend_bruteforce.restype = None
    L.oc_blend_bwd.argtypes = [C.c_int, C.c_int, C.c_int] + [P] * 13
    L.oc_blend_bwd.restype = None
    L.oc_blend_flow.argtypes = [C.c_int, C.c_int, C.c_int] + [P] * 13
    L.oc_blend_flow.restype = C.c_int64
    L.oc_blend_bwd_flow.argtypes = [C.c_int, C.c_int, C.c_int] + [P] * 16
    L.oc_blend_bwd_flow.restype = None
    L.oc_project_bwd.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.c_double] + [P] * 6
    L.oc_project_bwd.restype = None
    L.oc_project_bwd_flow.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.c_double] + [P] * 7
    L.oc_project_bwd_flow.restype = None
    L.oc_sh_basis.argtypes = [C.c_int, C.c_int, P, P]
    L.oc_sh_basis.restype = None
    L.oc_set_motion.argtypes = [C.c_int]
    L.oc_set_motion.restype = None
    L.oc_get_motion.restype = C.c_int
    L.oc_set_threads.argtypes = [C.c_int]
    L.oc_set_threads.restype = None
    L.oc_num_threads.restype = C.c_int
    L.oc_set_flag_margins.argtypes = [C.c_double, C.c_double, C.c_double]
    L.oc_set_flag_margins.restype = None
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = _load(_LIB_PATH)
    return _lib


class variant:
    """Context manager: every function of this module uses the oracle library at `path`
    (a build of an edited copy of the sources, see compile_library) until it exits.
    Test infrastructure for showing that a pin fails under a planted mistake."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.prev = _lib
        _lib = _load(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.prev


MOTION_LINEAR, MOTION_EXACT, MOTION_FROZEN_J = 0, 1, 2


class motion:
    """Context manager selecting the time stage's motion / covariance model (the readings
    of Eq. 13-14): MOTION_LINEAR (default: the 2D mean moves linearly, Eq. 13 as printed,
    Jacobian at the moved mean), MOTION_EXACT (the 2D mean is the exact projection of
    the moved mean), MOTION_FROZEN_J (linear motion, Jacobian at the camera stage's
    mean)."""

    def __init__(self, mode):
        self.mode = int(mode)

    def __enter__(self):
        self.prev = lib().oc_get_motion()
        lib().oc_set_motion(self.mode)
        return self

    def __exit__(self, *exc):
        lib().oc_set_motion(self.prev)


FLAG_MARGINS = (3e-5, 1e-5, 1e-5)  # default relative margins: alpha near 1/255, T' near 1e-4, power near 0


class flag_margins:
    """Context manager setting the relative margins of the blend's near-threshold flags
    (alpha near 1/255 or 0.99, T' near 1e-4, exponent near 0).  Bookkeeping only: images
    and decisions do not change.  For measuring how close FP32 evaluations come."""

    def __init__(self, alpha_rel=FLAG_MARGINS[0], t_rel=FLAG_MARGINS[1], power_rel=FLAG_MARGINS[2]):
        self.m = (float(alpha_rel), float(t_rel), float(power_rel))

    def __enter__(self):
        lib().oc_set_flag_margins(*self.m)
        return self

    def __exit__(self, *exc):
        lib().oc_set_flag_margins(*FLAG_MARGINS)


def set_threads(n):
    """OpenMP threads of the oracle (0 = all processors)."""
    lib().oc_set_threads(int(n))


def num_threads():
    return int(lib().oc_num_threads())


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _scene_struct(scene_arrays, n, deg):
    """scene_arrays: dict of arrays (any float dtype) -> (struct, keepalive list)."""
    keep = []
    s = _Scene()
    s.n = n
    s.sh_degree = deg
    for k in ("mean", "scale", "quat", "opacity", "t_mean", "t_scale", "velocity", "sh"):
        a = np.ascontiguousarray(scene_arrays[k], dtype=np.float64).reshape(-1)
        keep.append(a)
        setattr(s, k, a.ctypes.data_as(C.POINTER(C.c_double)))
    return s, keep


def _cam_struct(cam):
    c = _Camera()
    c.width, c.height = cam.width, cam.height
    for k in ("fx", "fy", "cx", "cy", "tan_fovx", "tan_fovy", "znear"):
        setattr(c, k, float(getattr(cam, k)))
    for i in range(9):
        c.R[i] = float(cam.R[i])
    for i in range(3):
        c.T[i] = float(cam.T[i])
        c.campos[i] = float(cam.campos[i])
    return c


def scene_dict(scene):
    return {k: getattr(scene, k) for k in ("mean", "scale", "quat", "opacity", "t_mean", "t_scale",
                                           "velocity", "sh")}


def project(scene, cam, t, prec="f32", arrays=None):
    """Camera stage + time stage for every Gaussian.  `arrays` overrides the
    parameters (e.g. float64 perturbed copies for finite differences)."""
    n, deg = scene.n, scene.sh_degree
    arr = scene_dict(scene) if arrays is None else arrays
    s, keep = _scene_struct(arr, n, deg)
    c = _cam_struct(cam)
    dt = np.float32 if prec == "f32" else np.float64
    out = {k: np.zeros((d, n), dt) for k, d in
           (("p", 3), ("u", 3), ("covc", 6), ("m0", 2), ("md", 2), ("rgb", 3), ("m", 2), ("conic", 3),
            ("mdt", 2))}
    out["amax"] = np.zeros(n, dt)
    out["w"] = np.zeros(n, dt)
    out["depth"] = np.zeros(n, np.float32)
    out["rect"] = np.zeros((4, n), np.int32)
    out["count"] = np.zeros(n, np.int32)
    out["margin"] = np.zeros(n, dt)
    f = getattr(lib(), "oc_project_" + prec)
    f(C.byref(s), C.byref(c), float(t), *[_p(out[k]) for k in
      ("p", "u", "covc", "m0", "md", "rgb", "m", "conic", "amax", "w", "depth", "rect", "count", "mdt",
       "margin")])
    del keep
    out["n"] = n
    return out


NEAR_DECISION = 1e-5


def near_decisions(scene, cam, t, rel=NEAR_DECISION):
    """Gaussians whose time-stage integer decisions lie within `rel` (relative) of their
    thresholds, evaluated in FP64: the temporal and near culls, the determinant's sign,
    the guard-band clamps, the discriminant floor, the radius ceiling and the rectangle
    floors (only the culls for a culled Gaussian).  Such a decision is one that FP32
    arithmetic in another order could take the other way; when a projection parity test
    fails, this count says whether the failure can be a rounding matter.  Returns
    (count, indices)."""
    m = project(scene, cam, t, "f64")["margin"]
    idx = np.nonzero(m < rel)[0]
    return int(idx.size), idx


def bin(proj, cam):
    n = proj["n"]
    count = np.ascontiguousarray(proj["count"], np.int32)
    I = int(count.astype(np.int64).sum())
    keys = np.zeros(max(I, 1), np.uint64)
    vals = np.zeros(max(I, 1), np.uint32)
    tiles = cam.tiles
    ranges = np.zeros(2 * tiles, np.uint32)
    got = lib().oc_bin(n, cam.width, cam.height, _p(np.ascontiguousarray(proj["rect"], np.int32)),
                       _p(count), _p(np.ascontiguousarray(proj["depth"], np.float32)),
                       _p(keys), _p(vals), _p(ranges))
    assert got == I
    return {"keys": keys[:I], "values": vals[:I], "ranges": ranges.reshape(tiles, 2), "I": I}


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def blend(proj, bins, cam, bg=(0.0, 0.0, 0.0), flow=False):
    """Eq. 4 per pixel.  flow=True also blends the screen velocity md of each splat with
    the same weights (the rendered optical flow of Sec. 3.3, background 0) into
    res["flow"] [2][H][W]."""
    n, W, H = proj["n"], cam.width, cam.height
    img = np.zeros((3, H, W))
    T = np.zeros((H, W))
    nc = np.zeros((H, W), np.int32)
    fl = np.zeros((H, W), np.int32)
    dh = np.zeros((H, W), np.uint64)
    vals = bins["values"] if bins["I"] > 0 else np.zeros(1, np.uint32)
    bgv = _f64(bg)
    if flow:
        fo = np.zeros((2, H, W))
        ne = lib().oc_blend_flow(n, W, H, _p(_f64(proj["m"])), _p(_f64(proj["conic"])), _p(_f64(proj["amax"])),
                                 _p(_f64(proj["rgb"])), _p(_f64(proj["mdt"])), _p(np.ascontiguousarray(vals)),
                                 _p(np.ascontiguousarray(bins["ranges"], np.uint32)), _p(bgv), _p(img), _p(fo),
                                 _p(T), _p(nc), _p(fl))
        return {"img": img, "flow": fo, "final_T": T, "n_contrib": nc, "flags": fl, "n_eval": int(ne)}
    ne = lib().oc_blend(n, W, H, _p(_f64(proj["m"])), _p(_f64(proj["conic"])), _p(_f64(proj["amax"])),
                        _p(_f64(proj["rgb"])), _p(np.ascontiguousarray(vals)),
                        _p(np.ascontiguousarray(bins["ranges"], np.uint32)), _p(bgv), _p(img), _p(T),
                        _p(nc), _p(fl), _p(dh))
    return {"img": img, "final_T": T, "n_contrib": nc, "flags": fl, "n_eval": int(ne), "dhash": dh}


def blend_bruteforce(proj, cam, bg=(0.0, 0.0, 0.0)):
    n, W, H = proj["n"], cam.width, cam.height
    img = np.zeros((3, H, W))
    T = np.zeros((H, W))
    nc = np.zeros((H, W), np.int32)
    fl = np.zeros((H, W), np.int32)
    lib().oc_blend_bruteforce(n, W, H, _p(_f64(proj["m"])), _p(_f64(proj["conic"])),
                              _p(_f64(proj["amax"])), _p(_f64(proj["rgb"])),
                              _p(np.ascontiguousarray(proj["rect"], np.int32)),
                              _p(np.ascontiguousarray(proj["count"], np.int32)),
                              _p(np.ascontiguousarray(proj["depth"], np.float32)), _p(_f64(bg)),
                              _p(img), _p(T), _p(nc), _p(fl))
    return {"img": img, "final_T": T, "n_contrib": nc, "flags": fl}


def blend_bwd(proj, bins, cam, dL_dimg, bg=(0.0, 0.0, 0.0), dL_dflow=None):
    """Adjoint of blend: splat-level gradients of sum(dL_dimg * img) (+ sum(dL_dflow *
    flow) when dL_dflow is given, then also g["mdt"], the gradient of the splats' flow
    velocities)."""
    n, W, H = proj["n"], cam.width, cam.height
    g = {"m": np.zeros((2, n)), "conic": np.zeros((3, n)), "amax": np.zeros(n), "rgb": np.zeros((3, n))}
    err = np.zeros(1)
    vals = bins["values"] if bins["I"] > 0 else np.zeros(1, np.uint32)
    if dL_dflow is not None:
        g["mdt"] = np.zeros((2, n))
        lib().oc_blend_bwd_flow(n, W, H, _p(_f64(proj["m"])), _p(_f64(proj["conic"])), _p(_f64(proj["amax"])),
                                _p(_f64(proj["rgb"])), _p(_f64(proj["mdt"])), _p(np.ascontiguousarray(vals)),
                                _p(np.ascontiguousarray(bins["ranges"], np.uint32)), _p(_f64(bg)),
                                _p(_f64(dL_dimg)), _p(_f64(dL_dflow)), _p(g["m"]), _p(g["conic"]),
                                _p(g["amax"]), _p(g["rgb"]), _p(g["mdt"]), _p(err))
    else:
        lib().oc_blend_bwd(n, W, H, _p(_f64(proj["m"])), _p(_f64(proj["conic"])), _p(_f64(proj["amax"])),
                           _p(_f64(proj["rgb"])), _p(np.ascontiguousarray(vals)),
                           _p(np.ascontiguousarray(bins["ranges"], np.uint32)), _p(_f64(bg)),
                           _p(_f64(dL_dimg)), _p(g["m"]), _p(g["conic"]), _p(g["amax"]), _p(g["rgb"]), _p(err))
    g["replay_rel_err"] = float(err[0])
    return g


def project_bwd(scene, cam, t, active, gsplat, arrays=None):
    """Parameter gradients from splat-level gradients, by complex step.
    Returns a dict in the scene's planar layout."""
    n, deg = scene.n, scene.sh_degree
    K = (deg + 1) ** 2
    P = 16 + 3 * K
    arr = scene_dict(scene) if arrays is None else arrays
    s, keep = _scene_struct(arr, n, deg)
    c = _cam_struct(cam)
    out = np.zeros((P, n))
    gmd = gsplat.get("mdt")
    lib().oc_project_bwd_flow(C.byref(s), C.byref(c), float(t), _p(np.ascontiguousarray(active, np.int32)),
                              _p(_f64(gsplat["m"])), _p(_f64(gsplat["conic"])), _p(_f64(gsplat["amax"])),
                              _p(_f64(gsplat["rgb"])), _p(_f64(gmd)) if gmd is not None else None, _p(out))
    del keep
    return unpack_params(out, K)


def unpack_params(flat, K):
    res, j = {}, 0
    for name, d in PARAM_BLOCKS:
        res[name] = flat[j:j + d] if d > 1 else flat[j]
        j += d
    res["sh"] = flat[j:j + 3 * K].reshape(K, 3, -1)
    return res


def render(scene, cam, t, bg=(0.0, 0.0, 0.0), prec="f32", arrays=None, flow=False):
    """project -> bin -> blend.  Returns (projection, bins, blend result)."""
    proj = project(scene, cam, t, prec, arrays)
    bins = bin(proj, cam)
    res = blend(proj, bins, cam, bg, flow=flow)
    return proj, bins, res


def render_grad(scene, cam, t, dL_dimg, bg=(0.0, 0.0, 0.0), prec="f32", arrays=None, mask=None, dL_dflow=None):
    """Gradient of sum(dL_dimg * image) (+ sum(dL_dflow * flow)) with respect to every
    parameter.  `mask` (H, W) zeroes the upstream gradients at excluded pixels."""
    proj, bins, res = render(scene, cam, t, bg, prec, arrays, flow=dL_dflow is not None)
    gin = np.array(dL_dimg, dtype=np.float64)
    gfl = None if dL_dflow is None else np.array(dL_dflow, dtype=np.float64)
    if mask is not None:
        gin = gin * (~mask)[None]
        if gfl is not None:
            gfl = gfl * (~mask)[None]
    gs = blend_bwd(proj, bins, cam, gin, bg, dL_dflow=gfl)
    active = (proj["count"] > 0).astype(np.int32)
    gp = project_bwd(scene, cam, t, active, gs, arrays)
    return gp, gs, (proj, bins, res)


# ---------------- flow-gradient guided consistency loss (Sec. 3.3, Eq. 16-17) -------------
# Readings (the paper leaves these open):
#  * gradients by the 3x3 Sobel operator, Kx = [[-1,0,1],[-2,0,2],[-1,0,1]] (x along a
#    row), Ky its transpose, as a correlation over the pixels whose 3x3 neighbourhood
#    lies inside the image ("interior" pixels); N counts them;
#  * |grad I| over the RGB image = sqrt(sum over channels of Gx^2 + Gy^2);
#  * "normalized" = divided by its largest value over the interior, floored at
#    NORM_FLOOR (so that rounding noise of a flat image or flow is not blown up to 1);
#  * L = lam / N * sum_interior nM (1 - nI), M = sqrt(u^2 + v^2 + eps);
#  * the loss shapes the motion: its gradient is taken with respect to the flow, with
#    the image-edge weight (1 - nI) and both normalisers held constant.
SOBEL_X = np.array([[-1.0, 0.0, 1.0], [-2.0, 0.0, 2.0], [-1.0, 0.0, 1.0]])
NORM_FLOOR = 1e-6
SOBEL_Y = SOBEL_X.T.copy()


def sobel(f):
    """(Gx, Gy) of a 2D array over its interior pixels, shape (H-2, W-2): a plain sum over
    the nine taps."""
    f = np.asarray(f, np.float64)
    H, W = f.shape
    gx = np.zeros((H - 2, W - 2))
    gy = np.zeros((H - 2, W - 2))
    for j in range(3):
        for i in range(3):
            win = f[j:j + H - 2, i:i + W - 2]
            gx += SOBEL_X[j, i] * win
            gy += SOBEL_Y[j, i] * win
    return gx, gy


def flow_loss(img, flow, lam, eps, norms=None):
    """L_fg of Eq. 17 and dL/dflow ([2][H][W]).  `norms` = the two normalisers
    (max(max |grad M|, floor), max(max |grad I|, floor)) to use instead (finite-difference
    checks hold them fixed).  Returns (loss, dL_dflow, info)."""
    img = np.asarray(img, np.float64)
    flow = np.asarray(flow, np.float64)
    _, H, W = img.shape
    if H < 3 or W < 3:
        return 0.0, np.zeros_like(flow), {"N": 0, "max_gM": 0.0, "max_gI": 0.0}
    u, v = flow
    M = np.sqrt(u * u + v * v + eps)
    gxM, gyM = sobel(M)
    gM = np.sqrt(gxM * gxM + gyM * gyM)
    gI2 = np.zeros((H - 2, W - 2))
    for c in range(3):
        gx, gy = sobel(img[c])
        gI2 += gx * gx + gy * gy
    gI = np.sqrt(gI2)
    mM, mI = (max(gM.max(), NORM_FLOOR), max(gI.max(), NORM_FLOOR)) if norms is None else norms
    nM = gM / mM
    nI = gI / mI
    N = (H - 2) * (W - 2)
    loss = lam / N * float(np.sum(nM * (1.0 - nI)))
    # backward (edge weight and normalisers constant)
    wgt = lam / N * (1.0 - nI) / mM
    safe = np.where(gM > 0, gM, 1.0)
    cx = np.where(gM > 0, wgt * gxM / safe, 0.0)
    cy = np.where(gM > 0, wgt * gyM / safe, 0.0)
    dM = np.zeros((H, W))
    for j in range(3):
        for i in range(3):
            dM[j:j + H - 2, i:i + W - 2] += SOBEL_X[j, i] * cx + SOBEL_Y[j, i] * cy
    Ms = np.where(M > 0, M, 1.0)  # M = 0 only with eps = 0 at zero flow: gradient 0 there
    dflow = np.stack([np.where(M > 0, dM * u / Ms, 0.0), np.where(M > 0, dM * v / Ms, 0.0)])
    return loss, dflow, {"N": N, "max_gM": float(mM), "max_gI": float(mI)}


def sh_basis(deg, dirs):
    dirs = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    K = (deg + 1) ** 2
    Y = np.zeros((dirs.shape[0], K))
    lib().oc_sh_basis(deg, dirs.shape[0], _p(dirs), _p(Y))
    return Y
