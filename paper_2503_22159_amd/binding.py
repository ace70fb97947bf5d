"""ctypes binding of libd4dgs.so (include/d4dgs.h).

Argument marshalling only: every step of the render path runs in the library's HIP
kernels.  Structures mirror the C header field for field.  Importing this module
loads the library and raises if it is missing -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libd4dgs.so")

ABI_VERSION = 8
MOTION_LINEAR, MOTION_EXACT, MOTION_FROZEN_J = 0, 1, 2  # d4dgs_motion
TILE = 16
CAM_REC_FLOATS = 19
REC_FLOATS = 12
GRAD_FLOATS = 12

OK, ERR_INVALID_ARG, ERR_OUT_OF_MEMORY, ERR_CAPACITY, ERR_HIP, ERR_BUSY, ERR_NOT_FOUND, ERR_TIMEOUT = range(8)
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "OUT_OF_MEMORY", 3: "CAPACITY", 4: "HIP", 5: "BUSY",
                6: "NOT_FOUND", 7: "TIMEOUT"}

_fp = C.POINTER(C.c_float)
_u32p = C.POINTER(C.c_uint32)


class Scene(C.Structure):
    _fields_ = [("n", C.c_int32), ("sh_degree", C.c_int32), ("mean", C.c_void_p), ("scale", C.c_void_p),
                ("quat", C.c_void_p), ("opacity", C.c_void_p), ("t_mean", C.c_void_p), ("t_scale", C.c_void_p),
                ("velocity", C.c_void_p), ("sh", C.c_void_p)]


class Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("tan_fovx", C.c_float), ("tan_fovy", C.c_float),
                ("znear", C.c_float), ("R", C.c_float * 9), ("T", C.c_float * 3), ("campos", C.c_float * 3)]


class CamCache(C.Structure):
    _fields_ = [("rec", C.c_void_p), ("capacity", C.c_int32), ("valid", C.c_int32), ("cam", Camera),
                ("scene_key", C.c_void_p), ("scene_n", C.c_int32), ("scene_sh_degree", C.c_int32),
                ("hits", C.c_uint64), ("misses", C.c_uint64)]


class Splats(C.Structure):
    _fields_ = [("capacity", C.c_int32), ("rec", C.c_void_p), ("count", C.c_void_p), ("offset", C.c_void_p),
                ("partial", C.c_void_p), ("mdot", C.c_void_p), ("motion", C.c_int32)]


class Bins(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("keys", C.c_void_p), ("values", C.c_void_p), ("ranges", C.c_void_p),
                ("num_instances", C.c_void_p), ("order", C.c_void_p)]


class Grads(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("mean", "scale", "quat", "opacity", "t_mean", "t_scale", "velocity", "sh",
                                          "split_grad_t", "split_grad_xyz", "split_count")]


class SceneArrays(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("mean", "scale", "quat", "opacity", "t_mean", "t_scale", "velocity", "sh")]


class ServeConfig(C.Structure):
    _fields_ = [("max_inflight", C.c_int32), ("max_batch", C.c_int32), ("scratch_budget_bytes", C.c_int64),
                ("n_streams", C.c_int32), ("bg", C.c_float * 3), ("max_instances_per_pixel_x1000", C.c_int64),
                ("max_queue", C.c_int32)]


class ReqStats(C.Structure):
    _fields_ = [("submit_ns", C.c_int64), ("admit_ns", C.c_int64), ("start_ns", C.c_int64), ("done_ns", C.c_int64),
                ("num_instances", C.c_int64), ("status", C.c_int32), ("batch_size", C.c_int32)]


class ServeStats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("submitted", "completed", "rejected", "retried", "queued", "inflight",
                                          "batches", "arena_bytes", "arena_peak_bytes")]


class D4Error(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


EXPORTS = ("d4dgs_abi_version", "d4dgs_last_error", "d4dgs_workspace_size", "d4dgs_workspace_init",
           "d4dgs_project", "d4dgs_project_bin", "d4dgs_bin_sort",
           "d4dgs_bin_sort_sync", "d4dgs_render_fwd", "d4dgs_render_fwd_timed", "d4dgs_render_bwd", "d4dgs_serve_create",
           "d4dgs_serve_submit", "d4dgs_serve_poll", "d4dgs_serve_wait", "d4dgs_serve_stats_get",
           "d4dgs_serve_destroy", "d4dgs_render_times", "d4dgs_render_fwd_flow", "d4dgs_flow_loss_workspace_size",
           "d4dgs_flow_loss", "d4dgs_render_bwd_flow", "d4dgs_bin_sort_noalloc",
           "d4dgs_render_bwd_timed", "d4dgs_spatial_order_workspace_size", "d4dgs_spatial_order",
           "d4dgs_scene_permute")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libd4dgs.so not built ({LIB_PATH}); run `python -m paper_2503_22159_amd.build`")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "d4dgs_abi_version": (C.c_int32, []),
        "d4dgs_last_error": (C.c_char_p, []),
        "d4dgs_workspace_size": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int64, C.POINTER(C.c_size_t)]),
        "d4dgs_project": (C.c_int, [C.POINTER(Scene), C.POINTER(Camera), C.c_float, C.POINTER(CamCache),
                                    C.POINTER(Splats), P]),
        "d4dgs_workspace_init": (C.c_int, [P, C.c_size_t, C.c_int32, C.c_int32, C.c_int32, C.c_int64, P]),
        "d4dgs_project_bin": (C.c_int, [C.POINTER(Scene), C.POINTER(Camera), C.c_float, C.POINTER(CamCache),
                                        C.POINTER(Splats), P, C.c_size_t, C.POINTER(Bins), P, P]),
        "d4dgs_bin_sort": (C.c_int, [C.POINTER(Splats), C.c_int32, C.c_int32, C.c_int32, P, C.c_size_t,
                                     C.POINTER(Bins), P, P]),
        "d4dgs_bin_sort_noalloc": (C.c_int, [C.POINTER(Splats), C.c_int32, C.c_int32, C.c_int32,
                                             C.POINTER(Bins), P, P]),
        "d4dgs_bin_sort_sync": (C.c_int, [C.POINTER(Splats), C.c_int32, C.c_int32, C.c_int32, P, C.c_size_t,
                                          C.POINTER(Bins), C.POINTER(C.c_int64), P]),
        "d4dgs_render_fwd": (C.c_int, [C.POINTER(Splats), C.POINTER(Bins), C.c_int32, C.c_int32,
                                       C.POINTER(C.c_float * 3), P, P, P, P]),
        "d4dgs_render_fwd_timed": (C.c_int, [C.POINTER(Splats), C.POINTER(Bins), C.c_int32, C.c_int32,
                                             C.POINTER(C.c_float * 3), P, P, P, P, P, P]),
        "d4dgs_render_bwd": (C.c_int, [C.POINTER(Scene), C.POINTER(Camera), C.c_float, C.POINTER(Splats),
                                       C.POINTER(Bins), C.POINTER(C.c_float * 3), P, P, P, P, C.POINTER(Grads), P]),
        "d4dgs_render_bwd_timed": (C.c_int, [C.POINTER(Scene), C.POINTER(Camera), C.c_float, C.POINTER(Splats),
                                             C.POINTER(Bins), C.POINTER(C.c_float * 3), P, P, P, P, C.POINTER(Grads),
                                             C.POINTER(C.c_void_p), P]),
        "d4dgs_spatial_order_workspace_size": (C.c_int, [C.c_int32, C.POINTER(C.c_size_t)]),
        "d4dgs_spatial_order": (C.c_int, [C.POINTER(Scene), P, P, C.c_size_t, P]),
        "d4dgs_scene_permute": (C.c_int, [C.POINTER(Scene), P, C.POINTER(SceneArrays), P]),
        "d4dgs_serve_create": (C.c_int, [C.POINTER(Scene), C.POINTER(ServeConfig), C.POINTER(C.c_void_p)]),
        "d4dgs_serve_submit": (C.c_int, [P, C.POINTER(Camera), C.c_float, P, C.POINTER(C.c_uint64)]),
        "d4dgs_serve_poll": (C.c_int, [P, C.c_uint64, C.POINTER(C.c_int32), C.POINTER(ReqStats)]),
        "d4dgs_serve_wait": (C.c_int, [P, C.c_uint64, C.c_int64, C.POINTER(ReqStats)]),
        "d4dgs_serve_stats_get": (C.c_int, [P, C.POINTER(ServeStats)]),
        "d4dgs_serve_destroy": (C.c_int, [P]),
        "d4dgs_render_times": (C.c_int, [C.POINTER(Scene), C.POINTER(Camera), C.c_int32, C.POINTER(C.c_float),
                                         C.POINTER(CamCache), C.POINTER(Splats), C.POINTER(Bins),
                                         C.POINTER(C.c_void_p), C.c_size_t, C.POINTER(C.c_float * 3),
                                         C.POINTER(C.c_void_p), P, P]),
        "d4dgs_render_fwd_flow": (C.c_int, [C.POINTER(Splats), C.POINTER(Bins), C.c_int32, C.c_int32,
                                            C.POINTER(C.c_float * 3), P, P, P, P, P]),
        "d4dgs_flow_loss_workspace_size": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
        "d4dgs_flow_loss": (C.c_int, [P, P, C.c_int32, C.c_int32, C.c_float, C.c_float, P, C.c_size_t, P, P, P]),
        "d4dgs_render_bwd_flow": (C.c_int, [C.POINTER(Scene), C.POINTER(Camera), C.c_float, C.POINTER(Splats),
                                            C.POINTER(Bins), C.POINTER(C.c_float * 3), P, P, P, P, P,
                                            C.POINTER(Grads), P]),
    }
    for name, (res, args) in sig.items():
        try:
            f = getattr(L, name)
        except AttributeError:
            continue  # reported by exported_symbols(); calling it raises AttributeError
        f.restype = res
        f.argtypes = args
    if L.d4dgs_abi_version() != ABI_VERSION:
        raise ImportError("libd4dgs ABI version mismatch")
    return L


lib = _load()


def last_error():
    return lib.d4dgs_last_error().decode()


def check(status):
    if status != OK:
        raise D4Error(status, last_error())
    return status


def camera_struct(cam):
    """From an object with the fields of paper_2503_22159_amd.inputs.Camera."""
    c = Camera()
    c.width, c.height = int(cam.width), int(cam.height)
    for k in ("fx", "fy", "cx", "cy", "tan_fovx", "tan_fovy", "znear"):
        setattr(c, k, float(getattr(cam, k)))
    for i in range(9):
        c.R[i] = float(cam.R[i])
    for i in range(3):
        c.T[i] = float(cam.T[i])
        c.campos[i] = float(cam.campos[i])
    return c


def workspace_size(n, width, height, max_instances):
    b = C.c_size_t(0)
    check(lib.d4dgs_workspace_size(n, width, height, max_instances, C.byref(b)))
    return b.value
