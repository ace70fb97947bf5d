"""Python handle on the library's continuous-batching render server (d4dgs_serve_*).

    srv = Server(device_scene, max_inflight=64, max_batch=16, budget_bytes=8 << 30, n_streams=4)
    ticket = srv.submit(cam, t, out)      # out: (3, H, W) float32 CUDA tensor
    stats = srv.wait(ticket)              # dict with submit/admit/start/done ns, status
    srv.close()

The scheduler runs in a native thread inside the library; these methods only marshal
arguments.  `plain()` builds the same server restricted to one request at a time on one
stream with no batching -- the sequential single-request renderer used as the baseline.
"""
from __future__ import annotations

import ctypes as C

from . import binding as B


class Server:
    def __init__(self, scene, max_inflight=64, max_batch=16, budget_bytes=8 << 30, n_streams=4,
                 bg=(0.0, 0.0, 0.0), instances_per_pixel=1.0, max_queue=0):
        self.scene = scene  # keeps the parameter tensors alive
        cfg = B.ServeConfig()
        cfg.max_inflight = int(max_inflight)
        cfg.max_batch = int(max_batch)
        cfg.scratch_budget_bytes = int(budget_bytes)
        cfg.n_streams = int(n_streams)
        for i in range(3):
            cfg.bg[i] = float(bg[i])
        cfg.max_instances_per_pixel_x1000 = int(round(1000 * instances_per_pixel))
        cfg.max_queue = int(max_queue)
        self._s = scene.struct()
        h = C.c_void_p()
        B.check(B.lib.d4dgs_serve_create(C.byref(self._s), C.byref(cfg), C.byref(h)))
        self.h = h
        self.cfg = cfg

    @classmethod
    def plain(cls, scene, budget_bytes=8 << 30, bg=(0.0, 0.0, 0.0), instances_per_pixel=1.0):
        return cls(scene, max_inflight=1, max_batch=1, budget_bytes=budget_bytes, n_streams=1, bg=bg,
                   instances_per_pixel=instances_per_pixel, max_queue=1 << 30)

    def submit(self, cam, t, out):
        assert out.is_cuda and out.dtype.is_floating_point and out.is_contiguous()
        assert tuple(out.shape) == (3, cam.height, cam.width)
        tk = C.c_uint64(0)
        B.check(B.lib.d4dgs_serve_submit(self.h, C.byref(B.camera_struct(cam)), float(t),
                                         C.c_void_p(out.data_ptr()), C.byref(tk)))
        return tk.value

    @staticmethod
    def _stats(st):
        return {k: getattr(st, k) for k, _ in B.ReqStats._fields_}

    def poll(self, ticket):
        done = C.c_int32(0)
        st = B.ReqStats()
        B.check(B.lib.d4dgs_serve_poll(self.h, C.c_uint64(ticket), C.byref(done), C.byref(st)))
        return self._stats(st) if done.value else None

    def wait(self, ticket, timeout_s=30.0):
        st = B.ReqStats()
        B.check(B.lib.d4dgs_serve_wait(self.h, C.c_uint64(ticket), C.c_int64(int(timeout_s * 1e9)), C.byref(st)))
        return self._stats(st)

    def stats(self):
        st = B.ServeStats()
        B.check(B.lib.d4dgs_serve_stats_get(self.h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in B.ServeStats._fields_}

    def close(self):
        if self.h:
            B.check(B.lib.d4dgs_serve_destroy(self.h))
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
