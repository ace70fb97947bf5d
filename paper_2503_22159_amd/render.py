"""PyTorch-facing wrappers of libd4dgs.

PyTorch supplies device memory and the current HIP stream; every stage of the render
path runs in the library's kernels (binding.py marshals arguments only).

    scene = DeviceScene.from_inputs(inputs_scene)          # resident parameters
    img, state = render_forward(scene, cam, t, bg)          # project -> bin/sort -> blend
    grads = render_backward(scene, cam, t, bg, state, dL)   # adjoint, all parameters
    img = render(params..., cam=..., t=...)                 # autograd.Function
    r = Renderer(scene, width, height); r.render(cam, t)    # fixed buffers for loops
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import binding as B

FIELDS = ("mean", "scale", "quat", "opacity", "t_mean", "t_scale", "velocity", "sh")


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def tiles_of(width, height):
    return ((width + B.TILE - 1) // B.TILE) * ((height + B.TILE - 1) // B.TILE)


def default_capacity(n, width, height):
    """Instance capacity: enough for the synthetic workloads' overlap (about 4 tiles per
    Gaussian) with headroom; render_forward grows it on overflow."""
    return int(max(1 << 16, 4 * n, 2 * tiles_of(width, height)))


class DeviceScene:
    """Scene parameters on the GPU: planar float32 tensors (see inputs.Scene)."""

    def __init__(self, tensors: dict, sh_degree: int):
        self.t = {k: tensors[k].contiguous() for k in FIELDS}
        for k in FIELDS:
            assert self.t[k].dtype == torch.float32 and self.t[k].is_cuda, k
        self.n = int(self.t["opacity"].numel())
        self.sh_degree = int(sh_degree)
        assert 0 <= self.sh_degree <= 3, "sh_degree must be 0..3"
        # the kernels index these planar arrays by n: a short one would be read out of bounds
        per = {"mean": 3, "scale": 3, "quat": 4, "opacity": 1, "t_mean": 1, "t_scale": 1, "velocity": 3,
               "sh": 3 * (self.sh_degree + 1) ** 2}
        for k, m in per.items():
            assert self.t[k].numel() == m * self.n, (k, tuple(self.t[k].shape), m, self.n)

    @classmethod
    def from_inputs(cls, scene, device="cuda"):
        return cls({k: torch.from_numpy(np.ascontiguousarray(getattr(scene, k))).to(device) for k in FIELDS},
                   scene.sh_degree)

    def struct(self):
        s = B.Scene()
        s.n = self.n
        s.sh_degree = self.sh_degree
        for k in FIELDS:
            setattr(s, k, self.t[k].data_ptr())
        return s


def spatial_order(scene: DeviceScene):
    """perm (int32 [n], device): the library's spatial (3D Morton) order of the scene's
    Gaussians (d4dgs_spatial_order)."""
    dev = scene.t["mean"].device
    perm = torch.empty(max(scene.n, 1), dtype=torch.int32, device=dev)
    nb = C.c_size_t(0)
    B.check(B.lib.d4dgs_spatial_order_workspace_size(scene.n, C.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    s = scene.struct()
    B.check(B.lib.d4dgs_spatial_order(C.byref(s), _ptr(perm), _ptr(ws), ws.numel(), _stream()))
    return perm[:scene.n]


def permute_scene(scene: DeviceScene, perm):
    """A new DeviceScene holding the scene's Gaussians in the order perm
    (d4dgs_scene_permute): Gaussian j of the result is Gaussian perm[j] of the input."""
    out = {k: torch.empty_like(scene.t[k]) for k in FIELDS}
    a = B.SceneArrays()
    for k in FIELDS:
        setattr(a, k, out[k].data_ptr())
    s = scene.struct()
    B.check(B.lib.d4dgs_scene_permute(C.byref(s), _ptr(perm), C.byref(a), _stream()))
    return DeviceScene(out, scene.sh_degree)


def spatially_ordered(scene: DeviceScene):
    """(reordered scene, perm): the scene stored in the library's spatial order."""
    perm = spatial_order(scene)
    return permute_scene(scene, perm), perm


class FrameState:
    """Device buffers of one rendered frame (splat record, sorted bins, replay state)."""

    def __init__(self, n, width, height, capacity, device="cuda", flow=False, motion=0, tile_order=True):
        self.n, self.width, self.height, self.capacity = n, width, height, int(capacity)
        self.motion = int(motion)  # d4dgs_motion of the time stage
        dev = device
        nn = max(n, 1)
        self.rec = torch.empty(nn * B.REC_FLOATS, dtype=torch.float32, device=dev)
        self.count = torch.empty(nn, dtype=torch.int32, device=dev)
        self.offset = torch.empty(nn, dtype=torch.int32, device=dev)
        self.partial = torch.empty((nn + 255) // 256, dtype=torch.int32, device=dev)
        self.keys = torch.empty(self.capacity, dtype=torch.int64, device=dev)
        self.values = torch.empty(self.capacity, dtype=torch.int32, device=dev)
        self.ranges = torch.empty(2 * tiles_of(width, height), dtype=torch.int32, device=dev)
        # tiles longest list first, written by the binning (scheduling of the per-tile kernels)
        self.order = torch.empty(max(tiles_of(width, height), 1), dtype=torch.int32, device=dev) if tile_order else None
        self.num_inst = torch.zeros(1, dtype=torch.int64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.ws = torch.empty(B.workspace_size(n, width, height, self.capacity), dtype=torch.uint8, device=dev)
        # screen velocity of each splat (written by the projection when the flow is wanted)
        self.mdot = torch.empty(nn * 2, dtype=torch.float32, device=dev) if flow else None
        self.flow = None
        self.img = None
        self.final_T = None
        self.n_contrib = None
        self.inst_grads = None

    def splats(self):
        s = B.Splats()
        s.capacity = max(self.n, 1)
        s.rec, s.count, s.offset, s.partial = (self.rec.data_ptr(), self.count.data_ptr(),
                                               self.offset.data_ptr(), self.partial.data_ptr())
        s.mdot = self.mdot.data_ptr() if self.mdot is not None else None
        s.motion = self.motion
        return s

    def bins(self):
        b = B.Bins()
        b.capacity = self.capacity
        b.keys, b.values, b.ranges, b.num_instances = (self.keys.data_ptr(), self.values.data_ptr(),
                                                       self.ranges.data_ptr(), self.num_inst.data_ptr())
        b.order = self.order.data_ptr() if self.order is not None else None
        return b


class CamCache:
    """Device buffer + bookkeeping of the camera-stage cache (Alg. 1)."""

    def __init__(self, capacity, device="cuda"):
        self.buf = torch.empty(max(capacity, 1) * B.CAM_REC_FLOATS, dtype=torch.float32, device=device)
        self.c = B.CamCache()
        self.c.rec = self.buf.data_ptr()
        self.c.capacity = max(capacity, 1)
        self.c.valid = 0

    def invalidate(self):
        self.c.valid = 0


class SharedCameraOrder:
    """Stream ordering for one CamCache shared by renderers on several streams.

    The cache is hit or missed on the host, when a call is made; its record is written on
    the device by the missing call's camera stage.  So a miss (the first frame of a camera)
    must run after every frame the other streams have queued, which may still read the
    previous camera's record, and the other streams' frames of the new camera must run
    after the miss has written it: before_miss / after_miss around the call that misses,
    before_hit before every other call (it waits once per stream and camera)."""

    def __init__(self, streams):
        self.streams = list(streams)
        self.fill = torch.cuda.Event()
        self.read = [torch.cuda.Event() for _ in self.streams]
        self.waited = [True] * len(self.streams)

    def before_miss(self, s):
        for q, st in enumerate(self.streams):
            if q != s:
                self.read[q].record(st)
                self.streams[s].wait_event(self.read[q])

    def after_miss(self, s):
        self.fill.record(self.streams[s])
        self.waited = [q == s for q in range(len(self.streams))]

    def before_hit(self, s):
        if not self.waited[s]:
            self.streams[s].wait_event(self.fill)
            self.waited[s] = True


def _bg(bg):
    a = (C.c_float * 3)()
    for i in range(3):
        a[i] = float(bg[i])
    return a


def project(scene: DeviceScene, cam, t, st: FrameState, cache: CamCache | None = None):
    s = scene.struct()
    sp = st.splats()
    B.check(B.lib.d4dgs_project(C.byref(s), C.byref(B.camera_struct(cam)), float(t),
                                C.byref(cache.c) if cache is not None else None, C.byref(sp), _stream()))


def bin_sort(st: FrameState, sync=False):
    sp, bn = st.splats(), st.bins()
    if sync:
        ni = C.c_int64(0)
        r = B.lib.d4dgs_bin_sort_sync(C.byref(sp), st.n, st.width, st.height, _ptr(st.ws), st.ws.numel(),
                                      C.byref(bn), C.byref(ni), _stream())
        if r == B.ERR_CAPACITY:
            return int(ni.value)
        B.check(r)
        return int(ni.value)
    B.check(B.lib.d4dgs_bin_sort(C.byref(sp), st.n, st.width, st.height, _ptr(st.ws), st.ws.numel(), C.byref(bn),
                                 _ptr(st.status), _stream()))
    return None


def blend(st: FrameState, bg=(0.0, 0.0, 0.0), keep_state=True, img=None):
    H, W = st.height, st.width
    dev = st.rec.device
    st.img = img if img is not None else torch.empty((3, H, W), dtype=torch.float32, device=dev)
    if keep_state:
        st.final_T = torch.empty((H, W), dtype=torch.float32, device=dev)
        st.n_contrib = torch.empty((H, W), dtype=torch.int32, device=dev)
    sp, bn = st.splats(), st.bins()
    B.check(B.lib.d4dgs_render_fwd(C.byref(sp), C.byref(bn), W, H, C.byref(_bg(bg)), _ptr(st.img),
                                   _ptr(st.final_T) if keep_state else None,
                                   _ptr(st.n_contrib) if keep_state else None, _stream()))
    return st.img


def render_forward(scene: DeviceScene, cam, t, bg=(0.0, 0.0, 0.0), capacity=None, keep_state=True,
                   cache: CamCache | None = None, motion=0):
    """Full forward with exact instance capacity handling (synchronises once to read the
    instance count; grows the capacity and re-sorts on overflow)."""
    cap = capacity or default_capacity(scene.n, cam.width, cam.height)
    st = FrameState(scene.n, cam.width, cam.height, cap, scene.t["mean"].device, motion=motion)
    project(scene, cam, t, st, cache)
    ni = bin_sort(st, sync=True)
    if ni > st.capacity:
        # the scan consumed the per-block sums in place: project again into larger buffers
        st = FrameState(scene.n, cam.width, cam.height, int(ni * 1.25) + 1024, scene.t["mean"].device,
                        motion=motion)
        project(scene, cam, t, st, cache)
        ni2 = bin_sort(st, sync=True)
        assert ni2 == ni
    st.num_instances = ni
    img = blend(st, bg, keep_state)
    return img, st


def grads_like(scene: DeviceScene, split_stats=False):
    """Zeroed gradient arrays; with split_stats also the splitting statistics
    (split_grad_t, split_grad_xyz float [n]; split_count int32 [n]) that every backward
    call accumulates: |dL/dmu_t| and |dL/dmu| of the view for each drawn Gaussian."""
    g = {k: torch.zeros_like(scene.t[k]) for k in FIELDS}
    if split_stats:
        dev = scene.t["mean"].device
        g["split_grad_t"] = torch.zeros(scene.n, dtype=torch.float32, device=dev)
        g["split_grad_xyz"] = torch.zeros(scene.n, dtype=torch.float32, device=dev)
        g["split_count"] = torch.zeros(scene.n, dtype=torch.int32, device=dev)
    return g


def render_backward(scene: DeviceScene, cam, t, bg, st: FrameState, dL_dimg, grads=None, dL_dflow=None,
                    events=None):
    """Adds d(sum dL_dimg * img [+ sum dL_dflow * flow])/d(params) into `grads` (created
    zeroed if None).  dL_dflow needs a frame rendered with the flow.  events: optional four
    torch.cuda.Event (timing enabled), set to the start and end of the blend adjoint and
    of the projection adjoint kernels (colour only)."""
    if grads is None:
        grads = grads_like(scene)
    dL = dL_dimg.contiguous().float()
    if getattr(st, "inst_grads", None) is None:
        st.inst_grads = torch.empty(max(st.capacity, 1) * B.GRAD_FLOATS, dtype=torch.float32, device=dL.device)
    g = B.Grads()
    for k in FIELDS:
        setattr(g, k, grads[k].data_ptr())
    for k in ("split_grad_t", "split_grad_xyz", "split_count"):
        if k in grads:
            setattr(g, k, grads[k].data_ptr())
    s = scene.struct()
    if dL_dflow is None and events is not None:
        ev = (C.c_void_p * 4)(*[e.cuda_event for e in events])
        B.check(B.lib.d4dgs_render_bwd_timed(C.byref(s), C.byref(B.camera_struct(cam)), float(t),
                                             C.byref(st.splats()), C.byref(st.bins()), C.byref(_bg(bg)),
                                             _ptr(st.final_T), _ptr(st.n_contrib), _ptr(dL), _ptr(st.inst_grads),
                                             C.byref(g), ev, _stream()))
    elif dL_dflow is None:
        B.check(B.lib.d4dgs_render_bwd(C.byref(s), C.byref(B.camera_struct(cam)), float(t), C.byref(st.splats()),
                                       C.byref(st.bins()), C.byref(_bg(bg)), _ptr(st.final_T), _ptr(st.n_contrib),
                                       _ptr(dL), _ptr(st.inst_grads), C.byref(g), _stream()))
    else:
        dF = dL_dflow.contiguous().float()
        B.check(B.lib.d4dgs_render_bwd_flow(C.byref(s), C.byref(B.camera_struct(cam)), float(t),
                                            C.byref(st.splats()), C.byref(st.bins()), C.byref(_bg(bg)),
                                            _ptr(st.final_T), _ptr(st.n_contrib), _ptr(dL), _ptr(dF),
                                            _ptr(st.inst_grads), C.byref(g), _stream()))
    return grads


def render_forward_flow(scene: DeviceScene, cam, t, bg=(0.0, 0.0, 0.0), capacity=None, keep_state=True,
                        cache: CamCache | None = None, motion=0):
    """Forward render with the optical flow of Sec. 3.3 (each splat's screen velocity
    blended with the colour weights).  Returns (img [3,H,W], flow [2,H,W], state)."""
    cap = capacity or default_capacity(scene.n, cam.width, cam.height)
    dev = scene.t["mean"].device
    st = FrameState(scene.n, cam.width, cam.height, cap, dev, flow=True, motion=motion)
    project(scene, cam, t, st, cache)
    ni = bin_sort(st, sync=True)
    if ni > st.capacity:
        st = FrameState(scene.n, cam.width, cam.height, int(ni * 1.25) + 1024, dev, flow=True, motion=motion)
        project(scene, cam, t, st, cache)
        assert bin_sort(st, sync=True) == ni
    st.num_instances = ni
    H, W = cam.height, cam.width
    st.img = torch.empty((3, H, W), dtype=torch.float32, device=dev)
    st.flow = torch.empty((2, H, W), dtype=torch.float32, device=dev)
    if keep_state:
        st.final_T = torch.empty((H, W), dtype=torch.float32, device=dev)
        st.n_contrib = torch.empty((H, W), dtype=torch.int32, device=dev)
    B.check(B.lib.d4dgs_render_fwd_flow(C.byref(st.splats()), C.byref(st.bins()), W, H, C.byref(_bg(bg)),
                                        _ptr(st.img), _ptr(st.flow), _ptr(st.final_T) if keep_state else None,
                                        _ptr(st.n_contrib) if keep_state else None, _stream()))
    return st.img, st.flow, st


def flow_loss(img, flow, lam, eps=1e-6, grad=True):
    """Flow-gradient guided consistency loss (Eq. 17) of a rendered image [3,H,W] and flow
    [2,H,W]; returns (loss as a 1-element tensor, dL/dflow or None)."""
    img = img.contiguous().float()
    flow = flow.contiguous().float()
    H, W = int(img.shape[1]), int(img.shape[2])
    nb = C.c_size_t(0)
    B.check(B.lib.d4dgs_flow_loss_workspace_size(W, H, C.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=img.device)
    loss = torch.empty(1, dtype=torch.float32, device=img.device)
    dflow = torch.empty_like(flow) if grad else None
    B.check(B.lib.d4dgs_flow_loss(_ptr(img), _ptr(flow), W, H, float(lam), float(eps), _ptr(ws), ws.numel(),
                                  _ptr(loss), _ptr(dflow), _stream()))
    return loss, dflow


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, cam, t, bg, sh_degree, capacity, *params):
        scene = DeviceScene(dict(zip(FIELDS, [p.detach() for p in params])), sh_degree)
        img, st = render_forward(scene, cam, t, bg, capacity)
        ctx.scene, ctx.cam, ctx.t, ctx.bg, ctx.st = scene, cam, t, bg, st
        return img

    @staticmethod
    def backward(ctx, dL_dimg):
        g = render_backward(ctx.scene, ctx.cam, ctx.t, ctx.bg, ctx.st, dL_dimg)
        return (None, None, None, None, None) + tuple(g[k] for k in FIELDS)


class _RenderFlowFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, cam, t, bg, sh_degree, capacity, *params):
        scene = DeviceScene(dict(zip(FIELDS, [p.detach() for p in params])), sh_degree)
        img, flow, st = render_forward_flow(scene, cam, t, bg, capacity)
        ctx.scene, ctx.cam, ctx.t, ctx.bg, ctx.st = scene, cam, t, bg, st
        return img, flow

    @staticmethod
    def backward(ctx, dL_dimg, dL_dflow):
        if dL_dimg is None:
            dL_dimg = torch.zeros_like(ctx.st.img)
        if dL_dflow is None:
            dL_dflow = torch.zeros_like(ctx.st.flow)
        g = render_backward(ctx.scene, ctx.cam, ctx.t, ctx.bg, ctx.st, dL_dimg, dL_dflow=dL_dflow)
        return (None, None, None, None, None) + tuple(g[k] for k in FIELDS)


class _FlowLossFn(torch.autograd.Function):
    """Eq. 17; the gradient flows to the flow only (the image-edge weight and the
    normalisers are constants of the loss)."""

    @staticmethod
    def forward(ctx, img, flow, lam, eps):
        loss, dflow = flow_loss(img.detach(), flow.detach(), lam, eps, grad=True)
        ctx.save_for_backward(dflow)
        return loss[0]

    @staticmethod
    def backward(ctx, g):
        (dflow,) = ctx.saved_tensors
        return None, dflow * g, None, None


def render_with_flow(mean, scale, quat, opacity, t_mean, t_scale, velocity, sh, *, cam, t, sh_degree,
                     bg=(0.0, 0.0, 0.0), capacity=None):
    """Differentiable render of one (camera, t) view returning (image, optical flow)."""
    return _RenderFlowFn.apply(cam, float(t), tuple(bg), int(sh_degree), capacity, mean, scale, quat, opacity,
                               t_mean, t_scale, velocity, sh)


def flow_gradient_loss(img, flow, lam, eps=1e-6):
    """Differentiable flow-gradient guided consistency loss (Eq. 17)."""
    return _FlowLossFn.apply(img, flow, float(lam), float(eps))


def render(mean, scale, quat, opacity, t_mean, t_scale, velocity, sh, *, cam, t, sh_degree, bg=(0.0, 0.0, 0.0),
           capacity=None):
    """Differentiable render of one (camera, t) view; gradients flow to all eight
    parameter tensors (planar layout, float32, CUDA)."""
    return _RenderFn.apply(cam, float(t), tuple(bg), int(sh_degree), capacity, mean, scale, quat, opacity, t_mean,
                           t_scale, velocity, sh)


class Renderer:
    """Fixed device buffers for repeated frames of one resolution (timing loops,
    sweeps).  Fully asynchronous: no host synchronisation per frame.  The argument
    structs of the entry points are built once (camera structs once per camera
    object: cameras passed here are treated as immutable), so a frame costs two
    foreign calls on the host: d4dgs_project_bin (projection and binning) and the
    blend.  project() + bin_sort() run the same stages through the separate calls."""

    def __init__(self, scene: DeviceScene, width, height, capacity=None, cache=True, keep_state=False,
                 tile_order=True):
        """cache: True (a camera-stage cache of its own), False, or a CamCache shared with
        other renderers (on other streams: see SharedCameraOrder)."""
        self.scene = scene
        self.width, self.height = int(width), int(height)
        dev = scene.t["mean"].device
        self.st = FrameState(scene.n, self.width, self.height,
                             capacity or default_capacity(scene.n, width, height), dev, tile_order=tile_order)
        if isinstance(cache, CamCache):
            self.cache = cache
        else:
            self.cache = CamCache(scene.n, dev) if cache else None
        self.keep_state = keep_state
        self.img = torch.empty((3, self.height, self.width), dtype=torch.float32, device=dev)
        if keep_state:
            self.st.final_T = torch.empty((self.height, self.width), dtype=torch.float32, device=dev)
            self.st.n_contrib = torch.empty((self.height, self.width), dtype=torch.int32, device=dev)
        st = self.st
        self._scene_s = scene.struct()
        self._sp = st.splats()
        self._bn = st.bins()
        self._cache_p = C.byref(self.cache.c) if self.cache is not None else None
        self._ws = (_ptr(st.ws), st.ws.numel())
        self._status = _ptr(st.status)
        self._img = _ptr(self.img)
        self._state = (_ptr(st.final_T), _ptr(st.n_contrib)) if keep_state else (None, None)
        self._cams = {}
        self._bgs = {}
        # the fused projection + binning needs the workspace's tile counters zero once
        B.check(B.lib.d4dgs_workspace_init(self._ws[0], self._ws[1], st.n, self.width, self.height, st.capacity,
                                           _stream()))
        torch.cuda.synchronize(dev)

    def _cam(self, cam):
        hit = self._cams.get(id(cam))
        if hit is None or hit[0] is not cam:
            hit = (cam, B.camera_struct(cam))
            self._cams[id(cam)] = hit
        return hit[1]

    def _bg(self, bg):
        key = tuple(float(x) for x in bg)
        a = self._bgs.get(key)
        if a is None:
            a = self._bgs[key] = _bg(key)
        return a

    def project(self, cam, t, stream=None):
        assert cam.width == self.width and cam.height == self.height
        B.check(B.lib.d4dgs_project(C.byref(self._scene_s), C.byref(self._cam(cam)), float(t), self._cache_p,
                                    C.byref(self._sp), stream or _stream()))

    def project_bin(self, cam, t, stream=None):
        """project() + bin_sort() in one call, with fewer kernels (same output)."""
        assert cam.width == self.width and cam.height == self.height
        B.check(B.lib.d4dgs_project_bin(C.byref(self._scene_s), C.byref(self._cam(cam)), float(t), self._cache_p,
                                        C.byref(self._sp), self._ws[0], self._ws[1], C.byref(self._bn),
                                        self._status, stream or _stream()))

    def bin_sort(self, stream=None):
        B.check(B.lib.d4dgs_bin_sort(C.byref(self._sp), self.st.n, self.width, self.height, self._ws[0],
                                     self._ws[1], C.byref(self._bn), self._status, stream or _stream()))

    def blend(self, bg=(0.0, 0.0, 0.0), stream=None, events=None):
        """events: optional (start, stop) torch.cuda.Event pair (timing enabled), set to the
        blend kernel's own start and end."""
        if events is None:
            B.check(B.lib.d4dgs_render_fwd(C.byref(self._sp), C.byref(self._bn), self.width, self.height,
                                           C.byref(self._bg(bg)), self._img, self._state[0], self._state[1],
                                           stream or _stream()))
        else:
            B.check(B.lib.d4dgs_render_fwd_timed(C.byref(self._sp), C.byref(self._bn), self.width, self.height,
                                                 C.byref(self._bg(bg)), self._img, self._state[0], self._state[1],
                                                 events[0].cuda_event, events[1].cuda_event, stream or _stream()))
        return self.img

    def render(self, cam, t, bg=(0.0, 0.0, 0.0)):
        stream = _stream()
        self.project_bin(cam, t, stream)
        return self.blend(bg, stream)

    def backward(self, cam, t, dL_dimg, grads, bg=(0.0, 0.0, 0.0), events=None):
        """Adjoint of the last render() (needs keep_state=True); adds into grads.  events:
        as render_backward."""
        assert self.keep_state
        if getattr(self.st, "inst_grads", None) is None:
            self.st.inst_grads = torch.empty(self.st.capacity * B.GRAD_FLOATS, dtype=torch.float32,
                                             device=self.img.device)
        return render_backward(self.scene, cam, t, bg, self.st, dL_dimg, grads, events=events)

    def overflowed(self):
        """True if any frame since the last reset exceeded the instance capacity."""
        return int(self.st.status.item()) != 0


class TimesRenderer:
    """Fixed buffers for T frames of one camera at T times, rendered by one
    d4dgs_render_times call (camera stage once, batched time stages, per-frame binning
    and blending on the library's own streams)."""

    def __init__(self, scene: DeviceScene, width, height, T, capacity=None, cache=True, tile_order=True):
        self.scene = scene
        self.width, self.height, self.T = int(width), int(height), int(T)
        dev = scene.t["mean"].device
        cap = capacity or default_capacity(scene.n, width, height)
        self.frames = [FrameState(scene.n, self.width, self.height, cap, dev, tile_order=tile_order)
                       for _ in range(self.T)]
        self.imgs = [torch.empty((3, self.height, self.width), dtype=torch.float32, device=dev) for _ in range(self.T)]
        self.cache = CamCache(scene.n, dev) if cache else None
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self._scene_s = scene.struct()
        self._sp = (B.Splats * self.T)(*[f.splats() for f in self.frames])
        self._bn = (B.Bins * self.T)(*[f.bins() for f in self.frames])
        self._ws = (C.c_void_p * self.T)(*[f.ws.data_ptr() for f in self.frames])
        self._ws_bytes = min(f.ws.numel() for f in self.frames)
        self._img = (C.c_void_p * self.T)(*[im.data_ptr() for im in self.imgs])
        self._t = (C.c_float * self.T)()
        self._cams = {}

    def render(self, cam, times, bg=(0.0, 0.0, 0.0), stream=None):
        """Renders self.T frames at `times` (length T); returns the T image tensors."""
        assert cam.width == self.width and cam.height == self.height and len(times) == self.T
        hit = self._cams.get(id(cam))
        if hit is None or hit[0] is not cam:
            hit = (cam, B.camera_struct(cam))
            self._cams[id(cam)] = hit
        for i, t in enumerate(times):
            self._t[i] = float(t)
        B.check(B.lib.d4dgs_render_times(C.byref(self._scene_s), C.byref(hit[1]), self.T, self._t,
                                         C.byref(self.cache.c) if self.cache is not None else None, self._sp,
                                         self._bn, self._ws, self._ws_bytes, C.byref(_bg(bg)), self._img,
                                         _ptr(self.status), stream or _stream()))
        return self.imgs

    def overflowed(self):
        return int(self.status.item()) != 0
