"""Torch-facing API of the HIP renderer: device tensors in, device tensors out.

PyTorch supplies device memory and streams; every computation runs in
libgeer.so.  Scene tensors use the library layout (float32, CUDA/HIP device,
contiguous): mean [3,N], scale [3,N], quat [4,N], opacity [N], sh [K*3,N].
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib

_contexts = {}


def context(device: int = 0):
    """The per-device library context (created on first use)."""
    if device not in _contexts:
        L = _lib.load()
        h = C.c_void_p()
        _lib.check(L.geer_create(int(device), C.byref(h)))
        _contexts[device] = h
    return _contexts[device]


def set_profiling(enable: bool, device: int = 0):
    _lib.check(_lib.load().geer_set_profiling(context(device), 1 if enable else 0), context(device))


def check_errors(device: int = 0, stream=None):
    """Waits for the work on `stream` (the current stream by default) and
    raises GeerError (status STALLED) if an earlier forward's association
    sort gave up on its bounded wait: that forward's outputs are invalid."""
    ctx = context(device)
    st = (stream or torch.cuda.current_stream(device)).cuda_stream
    _lib.check(_lib.load().geer_check(ctx, C.c_void_p(st)), ctx)


def profile_read(max_records: int = 64, device: int = 0):
    """Stage timings of the most recent renders (oldest first)."""
    recs = (_lib.GeerProfileRecord * max_records)()
    n = _lib.load().geer_profile_read(context(device), recs, max_records)
    if n < 0:
        raise _lib.GeerError(-n, "profile read failed")
    return [{k: getattr(recs[i], k) for k, _ in _lib.GeerProfileRecord._fields_} for i in range(n)]


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _check_scene(scene: dict):
    n = scene["mean"].shape[1]
    deg = int(scene["sh_degree"])
    shapes = {"mean": (3, n), "scale": (3, n), "quat": (4, n), "opacity": (n,), "sh": ((deg + 1) ** 2 * 3, n)}
    for k, shp in shapes.items():
        t = scene[k]
        if tuple(t.shape) != shp or t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("scene[%r] must be a contiguous float32 device tensor of shape %s, got %s %s %s"
                             % (k, shp, tuple(t.shape), t.dtype, t.device))
    return n, deg


def scene_from_numpy(s, device="cuda") -> dict:
    """Upload a host scene (the layout of the synthetic-scene module)."""
    return dict(mean=torch.as_tensor(s.mean, device=device).contiguous(),
                scale=torch.as_tensor(s.scale, device=device).contiguous(),
                quat=torch.as_tensor(s.quat, device=device).contiguous(),
                opacity=torch.as_tensor(s.opacity, device=device).contiguous(),
                sh=torch.as_tensor(s.sh, device=device).contiguous(),
                sh_degree=int(s.sh_degree))


class Frame:
    """Forward state kept by the library for the backward (geer_frame)."""

    def __init__(self, handle, ctx, cams):
        self.handle = handle
        self.ctx = ctx
        self.cams = cams

    def stats(self) -> dict:
        st = _lib.GeerFrameStats()
        _lib.check(_lib.load().geer_frame_get_stats(self.handle, C.byref(st)), self.ctx)
        return {k: int(getattr(st, k)) for k, _ in _lib.GeerFrameStats._fields_}

    def export(self, which: int) -> np.ndarray:
        L = _lib.load()
        nbytes = int(L.geer_frame_buffer_bytes(self.handle, which))
        out = np.zeros(max(nbytes // 4, 1), np.uint32)
        _lib.check(L.geer_frame_export(self.handle, which, C.c_void_p(out.ctypes.data), nbytes), self.ctx)
        return out[: nbytes // 4]

    def release(self):
        if self.handle:
            _lib.load().geer_frame_release(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def view_pixels(cams):
    return [int(c["width"]) * int(c["height"]) for c in cams]


def render(scene: dict, cams, opts: dict | None = None, keep_frame: bool = False, out=None, want_depth=True,
           want_trans=True):
    """Render the views `cams` (list of camera dicts).  Returns
    (rgb [sum 3*H*W], depth [sum H*W] | None, trans | None, Frame | None) as
    flat concatenations in view order (see views_of to split them)."""
    n, deg = _check_scene(scene)
    dev = scene["mean"].device
    ctx = context(dev.index or 0)
    npix = sum(view_pixels(cams))
    if out is None:
        rgb = torch.empty(3 * npix, device=dev, dtype=torch.float32)
        depth = torch.empty(npix, device=dev, dtype=torch.float32) if want_depth else None
        trans = torch.empty(npix, device=dev, dtype=torch.float32) if want_trans else None
    else:
        rgb, depth, trans = out
    views = (_lib.GeerView * len(cams))(*[_lib.make_view(c) for c in cams])
    sc = _lib.GeerScene()
    sc.n, sc.sh_degree, sc.reserved = n, deg, 0
    sc.mean, sc.scale, sc.quat, sc.opacity, sc.sh = (scene[k].data_ptr() for k in
                                                    ("mean", "scale", "quat", "opacity", "sh"))
    op = _lib.make_opts(**(opts or {}))
    fh = C.c_void_p()
    stream = torch.cuda.current_stream(dev).cuda_stream
    _lib.check(_lib.load().geer_render(ctx, C.byref(sc), len(cams), views, C.byref(op), _ptr(rgb), _ptr(depth),
                                       _ptr(trans), C.byref(fh) if keep_frame else None, C.c_void_p(stream)), ctx)
    frame = Frame(fh, ctx, cams) if keep_frame else None
    return rgb, depth, trans, frame


def render_static(scene: dict, cams, opts: dict | None = None, out=None, want_depth=True, want_trans=True):
    """The same forward as render(), through the library's allocation-free
    entry point: every intermediate buffer lives in its fixed device array
    (the outputs are the caller's).  Waits for the stream; raises GeerError
    (GEER_ERR_CAPACITY) when the scene or its association list does not fit
    the array.  Returns (rgb, depth | None, trans | None)."""
    n, deg = _check_scene(scene)
    dev = scene["mean"].device
    ctx = context(dev.index or 0)
    npix = sum(view_pixels(cams))
    if out is None:
        rgb = torch.empty(3 * npix, device=dev, dtype=torch.float32)
        depth = torch.empty(npix, device=dev, dtype=torch.float32) if want_depth else None
        trans = torch.empty(npix, device=dev, dtype=torch.float32) if want_trans else None
    else:
        rgb, depth, trans = out
    views = (_lib.GeerView * len(cams))(*[_lib.make_view(c) for c in cams])
    sc = _lib.GeerScene()
    sc.n, sc.sh_degree, sc.reserved = n, deg, 0
    sc.mean, sc.scale, sc.quat, sc.opacity, sc.sh = (scene[k].data_ptr() for k in
                                                    ("mean", "scale", "quat", "opacity", "sh"))
    op = _lib.make_opts(**(opts or {}))
    stream = torch.cuda.current_stream(dev).cuda_stream
    _lib.check(_lib.load().geer_render_static(ctx, C.byref(sc), len(cams), views, C.byref(op), _ptr(rgb),
                                              _ptr(depth), _ptr(trans), C.c_void_p(stream)), ctx)
    return rgb, depth, trans


def views_of(flat: torch.Tensor, cams, channels: int):
    """Split a flat concatenated output into per-view [C,H,W] tensors."""
    outs, off = [], 0
    for c in cams:
        hw = int(c["width"]) * int(c["height"])
        outs.append(flat[off: off + channels * hw].view(channels, int(c["height"]), int(c["width"])))
        off += channels * hw
    return outs


def backward(frame: Frame, scene: dict, dl_drgb: torch.Tensor, accumulate: bool = False, grads=None):
    """Gradients of the loss with respect to the scene given dL/dRGB (same
    layout as the forward's rgb).  Returns a dict of tensors in the scene
    layout (App. C chain, computed by the library)."""
    n, deg = _check_scene(scene)
    dev = scene["mean"].device
    if grads is None:
        grads = {k: torch.zeros_like(scene[k]) if accumulate else torch.empty_like(scene[k])
                 for k in ("mean", "scale", "quat", "opacity", "sh")}
    g = dl_drgb.contiguous()
    stream = torch.cuda.current_stream(dev).cuda_stream
    _lib.check(_lib.load().geer_render_backward(frame.ctx, frame.handle, _ptr(g), _ptr(grads["mean"]),
                                                _ptr(grads["scale"]), _ptr(grads["quat"]), _ptr(grads["opacity"]),
                                                _ptr(grads["sh"]), 1 if accumulate else 0, C.c_void_p(stream)),
               frame.ctx)
    return grads


def l1_loss(rgb: torch.Tensor, target: torch.Tensor, mask: torch.Tensor):
    """L1 over valid rays of one view: returns (loss [1], dL/drgb) computed on
    the device; rgb, target: [3*P] planar, mask: uint8 [P]."""
    dev = rgb.device
    P = mask.numel()
    dl = torch.empty_like(rgb)
    loss = torch.empty(1, device=dev, dtype=torch.float32)
    ctx = context(dev.index or 0)
    stream = torch.cuda.current_stream(dev).cuda_stream
    _lib.check(_lib.load().geer_l1_loss(ctx, P, _ptr(rgb.contiguous()), _ptr(target.contiguous()),
                                        _ptr(mask.contiguous()), _ptr(dl), _ptr(loss), C.c_void_p(stream)), ctx)
    return loss, dl


def reproject(beap: torch.Tensor, cam: dict, native_size=None, with_valid: bool = True):
    """Resamples a rendered BEAP image of `cam` ([C, H, W] or flat C*H*W,
    float32 on the device) onto the camera's native sensor (App. E inverse
    interpolation).  Returns (native [C, Hn, Wn], valid [Hn, Wn] uint8 or
    None); native_size = (Wn, Hn), default the grid's size."""
    w, h = int(cam["width"]), int(cam["height"])
    if beap.numel() % (w * h) != 0 or beap.dtype != torch.float32 or not beap.is_cuda:
        raise ValueError("beap must be a float32 device tensor of C x %d x %d values" % (h, w))
    C_ = beap.numel() // (w * h)
    nw, nh = native_size if native_size else (w, h)
    dev = beap.device
    src = beap.contiguous()
    out = torch.empty(C_ * nw * nh, device=dev, dtype=torch.float32)
    valid = torch.empty(nw * nh, device=dev, dtype=torch.uint8) if with_valid else None
    ctx = context(dev.index or 0)
    st = torch.cuda.current_stream(dev).cuda_stream
    _lib.check(_lib.load().geer_reproject(ctx, C.byref(_lib.make_view(cam)), int(nw), int(nh), C_, _ptr(src),
                                          _ptr(out), _ptr(valid), C.c_void_p(st)), ctx)
    return out.view(C_, nh, nw), (valid.view(nh, nw) if valid is not None else None)


class _Render(torch.autograd.Function):
    """Differentiable render: RGB depends on (mean, scale, quat, opacity, sh);
    depth and transmittance are returned without gradient."""

    @staticmethod
    def forward(ctx, mean, scale, quat, opacity, sh, sh_degree, cams, opts):
        scene = dict(mean=mean, scale=scale, quat=quat, opacity=opacity, sh=sh, sh_degree=sh_degree)
        rgb, depth, trans, frame = render(scene, cams, opts=opts, keep_frame=True)
        ctx.frame = frame
        ctx.sh_degree = sh_degree
        ctx.save_for_backward(mean, scale, quat, opacity, sh)
        ctx.mark_non_differentiable(depth, trans)
        return rgb, depth, trans

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_trans):
        mean, scale, quat, opacity, sh = ctx.saved_tensors
        scene = dict(mean=mean, scale=scale, quat=quat, opacity=opacity, sh=sh, sh_degree=ctx.sh_degree)
        if g_rgb is None:
            g_rgb = torch.zeros(3 * sum(view_pixels(ctx.frame.cams)), device=mean.device)
        grads = backward(ctx.frame, scene, g_rgb)
        ctx.frame.release()
        return grads["mean"], grads["scale"], grads["quat"], grads["opacity"], grads["sh"], None, None, None


def render_differentiable(scene: dict, cams, opts: dict | None = None):
    """torch.autograd entry point: returns (rgb, depth, trans) flat tensors;
    backward() on a function of rgb fills .grad of the scene tensors."""
    return _Render.apply(scene["mean"], scene["scale"], scene["quat"], scene["opacity"], scene["sh"],
                         int(scene["sh_degree"]), cams, opts)


def _scene_struct(scene: dict):
    n, deg = _check_scene(scene)
    sc = _lib.GeerScene()
    sc.n, sc.sh_degree, sc.reserved = n, deg, 0
    sc.mean, sc.scale, sc.quat, sc.opacity, sc.sh = (scene[k].data_ptr() for k in
                                                    ("mean", "scale", "quat", "opacity", "sh"))
    return sc


def _views(cams):
    return (_lib.GeerView * len(cams))(*[_lib.make_view(c) for c in cams])


def plan_workspace_bytes(scene: dict, cams, entry_capacity: int, opts: dict | None = None) -> int:
    """Device workspace (bytes) of a plan for this batch shape."""
    ctx = context(scene["mean"].device.index or 0)
    out = C.c_int64()
    _lib.check(_lib.load().geer_plan_workspace_bytes(ctx, C.byref(_scene_struct(scene)), len(cams), _views(cams),
                                                     C.byref(_lib.make_opts(**(opts or {}))), int(entry_capacity),
                                                     C.byref(out)), ctx)
    return int(out.value)


class Plan:
    """A captured forward for a fixed batch shape (geer_plan): every launch
    renders new cameras of the same grid sizes into the plan's outputs with
    one graph replay.  `workspace` is an optional uint8 device tensor (shared
    only by plans launched on one stream); `out` = (rgb, depth, trans)."""

    def __init__(self, scene: dict, cams, entry_capacity: int, opts: dict | None = None, workspace=None,
                 out=None):
        dev = scene["mean"].device
        self.ctx = context(dev.index or 0)
        self.scene = scene  # keeps the scene tensors alive
        self.shapes = [(int(c["width"]), int(c["height"])) for c in cams]
        npix = sum(view_pixels(cams))
        if out is None:
            out = (torch.empty(3 * npix, device=dev), torch.empty(npix, device=dev), torch.empty(npix, device=dev))
        self.rgb, self.depth, self.trans = out
        self.workspace = workspace
        ws_ptr = C.c_void_p(workspace.data_ptr()) if workspace is not None else None
        ws_bytes = workspace.numel() if workspace is not None else 0
        h = C.c_void_p()
        _lib.check(_lib.load().geer_plan_create(self.ctx, C.byref(_scene_struct(scene)), len(cams), _views(cams),
                                                C.byref(_lib.make_opts(**(opts or {}))), int(entry_capacity), ws_ptr,
                                                ws_bytes, _ptr(self.rgb), _ptr(self.depth), _ptr(self.trans),
                                                C.byref(h)), self.ctx)
        self.handle = h

    def launch(self, cams, stream=None):
        if stream is None:
            stream = torch.cuda.current_stream()
        _lib.check(_lib.load().geer_plan_launch(self.handle, _views(cams), C.c_void_p(stream.cuda_stream)), self.ctx)

    def status(self) -> dict:
        """Outcome of the last launch (waits for it): PBF pairs, capacity,
        whether they overflowed it and whether a sort stalled -- either way
        the launch's outputs are invalid and must be rendered again."""
        e, cap = C.c_int64(), C.c_int64()
        st = _lib.load().geer_plan_entries(self.handle, C.byref(e), C.byref(cap))
        if st not in (0, _lib.ERR_CAPACITY, _lib.ERR_STALLED):
            _lib.check(st, self.ctx)
        return dict(entries=int(e.value), capacity=int(cap.value), overflow=int(e.value) > int(cap.value),
                    stalled=st == _lib.ERR_STALLED)

    def entries(self):
        """(entries, capacity, overflowed) of the last launch (waits for it);
        raises GeerError if a sort stalled."""
        s = self.status()
        if s["stalled"]:
            _lib.check(_lib.ERR_STALLED, self.ctx)
        return s["entries"], s["capacity"], s["overflow"]

    def stats(self) -> dict:
        """Device-counted statistics of the last launch (waits for it)."""
        st = _lib.GeerFrameStats()
        _lib.check(_lib.load().geer_plan_get_stats(self.handle, C.byref(st)), self.ctx)
        return {k: int(getattr(st, k)) for k, _ in _lib.GeerFrameStats._fields_}

    def mark_stalled(self):
        """Test hook: reports the last launch as stalled (host-side flag)."""
        _lib.check(_lib.load().geer_debug_mark_stalled(self.ctx, self.handle), self.ctx)

    def device_bytes(self) -> int:
        return int(_lib.load().geer_plan_device_bytes(self.handle))

    def destroy(self):
        if self.handle:
            _lib.load().geer_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class TrainPlan(Plan):
    """A captured batched training step (geer_train_plan): per view the
    forward, the L1 loss against `target` over `mask` (every ray when None)
    and the backward; every launch fills rgb, loss ([1]) and the scene-shaped
    gradient tensors in `grads` with the gradient of the mean of the views'
    L1 losses.  `target` / `mask` / rgb use the concatenated per-view layout
    of render()."""

    def __init__(self, scene: dict, cams, entry_capacity: int, target: torch.Tensor, mask=None,
                 opts: dict | None = None, workspace=None):
        dev = scene["mean"].device
        self.ctx = context(dev.index or 0)
        self.scene = scene
        self.shapes = [(int(c["width"]), int(c["height"])) for c in cams]
        npix = sum(view_pixels(cams))
        self.target = target.contiguous()
        self.mask = mask.contiguous() if mask is not None else None
        if self.target.numel() != 3 * npix or (self.mask is not None and self.mask.numel() != npix):
            raise ValueError("target must hold 3 x %d values and mask %d" % (npix, npix))
        self.rgb = torch.empty(3 * npix, device=dev)
        self.depth = self.trans = None
        self.loss = torch.zeros(1, device=dev)
        self.grads = {k: torch.empty_like(scene[k]) for k in ("mean", "scale", "quat", "opacity", "sh")}
        self.workspace = workspace
        ws_ptr = C.c_void_p(workspace.data_ptr()) if workspace is not None else None
        ws_bytes = workspace.numel() if workspace is not None else 0
        g = self.grads
        h = C.c_void_p()
        _lib.check(_lib.load().geer_train_plan_create(
            self.ctx, C.byref(_scene_struct(scene)), len(cams), _views(cams), C.byref(_lib.make_opts(**(opts or {}))),
            int(entry_capacity), ws_ptr, ws_bytes, _ptr(self.target), _ptr(self.mask), _ptr(self.rgb),
            _ptr(self.loss), _ptr(g["mean"]), _ptr(g["scale"]), _ptr(g["quat"]), _ptr(g["opacity"]), _ptr(g["sh"]),
            C.byref(h)), self.ctx)
        self.handle = h


def train_plan_workspace_bytes(scene: dict, cams, entry_capacity: int, opts: dict | None = None) -> int:
    ctx = context(scene["mean"].device.index or 0)
    out = C.c_int64()
    _lib.check(_lib.load().geer_train_plan_workspace_bytes(ctx, C.byref(_scene_struct(scene)), len(cams),
                                                           _views(cams), C.byref(_lib.make_opts(**(opts or {}))),
                                                           int(entry_capacity), C.byref(out)), ctx)
    return int(out.value)
