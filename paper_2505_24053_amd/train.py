"""Training around the renderer: the optimiser's raw parameters, the fused
Adam step and the clone / split / prune refinement (geer_adam_step,
geer_densify).  Tensors are device float32; every computation runs in
libgeer.so.

Raw rows of a state of n Gaussians with SH degree d (K = (d + 1)^2), one
tensor [11 + 3K, n]: mean 3, log scale 3, quaternion 4, opacity logit 1, SH
3K.  The activated scale exp(log s) and opacity sigmoid(logit) live beside
it; scene() gives the renderer's view of the state.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import _lib, renderer


def rows(sh_degree: int) -> int:
    return 11 + 3 * (sh_degree + 1) ** 2


class TrainState:
    """Raw parameters, activated scale and opacity, Adam moments and the
    refinement statistics of one scene on one device."""

    def __init__(self, raw: torch.Tensor, sh_degree: int, m=None, v=None, accum=None, count=None,
                 scale=None, opacity=None, activate=True):
        if raw.dim() != 2 or raw.shape[0] != rows(sh_degree) or raw.dtype != torch.float32 or not raw.is_cuda:
            raise ValueError("raw must be a float32 device tensor [%d, n]" % rows(sh_degree))
        self.raw = raw.contiguous()
        self.sh_degree = int(sh_degree)
        n = self.raw.shape[1]
        dev = self.raw.device
        z = lambda *shape: torch.zeros(*shape, device=dev, dtype=torch.float32)  # noqa: E731
        self.m = m if m is not None else z(self.raw.shape)
        self.v = v if v is not None else z(self.raw.shape)
        self.accum = accum if accum is not None else z(n)
        self.count = count if count is not None else z(n)
        self.scale = scale if scale is not None else z(3, n)
        self.opacity = opacity if opacity is not None else z(n)
        self.ctx = renderer.context(dev.index or 0)
        if activate:
            _lib.check(_lib.load().geer_activate(self.ctx, C.byref(self.struct()),
                                                 C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)), self.ctx)

    @property
    def n(self) -> int:
        return int(self.raw.shape[1])

    @classmethod
    def from_scene(cls, scene, device="cuda"):
        """From a host scene (linear scales, opacities in (0, 1))."""
        op = np.clip(scene.opacity.astype(np.float64), 1e-6, 1 - 1e-6)
        raw = np.concatenate([scene.mean, np.log(scene.scale.astype(np.float64)), scene.quat,
                              np.log(op / (1 - op))[None], scene.sh]).astype(np.float32)
        return cls(torch.as_tensor(raw, device=device), scene.sh_degree)

    def struct(self):
        t = _lib.GeerTrainState()
        t.n, t.sh_degree, t.reserved = self.n, self.sh_degree, 0
        for k in ("raw", "scale", "opacity", "m", "v", "accum", "count"):
            setattr(t, k, getattr(self, k).data_ptr())
        return t

    def scene(self) -> dict:
        """The renderer's scene: (mean, activated scale, quaternion,
        activated opacity, SH), sharing this state's memory."""
        return dict(mean=self.raw[0:3], scale=self.scale, quat=self.raw[6:10], opacity=self.opacity,
                    sh=self.raw[11:], sh_degree=self.sh_degree)

    def adam_step(self, grads: dict, step: int, lr=(1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3), betas=(0.9, 0.999),
                  eps=1e-15, stats=True):
        """One fused Adam step on the renderer's gradients (dict with the
        scene's keys), bias-corrected for step `step` (>= 1)."""
        o = _lib.GeerAdamOpts()
        o.lr_mean, o.lr_scale, o.lr_quat, o.lr_opacity, o.lr_sh = (float(x) for x in lr)
        o.beta1, o.beta2, o.eps, o.step, o.reserved = float(betas[0]), float(betas[1]), float(eps), int(step), 0
        t = self.struct()
        if not stats:
            t.accum = t.count = None
        g = [grads[k].contiguous() for k in ("mean", "scale", "quat", "opacity", "sh")]
        st = torch.cuda.current_stream(self.raw.device).cuda_stream
        _lib.check(_lib.load().geer_adam_step(self.ctx, C.byref(t), C.byref(o), *[C.c_void_p(x.data_ptr()) for x in g],
                                              C.c_void_p(st)), self.ctx)

    def densify(self, noise: torch.Tensor, grad_threshold=2e-4, split_scale=0.1, min_opacity=0.005,
                split_shrink=1.6) -> "TrainState":
        """The refined state (a new one; this one is unchanged).  noise:
        standard normal draws [6, n] for the split children's offsets."""
        n = self.n
        cap = max(2 * n, 1)
        dev = self.raw.device
        R = rows(self.sh_degree)
        bufs = {k: torch.empty(R * cap if k in ("raw", "m", "v") else (3 * cap if k == "scale" else cap),
                               device=dev, dtype=torch.float32)
                for k in ("raw", "scale", "opacity", "m", "v", "accum", "count")}
        out = _lib.GeerTrainState()
        out.n, out.sh_degree, out.reserved = cap, self.sh_degree, 0
        for k, b in bufs.items():
            setattr(out, k, b.data_ptr())
        o = _lib.GeerDensifyOpts()
        o.grad_threshold, o.split_scale = float(grad_threshold), float(split_scale)
        o.min_opacity, o.split_shrink = float(min_opacity), float(split_shrink)
        noise = noise.contiguous()
        if tuple(noise.shape) != (6, n):
            raise ValueError("noise must be [6, %d]" % n)
        st = torch.cuda.current_stream(dev).cuda_stream
        _lib.check(_lib.load().geer_densify(self.ctx, C.byref(self.struct()), C.byref(o), C.c_void_p(noise.data_ptr()),
                                            C.byref(out), C.c_void_p(st)), self.ctx)
        m = int(out.n)
        view = lambda k, r: bufs[k][: r * m].view(r, m) if r > 1 else bufs[k][:m]  # noqa: E731
        return TrainState(view("raw", R), self.sh_degree, m=view("m", R), v=view("v", R), accum=view("accum", 1),
                          count=view("count", 1), scale=view("scale", 3), opacity=view("opacity", 1), activate=False)


def logit(p: float) -> float:
    return math.log(p / (1 - p))
