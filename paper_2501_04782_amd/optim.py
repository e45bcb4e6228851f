"""Fused Adan optimizer (Sec. 4.1: Adan, learning rate 0.01 with exponential
decay 0.99995 per step) over the scene's FP32 parameter tensors, one
``gv_adan_step`` launch per step (argument marshalling only)."""
from __future__ import annotations

import ctypes
from typing import Dict, Sequence

import torch

from . import _lib as L
from .raster import _stream


class Adan:
    """Adan over up to 16 FP32 tensors (updated in place).  ``step(grads)``
    takes the gradients in the same order as ``params``."""

    def __init__(self, params: Sequence[torch.Tensor], lr: float = 0.01, gamma: float = 0.99995,
                 betas=(0.02, 0.08, 0.01), eps: float = 1e-8, weight_decay: float = 0.0):
        params = list(params)
        if not 1 <= len(params) <= L.GV_ADAN_MAX_TENSORS:
            raise ValueError(f"Adan takes 1..{L.GV_ADAN_MAX_TENSORS} tensors")
        for p in params:
            if p.dtype != torch.float32 or not p.is_contiguous() or not p.is_cuda:
                raise ValueError("Adan parameters must be contiguous float32 device tensors")
        self.params = params
        self.states = [torch.zeros((4,) + tuple(p.shape), device=p.device) for p in params]
        self.lr0, self.gamma, self.betas, self.eps, self.wd = lr, gamma, betas, eps, weight_decay
        self.k = 0

    def lr(self) -> float:
        return self.lr0 * self.gamma ** self.k

    def step(self, grads: Sequence[torch.Tensor]) -> None:
        grads = list(grads)
        if len(grads) != len(self.params):
            raise ValueError("one gradient per parameter tensor")
        n = len(self.params)
        for p, g in zip(self.params, grads):
            if g.shape != p.shape or g.dtype != torch.float32 or not g.is_contiguous():
                raise ValueError("gradients must match the parameters (contiguous float32)")
        P = (ctypes.c_void_p * n)(*[p.data_ptr() for p in self.params])
        G = (ctypes.c_void_p * n)(*[g.data_ptr() for g in grads])
        S = (ctypes.c_void_p * n)(*[s.data_ptr() for s in self.states])
        C = (ctypes.c_int64 * n)(*[p.numel() for p in self.params])
        hp = L.GvAdanParams(self.lr(), self.betas[0], self.betas[1], self.betas[2], self.eps, self.wd, self.k, 0)
        L.check(L.load().gv_adan_step(n, P, G, S, C, ctypes.byref(hp), _stream()), "gv_adan_step")
        self.k += 1

    @classmethod
    def for_scene(cls, scene, **kw) -> "Adan":
        """All FP32 parameter tensors of a raster.Scene."""
        names = [k for k in ("means", "log_scales", "quats", "opacity_logits", "colors", "mean_coeffs", "ctrl",
                             "scale_coeffs", "quat_coeffs", "sh") if getattr(scene, k) is not None]
        opt = cls([getattr(scene, k) for k in names], **kw)
        opt.names = names
        return opt

    def step_grads(self, grads: Dict[str, torch.Tensor]) -> None:
        """Step with a gradient dict as returned by render_batch (for_scene order)."""
        self.step([grads[k] for k in self.names])
