"""Torch-facing binding of the gfx950 rasterizer (libgv.so).

Every computation runs in the library's HIP kernels; this module only checks
tensor shapes/dtypes, passes device pointers and the current HIP stream, and
wraps the calls in ``torch.autograd.Function`` objects.  Names follow the C ABI
(include/gv.h): ``render_fwd``, ``render_bwd``, ``render_batch``,
``project_fwd``, ``BatchGraph``.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t: torch.Tensor, shape, dtype, name: str):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)} != {tuple(shape)}")
    if t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype} != {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


@dataclasses.dataclass
class Camera:
    """Pinhole intrinsics shared by all frames (Sec. 3.4) + rasterizer constants."""
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    near_plane: float = 0.01
    dilation: float = 0.3
    bg: tuple = (0.0, 0.0, 0.0)

    @classmethod
    def of(cls, c) -> "Camera":
        return cls(int(c.width), int(c.height), float(c.fx), float(c.fy), float(c.cx), float(c.cy),
                   float(c.near_plane), float(c.dilation), tuple(float(x) for x in c.bg))

    def c(self) -> L.GvCamera:
        g = L.GvCamera()
        g.width, g.height = self.width, self.height
        g.fx, g.fy, g.cx, g.cy = self.fx, self.fy, self.cx, self.cy
        g.near_plane, g.dilation = self.near_plane, self.dilation
        for i in range(3):
            g.bg[i] = self.bg[i]
        return g


class Scene:
    """Gaussian parameters on the device, planar [C][N] (fp32 or bf16)."""

    FIELDS = ("means", "log_scales", "quats", "opacity_logits", "colors")
    ROWS = dict(means=3, log_scales=3, quats=4, opacity_logits=None, colors=3)
    OPTIONAL = ("mean_coeffs", "ctrl", "scale_coeffs", "quat_coeffs", "sh")
    SH_DEGREE = {3: 1, 8: 2, 15: 3}

    def __init__(self, means, log_scales, quats, opacity_logits, colors, mean_coeffs=None, ctrl=None,
                 scale_coeffs=None, quat_coeffs=None, sh=None):
        """Time dependence (Sec. 3.2, Eq. 2-3), all optional: ``mean_coeffs``
        [3][3][N] cubic mean; ``ctrl`` [M][3][N] B-spline control points (then
        ``means`` is not read); ``scale_coeffs`` [3][3][N] and ``quat_coeffs``
        [3][4][N] cubic log-scales and quaternion.  View-dependent colour
        (Sec. 3.1): ``sh`` [(D+1)^2-1][3][N], SH coefficients of degrees 1..D
        (``colors`` is the degree-0 term)."""
        self.means, self.log_scales, self.quats = means, log_scales, quats
        self.opacity_logits, self.colors, self.mean_coeffs = opacity_logits, colors, mean_coeffs
        self.ctrl, self.scale_coeffs, self.quat_coeffs, self.sh = ctrl, scale_coeffs, quat_coeffs, sh
        dt = log_scales.dtype
        if dt not in (torch.float32, torch.bfloat16):
            raise ValueError("parameters must be float32 or bfloat16")
        n = opacity_logits.shape[-1]
        for f in self.FIELDS:
            rows = self.ROWS[f]
            if f == "means" and means is None and ctrl is not None:
                continue
            _need(getattr(self, f), (n,) if rows is None else (rows, n), dt, f)
        if mean_coeffs is not None:
            _need(mean_coeffs, (3, 3, n), dt, "mean_coeffs")
        if ctrl is not None:
            if mean_coeffs is not None:
                raise ValueError("a scene has either B-spline control points or cubic mean coefficients")
            if ctrl.dim() != 3 or not (4 <= ctrl.shape[0] <= L.GV_MAX_CTRL):
                raise ValueError(f"ctrl must be [M][3][N] with 4 <= M <= {L.GV_MAX_CTRL}")
            _need(ctrl, (ctrl.shape[0], 3, n), dt, "ctrl")
        if scale_coeffs is not None:
            _need(scale_coeffs, (3, 3, n), dt, "scale_coeffs")
        if quat_coeffs is not None:
            _need(quat_coeffs, (3, 4, n), dt, "quat_coeffs")
        self.sh_degree = 0
        if sh is not None:
            if sh.dim() != 3 or int(sh.shape[0]) not in self.SH_DEGREE:
                raise ValueError("sh must be [(D+1)^2-1][3][N] with D in 1..3")
            _need(sh, (sh.shape[0], 3, n), dt, "sh")
            self.sh_degree = self.SH_DEGREE[int(sh.shape[0])]
        self.dtype = L.GV_BF16 if dt == torch.bfloat16 else L.GV_F32
        self.n = int(n)

    @property
    def device(self):
        return self.log_scales.device

    @property
    def n_ctrl(self) -> int:
        return 0 if self.ctrl is None else int(self.ctrl.shape[0])

    @classmethod
    def from_synth(cls, s, device="cuda") -> "Scene":
        """From a gv_synth.Scene (storage arrays)."""
        def t(a):
            if a is None:
                return None
            if s.dtype == "bf16":
                return torch.from_numpy(np.ascontiguousarray(a).view(np.int16)).to(device).view(torch.bfloat16)
            return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
        return cls(t(s.means), t(s.log_scales), t(s.quats), t(s.opacity_logits), t(s.colors), t(s.mean_coeffs),
                   t(getattr(s, "ctrl", None)), t(getattr(s, "scale_coeffs", None)),
                   t(getattr(s, "quat_coeffs", None)), t(getattr(s, "sh", None)))

    def c(self) -> L.GvScene:
        g = L.GvScene()
        g.n, g.dtype = self.n, self.dtype
        ptr = lambda x: None if x is None else x.data_ptr()  # noqa: E731
        g.means, g.log_scales, g.quats = ptr(self.means), ptr(self.log_scales), ptr(self.quats)
        g.opacity_logits, g.colors = ptr(self.opacity_logits), ptr(self.colors)
        g.mean_coeffs = ptr(self.mean_coeffs)
        g.n_ctrl, g.ctrl = self.n_ctrl, ptr(self.ctrl)
        g.scale_coeffs, g.quat_coeffs = ptr(self.scale_coeffs), ptr(self.quat_coeffs)
        g.sh_degree, g.sh = self.sh_degree, ptr(self.sh)
        return g


def grad_buffers(scene: Scene) -> dict:
    """FP32 gradient outputs shaped like the scene's parameters."""
    dev = scene.device
    n = scene.n
    g = dict(means=torch.zeros(3, n, device=dev), log_scales=torch.zeros(3, n, device=dev),
             quats=torch.zeros(4, n, device=dev), opacity_logits=torch.zeros(n, device=dev),
             colors=torch.zeros(3, n, device=dev))
    for k in Scene.OPTIONAL:
        v = getattr(scene, k)
        g[k] = None if v is None else torch.zeros(v.shape, device=dev)
    g["intrinsics"] = torch.zeros(4, device=dev)  # dL/d(fx, fy, cx, cy)
    return g


def _grads_c(g: dict) -> L.GvGrads:
    s = L.GvGrads()
    for k in ("means", "log_scales", "quats", "opacity_logits", "colors") + Scene.OPTIONAL + ("intrinsics",):
        t = g.get(k)
        if t is not None:
            _need(t, t.shape, torch.float32, f"grad {k}")
        setattr(s, k, None if t is None else t.data_ptr())
    return s


class Workspace:
    """Caller-owned scratch memory of one render call (see gv_workspace_bytes)."""

    def __init__(self, camera: Camera, n: int, frames: int, k_capacity: int, device="cuda"):
        lib = L.load()
        out = ctypes.c_size_t()
        L.check(lib.gv_workspace_bytes(ctypes.byref(camera.c()), int(n), int(frames), int(k_capacity),
                                       ctypes.byref(out)), "gv_workspace_bytes")
        self.nbytes = int(out.value)
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.camera, self.n, self.frames, self.k_capacity = camera, int(n), int(frames), int(k_capacity)

    @property
    def ptr(self):
        return ctypes.c_void_p(self.buf.data_ptr())

    def status(self) -> dict:
        w = (ctypes.c_uint32 * 4)()
        L.check(L.load().gv_device_status(self.ptr, w), "gv_device_status")
        return dict(overflow=int(w[0]), nonfinite=int(w[1]), intersections=int(w[2]) | (int(w[3]) << 32))


def project_fwd(scene: Scene, camera: Camera, pose7: torch.Tensor, t: float, ws: Workspace):
    """Per-Gaussian records (u, v, A00, A01, A11, depth, opacity, 0) and tile counts."""
    _need(pose7, (7,), torch.float32, "pose7")
    rec = torch.empty(scene.n, 8, device=pose7.device)
    cnt = torch.empty(scene.n, dtype=torch.int32, device=pose7.device)
    L.check(L.load().gv_project_fwd(ctypes.byref(scene.c()), ctypes.byref(camera.c()), _ptr(pose7), float(t),
                                    _ptr(rec), _ptr(cnt), ws.ptr, ws.nbytes, _stream()), "gv_project_fwd")
    return rec, cnt


def render_fwd(scene: Scene, camera: Camera, pose7: torch.Tensor, t: float, ws: Workspace,
               image: Optional[torch.Tensor] = None, T_final: Optional[torch.Tensor] = None):
    """One frame: image [3][H][W] (and T_final [H][W])."""
    _need(pose7, (7,), torch.float32, "pose7")
    H, W = camera.height, camera.width
    if image is None:
        image = torch.empty(3, H, W, device=pose7.device)
    _need(image, (3, H, W), torch.float32, "image")
    if T_final is not None:
        _need(T_final, (H, W), torch.float32, "T_final")
    L.check(L.load().gv_render_fwd(ctypes.byref(scene.c()), ctypes.byref(camera.c()), _ptr(pose7), float(t),
                                   _ptr(image), _ptr(T_final), ws.ptr, ws.nbytes, _stream()), "gv_render_fwd")
    return image


def render_fwd_noalloc(scene: Scene, camera: Camera, pose7: torch.Tensor, t: float, image: torch.Tensor,
                       T_final: Optional[torch.Tensor] = None) -> torch.Tensor:
    """render_fwd into caller-given outputs with the library's fixed scratch
    instead of a workspace (no device allocation; calls on one GPU must not
    overlap)."""
    _need(pose7, (7,), torch.float32, "pose7")
    H, W = camera.height, camera.width
    _need(image, (3, H, W), torch.float32, "image")
    if T_final is not None:
        _need(T_final, (H, W), torch.float32, "T_final")
    L.check(L.load().gv_render_fwd_noalloc(ctypes.byref(scene.c()), ctypes.byref(camera.c()), _ptr(pose7), float(t),
                                           _ptr(image), _ptr(T_final), _stream()), "gv_render_fwd_noalloc")
    return image


def render_bwd(scene: Scene, camera: Camera, pose7: torch.Tensor, t: float, ws: Workspace, image: torch.Tensor,
               dL_dimage: Optional[torch.Tensor] = None, target: Optional[torch.Tensor] = None,
               loss_scale: float = 0.0, grads: Optional[dict] = None, dL_dpose7: Optional[torch.Tensor] = None,
               accumulate: bool = False):
    """Backward of the last render_fwd on ``ws``; returns (grads, dL_dpose7)."""
    H, W = camera.height, camera.width
    flags = L.GV_ACCUMULATE if accumulate else 0
    if target is not None:
        _need(target, (3, H, W), torch.float32, "target")
        flags |= L.GV_LOSS_L2
    else:
        _need(dL_dimage, (3, H, W), torch.float32, "dL_dimage")
    if grads is None:
        grads = grad_buffers(scene)
    if dL_dpose7 is None:
        dL_dpose7 = torch.empty(7, device=pose7.device)
    L.check(L.load().gv_render_bwd(ctypes.byref(scene.c()), ctypes.byref(camera.c()), _ptr(pose7), float(t),
                                   _ptr(image), _ptr(dL_dimage), _ptr(target), float(loss_scale), flags,
                                   ctypes.byref(_grads_c(grads)), _ptr(dL_dpose7), ws.ptr, ws.nbytes, _stream()),
            "gv_render_bwd")
    return grads, dL_dpose7


def _batch_args(scene, camera, poses, times, ws, targets, dL_dimages, flags, images, loss, grads, dL_dposes):
    F = int(poses.shape[0])
    H, W = camera.height, camera.width
    _need(poses, (F, 7), torch.float32, "poses")
    if times is not None:
        _need(times, (F,), torch.float32, "times")
    _need(images, (F, 3, H, W), torch.float32, "images")
    if targets is not None:
        _need(targets, (F, 3, H, W), torch.float32, "targets")
    if dL_dimages is not None:
        _need(dL_dimages, (F, 3, H, W), torch.float32, "dL_dimages")
    if loss is not None:
        _need(loss, (F,), torch.float32, "loss")
    if dL_dposes is not None:
        _need(dL_dposes, (F, 7), torch.float32, "dL_dposes")
    gs = _grads_c(grads) if grads is not None else None
    return (ctypes.byref(scene.c()), ctypes.byref(camera.c()), _ptr(poses), _ptr(times), F, _ptr(targets),
            _ptr(dL_dimages), flags, _ptr(images), _ptr(loss), None if gs is None else ctypes.byref(gs),
            _ptr(dL_dposes), ws.ptr, ws.nbytes), gs


def render_batch(scene: Scene, camera: Camera, poses: torch.Tensor, times: Optional[torch.Tensor], ws: Workspace,
                 targets: Optional[torch.Tensor] = None, dL_dimages: Optional[torch.Tensor] = None,
                 forward: bool = True, backward: bool = True, images: Optional[torch.Tensor] = None,
                 loss: Optional[torch.Tensor] = None, grads: Optional[dict] = None,
                 dL_dposes: Optional[torch.Tensor] = None, accumulate: bool = False) -> dict:
    """All frames of a clip in one launch sequence (no host synchronisation)."""
    F = int(poses.shape[0])
    dev = poses.device
    H, W = camera.height, camera.width
    flags = (L.GV_FWD if forward else 0) | (L.GV_BWD if backward else 0) | (L.GV_ACCUMULATE if accumulate else 0)
    if targets is not None:
        flags |= L.GV_LOSS_L2
    if images is None:
        images = torch.empty(F, 3, H, W, device=dev)
    if targets is not None and loss is None:
        loss = torch.empty(F, device=dev)
    if backward and grads is None:
        grads = grad_buffers(scene)
    if backward and dL_dposes is None:
        dL_dposes = torch.empty(F, 7, device=dev)
    args, _keep = _batch_args(scene, camera, poses, times, ws, targets, dL_dimages, flags, images, loss, grads,
                              dL_dposes)
    L.check(L.load().gv_render_batch(*args, _stream()), "gv_render_batch")
    return dict(images=images, loss=loss, grads=grads, dL_dposes=dL_dposes)


def render_batch_timed(scene: Scene, camera: Camera, poses: torch.Tensor, times: Optional[torch.Tensor],
                       ws: Workspace, targets: Optional[torch.Tensor] = None,
                       dL_dimages: Optional[torch.Tensor] = None, out: Optional[dict] = None) -> dict:
    """One forward+backward of the clip with HIP events between the stages
    (synchronous); returns {stage name: ms} and the outputs."""
    F = int(poses.shape[0])
    dev = poses.device
    H, W = camera.height, camera.width
    flags = L.GV_FWD | L.GV_BWD | (L.GV_LOSS_L2 if targets is not None else 0)
    out = out or {}
    images = out.get("images") if out.get("images") is not None else torch.empty(F, 3, H, W, device=dev)
    loss = out.get("loss") if out.get("loss") is not None else (torch.empty(F, device=dev) if targets is not None
                                                                else None)
    grads = out.get("grads") or grad_buffers(scene)
    dposes = out.get("dL_dposes") if out.get("dL_dposes") is not None else torch.empty(F, 7, device=dev)
    args, _keep = _batch_args(scene, camera, poses, times, ws, targets, dL_dimages, flags, images, loss, grads, dposes)
    ms = (ctypes.c_float * L.GV_STAGES)()
    L.check(L.load().gv_render_batch_timed(*args, _stream(), ms), "gv_render_batch_timed")
    return dict(stage_ms={name: float(ms[i]) for i, name in enumerate(L.STAGE_NAMES)},
                images=images, loss=loss, grads=grads, dL_dposes=dposes)


def autotune(scene: Scene, camera: Camera, poses: torch.Tensor, times: Optional[torch.Tensor], ws: Workspace,
             targets: torch.Tensor, cache_path: Optional[str] = None) -> dict:
    """Time the candidate kernel settings on this clip and install the fastest."""
    F = int(poses.shape[0])
    dev = poses.device
    images = torch.empty(F, 3, camera.height, camera.width, device=dev)
    loss = torch.empty(F, device=dev)
    grads = grad_buffers(scene)
    dposes = torch.empty(F, 7, device=dev)
    args, _keep = _batch_args(scene, camera, poses, times, ws, targets, None, L.GV_FWD | L.GV_BWD | L.GV_LOSS_L2,
                              images, loss, grads, dposes)
    # gv_autotune takes (scene, cam, poses, times, F, targets, images, loss, grads, dposes, ws, bytes, path, out)
    t = L.GvTuning()
    L.check(L.load().gv_autotune(args[0], args[1], args[2], args[3], args[4], args[5], args[8], args[9], args[10],
                                 args[11], args[12], args[13], None if cache_path is None else cache_path.encode(),
                                 ctypes.byref(t)), "gv_autotune")
    return dict(batch=int(t.batch), sort_cap=int(t.sort_cap), compact=int(t.compact), bwd_batch=int(t.bwd_batch))


def get_tuning() -> dict:
    t = L.GvTuning()
    L.check(L.load().gv_get_tuning(ctypes.byref(t)), "gv_get_tuning")
    return dict(batch=int(t.batch), sort_cap=int(t.sort_cap), compact=int(t.compact), bwd_batch=int(t.bwd_batch))


def set_tuning(batch: int, sort_cap: int, compact: int = 0, bwd_batch: int = 0) -> None:
    """Install a tuning (bwd_batch 0 = same as batch)."""
    t = L.GvTuning()
    t.batch, t.sort_cap, t.compact, t.bwd_batch = int(batch), int(sort_cap), int(compact), int(bwd_batch)
    L.check(L.load().gv_set_tuning(ctypes.byref(t)), "gv_set_tuning")


class BatchGraph:
    """A gv_render_batch call captured once into a HIP graph (all buffers fixed)."""

    def __init__(self, scene: Scene, camera: Camera, poses, times, ws: Workspace, targets=None, dL_dimages=None,
                 backward=True):
        F = int(poses.shape[0])
        dev = poses.device
        H, W = camera.height, camera.width
        self.images = torch.empty(F, 3, H, W, device=dev)
        self.loss = torch.empty(F, device=dev) if targets is not None else None
        self.grads = grad_buffers(scene) if backward else None
        self.dL_dposes = torch.empty(F, 7, device=dev) if backward else None
        flags = L.GV_FWD | (L.GV_BWD if backward else 0) | (L.GV_LOSS_L2 if targets is not None else 0)
        self._refs = (scene, camera, poses, times, ws, targets, dL_dimages)
        args, self._gs = _batch_args(scene, camera, poses, times, ws, targets, dL_dimages, flags, self.images,
                                     self.loss, self.grads, self.dL_dposes)
        h = ctypes.c_void_p()
        torch.cuda.synchronize()
        L.check(L.load().gv_batch_graph_create(*args, ctypes.byref(h)), "gv_batch_graph_create")
        self._h = h

    def launch(self):
        L.check(L.load().gv_batch_graph_launch(self._h, _stream()), "gv_batch_graph_launch")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.load().gv_batch_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def estimate_capacity(scene: Scene, camera: Camera, poses: torch.Tensor, times: Optional[torch.Tensor],
                      margin: float = 1.3, sample: int = 3) -> int:
    """Intersection capacity for a clip, from the exact tile counts of a few
    frames (first, middle, last) scaled to all frames with a margin."""
    F = int(poses.shape[0])
    ws = Workspace(camera, scene.n, 1, 0, device=poses.device)
    idx = sorted({0, F // 2, F - 1})[:max(1, sample)]
    worst = 0
    for f in idx:
        t = float(times[f]) if times is not None else 0.0
        _, cnt = project_fwd(scene, camera, poses[f].contiguous(), t, ws)
        worst = max(worst, int(cnt.sum().item()))
    return int(math.ceil(worst * margin * F)) + 1024


# ---------------------------------------------------------------------------
# autograd
# ---------------------------------------------------------------------------

def _raise_on_overflow(ws: Workspace, where: str) -> None:
    """The batched forward never synchronises; an autograd caller gets its
    images back only after the status words have been read (one small copy),
    so an exceeded intersection capacity raises instead of returning
    unwritten images."""
    st = ws.status()
    if st["overflow"]:
        raise L.GvError(L.GV_ERR_CAPACITY, f"{where}: {st['intersections']} intersections for a capacity of "
                                           f"{ws.k_capacity}")


class RasterizeFrame(torch.autograd.Function):
    """image = render(params, pose) for one frame; backward through render_bwd.
    The workspace must not be reused by another forward before backward."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, colors, pose7, camera, ws, t):
        scene = Scene(means, log_scales, quats, opacity_logits, colors)
        image = render_fwd(scene, camera, pose7, t, ws)
        ctx.save_for_backward(means, log_scales, quats, opacity_logits, colors, pose7, image)
        ctx.camera, ctx.ws, ctx.t = camera, ws, t
        return image

    @staticmethod
    def backward(ctx, dimage):
        means, log_scales, quats, opacity_logits, colors, pose7, image = ctx.saved_tensors
        scene = Scene(means, log_scales, quats, opacity_logits, colors)
        g, dpose = render_bwd(scene, ctx.camera, pose7, ctx.t, ctx.ws, image, dL_dimage=dimage.contiguous())
        return (g["means"], g["log_scales"], g["quats"], g["opacity_logits"], g["colors"], dpose, None, None, None)


class RasterizeClip(torch.autograd.Function):
    """images [F][3][H][W] of a clip with per-frame poses; gradients of the
    shared parameters are summed over frames, pose gradients are per frame.
    mean_coeffs (cubic means) and sh (view-dependent colour) may be None."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, colors, mean_coeffs, sh, poses, times, camera, ws):
        scene = Scene(means, log_scales, quats, opacity_logits, colors, mean_coeffs, sh=sh)
        out = render_batch(scene, camera, poses, times, ws, forward=True, backward=False)
        _raise_on_overflow(ws, "RasterizeClip")
        ctx.save_for_backward(means, log_scales, quats, opacity_logits, colors, mean_coeffs, sh, poses, times,
                              out["images"])
        ctx.camera, ctx.ws = camera, ws
        return out["images"]

    @staticmethod
    def backward(ctx, dimages):
        means, log_scales, quats, opacity_logits, colors, mean_coeffs, sh, poses, times, images = ctx.saved_tensors
        scene = Scene(means, log_scales, quats, opacity_logits, colors, mean_coeffs, sh=sh)
        out = render_batch(scene, ctx.camera, poses, times, ctx.ws, dL_dimages=dimages.contiguous(), forward=False,
                           backward=True, images=images)
        g = out["grads"]
        return (g["means"], g["log_scales"], g["quats"], g["opacity_logits"], g["colors"], g["mean_coeffs"],
                g["sh"], out["dL_dposes"], None, None, None)


class RasterizeDynamicClip(torch.autograd.Function):
    """Like RasterizeClip for Gaussians with the dynamics of Eq. 2-3: B-spline
    means (control points [M][3][N]) and cubic log-scales and quaternions
    (coefficients [3][3][N], [3][4][N]); frame times must lie in [0, 1]."""

    @staticmethod
    def forward(ctx, ctrl, log_scales, quats, opacity_logits, colors, scale_coeffs, quat_coeffs, poses, times,
                camera, ws):
        scene = Scene(None, log_scales, quats, opacity_logits, colors, ctrl=ctrl, scale_coeffs=scale_coeffs,
                      quat_coeffs=quat_coeffs)
        out = render_batch(scene, camera, poses, times, ws, forward=True, backward=False)
        _raise_on_overflow(ws, "RasterizeDynamicClip")
        ctx.save_for_backward(ctrl, log_scales, quats, opacity_logits, colors, scale_coeffs, quat_coeffs, poses,
                              times, out["images"])
        ctx.camera, ctx.ws = camera, ws
        return out["images"]

    @staticmethod
    def backward(ctx, dimages):
        ctrl, log_scales, quats, opacity_logits, colors, scale_coeffs, quat_coeffs, poses, times, images = \
            ctx.saved_tensors
        scene = Scene(None, log_scales, quats, opacity_logits, colors, ctrl=ctrl, scale_coeffs=scale_coeffs,
                      quat_coeffs=quat_coeffs)
        out = render_batch(scene, ctx.camera, poses, times, ctx.ws, dL_dimages=dimages.contiguous(), forward=False,
                           backward=True, images=images)
        g = out["grads"]
        return (g["ctrl"], g["log_scales"], g["quats"], g["opacity_logits"], g["colors"], g["scale_coeffs"],
                g["quat_coeffs"], out["dL_dposes"], None, None, None)


def visibility_counts(scene: Scene, camera: Camera, poses: torch.Tensor, times: Optional[torch.Tensor],
                      ws: Workspace, images: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Per Gaussian, the number of frames in which it contributes to at least
    one pixel (int32 [N]); the frames are rendered into ``images``."""
    F = int(poses.shape[0])
    dev = poses.device
    if images is None:
        images = torch.empty(F, 3, camera.height, camera.width, device=dev)
    counts = torch.empty(scene.n, dtype=torch.int32, device=dev)
    sc, cam = scene.c(), camera.c()
    L.check(L.load().gv_visibility_counts(ctypes.byref(sc), ctypes.byref(cam), poses.data_ptr(),
                                          None if times is None else times.data_ptr(), F, images.data_ptr(),
                                          counts.data_ptr(), ws.ptr, ws.nbytes, _stream()), "gv_visibility_counts")
    return counts


def gaussian_pyramid(images: torch.Tensor, levels: int):
    """[images, level 1, ..., level levels-1] of [..., H, W] FP32 frames
    (binomial 5-tap blur + decimation by 2, mirrored borders)."""
    if images.dtype != torch.float32 or not images.is_contiguous() or not images.is_cuda:
        raise ValueError("images must be a contiguous float32 device tensor")
    lead = images.shape[:-2]
    H, W = int(images.shape[-2]), int(images.shape[-1])
    planes = int(np.prod(lead)) if len(lead) else 1
    n = ctypes.c_int64()
    L.check(L.load().gv_pyramid_floats(planes, H, W, levels, ctypes.byref(n)), "gv_pyramid_floats")
    out = torch.empty(max(int(n.value), 1), device=images.device)
    L.check(L.load().gv_gaussian_pyramid(images.data_ptr(), planes, H, W, levels, out.data_ptr(), _stream()),
            "gv_gaussian_pyramid")
    res, off, h, w = [images], 0, H, W
    for _ in range(1, levels):
        h, w = (h + 1) // 2, (w + 1) // 2
        res.append(out[off:off + planes * h * w].view(*lead, h, w))
        off += planes * h * w
    return res
