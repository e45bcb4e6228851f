"""Torch binding of the camera-motion Neural ODE kernels (Eq. 1, Sec. 3.4).

theta [5191] packs the 8 -> 64 -> 64 -> 7 tanh MLP (W1[64][8], b1[64],
W2[64][64], b2[64], W3[7][64], b3[7]); z0 [7] is the initial state
(qw, qx, qy, qz, tx, ty, tz).  ``camera_ode_fwd`` integrates with RK4
(``substeps`` per frame interval, frames at t = f/(F-1)) and returns the
per-frame world->camera poses [F][7]; ``camera_ode_bwd`` is the discrete
adjoint.  All arithmetic runs in the library's kernels.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from .raster import Camera, Scene, Workspace, _grads_c, _need, _ptr, _stream, grad_buffers

N_THETA = 5191


class OdeWorkspace:
    def __init__(self, frames: int, substeps: int, device="cuda"):
        out = ctypes.c_size_t()
        L.check(L.load().gv_camera_ode_workspace_bytes(int(frames), int(substeps), ctypes.byref(out)),
                "gv_camera_ode_workspace_bytes")
        self.nbytes = int(out.value)
        # at least one aligned block so the pointer is valid even for F = 1
        self.buf = torch.empty(max(self.nbytes, 256), dtype=torch.uint8, device=device)
        self.frames, self.substeps = int(frames), int(substeps)

    @property
    def ptr(self):
        return ctypes.c_void_p(self.buf.data_ptr())


def camera_ode_fwd(theta: torch.Tensor, z0: torch.Tensor, frames: int, substeps: int, ws: OdeWorkspace,
                   poses: torch.Tensor = None) -> torch.Tensor:
    _need(theta, (N_THETA,), torch.float32, "theta")
    _need(z0, (7,), torch.float32, "z0")
    if poses is None:
        poses = torch.empty(frames, 7, device=theta.device)
    _need(poses, (frames, 7), torch.float32, "poses")
    L.check(L.load().gv_camera_ode_fwd(_ptr(theta), _ptr(z0), int(frames), int(substeps), _ptr(poses), ws.ptr,
                                       ws.buf.numel(), _stream()), "gv_camera_ode_fwd")
    return poses


def camera_ode_bwd(theta: torch.Tensor, z0: torch.Tensor, frames: int, substeps: int, dL_dposes: torch.Tensor,
                   ws: OdeWorkspace, dtheta: torch.Tensor = None, dz0: torch.Tensor = None):
    _need(dL_dposes, (frames, 7), torch.float32, "dL_dposes")
    if dtheta is None:
        dtheta = torch.empty(N_THETA, device=theta.device)
    if dz0 is None:
        dz0 = torch.empty(7, device=theta.device)
    L.check(L.load().gv_camera_ode_bwd(_ptr(theta), _ptr(z0), int(frames), int(substeps), _ptr(dL_dposes),
                                       _ptr(dtheta), _ptr(dz0), ws.ptr, ws.buf.numel(), _stream()),
            "gv_camera_ode_bwd")
    return dtheta, dz0


def pose_error(poses: torch.Tensor, ref_poses: torch.Tensor) -> dict:
    """Trajectory error of a camera path against a reference pose table
    (gv_pose_error): root mean square distance of the camera centres, mean
    relative rotation angle (radians) and the per-frame values.  Reads the
    results back (synchronises the stream)."""
    F = int(poses.shape[0])
    _need(poses, (F, 7), torch.float32, "poses")
    _need(ref_poses, (F, 7), torch.float32, "ref_poses")
    per_frame = torch.empty(F, 2, device=poses.device)
    summary = torch.empty(2, device=poses.device)
    L.check(L.load().gv_pose_error(_ptr(poses), _ptr(ref_poses), F, _ptr(per_frame), _ptr(summary), _stream()),
            "gv_pose_error")
    pf, sm = per_frame.cpu().numpy(), summary.cpu().numpy()
    return dict(translation_rmse=float(sm[0]), mean_angle=float(sm[1]), translation=pf[:, 0], angle=pf[:, 1])


class CameraODE(torch.autograd.Function):
    """poses = ODE(theta, z0); backward through the discrete adjoint."""

    @staticmethod
    def forward(ctx, theta, z0, frames, substeps, ws):
        poses = camera_ode_fwd(theta, z0, frames, substeps, ws)
        ctx.save_for_backward(theta, z0)
        ctx.frames, ctx.substeps, ctx.ws = frames, substeps, ws
        return poses

    @staticmethod
    def backward(ctx, dposes):
        theta, z0 = ctx.saved_tensors
        dtheta, dz0 = camera_ode_bwd(theta, z0, ctx.frames, ctx.substeps, dposes.contiguous(), ctx.ws)
        return dtheta, dz0, None, None, None


class FitGraph:
    """One learned-camera fitting step as a single HIP graph: camera ODE forward,
    batched raster forward+backward (fused L2 against ``targets`` or an explicit
    ``dL_dimages``), camera ODE adjoint.  All buffers are fixed at creation."""

    def __init__(self, scene: Scene, camera: Camera, theta, z0, frames: int, substeps: int, times, ws: Workspace,
                 targets=None, dL_dimages=None):
        dev = theta.device
        H, W = camera.height, camera.width
        _need(theta, (N_THETA,), torch.float32, "theta")
        _need(z0, (7,), torch.float32, "z0")
        self.ode_ws = OdeWorkspace(frames, substeps, device=dev)
        self.poses = torch.empty(frames, 7, device=dev)
        self.images = torch.empty(frames, 3, H, W, device=dev)
        self.loss = torch.empty(frames, device=dev) if targets is not None else None
        self.grads = grad_buffers(scene)
        self.dL_dposes = torch.empty(frames, 7, device=dev)
        self.dtheta = torch.empty(N_THETA, device=dev)
        self.dz0 = torch.empty(7, device=dev)
        self._refs = (scene, camera, theta, z0, times, ws, targets, dL_dimages)
        self._gs = _grads_c(self.grads)
        h = ctypes.c_void_p()
        torch.cuda.synchronize()
        L.check(L.load().gv_fit_graph_create(
            ctypes.byref(scene.c()), ctypes.byref(camera.c()), _ptr(theta), _ptr(z0), int(substeps),
            self.ode_ws.ptr, self.ode_ws.buf.numel(), _ptr(times), int(frames), _ptr(targets), _ptr(dL_dimages),
            _ptr(self.poses), _ptr(self.images), _ptr(self.loss), ctypes.byref(self._gs), _ptr(self.dL_dposes),
            _ptr(self.dtheta), _ptr(self.dz0), ws.ptr, ws.nbytes, ctypes.byref(h)), "gv_fit_graph_create")
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
