"""Shared helpers of the GPU parity tests: HIP path vs the FP64 oracle.

Tolerances (written here, used by every parity test):

* pixels: max |C_gpu - C_oracle| <= 1e-4 (FP32 compositing), over pixels whose
  discrete decisions are not within rounding of a threshold;
* gradients: per tensor ||g_gpu - g_oracle||_2 / ||g_oracle||_2 <= 1e-3, with
  the same explicit upstream gradient on both sides, zeroed at those pixels.

A pixel is "knife-edge" when the oracle reports a relative margin below
MARGIN_TOL for one of its decisions: the 3-sigma cut (q = 9), the alpha >= 1/255
test, the T(1 - alpha) < 1e-4 stop, or (gradients only) the alpha <= 0.99
clamp.  The bounds come from the kernel's FP32 arithmetic: the conic is
rounded once (2^-24), the tile-local centre is rounded once from FP64 (an
absolute error below 1e-6 px for a centre within 16 px plus 3 sigma of the
tile), which bounds the relative error of q by ~2e-6; exp2 adds about one ulp
and the q error is amplified by q/2 in alpha, about 1e-5 at q = 9; the
transmittance compounds the alpha errors of up to a few hundred entries.
"""
from __future__ import annotations

import numpy as np
import torch

import gv_synth
import oracle
from paper_2501_04782_amd import raster

PIXEL_TOL = 1e-4
GRAD_TOL = 1e-3
MARGIN_TOL = np.array([2e-5, 1e-4, 2e-3, 1e-4])


def knife_edge(margins: np.ndarray, grads: bool = False, widen: float = 1.0) -> np.ndarray:
    """widen > 1 also sets aside pixels whose decisions could move when the
    two sides' inputs differ slightly (e.g. poses integrated in FP32 vs FP64)."""
    m = margins.reshape(-1, 4)
    k = 4 if grads else 3
    return (m[:, :k] < widen * MARGIN_TOL[None, :k]).any(axis=1)


def rel_err(got, ref) -> float:
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / den) if den > 0 else float(np.linalg.norm(got))


def device_inputs(w: dict, device="cuda"):
    scene = raster.Scene.from_synth(w["scene"], device)
    cam = raster.Camera.of(w["camera"])
    poses = torch.from_numpy(np.ascontiguousarray(w["poses"], dtype=np.float32)).to(device)
    times = torch.from_numpy(np.ascontiguousarray(w["times"], dtype=np.float32)).to(device)
    return scene, cam, poses, times


def workspace_for(scene, cam, poses, times, margin=1.5):
    cap = raster.estimate_capacity(scene, cam, poses, times, margin=margin)
    return raster.Workspace(cam, scene.n, int(poses.shape[0]), cap, device=poses.device)


def oracle_frame(w: dict, f: int, pixels=None, dL_dC=None, grads=None):
    return oracle.render_frame(w["scene"], w["camera"], w["poses"][f].astype(np.float64), float(w["times"][f]),
                               pixels=pixels, dL_dC=dL_dC, grads=grads)


def planar_to_pixels(img: np.ndarray) -> np.ndarray:
    """[3][H][W] -> [H*W][3]"""
    return img.reshape(3, -1).T


def compare_image(gpu_img: np.ndarray, ref: dict, label: str):
    """gpu_img [3][H][W] against an oracle full-frame result; returns stats."""
    ke = knife_edge(ref["margins"])
    d = np.abs(planar_to_pixels(gpu_img) - ref["color"]).max(axis=1)
    bad = (d > PIXEL_TOL) & ~ke
    worst = float(d[~ke].max()) if (~ke).any() else 0.0
    assert not bad.any(), f"{label}: {bad.sum()} pixels off by > {PIXEL_TOL} (max {d.max():.3e}); knife-edge {ke.sum()}"
    return dict(max_abs=worst, knife_edge=int(ke.sum()), pixels=int(d.size))


def compare_grads(gpu: dict, ref: dict, label: str, names=None):
    out = {}
    names = names or [k for k in ("means", "log_scales", "quats", "opacity_logits", "colors", "mean_coeffs", "ctrl",
                                  "scale_coeffs", "quat_coeffs", "sh", "intrinsics")
                      if ref.get(k) is not None and not (k == "means" and ref.get("ctrl") is not None)]
    for k in names:
        g = gpu[k].detach().cpu().numpy() if isinstance(gpu[k], torch.Tensor) else gpu[k]
        e = rel_err(g, ref[k])
        out[k] = e
        assert e <= GRAD_TOL, f"{label}: grad {k} relative error {e:.3e} > {GRAD_TOL}"
    return out
