"""Shared helpers of the GPU parity tests: HIP path vs the FP64 oracle.

Tolerances (written here, used by every parity test):

* pixels: |C_gpu - C_oracle| <= 1e-4 (FP32 compositing) at every pixel whose
  discrete decisions are not within rounding of a threshold;
* set-aside pixels (a decision within rounding of its threshold) are still
  checked, against the looser bound the flipped decision allows:
  |C_gpu - C_oracle| <= 1e-4 + stake * colour range, where the oracle's stake
  is the blending weight those decisions control (alpha*T of an entry at the
  3-sigma or 1/255 cut, the remaining transmittance at the stop);
* at most SET_ASIDE_MAX (1 %) of a test's checked pixels may be set aside:
  with the margins below, a pixel reached by m entries inside their
  footprint is set aside with probability of about m times the relative
  width of the bands (a few 1e-5 per entry and decision), which is 0-0.5 % of
  the pixels of the test scenes (the most in the densest tiles, where many
  pixels stop); the fraction checked against a bound looser than twice the
  pixel tolerance is reported;
* gradients: per tensor ||g_gpu - g_oracle||_2 / ||g_oracle||_2 <= 1e-3, and
  element by element |g_gpu - g_oracle| <= 3e-3 |g_oracle| + 1e-6 max|g_oracle|,
  with the same explicit upstream gradient on both sides, zeroed at set-aside
  pixels (which removes them from both sides exactly).  The elementwise bar
  catches an error confined to a few Gaussians, which the norm would hide;
  its relative part allows for ill-conditioned elements: for a needle-like
  Gaussian (scales e^-1 and e^-5) the quaternion gradient passes through
  the conic's inverse and the rotation of a 3000:1 covariance, which turn
  the FP32 rounding of the per-pixel moments (~1e-7) into element errors of
  up to 1.05e-3 (measured), while the tensor's norm error stays at 6e-6;
* gradients of shared parameters summed over a clip's frames (one set of
  Gaussians serves every frame, Sec. 3.2, under the L2 loss over all
  frames, Sec. 4.1) may also be off by SUM_RTOL times the sum over frames of
  the per-frame gradient's magnitude: the rounding error of a sum is bounded
  by a multiple of the unit roundoff times the sum of its terms' magnitudes,
  not of its result, and per-frame terms can cancel by a factor of several
  thousand (measured: a quaternion gradient of -0.21 from 32 frames whose
  terms sum to 1495 in magnitude, off by 7.4e-7 of that sum in FP32).

A pixel is set aside when the oracle reports a relative margin below
MARGIN_TOL for one of its decisions: the 3-sigma cut (q = 9), the alpha >= 1/255
test, the T(1 - alpha) < 1e-4 stop, or (gradients only) the alpha <= 0.99
clamp.  The bounds come from the kernel's FP32 arithmetic: the conic is
rounded once (2^-24), the tile-local centre is rounded once from FP64 (an
absolute error below 1e-6 px for a centre within 16 px plus 3 sigma of the
tile), which bounds the relative error of q by ~2e-6; exp2 adds about one ulp
and the q error is amplified by q/2 in alpha, about 1e-5 at q = 9; the
transmittance compounds the alpha errors of the entries in front: a factor
1 - alpha has a relative error of about alpha / (1 - alpha) times alpha's,
largest where q (and so alpha's error) is smallest, giving a few 1e-6 over a
few hundred entries (measured final transmittances differ from the oracle's
by at most 2.1e-6 relative), so the stop margin 2e-4 keeps a factor of 100.
"""
from __future__ import annotations

import numpy as np
import torch

import gv_synth
import oracle
from paper_2501_04782_amd import raster

PIXEL_TOL = 1e-4
GRAD_TOL = 1e-3
ELEM_RTOL = 3e-3          # elementwise gradient check: relative part
ELEM_ATOL = 1e-6          # elementwise gradient check: absolute part, times max|g_oracle|
SUM_RTOL = 1e-5           # elementwise, sums over frames: times the sum of the per-frame magnitudes (~170 ulp)
MARGIN_TOL = np.array([2e-5, 1e-4, 2e-4, 1e-4])
SET_ASIDE_MAX = 0.01      # fraction of a test's checked pixels that may be set aside
SH_BOUND = 0.75           # |Y_lm| <= sqrt((2l + 1) / (4 pi)) <= 0.75 for l <= 3


def knife_edge(margins: np.ndarray, grads: bool = False, widen: float = 1.0) -> np.ndarray:
    """widen > 1 also sets aside pixels whose decisions could move when the
    two sides' inputs differ slightly (e.g. poses integrated in FP32 vs FP64)."""
    m = margins.reshape(-1, 4)
    k = 4 if grads else 3
    return (m[:, :k] < widen * MARGIN_TOL[None, :k]).any(axis=1)


def colour_range(w: dict) -> float:
    """Largest per-channel spread of the colours a pixel blends (Gaussian
    colours, with SH terms bounded, and the background): a decision taken the
    other way moves a pixel by at most its stake times this."""
    s = w["scene"].as_f64() if hasattr(w["scene"], "as_f64") else w["scene"]
    col = np.asarray(s["colors"], np.float64).reshape(3, -1)
    bg = np.asarray(w["camera"].bg, np.float64)
    sh = s.get("sh")
    spread = np.zeros(3)
    if sh is not None:
        spread = SH_BOUND * np.abs(np.asarray(sh, np.float64)).sum(axis=0).max(axis=-1)
    hi = np.maximum(col.max(axis=1, initial=-np.inf) + spread, bg) if col.size else bg
    lo = np.minimum(col.min(axis=1, initial=np.inf) - spread, bg) if col.size else bg
    return float(np.max(hi - lo))


def rel_err(got, ref) -> float:
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / den) if den > 0 else float(np.linalg.norm(got))


def elem_check(got, ref, label: str, mag=None) -> float:
    """Elementwise bar; returns the worst |d| / (ELEM_RTOL |ref| + ELEM_ATOL max|ref|
    [+ SUM_RTOL mag]), where mag (same shape as ref) is the sum over frames of
    the per-frame gradient's magnitude for a gradient summed over frames."""
    got = np.asarray(got, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    assert np.all(np.isfinite(got)), f"{label}: non-finite gradient values"
    if ref.size == 0:
        return 0.0
    scale = np.abs(ref).max()
    bound = ELEM_RTOL * np.abs(ref) + ELEM_ATOL * scale
    if mag is not None:
        bound = bound + SUM_RTOL * np.asarray(mag, np.float64).reshape(-1)
    d = np.abs(got - ref)
    if scale == 0.0:
        assert np.all(d == 0.0), f"{label}: oracle gradient is zero, GPU max |g| {d.max():.3e}"
        return 0.0
    ratio = d / bound
    worst = int(np.argmax(ratio))
    assert ratio[worst] <= 1.0, (f"{label}: {(ratio > 1).sum()} of {ref.size} elements off; worst index {worst}: "
                                 f"gpu {got[worst]:.6e} oracle {ref[worst]:.6e} (bound {bound[worst]:.2e})")
    return float(ratio[worst])


def device_inputs(w: dict, device="cuda"):
    scene = raster.Scene.from_synth(w["scene"], device)
    cam = raster.Camera.of(w["camera"])
    poses = torch.from_numpy(np.ascontiguousarray(w["poses"], dtype=np.float32)).to(device)
    times = torch.from_numpy(np.ascontiguousarray(w["times"], dtype=np.float32)).to(device)
    return scene, cam, poses, times


def workspace_for(scene, cam, poses, times, margin=1.5):
    cap = raster.estimate_capacity(scene, cam, poses, times, margin=margin)
    return raster.Workspace(cam, scene.n, int(poses.shape[0]), cap, device=poses.device)


def oracle_frame(w: dict, f: int, pixels=None, dL_dC=None, grads=None, widen: float = 1.0, tile: int = 0):
    """Oracle render of frame f (with the per-pixel stake of set-aside
    decisions); tile > 0 takes the oracle's tiled form, whose results are
    identical to the per-pixel definition (margins below 1e-3, the only ones
    used here, included) and which whole full-size frames need."""
    return oracle.render_frame(w["scene"], w["camera"], w["poses"][f].astype(np.float64), float(w["times"][f]),
                               pixels=pixels, dL_dC=dL_dC, grads=grads, stake_tol=widen * MARGIN_TOL[:3], tile=tile)


def oracle_clip_grads(w: dict, dls, frames=None, pixels=None, tile: int = 0):
    """The oracle's gradients of sum_f sum_p dls[k][p] . C_f[p] over the listed
    frames (all by default), frame by frame: the sums over frames, the
    per-frame pose gradients [F][7] and, per element, the sum over frames of
    the per-frame gradient's magnitude (the scale of the sum's rounding)."""
    frames = range(w["frames"]) if frames is None else frames
    pixels = [None] * len(frames) if pixels is None else pixels
    total = oracle.zero_grads(w["scene"])
    mag = oracle.zero_grads(w["scene"])
    dposes = np.zeros((len(w["poses"]), 7))
    for f, pix, dl in zip(frames, pixels, dls):
        gf = oracle_frame(w, f, pixels=pix, dL_dC=dl, grads=oracle.zero_grads(w["scene"]), tile=tile)["grads"]
        for k, v in gf.items():
            if v is not None and k != "pose":
                total[k] += v
                mag[k] += np.abs(v)
        dposes[f] = gf["pose"]
    total["pose"] = mag["pose"] = None
    return total, dposes, mag


def planar_to_pixels(img: np.ndarray) -> np.ndarray:
    """[3][H][W] -> [H*W][3]"""
    return img.reshape(3, -1).T


class PixelTally:
    """Counts of a test's checked, set-aside and loosely checked pixels; the
    set-aside fraction is asserted once the test has seen all its pixels."""

    def __init__(self, label: str):
        self.label, self.checked, self.set_aside, self.loose, self.worst = label, 0, 0, 0, 0.0

    def add(self, got: np.ndarray, ref: dict, crange: float, widen: float = 1.0, where: str = ""):
        """got [P][3] against the oracle result ref at the same pixels."""
        d = np.abs(np.asarray(got, np.float64) - ref["color"]).max(axis=1)
        ke = knife_edge(ref["margins"], widen=widen) | (ref["stake"] > 0)
        allow = PIXEL_TOL + ref["stake"] * crange
        bad = d > allow
        i = int(np.argmax(d - allow))
        assert not bad.any(), (f"{self.label}{where}: {bad.sum()} pixels off; worst pixel #{i}: |d| {d[i]:.3e} > "
                               f"{allow[i]:.3e} (stake {ref['stake'][i]:.2e}, set aside {bool(ke[i])})")
        self.checked += d.size
        self.set_aside += int(ke.sum())
        self.loose += int((ref["stake"] * crange > PIXEL_TOL).sum())
        if (~ke).any():
            self.worst = max(self.worst, float(d[~ke].max()))
        return d

    def finish(self, set_aside_max: float = SET_ASIDE_MAX) -> dict:
        n = max(self.checked, 1)
        fa = self.set_aside / n
        assert fa <= set_aside_max, f"{self.label}: {self.set_aside}/{self.checked} pixels set aside ({fa:.2%})"
        return dict(max_abs=self.worst, set_aside=self.set_aside, loose=self.loose, pixels=self.checked)


def compare_image(gpu_img: np.ndarray, ref: dict, label: str, crange: float, tally: PixelTally = None):
    """gpu_img [3][H][W] against an oracle full-frame result; with a tally the
    fractions are asserted by the caller's tally.finish(), else here."""
    own = tally is None
    tally = tally or PixelTally(label)
    tally.add(planar_to_pixels(gpu_img), ref, crange)
    return tally.finish() if own else None


def compare_grads(gpu: dict, ref: dict, label: str, names=None, mag: dict = None):
    """Every gradient tensor the oracle gives: norm-wise and elementwise bars
    (mag: per-tensor sums over frames of per-frame magnitudes, for gradients
    summed over a clip)."""
    out = {}
    names = names or [k for k in ("means", "log_scales", "quats", "opacity_logits", "colors", "mean_coeffs", "ctrl",
                                  "scale_coeffs", "quat_coeffs", "sh", "intrinsics")
                      if ref.get(k) is not None and not (k == "means" and ref.get("ctrl") is not None)]
    for k in names:
        g = gpu[k].detach().cpu().numpy() if isinstance(gpu[k], torch.Tensor) else gpu[k]
        e = rel_err(g, ref[k])
        assert e <= GRAD_TOL, f"{label}: grad {k} relative error {e:.3e} > {GRAD_TOL}"
        r = elem_check(g, ref[k], f"{label}: grad {k}", None if mag is None else mag.get(k))
        out[k] = (round(e, 9), round(r, 3))
    return out


def compare_poses(gpu, ref, label: str):
    """Per-frame pose gradients: norm-wise and elementwise bars."""
    g = gpu.detach().cpu().numpy() if isinstance(gpu, torch.Tensor) else np.asarray(gpu)
    e = rel_err(g, ref)
    assert e <= GRAD_TOL, f"{label}: pose gradient relative error {e:.3e}"
    elem_check(g, ref, f"{label}: pose gradient")
    return e


# ------------------------------------------------------- tile buckets


def tile_buckets(w: dict, f: int, tile: int = 16) -> np.ndarray:
    """Entries per tile of frame f from the oracle's projection: Gaussians
    (opacity >= 1/255) whose 3-sigma ellipse meets the tile's pixel-centre box
    (minimum of the quadratic form over the box <= 9)."""
    cam = w["camera"]
    p = oracle.project(w["scene"], cam, w["poses"][f].astype(np.float64), float(w["times"][f]))
    ok = (p["valid"] > 0) & (p["opacity"] >= 1 / 255)
    u, v, a, b, c = p["u"][ok], p["v"][ok], p["A00"][ok], p["A01"][ok], p["A11"][ok]
    hx, hy = 3 * np.sqrt(p["cov00"][ok]), 3 * np.sqrt(p["cov11"][ok])
    TX, TY = (cam.width + tile - 1) // tile, (cam.height + tile - 1) // tile
    # tiles whose centre range [t*tile + 0.5, t*tile + tile - 0.5] meets [u - hx, u + hx]
    tx0 = np.clip(np.ceil((u - hx - tile + 0.5) / tile), 0, TX).astype(np.int64)
    tx1 = np.clip(np.floor((u + hx - 0.5) / tile), -1, TX - 1).astype(np.int64)
    ty0 = np.clip(np.ceil((v - hy - tile + 0.5) / tile), 0, TY).astype(np.int64)
    ty1 = np.clip(np.floor((v + hy - 0.5) / tile), -1, TY - 1).astype(np.int64)
    nx, ny = np.maximum(tx1 - tx0 + 1, 0), np.maximum(ty1 - ty0 + 1, 0)
    cnt = nx * ny
    gi = np.repeat(np.arange(u.size), cnt)
    k = np.arange(gi.size) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    tx = tx0[gi] + k % nx[gi]
    ty = ty0[gi] + k // nx[gi]
    x0, x1 = tx * tile + 0.5, np.minimum(tx * tile + tile - 0.5, cam.width - 0.5)
    y0, y1 = ty * tile + 0.5, np.minimum(ty * tile + tile - 0.5, cam.height - 0.5)
    U, V, A, B, C = u[gi], v[gi], a[gi], b[gi], c[gi]
    dx0, dx1, dy0, dy1 = x0 - U, x1 - U, y0 - V, y1 - V
    best = np.where((dx0 <= 0) & (dx1 >= 0) & (dy0 <= 0) & (dy1 >= 0), 0.0, np.inf)
    for dx in (dx0, dx1):
        dy = np.clip(-B * dx / C, dy0, dy1)
        best = np.minimum(best, A * dx * dx + 2 * B * dx * dy + C * dy * dy)
    for dy in (dy0, dy1):
        dx = np.clip(-B * dy / A, dx0, dx1)
        best = np.minimum(best, A * dx * dx + 2 * B * dx * dy + C * dy * dy)
    hit = best <= 9.0
    return np.bincount((ty * TX + tx)[hit], minlength=TX * TY)
