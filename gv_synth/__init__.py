"""Seeded synthetic inputs for the Gaussian rasterizer workloads.

This module only *draws* inputs: scenes, camera intrinsics, camera
trajectories, target frames and small adversarial scenes.  It contains none of
the renderer's arithmetic (no projection, compositing or gradients), so that
both the FP64 oracle and the HIP path can take their inputs from it without
sharing any code with each other.

Recipe (stand-in for the paper's DL3DV 540p and DAVIS 480p videos, Sec. 4.1,
which are not available): every quantity is drawn in FP64 from
``numpy.random.default_rng(seed)`` (PCG64) in the fixed order

    means, log-scales, quaternions (normalised), opacity logits, colours,
    [cubic mean coefficients], [trajectory], [targets]

and then rounded to nearest-even into its storage type (fp32, or bf16 for the
large clip).  All tensors are planar ``[C][N]``.  Gaussians follow Sec. 3.1:
mean, covariance as (RS)(RS)^T from a rotation quaternion and per-axis scales,
colour, opacity; colour is RGB (spherical harmonics of degree 0) and opacity
is constant in time (Eq. 3).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "Camera", "Scene", "WORKLOADS", "make_camera", "make_scene", "make_trajectory",
    "make_times", "make_targets", "make_workload", "round_bf16", "bf16_bits_to_f64",
    "adversarial_scene", "identity_poses", "init_mlp_theta",
]


# --------------------------------------------------------------------------
# storage helpers
# --------------------------------------------------------------------------

def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round FP64 values to bf16 (round-to-nearest-even, 8-bit significand).

    Returns the rounded values as FP64 (exactly representable in bf16).  Only
    normal, finite values occur in the workloads; zeros pass through.
    """
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                     # x = m * 2**e, 0.5 <= |m| < 1
    r = np.rint(m * 256.0) / 256.0         # 8 significant bits, half-to-even
    return np.ldexp(r, e)


def f64_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """bf16 bit patterns (uint16) of values already rounded by round_bf16."""
    f32 = np.asarray(x, dtype=np.float64).astype(np.float32)   # exact
    return (f32.view(np.uint32) >> 16).astype(np.uint16)


def bf16_bits_to_f64(bits: np.ndarray) -> np.ndarray:
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


# --------------------------------------------------------------------------
# containers
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Camera:
    """Pinhole intrinsics shared by every frame of a clip (Sec. 3.4)."""
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    near_plane: float = 0.01
    dilation: float = 0.3
    bg: tuple = (0.0, 0.0, 0.0)


@dataclasses.dataclass
class Scene:
    """Gaussian parameters in storage precision, planar [C][N].

    ``dtype`` is "f32" (float32 arrays) or "bf16" (uint16 bit patterns).
    Optional time dependence (all None for a static scene):

    * ``mean_coeffs`` [3 coeff][3 xyz][N]: a1..a3 of the cubic mean
      mu(t) = mu0 + a1 t + a2 t^2 + a3 t^3;
    * ``ctrl`` [M][3 xyz][N]: control points of the clamped cubic B-spline
      mean (then ``means`` holds the centre the points were drawn around);
    * ``scale_coeffs`` [3 coeff][3][N] and ``quat_coeffs`` [3 coeff][4][N]:
      b1..b3 and r1..r3 of the cubic log-scales and quaternion.

    ``sh`` [(D+1)^2 - 1][3][N] holds spherical-harmonics coefficients of
    degrees 1..D for a view-dependent colour (``colors`` is the l = 0 term).
    """
    dtype: str
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    colors: np.ndarray
    mean_coeffs: Optional[np.ndarray] = None
    ctrl: Optional[np.ndarray] = None
    scale_coeffs: Optional[np.ndarray] = None
    quat_coeffs: Optional[np.ndarray] = None
    sh: Optional[np.ndarray] = None

    OPTIONAL = ("mean_coeffs", "ctrl", "scale_coeffs", "quat_coeffs", "sh")

    @property
    def n(self) -> int:
        return int(self.opacity_logits.shape[-1])

    def fields(self):
        names = ["means", "log_scales", "quats", "opacity_logits", "colors"]
        names += [k for k in self.OPTIONAL if getattr(self, k) is not None]
        return names

    def as_f64(self) -> dict:
        """Exact FP64 values of the stored numbers."""
        out = {}
        for k in self.fields():
            a = getattr(self, k)
            out[k] = bf16_bits_to_f64(a) if self.dtype == "bf16" else np.asarray(a, np.float32).astype(np.float64)
        for k in self.OPTIONAL:
            out[k] = out.get(k)
        return out


# --------------------------------------------------------------------------
# workloads (shapes and distributions of the benchmark configurations)
# --------------------------------------------------------------------------

WORKLOADS = {
    # single 128x128 frame, 2k Gaussians, fixed camera looking down +z
    "frame128_n2k": dict(width=128, height=128, n=2000, frames=1, focal=128.0,
                          z=(2.0, 6.0), log_scale=(-3.5, 0.3), trajectory=None,
                          dtype="f32", cubic=False),
    # single 960x540 frame, 100k Gaussians
    "frame540p_n100k": dict(width=960, height=540, n=100_000, frames=1, focal=960.0,
                            z=(2.0, 10.0), log_scale=(-4.5, 0.5), trajectory=None,
                            dtype="f32", cubic=False),
    # 50-frame 960x540 clip, 200k shared Gaussians, smooth camera trajectory
    "clip540p_f50_n200k": dict(width=960, height=540, n=200_000, frames=50, focal=960.0,
                               z=(2.0, 10.0), log_scale=(-4.5, 0.5), trajectory="smooth",
                               dtype="f32", cubic=False),
    # camera-ODE fitting step: 100 frames
    "clip540p_f100_n200k": dict(width=960, height=540, n=200_000, frames=100, focal=960.0,
                                z=(2.0, 10.0), log_scale=(-4.5, 0.5), trajectory="smooth",
                                dtype="f32", cubic=False),
    # large clip, bf16 parameters, cubic means, static camera
    "clip1080p_f32_n500k_bf16": dict(width=1920, height=1080, n=500_000, frames=32, focal=1920.0,
                                     z=(2.0, 10.0), log_scale=(-4.5, 0.5), trajectory=None,
                                     dtype="bf16", cubic=True),
    # the benchmark clip with Eq. 2-3 dynamics: B-spline means (8 control
    # points) and cubic log-scales and quaternions
    "clip540p_f50_n200k_dyn": dict(width=960, height=540, n=200_000, frames=50, focal=960.0,
                                   z=(2.0, 10.0), log_scale=(-4.5, 0.5), trajectory="smooth",
                                   dtype="f32", cubic=False, n_ctrl=8, poly_cov=True),
    # the benchmark clip with view-dependent colour: SH of degree 3
    "clip540p_f50_n200k_sh3": dict(width=960, height=540, n=200_000, frames=50, focal=960.0,
                                   z=(2.0, 10.0), log_scale=(-4.5, 0.5), trajectory="smooth",
                                   dtype="f32", cubic=False, sh_degree=3),
}


def make_camera(width: int, height: int, focal: float, **kw) -> Camera:
    """Pinhole camera with the principal point at the image centre."""
    return Camera(width=width, height=height, fx=float(focal), fy=float(focal),
                  cx=width / 2.0, cy=height / 2.0, **kw)


def _store(x: np.ndarray, dtype: str) -> np.ndarray:
    if dtype == "f32":
        return np.ascontiguousarray(x.astype(np.float32))
    if dtype == "bf16":
        return np.ascontiguousarray(f64_to_bf16_bits(round_bf16(x)))
    raise ValueError(dtype)


def make_scene(rng: np.random.Generator, n: int, z=(2.0, 6.0), log_scale=(-3.5, 0.3),
               dtype: str = "f32", cubic: bool = False, xy=(-1.0, 1.0),
               coeff_std: float = 0.05, n_ctrl: int = 0, poly_cov: bool = False,
               ctrl_std: float = 0.05, sh_degree: int = 0, sh_std: float = 0.1) -> Scene:
    """Draw N Gaussians: means x,y ~ U[xy], z ~ U[z]; log-scales ~ N(mu, sd);
    quaternions ~ N(0, I4) normalised; opacity logits ~ N(0, 1); RGB ~ U[0,1];
    optional cubic mean coefficients ~ N(0, coeff_std).  Then, in this order:
    n_ctrl > 0 control points P_i = mean + N(0, ctrl_std) per axis, and with
    poly_cov the cubic log-scale and quaternion coefficients ~ N(0, coeff_std),
    and with sh_degree D > 0 the SH coefficients of degrees 1..D ~ N(0, sh_std)."""
    means = np.empty((3, n))
    means[0] = rng.uniform(xy[0], xy[1], n)
    means[1] = rng.uniform(xy[0], xy[1], n)
    means[2] = rng.uniform(z[0], z[1], n)
    log_scales = rng.normal(log_scale[0], log_scale[1], (3, n))
    q = rng.normal(0.0, 1.0, (4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    opacity_logits = rng.normal(0.0, 1.0, n)
    colors = rng.uniform(0.0, 1.0, (3, n))
    coeffs = rng.normal(0.0, coeff_std, (3, 3, n)) if cubic else None
    ctrl = means[None] + rng.normal(0.0, ctrl_std, (n_ctrl, 3, n)) if n_ctrl > 0 else None
    sc = rng.normal(0.0, coeff_std, (3, 3, n)) if poly_cov else None
    qc = rng.normal(0.0, coeff_std, (3, 4, n)) if poly_cov else None
    sh = rng.normal(0.0, sh_std, ((sh_degree + 1) ** 2 - 1, 3, n)) if sh_degree > 0 else None
    opt = lambda a: None if a is None else _store(a, dtype)  # noqa: E731
    return Scene(dtype=dtype, means=_store(means, dtype), log_scales=_store(log_scales, dtype),
                 quats=_store(q, dtype), opacity_logits=_store(opacity_logits, dtype),
                 colors=_store(colors, dtype), mean_coeffs=opt(coeffs), ctrl=opt(ctrl),
                 scale_coeffs=opt(sc), quat_coeffs=opt(qc), sh=opt(sh))


def identity_poses(frames: int) -> np.ndarray:
    p = np.zeros((frames, 7), np.float32)
    p[:, 0] = 1.0
    return p


def _axis_angle_quat(axis: np.ndarray, angle: float) -> np.ndarray:
    axis = axis / np.linalg.norm(axis)
    return np.concatenate([[math.cos(angle / 2)], math.sin(angle / 2) * axis])


def _slerp(qa: np.ndarray, qb: np.ndarray, s: float) -> np.ndarray:
    d = float(np.dot(qa, qb))
    if d < 0.0:
        qb, d = -qb, -d
    if d > 1.0 - 1e-12:
        q = qa + s * (qb - qa)
        return q / np.linalg.norm(q)
    th = math.acos(d)
    return (math.sin((1 - s) * th) * qa + math.sin(s * th) * qb) / math.sin(th)


def make_trajectory(rng: np.random.Generator, frames: int, amp: float = 0.2,
                    period=(20.0, 80.0), max_deg: float = 10.0) -> np.ndarray:
    """Smooth world->camera poses [F][7] = (qw, qx, qy, qz, tx, ty, tz).

    Translation per axis: sum of 3 sinusoids of amplitude ``amp``, period
    U[period], phase U[0, 2pi).  Rotation: slerp between two rotations, each a
    random axis with angle U[0, max_deg] degrees, parameter f/(F-1).
    """
    P = rng.uniform(period[0], period[1], (3, 3))
    phi = rng.uniform(0.0, 2 * math.pi, (3, 3))
    ax_a = rng.normal(0.0, 1.0, 3)
    ang_a = math.radians(rng.uniform(0.0, max_deg))
    ax_b = rng.normal(0.0, 1.0, 3)
    ang_b = math.radians(rng.uniform(0.0, max_deg))
    qa, qb = _axis_angle_quat(ax_a, ang_a), _axis_angle_quat(ax_b, ang_b)
    poses = np.zeros((frames, 7))
    for f in range(frames):
        s = f / (frames - 1) if frames > 1 else 0.0
        poses[f, :4] = _slerp(qa, qb, s)
        for axis in range(3):
            poses[f, 4 + axis] = sum(amp * math.sin(2 * math.pi * f / P[axis, k] + phi[axis, k])
                                     for k in range(3))
    return poses.astype(np.float32)


def make_times(frames: int) -> np.ndarray:
    """Normalised frame times t_f = f/(F-1) in [0, 1] (t = 0 for one frame)."""
    if frames == 1:
        return np.zeros(1, np.float32)
    return (np.arange(frames, dtype=np.float64) / (frames - 1)).astype(np.float32)


def make_targets(rng: np.random.Generator, frames: int, height: int, width: int) -> np.ndarray:
    """Target frames ~ U[0,1], [F][3][H][W] fp32, drawn frame by frame (the
    same stream as one draw of the whole array)."""
    out = np.empty((frames, 3, height, width), np.float32)
    for f in range(frames):
        out[f] = rng.random((3, height, width))
    return out


def make_workload(name: str, seed: int = 0, targets: bool = True, n: Optional[int] = None,
                  frames: Optional[int] = None) -> dict:
    """Build one named workload: scene, camera, poses [F][7], times [F] and,
    optionally, U[0,1] targets.  ``n``/``frames`` override the sizes (the
    distributions stay the same) for reduced-size test cases."""
    w = WORKLOADS[name]
    n = w["n"] if n is None else n
    F = w["frames"] if frames is None else frames
    rng = np.random.default_rng(seed)
    scene = make_scene(rng, n, z=w["z"], log_scale=w["log_scale"], dtype=w["dtype"], cubic=w["cubic"],
                       n_ctrl=w.get("n_ctrl", 0), poly_cov=w.get("poly_cov", False),
                       sh_degree=w.get("sh_degree", 0))
    cam = make_camera(w["width"], w["height"], w["focal"])
    poses = make_trajectory(rng, F) if w["trajectory"] == "smooth" else identity_poses(F)
    times = make_times(F)
    tg = make_targets(rng, F, cam.height, cam.width) if targets else None
    return dict(name=name, scene=scene, camera=cam, poses=poses, times=times, targets=tg, frames=F, n=n)


# --------------------------------------------------------------------------
# adversarial scenes for edge-case tests
# --------------------------------------------------------------------------

def adversarial_scene(rng: np.random.Generator, n: int, kind: str, width: int = 48, height: int = 40,
                      focal: float = 48.0) -> tuple:
    """Small scenes that stress one edge of the renderer.

    kinds: "huge" (a few Gaussians covering the whole image among small ones),
    "offscreen" (most Gaussians outside the frustum), "near" (Gaussians close
    to the near plane), "ties" (many exactly equal depths), "zero_opacity"
    (opacity logits of -40), "dense" (many overlapping Gaussians, early
    termination), "elongated" (needle-like covariances).
    """
    cam = make_camera(width, height, focal)
    means = np.empty((3, n))
    means[0] = rng.uniform(-1, 1, n)
    means[1] = rng.uniform(-1, 1, n)
    means[2] = rng.uniform(2, 6, n)
    ls = rng.normal(-2.5, 0.4, (3, n))
    q = rng.normal(0, 1, (4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    eta = rng.normal(0, 1, n)
    col = rng.uniform(0, 1, (3, n))
    if kind == "huge":
        k = max(1, n // 20)
        ls[:, :k] = rng.uniform(0.0, 1.0, (3, k))
    elif kind == "offscreen":
        k = (3 * n) // 4
        means[0, :k] = rng.choice([-1, 1], k) * rng.uniform(3, 20, k)
        means[1, :k] = rng.uniform(-5, 5, k)
    elif kind == "near":
        means[2] = rng.uniform(0.05, 0.6, n)
        means[0] *= means[2] / 4
        means[1] *= means[2] / 4
        ls -= 1.5
    elif kind == "ties":
        means[2] = rng.choice([2.0, 3.0, 4.0], n)
    elif kind == "zero_opacity":
        eta[:] = -40.0
    elif kind == "dense":
        eta = rng.normal(3.0, 0.5, n)
        ls = rng.normal(-1.8, 0.2, (3, n))
    elif kind == "elongated":
        ls[0] = rng.normal(-1.0, 0.2, n)
        ls[1] = rng.normal(-5.0, 0.2, n)
        ls[2] = rng.normal(-5.0, 0.2, n)
    else:
        raise ValueError(kind)
    scene = Scene(dtype="f32", means=_store(means, "f32"), log_scales=_store(ls, "f32"),
                  quats=_store(q, "f32"), opacity_logits=_store(eta, "f32"), colors=_store(col, "f32"))
    return scene, cam


# --------------------------------------------------------------------------
# camera-ODE parameters
# --------------------------------------------------------------------------

def init_mlp_theta(rng: np.random.Generator, last_layer_scale: float = 0.1, hidden: int = 64,
                   state: int = 7) -> np.ndarray:
    """Parameters of the 8 -> 64 -> 64 -> 7 vector-field MLP as one FP64 vector
    (W1 [64][8], b1, W2 [64][64], b2, W3 [7][64], b3): each layer's weights and
    bias ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)), the last layer scaled by
    ``last_layer_scale`` (a small initial camera velocity)."""
    def layer(fan_out, fan_in, scale=1.0):
        b = 1.0 / np.sqrt(fan_in)
        return rng.uniform(-b, b, (fan_out, fan_in)) * scale, rng.uniform(-b, b, fan_out) * scale
    W1, b1 = layer(hidden, state + 1)
    W2, b2 = layer(hidden, hidden)
    W3, b3 = layer(state, hidden, last_layer_scale)
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])
