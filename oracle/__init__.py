"""FP64 CPU oracle for the differentiable Gaussian rasterizer and the camera ODE.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  It shares
no code with the HIP path (``paper_2501_04782_amd``) and imports nothing from
it; the only module both sides use is ``gv_synth`` (seeded input draws).

* ``gvo_raster.c``: the tile-free, per-pixel definition of 3D Gaussian
  splatting image formation (paper Sec. 3.1) and its adjoint, in FP64, and a
  tiled form of it for speed (each pixel visits only the Gaussians whose
  footprint box meets its tile, in the same order, with identical results:
  ``tests/test_oracle_tiled.py``).
* ``camera_ode.py``: the camera-motion Neural ODE (Eq. 1, Sec. 3.4) with RK4
  and its discrete adjoint, in FP64 numpy.
* this file: ctypes marshalling around ``gvo_raster.c``, a clip loop and the
  L2 loss of Sec. 4.1.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

from . import camera_ode  # noqa: F401  (re-export)

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)


class _Frame(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("means", _dp), ("log_scales", _dp), ("quats", _dp), ("opacity_logits", _dp),
        ("colors", _dp), ("mean_coeffs", _dp),
        ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("fx", ctypes.c_double), ("fy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
        ("near_plane", ctypes.c_double), ("dilation", ctypes.c_double),
        ("bg", ctypes.c_double * 3), ("pose", ctypes.c_double * 7), ("t", ctypes.c_double),
        ("n_ctrl", ctypes.c_int32), ("ctrl", _dp), ("scale_coeffs", _dp), ("quat_coeffs", _dp),
        ("sh_degree", ctypes.c_int32), ("sh", _dp),
    ]


class _Grads(ctypes.Structure):
    _fields_ = [("means", _dp), ("log_scales", _dp), ("quats", _dp), ("opacity_logits", _dp),
                ("colors", _dp), ("mean_coeffs", _dp), ("pose", _dp),
                ("ctrl", _dp), ("scale_coeffs", _dp), ("quat_coeffs", _dp), ("sh", _dp), ("intrinsics", _dp)]

OPTIONAL = ("mean_coeffs", "ctrl", "scale_coeffs", "quat_coeffs", "sh")


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.gvo_project.argtypes = [ctypes.POINTER(_Frame), _dp]
        lib.gvo_project.restype = ctypes.c_int
        lib.gvo_render.argtypes = [ctypes.POINTER(_Frame), ctypes.c_int64, _i64p, _dp, _dp, _i64p, _dp,
                                   _dp, ctypes.POINTER(_Grads), ctypes.c_int, _dp, _dp]
        lib.gvo_render.restype = ctypes.c_int
        lib.gvo_render_tiled.argtypes = lib.gvo_render.argtypes + [ctypes.c_int]
        lib.gvo_render_tiled.restype = ctypes.c_int
        lib.gvo_bspline_basis.argtypes = [ctypes.c_int32, ctypes.c_double, _dp]
        lib.gvo_bspline_basis.restype = ctypes.c_int
        lib.gvo_sh_basis.argtypes = [ctypes.c_int32, _dp, _dp, _dp]
        lib.gvo_sh_basis.restype = ctypes.c_int
        lib.gvo_abi_version.restype = ctypes.c_int
        lib.gvo_contributors.argtypes = [ctypes.POINTER(_Frame), ctypes.POINTER(ctypes.c_uint8), ctypes.c_int]
        lib.gvo_contributors.restype = ctypes.c_int
        if lib.gvo_abi_version() != 7:
            raise RuntimeError("liboracle.so is stale: rebuild it (python -m oracle.build)")
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def scene_f64(scene) -> dict:
    """Accept a gv_synth.Scene or a dict of arrays; return contiguous FP64 arrays."""
    d = scene.as_f64() if hasattr(scene, "as_f64") else dict(scene)
    out = {}
    for k in ("means", "log_scales", "quats", "opacity_logits", "colors"):
        out[k] = np.ascontiguousarray(np.asarray(d[k], dtype=np.float64))
    for k in OPTIONAL:
        v = d.get(k)
        out[k] = None if v is None else np.ascontiguousarray(np.asarray(v, dtype=np.float64))
    if out["ctrl"] is not None and out["mean_coeffs"] is not None:
        raise ValueError("a scene has either B-spline control points or cubic mean coefficients")
    return out


def bspline_basis(n_ctrl: int, t: float) -> np.ndarray:
    """N_{i,3}(t), i < n_ctrl, of the clamped cubic B-spline of Eq. 2."""
    out = np.zeros(n_ctrl)
    if _load().gvo_bspline_basis(int(n_ctrl), float(t), _ptr(out)) != 0:
        raise ValueError(f"bspline_basis: need 4 <= n_ctrl <= 64 and 0 <= t <= 1 (got {n_ctrl}, {t})")
    return out


def sh_basis(degree: int, d, grad: bool = False):
    """Real SH Y_lm(d), 1 <= l <= degree, (l, m) ascending; with grad=True
    also the partials of each polynomial w.r.t. (x, y, z)."""
    d = np.ascontiguousarray(np.asarray(d, dtype=np.float64).reshape(3))
    nb = (degree + 1) ** 2 - 1
    out = np.zeros(max(nb, 1))
    g = np.zeros((max(nb, 1), 3))
    if _load().gvo_sh_basis(int(degree), _ptr(d), _ptr(out), _ptr(g)) != 0:
        raise ValueError(f"sh_basis: degree must be 0..3 (got {degree})")
    return (out[:nb], g[:nb]) if grad else out[:nb]


def sh_degree_of(sh) -> int:
    if sh is None:
        return 0
    nb = int(np.asarray(sh).shape[0])
    deg = {3: 1, 8: 2, 15: 3}.get(nb)
    if deg is None:
        raise ValueError(f"sh must hold 3, 8 or 15 coefficient rows (degree 1..3), got {nb}")
    return deg


def _frame(s: dict, cam, pose7, t: float):
    fr = _Frame()
    fr.n = int(s["opacity_logits"].shape[0])
    fr.means, fr.log_scales, fr.quats = _ptr(s["means"]), _ptr(s["log_scales"]), _ptr(s["quats"])
    fr.opacity_logits, fr.colors = _ptr(s["opacity_logits"]), _ptr(s["colors"])
    fr.mean_coeffs = _ptr(s["mean_coeffs"])
    fr.n_ctrl = 0 if s["ctrl"] is None else int(s["ctrl"].shape[0])
    fr.ctrl, fr.scale_coeffs, fr.quat_coeffs = _ptr(s["ctrl"]), _ptr(s["scale_coeffs"]), _ptr(s["quat_coeffs"])
    fr.sh_degree, fr.sh = sh_degree_of(s["sh"]), _ptr(s["sh"])
    fr.width, fr.height = int(cam.width), int(cam.height)
    fr.fx, fr.fy, fr.cx, fr.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    fr.near_plane, fr.dilation = float(cam.near_plane), float(cam.dilation)
    for k in range(3):
        fr.bg[k] = float(cam.bg[k])
    pose7 = np.asarray(pose7, dtype=np.float64).reshape(7)
    for k in range(7):
        fr.pose[k] = float(pose7[k])
    fr.t = float(t)
    return fr


PROJECT_FIELDS = ["valid", "u", "v", "cov00", "cov01", "cov11", "A00", "A01", "A11", "depth", "key",
                  "opacity", "Sxx", "Sxy", "Sxz", "Syy", "Syz", "Szz", "mx", "my"]


def project(scene, cam, pose7, t: float = 0.0) -> dict:
    """Per-Gaussian projection (mean, EWA covariance, conic, depth, opacity)."""
    s = scene_f64(scene)
    fr = _frame(s, cam, pose7, t)
    out = np.zeros((fr.n, 24))
    _load().gvo_project(ctypes.byref(fr), _ptr(out))
    return {k: out[:, i] for i, k in enumerate(PROJECT_FIELDS)}


def zero_grads(scene) -> dict:
    s = scene_f64(scene)
    n = s["opacity_logits"].shape[0]
    g = dict(means=np.zeros((3, n)), log_scales=np.zeros((3, n)), quats=np.zeros((4, n)),
             opacity_logits=np.zeros(n), colors=np.zeros((3, n)), pose=np.zeros(7), intrinsics=np.zeros(4))
    for k in OPTIONAL:
        g[k] = None if s[k] is None else np.zeros_like(s[k])
    return g


def render_frame(scene, cam, pose7, t: float = 0.0, pixels: Optional[np.ndarray] = None,
                 dL_dC: Optional[np.ndarray] = None, grads: Optional[dict] = None,
                 threads: int = 0, stake_tol: Optional[Sequence[float]] = None, tile: int = 0) -> dict:
    """Render one frame at the listed pixels (linear y*W+x; None = all).

    Returns color [P][3], T_final [P], n_contrib [P], margins [P][4] and, when
    dL_dC [P][3] is given, the gradient dict (accumulated into ``grads`` if
    passed) of sum_p dL_dC[p] . C[p].  With ``stake_tol`` (relative margins
    of the 3-sigma cut, the 1/255 cut and the stop) it also returns
    ``stake`` [P]: the blending weight that decisions within those margins
    control (an entry's alpha*T for a cut, the remaining transmittance for
    the stop), so that a pixel taken the other way at such a decision can
    differ by at most stake times the colour range.

    tile > 0 selects the tiled form: each pixel visits only the Gaussians whose
    footprint box meets its tile (in the same global order), with results
    identical to the per-pixel definition (margins from 1e-3 up may read
    larger); it is the fast form for timing and large frames.
    """
    s = scene_f64(scene)
    fr = _frame(s, cam, pose7, t)
    if pixels is None:
        npx = int(cam.width) * int(cam.height)
        pix_p = None
    else:
        pixels = np.ascontiguousarray(np.asarray(pixels, dtype=np.int64))
        npx = int(pixels.shape[0])
        assert npx == 0 or (pixels.min() >= 0 and pixels.max() < cam.width * cam.height)
        pix_p = pixels.ctypes.data_as(_i64p)
    color = np.zeros((npx, 3))
    T = np.zeros(npx)
    nc = np.zeros(npx, np.int64)
    mg = np.zeros((npx, 4))
    gstruct = None
    dl = None
    if dL_dC is not None:
        dl = np.ascontiguousarray(np.asarray(dL_dC, dtype=np.float64).reshape(npx, 3))
        if grads is None:
            grads = zero_grads(s)
        gstruct = _Grads(_ptr(grads["means"]), _ptr(grads["log_scales"]), _ptr(grads["quats"]),
                         _ptr(grads["opacity_logits"]), _ptr(grads["colors"]), _ptr(grads.get("mean_coeffs")),
                         _ptr(grads["pose"]), _ptr(grads.get("ctrl")), _ptr(grads.get("scale_coeffs")),
                         _ptr(grads.get("quat_coeffs")), _ptr(grads.get("sh")), _ptr(grads.get("intrinsics")))
    tol = stake = None
    if stake_tol is not None:
        tol = np.ascontiguousarray(np.asarray(stake_tol, dtype=np.float64).reshape(3))
        stake = np.zeros(npx)
    args = (ctypes.byref(fr), npx, pix_p, _ptr(color), _ptr(T), nc.ctypes.data_as(_i64p), _ptr(mg), _ptr(dl),
            ctypes.byref(gstruct) if gstruct is not None else None, int(threads), _ptr(tol), _ptr(stake))
    rc = _load().gvo_render_tiled(*args, int(tile)) if tile > 0 else _load().gvo_render(*args)
    if rc != 0:
        raise RuntimeError(f"gvo_render failed with code {rc}")
    out = dict(color=color, T_final=T, n_contrib=nc, margins=mg)
    if stake is not None:
        out["stake"] = stake
    if dl is not None:
        out["grads"] = grads
    return out


def contributors(scene, cam, pose7, t: float = 0.0, threads: int = 0) -> np.ndarray:
    """Bool per Gaussian: contributes to at least one pixel of the frame."""
    s = scene_f64(scene)
    fr = _frame(s, cam, pose7, t)
    out = np.zeros(fr.n, np.uint8)
    rc = _load().gvo_contributors(ctypes.byref(fr), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), int(threads))
    if rc != 0:
        raise RuntimeError(f"gvo_contributors failed with code {rc}")
    return out.astype(bool)


def visibility_counts(scene, cam, poses, times, threads: int = 0) -> np.ndarray:
    """Per Gaussian, the number of frames of the clip it contributes to."""
    counts = np.zeros(scene_f64(scene)["opacity_logits"].shape[0], np.int64)
    for f in range(len(poses)):
        counts += contributors(scene, cam, np.asarray(poses[f], np.float64), float(times[f]), threads)
    return counts


def render_image(scene, cam, pose7, t: float = 0.0, threads: int = 0) -> dict:
    """Whole frame as planar arrays: image [3][H][W], T_final [H][W], margins [H][W][4]."""
    r = render_frame(scene, cam, pose7, t, threads=threads)
    H, W = int(cam.height), int(cam.width)
    return dict(image=r["color"].T.reshape(3, H, W).copy(), T_final=r["T_final"].reshape(H, W),
                n_contrib=r["n_contrib"].reshape(H, W), margins=r["margins"].reshape(H, W, 4))


def l2_loss_and_grad(images: np.ndarray, targets: np.ndarray, per_frame: bool = False):
    """The L2 reconstruction loss of Sec. 4.1, read as the mean over all
    frames, channels and pixels of the squared difference, and its gradient
    with respect to the images (same shape).  With per_frame=True the loss is
    returned as each frame's share (leading axis = frames), which sums to the
    mean: share_f = sum over frame f of (image - target)^2 / (number of
    values in all frames)."""
    images = np.asarray(images, np.float64)
    targets = np.asarray(targets, np.float64)
    if images.shape != targets.shape:
        raise ValueError(f"images {images.shape} and targets {targets.shape} differ in shape")
    diff = images - targets
    sq = diff * diff
    grad = 2.0 * diff / diff.size
    if per_frame:
        return sq.reshape(sq.shape[0], -1).sum(axis=1) / diff.size, grad
    return float(np.mean(sq)), grad


def _rotation(q) -> np.ndarray:
    """Rotation matrix of the quaternion q (w, x, y, z) after normalisation."""
    q = np.asarray(q, np.float64)
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def trajectory_error(poses, ref_poses) -> dict:
    """Error of a camera trajectory against a reference pose table (the
    learned camera of Sec. 3.4 judged by per-frame poses).  Poses are
    world-to-camera 7-vectors (q_w, q_x, q_y, q_z, t_x, t_y, t_z), q not
    necessarily unit.  Per frame: the camera centre c = -R^T t and the
    rotation R; the translation error is |c - c_ref|, the rotation error the
    geodesic angle of R R_ref^T, atan2(sin, cos) with sin the norm of the
    matrix's skew part and cos = (trace - 1) / 2.  Returns the root mean square
    translation error, the mean angle (radians) and the per-frame values."""
    poses = np.asarray(poses, np.float64).reshape(-1, 7)
    ref = np.asarray(ref_poses, np.float64).reshape(-1, 7)
    if poses.shape != ref.shape:
        raise ValueError("pose tables differ in length")
    terr = np.zeros(len(poses))
    ang = np.zeros(len(poses))
    for f in range(len(poses)):
        R, Rr = _rotation(poses[f, :4]), _rotation(ref[f, :4])
        c = -R.T @ poses[f, 4:]
        cr = -Rr.T @ ref[f, 4:]
        terr[f] = np.linalg.norm(c - cr)
        D = R @ Rr.T
        s = 0.5 * np.linalg.norm([D[2, 1] - D[1, 2], D[0, 2] - D[2, 0], D[1, 0] - D[0, 1]])
        ang[f] = np.arctan2(s, 0.5 * (np.trace(D) - 1.0))
    n = max(len(poses), 1)
    return dict(translation_rmse=float(np.sqrt(np.sum(terr ** 2) / n)), mean_angle=float(np.sum(ang) / n),
                translation=terr, angle=ang)


def render_clip_grads(scene, cam, poses: np.ndarray, times: Sequence[float], frames: Sequence[int],
                      pixels: Sequence[np.ndarray], dL_dC: Sequence[np.ndarray], threads: int = 0, tile: int = 0):
    """Sum over the listed frames of the gradient of sum_p dL_dC[f][p] . C_f[p]
    (shared parameters summed over frames, poses per frame); tile > 0 takes
    the tiled form (identical results)."""
    grads = zero_grads(scene)
    dposes = np.zeros((len(poses), 7))
    colors = []
    for f, pix, dl in zip(frames, pixels, dL_dC):
        grads["pose"][:] = 0.0
        r = render_frame(scene, cam, poses[f], float(times[f]), pixels=pix, dL_dC=dl, grads=grads,
                         threads=threads, tile=tile)
        dposes[f] = grads["pose"]
        colors.append(r["color"])
    grads["pose"] = None
    return grads, dposes, colors
