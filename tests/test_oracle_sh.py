"""Pins of the oracle's view-dependent colour (Sec. 3.1: colour as spherical
harmonics of degree d_c; the stored RGB is the l = 0 term).

The basis is pinned by orthonormality on the sphere (Gauss quadrature, exact
for these polynomial degrees), by scipy's complex spherical harmonics (each
real function equals the matching real combination up to one sign), and its
gradient polynomials by finite differences; the rendering path by reduction
to the RGB path and by finite differences through the view direction, the
mean and the pose.
"""
import math

import numpy as np
import pytest
from scipy.special import sph_harm_y

import gv_synth
import oracle

LM = [(l, m) for l in range(1, 4) for m in range(-l, l + 1)]


def sphere_quadrature(nt=10, nphi=24):
    """Nodes and weights integrating polynomials of degree < 2 nt in cos(theta)
    and trigonometric degree < nphi in phi exactly."""
    z, wz = np.polynomial.legendre.leggauss(nt)
    phi = 2 * np.pi * np.arange(nphi) / nphi
    Z, PHI = np.meshgrid(z, phi, indexing="ij")
    s = np.sqrt(1 - Z * Z)
    dirs = np.stack([s * np.cos(PHI), s * np.sin(PHI), Z], -1).reshape(-1, 3)
    w = (wz[:, None] * np.full(nphi, 2 * np.pi / nphi)[None]).reshape(-1)
    return dirs, w


def test_basis_is_orthonormal_and_orthogonal_to_the_constant():
    dirs, w = sphere_quadrature()
    Y = np.stack([oracle.sh_basis(3, d) for d in dirs])  # [Q][15]
    gram = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(gram, np.eye(15), atol=1e-12)
    np.testing.assert_allclose((Y * w[:, None]).sum(0), 0.0, atol=1e-12)
    assert abs(w.sum() - 4 * np.pi) < 1e-12


def test_basis_matches_scipy_real_harmonics_up_to_sign():
    rng = np.random.default_rng(0)
    d = rng.normal(size=(200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    polar, az = np.arccos(d[:, 2]), np.arctan2(d[:, 1], d[:, 0])
    Y = np.stack([oracle.sh_basis(3, v) for v in d])
    for k, (l, m) in enumerate(LM):
        c = sph_harm_y(l, abs(m), polar, az)
        ref = c.real if m == 0 else math.sqrt(2) * (c.real if m > 0 else c.imag)
        sign = np.sign(np.dot(Y[:, k], ref))
        assert sign != 0
        np.testing.assert_allclose(Y[:, k], sign * ref, atol=1e-12, err_msg=str((l, m)))


@pytest.mark.parametrize("degree", [1, 2, 3])
def test_lower_degrees_are_prefixes(degree):
    d = np.array([0.3, -0.5, 0.81])
    d /= np.linalg.norm(d)
    np.testing.assert_array_equal(oracle.sh_basis(degree, d), oracle.sh_basis(3, d)[:(degree + 1) ** 2 - 1])


def test_gradient_polynomials_match_finite_differences():
    rng = np.random.default_rng(1)
    for _ in range(20):
        p = rng.normal(size=3)
        _, G = oracle.sh_basis(3, p, grad=True)
        for j in range(3):
            e = np.zeros(3)
            e[j] = 1e-6
            fd = (oracle.sh_basis(3, p + e) - oracle.sh_basis(3, p - e)) / 2e-6
            np.testing.assert_allclose(G[:, j], fd, rtol=1e-7, atol=1e-8)


def sh_case(seed, degree=3, n=30, W=32, H=24, sh_std=0.3):
    rng = np.random.default_rng(seed)
    cam = gv_synth.make_camera(W, H, float(W), bg=(0.1, 0.2, 0.3))
    mu = np.stack([rng.uniform(-0.7, 0.7, n), rng.uniform(-0.5, 0.5, n), rng.uniform(2, 5, n)])
    s = dict(means=mu, log_scales=rng.normal(-2.4, 0.4, (3, n)), quats=rng.normal(0, 1, (4, n)),
             opacity_logits=rng.normal(0.3, 1.0, n), colors=rng.uniform(0, 1, (3, n)),
             sh=rng.normal(0, sh_std, ((degree + 1) ** 2 - 1, 3, n)))
    pose = np.array([0.98, 0.08, -0.12, 0.05, 0.3, -0.2, 0.4])
    return s, cam, pose, rng


def test_zero_coefficients_reduce_to_rgb():
    s, cam, pose, rng = sh_case(2)
    s0 = dict(s)
    s0["sh"] = np.zeros_like(s["sh"])
    st = {k: v for k, v in s.items() if k != "sh"}
    dl = rng.normal(0, 1, (cam.width * cam.height, 3))
    a = oracle.render_frame(s0, cam, pose, dL_dC=dl)
    b = oracle.render_frame(st, cam, pose, dL_dC=dl)
    np.testing.assert_array_equal(a["color"], b["color"])
    for k in ("means", "log_scales", "quats", "opacity_logits", "colors", "pose"):
        np.testing.assert_allclose(a["grads"][k], b["grads"][k], rtol=1e-12, atol=1e-14)


def test_colour_follows_the_view_direction():
    """One isotropic Gaussian on the optical axis of a camera translated along
    +x: the colour at its centre is o * (rgb + sum k Y(d)) (+ background),
    with d the unit vector from the camera centre to the mean."""
    W = H = 33
    cam = gv_synth.make_camera(W, H, float(W), bg=(0.0, 0.0, 0.0))
    mu = np.array([[0.5], [0.0], [3.0]])
    kc = np.arange(45, dtype=float).reshape(15, 3, 1) * 0.01 - 0.2
    s = dict(means=mu, log_scales=np.full((3, 1), -1.0), quats=np.array([[1.0], [0.0], [0.0], [0.0]]),
             opacity_logits=np.array([2.0]), colors=np.array([[0.3], [0.4], [0.5]]), sh=kc)
    pose = np.array([1.0, 0, 0, 0, -0.5, 0.0, 0.0])  # camera centre at (0.5, 0, 0): the mean is straight ahead
    r = oracle.render_frame(s, cam, pose)
    centre = (H // 2) * W + W // 2
    o = 1 / (1 + math.exp(-2.0))
    d = np.array([0.0, 0.0, 1.0])
    col = s["colors"][:, 0] + oracle.sh_basis(3, d) @ kc[:, :, 0]
    np.testing.assert_allclose(r["color"][centre], o * col, rtol=1e-12)
    # seen from a camera centre at the origin the direction tilts towards +x
    pose2 = np.array([1.0, 0, 0, 0, 0.0, 0.0, 0.0])
    r2 = oracle.render_frame(s, cam, pose2)
    d2 = np.array([0.5, 0.0, 3.0]) / math.hypot(0.5, 3.0)
    p = oracle.project(s, cam, pose2)
    x, y = int(p["u"][0]), int(p["v"][0])
    dx, dy = x + 0.5 - p["u"][0], y + 0.5 - p["v"][0]
    A = np.array([[p["A00"][0], p["A01"][0]], [p["A01"][0], p["A11"][0]]])
    q = np.array([dx, dy]) @ A @ np.array([dx, dy])
    col2 = s["colors"][:, 0] + oracle.sh_basis(3, d2) @ kc[:, :, 0]
    np.testing.assert_allclose(r2["color"][y * W + x], o * math.exp(-q / 2) * col2, rtol=1e-10)


@pytest.mark.parametrize("degree", [1, 3])
def test_sh_adjoint_matches_central_differences(degree):
    s, cam, pose, rng = sh_case(7 + degree, degree=degree)
    full = oracle.render_frame(s, cam, pose)
    dl = rng.normal(0, 1, (cam.width * cam.height, 3))
    stable = (full["margins"] > 1e-3).all(axis=1)
    assert stable.mean() > 0.9
    dl[~stable] = 0.0
    g = oracle.render_frame(s, cam, pose, dL_dC=dl)["grads"]

    def L(p=pose):
        return float(np.sum(oracle.render_frame(s, cam, p)["color"] * dl))

    for name in ("sh", "means", "colors"):
        flat = s[name].reshape(-1)
        for i in rng.choice(flat.size, 30, replace=False):
            h = 1e-6 * max(1.0, abs(flat[i]))
            old = flat[i]
            flat[i] = old + h
            lp = L()
            flat[i] = old - h
            lm = L()
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            assert g[name].reshape(-1)[i] == pytest.approx(fd, rel=2e-5, abs=2e-7 * (1 + np.abs(g[name]).max())), \
                (name, i)
    for k in range(7):
        pp, pm = pose.copy(), pose.copy()
        pp[k] += 1e-6
        pm[k] -= 1e-6
        fd = (L(pp) - L(pm)) / 2e-6
        assert g["pose"][k] == pytest.approx(fd, rel=2e-5, abs=1e-6), ("pose", k)


def test_synthetic_sh_workload_shapes():
    w = gv_synth.make_workload("clip540p_f50_n200k_sh3", n=400, frames=2, targets=False)
    assert w["scene"].sh.shape == (15, 3, 400)
    w0 = gv_synth.make_workload("clip540p_f50_n200k", n=400, frames=2, targets=False)
    np.testing.assert_array_equal(w["scene"].colors, w0["scene"].colors)
