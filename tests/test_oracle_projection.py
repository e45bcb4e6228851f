"""Pins of the oracle's projection stage (steps 1-4 of the forward model).

Each test ties the oracle to something other than itself: scipy's rotation
routines, closed forms of special cases, the defining relation of the EWA
approximation (the 2D covariance is the push-forward of the 3D one by the
Jacobian of the mean's projection, checked against finite differences of the
oracle's own mean projection) and a Monte-Carlo estimate.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import gv_synth
import oracle


def one_gaussian(mu, log_s, q, eta=0.0, col=(1.0, 1.0, 1.0), coeffs=None):
    s = dict(means=np.array(mu, float).reshape(3, 1), log_scales=np.array(log_s, float).reshape(3, 1),
             quats=np.array(q, float).reshape(4, 1), opacity_logits=np.array([eta], float),
             colors=np.array(col, float).reshape(3, 1))
    s["mean_coeffs"] = None if coeffs is None else np.array(coeffs, float).reshape(3, 3, 1)
    return s


def rand_scene(rng, n):
    mu = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(2, 6, n)])
    q = rng.normal(0, 1, (4, n))
    return dict(means=mu, log_scales=rng.normal(-2.5, 0.5, (3, n)), quats=q,
                opacity_logits=rng.normal(0, 1, n), colors=rng.uniform(0, 1, (3, n)), mean_coeffs=None)


def scipy_R(q_wxyz):
    w, x, y, z = q_wxyz
    return Rotation.from_quat([x, y, z, w]).as_matrix()


CAM = gv_synth.make_camera(64, 48, 64.0)


def test_world_covariance_matches_scipy_rotation():
    """Sigma = (RS)(RS)^T (Sec. 3.1) with R from scipy's quaternion routine."""
    rng = np.random.default_rng(1)
    s = rand_scene(rng, 50)
    p = oracle.project(s, CAM, [1, 0, 0, 0, 0, 0, 0])
    for g in range(50):
        R = scipy_R(s["quats"][:, g])
        S = np.diag(np.exp(s["log_scales"][:, g]))
        Sig = (R @ S) @ (R @ S).T
        got = np.array([[p["Sxx"][g], p["Sxy"][g], p["Sxz"][g]],
                        [p["Sxy"][g], p["Syy"][g], p["Syz"][g]],
                        [p["Sxz"][g], p["Syz"][g], p["Szz"][g]]])
        np.testing.assert_allclose(got, Sig, rtol=1e-12, atol=1e-15)
        # eigenvalues are the squared scales
        np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(got)), np.sort(np.diag(S) ** 2), rtol=1e-9)


def test_camera_space_mean_matches_scipy_pose():
    rng = np.random.default_rng(2)
    s = rand_scene(rng, 40)
    qc = rng.normal(0, 1, 4)
    tc = rng.normal(0, 0.3, 3)
    pose = np.concatenate([qc, tc])
    p = oracle.project(s, CAM, pose)
    m = scipy_R(qc / np.linalg.norm(qc)) @ s["means"] + tc[:, None]
    ok = m[2] > CAM.near_plane
    np.testing.assert_allclose(p["mx"][ok], m[0][ok], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(p["my"][ok], m[1][ok], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(p["depth"][ok], m[2][ok], rtol=1e-12)
    # depth key is the fp32 rounding of the depth
    np.testing.assert_array_equal(p["key"][ok], m[2][ok].astype(np.float32).astype(np.float64))


def test_pinhole_special_points():
    """On the optical axis the mean lands on the principal point; at (x,0,z)
    it lands at cx + fx x / z."""
    cam = gv_synth.make_camera(100, 80, 90.0)
    s = one_gaussian([0, 0, 3], [-3, -3, -3], [1, 0, 0, 0])
    p = oracle.project(s, cam, [1, 0, 0, 0, 0, 0, 0])
    assert p["u"][0] == pytest.approx(cam.cx, abs=1e-12) and p["v"][0] == pytest.approx(cam.cy, abs=1e-12)
    s = one_gaussian([0.6, 0, 3], [-3, -3, -3], [1, 0, 0, 0])
    p = oracle.project(s, cam, [1, 0, 0, 0, 0, 0, 0])
    assert p["u"][0] == pytest.approx(cam.cx + 90.0 * 0.6 / 3.0, abs=1e-12)
    assert p["v"][0] == pytest.approx(cam.cy, abs=1e-12)


def test_isotropic_on_axis_closed_form():
    """Isotropic Gaussian on the optical axis: Sigma' = ((f s/z)^2 + dil) I,
    conic = I / ((f s/z)^2 + dil), for any rotation quaternion."""
    cam = gv_synth.make_camera(64, 64, 128.0)
    rng = np.random.default_rng(3)
    for z, ls in [(2.0, -3.0), (5.0, -2.0), (3.3, -4.1)]:
        q = rng.normal(0, 1, 4)
        p = oracle.project(one_gaussian([0, 0, z], [ls] * 3, q), cam, [1, 0, 0, 0, 0, 0, 0])
        var = (128.0 * np.exp(ls) / z) ** 2 + cam.dilation
        assert p["cov00"][0] == pytest.approx(var, rel=1e-12)
        assert p["cov11"][0] == pytest.approx(var, rel=1e-12)
        assert abs(p["cov01"][0]) < 1e-12 * var
        assert p["A00"][0] == pytest.approx(1 / var, rel=1e-12)
        assert p["A11"][0] == pytest.approx(1 / var, rel=1e-12)


def test_anisotropic_rotated_about_optical_axis_closed_form():
    """Scales (a, b, c) rotated by angle th about z, on the optical axis:
    Sigma' = (f/z)^2 R2 diag(a^2, b^2) R2^T + dil I with R2 the 2D rotation by
    th.  A transposed rotation would rotate by -th and fail."""
    cam = gv_synth.make_camera(64, 64, 100.0)
    z, a, b, th = 4.0, 0.05, 0.02, 0.7
    q = [np.cos(th / 2), 0, 0, np.sin(th / 2)]
    p = oracle.project(one_gaussian([0, 0, z], np.log([a, b, 0.03]), q), cam, [1, 0, 0, 0, 0, 0, 0])
    R2 = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    cov = (100.0 / z) ** 2 * R2 @ np.diag([a * a, b * b]) @ R2.T + cam.dilation * np.eye(2)
    np.testing.assert_allclose([p["cov00"][0], p["cov01"][0], p["cov11"][0]],
                               [cov[0, 0], cov[0, 1], cov[1, 1]], rtol=1e-12)


def _fd_jacobian_of_mean_projection(s, g, cam, pose, h=1e-6):
    Jn = np.zeros((2, 3))
    for k in range(3):
        sp = {kk: (None if v is None else v.copy()) for kk, v in s.items()}
        sm = {kk: (None if v is None else v.copy()) for kk, v in s.items()}
        sp["means"][k, g] += h
        sm["means"][k, g] -= h
        pp, pm = oracle.project(sp, cam, pose), oracle.project(sm, cam, pose)
        Jn[0, k] = (pp["u"][g] - pm["u"][g]) / (2 * h)
        Jn[1, k] = (pp["v"][g] - pm["v"][g]) / (2 * h)
    return Jn


def test_ewa_covariance_is_pushforward_by_projection_jacobian():
    """Sigma' - dil I == Jw Sigma Jw^T where Jw = d(u,v)/d(mu) is taken by
    central differences of the oracle's own projected means (off-axis
    Gaussians, rotated camera)."""
    rng = np.random.default_rng(4)
    s = rand_scene(rng, 8)
    qc = np.array([1.0, 0.05, -0.04, 0.03])
    pose = np.concatenate([qc, [0.1, -0.05, 0.2]])
    p = oracle.project(s, CAM, pose)
    for g in range(8):
        Jw = _fd_jacobian_of_mean_projection(s, g, CAM, pose)
        Sig = np.array([[p["Sxx"][g], p["Sxy"][g], p["Sxz"][g]],
                        [p["Sxy"][g], p["Syy"][g], p["Syz"][g]],
                        [p["Sxz"][g], p["Syz"][g], p["Szz"][g]]])
        expect = Jw @ Sig @ Jw.T
        got = np.array([[p["cov00"][g] - CAM.dilation, p["cov01"][g]], [p["cov01"][g], p["cov11"][g] - CAM.dilation]])
        np.testing.assert_allclose(got, expect, rtol=1e-6, atol=1e-9 * np.abs(expect).max())
        # conic is the inverse of the dilated covariance
        A = np.array([[p["A00"][g], p["A01"][g]], [p["A01"][g], p["A11"][g]]])
        np.testing.assert_allclose(A @ (got + CAM.dilation * np.eye(2)), np.eye(2), atol=1e-12)


def test_ewa_covariance_monte_carlo():
    """For a small Gaussian the exact perspective image of samples has the
    EWA covariance to first order (statistical tolerance)."""
    rng = np.random.default_rng(5)
    mu = np.array([0.4, -0.3, 3.0])
    q = np.array([0.9, 0.3, -0.2, 0.25])
    ls = np.log([0.004, 0.002, 0.003])
    cam = gv_synth.make_camera(128, 128, 128.0)
    pose = np.array([0.99, 0.02, 0.05, -0.03, 0.05, 0.02, 0.1])
    p = oracle.project(one_gaussian(mu, ls, q), cam, pose)
    R = scipy_R(q / np.linalg.norm(q))
    L = R @ np.diag(np.exp(ls))
    X = mu[:, None] + L @ rng.normal(0, 1, (3, 400_000))
    Rc = scipy_R(pose[:4] / np.linalg.norm(pose[:4]))
    m = Rc @ X + pose[4:, None]
    uv = np.stack([cam.fx * m[0] / m[2] + cam.cx, cam.fy * m[1] / m[2] + cam.cy])
    C = np.cov(uv)
    got = np.array([[p["cov00"][0] - cam.dilation, p["cov01"][0]], [p["cov01"][0], p["cov11"][0] - cam.dilation]])
    np.testing.assert_allclose(got, C, rtol=2e-2, atol=2e-2 * np.abs(C).max())
    np.testing.assert_allclose([p["u"][0], p["v"][0]], uv.mean(axis=1), atol=2e-3)


def test_cubic_mean_in_time():
    """mu(t) = mu0 + a1 t + a2 t^2 + a3 t^3 (polynomial motion basis)."""
    cam = gv_synth.make_camera(64, 64, 64.0)
    co = np.array([[0.1, -0.2, 0.05], [0.3, 0.1, -0.1], [-0.2, 0.05, 0.2]])  # [coeff][xyz]
    s = one_gaussian([0.1, 0.2, 3.0], [-3] * 3, [1, 0, 0, 0], coeffs=co)
    for t in [0.0, 0.37, 1.0]:
        p = oracle.project(s, cam, [1, 0, 0, 0, 0, 0, 0], t=t)
        mu = np.array([0.1, 0.2, 3.0]) + co[0] * t + co[1] * t ** 2 + co[2] * t ** 3
        assert p["mx"][0] == pytest.approx(mu[0], abs=1e-14)
        assert p["my"][0] == pytest.approx(mu[1], abs=1e-14)
        assert p["depth"][0] == pytest.approx(mu[2], abs=1e-14)


def test_culling_rules():
    cam = gv_synth.make_camera(32, 32, 32.0)
    base = rand_scene(np.random.default_rng(6), 5)
    base["means"][2, 0] = 0.005          # in front of the camera but before the near plane
    base["means"][2, 1] = -1.0           # behind the camera
    base["quats"][:, 2] = 0.0            # degenerate rotation
    base["log_scales"][0, 3] = np.nan    # non-finite parameter
    p = oracle.project(base, cam, [1, 0, 0, 0, 0, 0, 0])
    assert list(p["valid"]) == [0, 0, 0, 0, 1]
