"""Pins of the oracle's time evaluation (Sec. 3.2, Eq. 2-3): clamped cubic
B-spline means and cubic-polynomial log-scales and quaternions.

The basis is pinned by its defining properties (partition of unity, local
support, endpoint interpolation), by the Bernstein polynomials it reduces to
with four control points, and by scipy's B-spline evaluation; the rendering
path by its reduction to the already-pinned static and cubic-mean paths; the
adjoint by central finite differences.
"""
import math

import numpy as np
import pytest
from scipy.interpolate import BSpline

import gv_synth
import oracle


def knots(M):
    inner = [(j - 3) / (M - 3) for j in range(4, M)]
    return np.array([0.0] * 4 + inner + [1.0] * 4)


T_GRID = np.concatenate([np.linspace(0.0, 1.0, 201), [1e-12, 1 - 1e-12, 0.5 + 1e-13]])


@pytest.mark.parametrize("M", [4, 5, 8, 13])
def test_partition_of_unity_and_local_support(M):
    u = knots(M)
    for t in T_GRID:
        B = oracle.bspline_basis(M, t)
        assert abs(B.sum() - 1.0) < 1e-14, (M, t)
        assert (B >= -1e-16).all()
        for i in range(M):
            if not (u[i] <= t <= u[i + 4]):
                assert B[i] == 0.0, (M, t, i)
        assert (B > 0).sum() <= 4


@pytest.mark.parametrize("M", [4, 6, 9])
def test_endpoint_interpolation(M):
    B0, B1 = oracle.bspline_basis(M, 0.0), oracle.bspline_basis(M, 1.0)
    np.testing.assert_array_equal(B0, np.eye(M)[0])
    np.testing.assert_array_equal(B1, np.eye(M)[M - 1])


def test_four_control_points_are_bernstein():
    for t in T_GRID:
        B = oracle.bspline_basis(4, t)
        bern = [math.comb(3, i) * t ** i * (1 - t) ** (3 - i) for i in range(4)]
        np.testing.assert_allclose(B, bern, rtol=0, atol=1e-15)


@pytest.mark.parametrize("M", [5, 8, 11])
def test_matches_scipy_bspline(M):
    u = knots(M)
    for t in T_GRID:
        ref = np.array([BSpline(u, np.eye(M)[i], 3, extrapolate=False)(t) for i in range(M)])
        if t == 1.0:  # scipy leaves the closed right end to extrapolation
            ref = np.array([BSpline(u, np.eye(M)[i], 3, extrapolate=True)(t) for i in range(M)])
        np.testing.assert_allclose(oracle.bspline_basis(M, t), ref, rtol=0, atol=1e-14)


def test_invalid_arguments():
    with pytest.raises(ValueError):
        oracle.bspline_basis(3, 0.5)
    with pytest.raises(ValueError):
        oracle.bspline_basis(6, 1.5)


# ---------------------------------------------------------------------------
# rendering with time-dependent parameters
# ---------------------------------------------------------------------------

def dyn_case(seed, M=6, n=30, W=32, H=24):
    rng = np.random.default_rng(seed)
    cam = gv_synth.make_camera(W, H, float(W), bg=(0.1, 0.2, 0.3))
    mu = np.stack([rng.uniform(-0.7, 0.7, n), rng.uniform(-0.5, 0.5, n), rng.uniform(2, 5, n)])
    s = dict(means=mu, log_scales=rng.normal(-2.4, 0.4, (3, n)), quats=rng.normal(0, 1, (4, n)),
             opacity_logits=rng.normal(0.3, 1.0, n), colors=rng.uniform(0, 1, (3, n)),
             ctrl=mu[None] + rng.normal(0, 0.15, (M, 3, n)),
             scale_coeffs=rng.normal(0, 0.3, (3, 3, n)), quat_coeffs=rng.normal(0, 0.3, (3, 4, n)))
    pose = np.array([1.0, 0.03, -0.05, 0.02, 0.05, -0.03, 0.1])
    return s, cam, pose, rng


def static_at(s, t):
    """The static scene whose parameters are the dynamic scene's values at t."""
    M = s["ctrl"].shape[0]
    B = oracle.bspline_basis(M, t)
    mu = np.einsum("i,ikn->kn", B, s["ctrl"])
    pw = np.array([t, t * t, t * t * t])
    ls = s["log_scales"] + np.einsum("c,ckn->kn", pw, s["scale_coeffs"])
    q = s["quats"] + np.einsum("c,ckn->kn", pw, s["quat_coeffs"])
    return dict(means=mu, log_scales=ls, quats=q, opacity_logits=s["opacity_logits"], colors=s["colors"]), B, pw


@pytest.mark.parametrize("t", [0.0, 0.37, 0.5, 1.0])
def test_dynamic_frame_reduces_to_static_frame(t):
    s, cam, pose, rng = dyn_case(3)
    st, B, pw = static_at(s, t)
    dl = rng.normal(0, 1, (cam.width * cam.height, 3))
    rd = oracle.render_frame(s, cam, pose, t, dL_dC=dl)
    rs = oracle.render_frame(st, cam, pose, t, dL_dC=dl)
    np.testing.assert_allclose(rd["color"], rs["color"], rtol=0, atol=1e-12)
    gd, gs = rd["grads"], rs["grads"]
    # linear time evaluation: each coefficient gets its basis value times the static gradient
    np.testing.assert_allclose(gd["ctrl"], B[:, None, None] * gs["means"][None], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gd["log_scales"], gs["log_scales"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gd["scale_coeffs"], pw[:, None, None] * gs["log_scales"][None], rtol=1e-9,
                               atol=1e-12)
    np.testing.assert_allclose(gd["quats"], gs["quats"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gd["quat_coeffs"], pw[:, None, None] * gs["quats"][None], rtol=1e-9, atol=1e-12)
    np.testing.assert_array_equal(gd["means"], 0.0)  # the stored centre is unused with control points
    for k in ("opacity_logits", "colors", "pose"):
        np.testing.assert_allclose(gd[k], gs[k], rtol=1e-9, atol=1e-12)


def test_four_point_spline_equals_cubic_mean():
    """With M = 4 the spline is the cubic in power form: mu0 = P0,
    a1 = 3(P1-P0), a2 = 3(P0-2P1+P2), a3 = P3-3P2+3P1-P0."""
    s, cam, pose, rng = dyn_case(5, M=4)
    P = s["ctrl"]
    cub = dict(s)
    del cub["ctrl"]
    cub["means"] = P[0]
    cub["mean_coeffs"] = np.stack([3 * (P[1] - P[0]), 3 * (P[0] - 2 * P[1] + P[2]),
                                   P[3] - 3 * P[2] + 3 * P[1] - P[0]])
    for t in (0.0, 0.21, 0.8, 1.0):
        a = oracle.render_frame(s, cam, pose, t)["color"]
        b = oracle.render_frame(cub, cam, pose, t)["color"]
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-11)


def test_dynamic_adjoint_matches_central_differences():
    s, cam, pose, rng = dyn_case(7, M=5)
    t = 0.63
    full = oracle.render_frame(s, cam, pose, t)
    dl = rng.normal(0, 1, (cam.width * cam.height, 3))
    stable = (full["margins"] > 1e-3).all(axis=1)
    assert stable.mean() > 0.9
    dl[~stable] = 0.0
    g = oracle.render_frame(s, cam, pose, t, dL_dC=dl)["grads"]

    def L():
        return float(np.sum(oracle.render_frame(s, cam, pose, t)["color"] * dl))

    for name in ("ctrl", "scale_coeffs", "quat_coeffs", "log_scales", "quats"):
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


def test_synthetic_dynamic_workload_shapes():
    w = gv_synth.make_workload("clip540p_f50_n200k_dyn", n=500, frames=3, targets=False)
    sc = w["scene"]
    assert sc.ctrl.shape == (8, 3, 500) and sc.scale_coeffs.shape == (3, 3, 500)
    assert sc.quat_coeffs.shape == (3, 4, 500) and sc.mean_coeffs is None
    # static fields keep the same draws as the static workload (dynamic draws come last)
    w0 = gv_synth.make_workload("clip540p_f50_n200k", n=500, frames=3, targets=False)
    np.testing.assert_array_equal(sc.means, w0["scene"].means)
    np.testing.assert_array_equal(sc.colors, w0["scene"].colors)
