"""Pins of the oracle's per-pixel "stake": the blending weight that
decisions within rounding of a threshold control (the 3-sigma cut, the 1/255
opacity cut and the stop before T falls below 1e-4; the 3DGS compositing rule
that Sec. 3.1 relies on).  A comparison with an FP32 implementation sets such
pixels aside and checks them against the looser bound stake x colour range.

Closed forms: a single Gaussian whose 3-sigma ellipse or 1/255 contour passes
through the pixel centre (stake = its alpha, T = 1); a stack whose
transmittance reaches 1e-4 within the stop margin (stake = the transmittance
before the stop candidate); the cascade in which a cut entry in front widens
the stop window by its own alpha; and a pixel far from every threshold.
"""
import numpy as np
import pytest

import gv_synth
import oracle

TOL = [2e-5, 1e-4, 2e-3]
ID = [1, 0, 0, 0, 0, 0, 0]


def logit(p):
    return float(np.log(p / (1 - p)))


def one_iso(cam, z, var, o):
    """One isotropic Gaussian on the optical axis whose projected variance is
    `var` px^2 (dilation included)."""
    s = np.sqrt(var - cam.dilation) * z / cam.fx
    scene = dict(means=np.array([[0.0], [0.0], [z]]), log_scales=np.full((3, 1), np.log(s)),
                 quats=np.array([[1.0], [0], [0], [0]]), opacity_logits=np.array([logit(o)]),
                 colors=np.array([[0.9], [0.5], [0.1]]), mean_coeffs=None)
    return scene


def test_far_from_thresholds_has_zero_stake():
    rng = np.random.default_rng(0)
    cam = gv_synth.make_camera(48, 40, 48.0)
    scene = gv_synth.make_scene(rng, 200, z=(2.0, 6.0), log_scale=(-3.0, 0.3))
    r = oracle.render_frame(scene, cam, ID, stake_tol=TOL)
    m = r["margins"]
    clear = (m[:, 0] >= TOL[0]) & (m[:, 1] >= TOL[1]) & (m[:, 2] >= 3 * TOL[2])
    assert clear.sum() > 0.9 * len(clear)
    assert np.all(r["stake"][clear] == 0.0)
    assert np.all(r["stake"] >= 0.0) and np.all(r["stake"] <= 1.0 + 1e-12)


@pytest.mark.parametrize("delta", [1e-6, -1e-6, 1e-3])
def test_three_sigma_cut(delta):
    """Pixel centre at q = 9 (1 + delta) from one Gaussian: inside or just
    outside the cut, its weight o exp(-q/2) is at stake; far off, nothing."""
    cam = gv_synth.make_camera(41, 41, 41.0)   # centre pixel 20 has its centre on the axis
    r_px = 4.0                                 # the pixel 4 to the right
    q = 9.0 * (1.0 + delta)
    var = r_px * r_px / q
    o = 0.9
    scene = one_iso(cam, 3.0, var, o)
    pix = 20 * 41 + 24
    r = oracle.render_frame(scene, cam, ID, pixels=[pix], stake_tol=TOL)
    assert r["margins"][0, 0] == pytest.approx(abs(delta), rel=1e-6)
    expect = o * np.exp(-q / 2) if abs(delta) < TOL[0] else 0.0
    assert r["stake"][0] == pytest.approx(expect, rel=1e-9, abs=1e-15)
    # the pixel itself: blended only inside the cut
    assert r["n_contrib"][0] == (1 if delta < 0 else 0)


@pytest.mark.parametrize("delta", [5e-5, -5e-5])
def test_alpha_cut(delta):
    """alpha = (1/255)(1 + delta) at the pixel: alpha (with T = 1) at stake."""
    cam = gv_synth.make_camera(41, 41, 41.0)
    o = 0.05
    q = 2.0 * np.log(255.0 * o / (1.0 + delta))
    r_px = 3.0
    scene = one_iso(cam, 3.0, r_px * r_px / q, o)
    r = oracle.render_frame(scene, cam, ID, pixels=[20 * 41 + 23], stake_tol=TOL)
    assert r["margins"][0, 1] == pytest.approx(abs(delta), rel=1e-6)
    assert r["stake"][0] == pytest.approx((1.0 + delta) / 255.0, rel=1e-9)
    assert r["n_contrib"][0] == (1 if delta > 0 else 0)


def stacked(cam, px, py, alphas, colors=None):
    n = len(alphas)
    zs = 2.0 + 0.5 * np.arange(n)
    means = np.array([[(px + 0.5 - cam.cx) * z / cam.fx, (py + 0.5 - cam.cy) * z / cam.fy, z] for z in zs]).T
    cols = np.tile([[0.2], [0.5], [0.9]], n) if colors is None else colors
    return dict(means=means, log_scales=np.full((3, n), -3.0), quats=np.tile([[1.0], [0], [0], [0]], n),
                opacity_logits=np.array([logit(a) for a in alphas]), colors=cols, mean_coeffs=None)


def test_stop_within_margin_puts_remaining_transmittance_at_stake():
    """Three alpha = a entries at the pixel centre with (1-a)^3 = 1e-4 (1 + 1e-5):
    the third is blended with its stop decision 1e-5 from the threshold, so
    the transmittance before it, (1-a)^2, is at stake; a fourth entry (well
    below 1e-4) stops the pixel."""
    cam = gv_synth.make_camera(32, 32, 32.0)
    a = 1.0 - (1e-4 * (1.0 + 1e-5)) ** (1.0 / 3.0)
    r = oracle.render_frame(stacked(cam, 16, 16, [a] * 4), cam, ID, pixels=[16 * 32 + 16], stake_tol=TOL)
    assert r["n_contrib"][0] == 3
    assert r["margins"][0, 2] == pytest.approx(1e-5, rel=1e-4)
    assert r["stake"][0] == pytest.approx((1.0 - a) ** 2, rel=1e-9)


def test_cut_entry_in_front_widens_the_stop_window():
    """A first entry exactly at the 3-sigma cut (weight w = o e^-4.5) changes
    every later transmittance by up to a factor 1 - w, so a stop decision
    5e-3 from its threshold (outside the plain 2e-3 margin but inside
    2e-3 + w) also counts: stake = w + T before the stop candidate."""
    cam = gv_synth.make_camera(41, 41, 41.0)
    # entry 0: large isotropic Gaussian with the pixel exactly on its q = 9 contour
    r_px = 4.0
    q0 = 9.0 * (1.0 - 1e-7)
    var0 = r_px * r_px / q0
    z0 = 1.5
    s0 = np.sqrt(var0 - cam.dilation) * z0 / cam.fx
    w = 0.999 * np.exp(-q0 / 2)
    # entries 1..3 stacked on the pixel centre (24, 20), deeper
    a = 1.0 - (1e-4 * (1.0 + 5e-3) / (1.0 - w)) ** (1.0 / 3.0)
    st = stacked(cam, 24, 20, [a] * 3)
    scene = dict(means=np.concatenate([[[0.0], [0.0], [z0]], st["means"]], axis=1),
                 log_scales=np.concatenate([np.full((3, 1), np.log(s0)), st["log_scales"]], axis=1),
                 quats=np.concatenate([[[1.0], [0], [0], [0]], st["quats"]], axis=1),
                 opacity_logits=np.concatenate([[logit(0.999)], st["opacity_logits"]]),
                 colors=np.concatenate([[[0.1], [0.1], [0.1]], st["colors"]], axis=1), mean_coeffs=None)
    r = oracle.render_frame(scene, cam, ID, pixels=[20 * 41 + 24], stake_tol=TOL)
    assert r["n_contrib"][0] == 4
    assert r["margins"][0, 2] == pytest.approx(5e-3, rel=1e-3)
    T_before_last = (1.0 - w) * (1.0 - a) ** 2
    assert r["stake"][0] == pytest.approx(w + T_before_last, rel=1e-6)
    # without the cut entry the same stop margin is outside the window
    r2 = oracle.render_frame(st, cam, ID, pixels=[20 * 41 + 24], stake_tol=TOL)
    assert r2["stake"][0] == 0.0
