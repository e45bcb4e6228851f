"""Pins of the oracle's compositing stage (step 6 of the forward model).

Closed forms (one and two Gaussians, the four-stacked termination example in
tests/golden), the thresholds of the 3DGS compositing rule, and invariants of
image formation: partition of unity of the blending weights, zero opacity,
colour linearity, rigid-motion equivariance, mirror symmetry and invariance
to the storage order of the Gaussians.
"""
import json
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import gv_synth
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ID = [1, 0, 0, 0, 0, 0, 0]


def scene_of(means, log_scales, quats, etas, colors):
    return dict(means=np.array(means, float).reshape(3, -1), log_scales=np.array(log_scales, float).reshape(3, -1),
                quats=np.array(quats, float).reshape(4, -1), opacity_logits=np.array(etas, float).ravel(),
                colors=np.array(colors, float).reshape(3, -1), mean_coeffs=None)


def logit(p):
    return float(np.log(p / (1 - p)))


def at_pixel_centre(px, py, z, cam):
    """World point (identity camera) that projects exactly onto a pixel centre."""
    return [(px + 0.5 - cam.cx) * z / cam.fx, (py + 0.5 - cam.cy) * z / cam.fy, z]


def rand_scene(rng, n, z=(2, 6)):
    mu = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(z[0], z[1], n)])
    return dict(means=mu, log_scales=rng.normal(-2.6, 0.4, (3, n)), quats=rng.normal(0, 1, (4, n)),
                opacity_logits=rng.normal(0.5, 1, n), colors=rng.uniform(0, 1, (3, n)), mean_coeffs=None)


def test_golden_termination_four_stacked():
    g = json.load(open(os.path.join(GOLDEN, "termination_four_stacked.json")))
    cam = gv_synth.make_camera(g["width"], g["height"], g["focal"], bg=tuple(g["bg"]))
    px, py = g["pixel"]
    means = np.array([at_pixel_centre(px, py, z, cam) for z in g["depths"]]).T
    n = len(g["depths"])
    s = scene_of(means, np.full((3, n), -3.0), np.tile([[1.0], [0], [0], [0]], n), [logit(g["opacity"])] * n,
                 np.tile(np.array(g["color"])[:, None], n))
    r = oracle.render_frame(s, cam, ID, pixels=[py * g["width"] + px])
    np.testing.assert_allclose(r["color"][0], g["expected_color"], rtol=0, atol=1e-12)
    assert r["T_final"][0] == pytest.approx(g["expected_T_final"], rel=1e-9)
    assert r["n_contrib"][0] == g["expected_n_contrib"]


def test_three_stacked_distinct_colours_closed_form():
    cam = gv_synth.make_camera(32, 32, 32.0, bg=(0.3, 0.6, 0.9))
    zs = [2.0, 3.0, 4.0]
    a = 0.6
    cols = np.array([[0.9, 0.1, 0.2], [0.2, 0.8, 0.3], [0.1, 0.3, 0.7]]).T  # [3][n]
    means = np.array([at_pixel_centre(10, 20, z, cam) for z in zs]).T
    # store them far-to-near so the depth sort has work to do
    s = scene_of(means[:, ::-1], np.full((3, 3), -3.0), np.tile([[1.0], [0], [0], [0]], 3), [logit(a)] * 3,
                 cols[:, ::-1])
    r = oracle.render_frame(s, cam, ID, pixels=[20 * 32 + 10])
    bg = np.array(cam.bg)
    expect = cols[:, 0] * a + cols[:, 1] * a * (1 - a) + cols[:, 2] * a * (1 - a) ** 2 + bg * (1 - a) ** 3
    np.testing.assert_allclose(r["color"][0], expect, atol=1e-12)
    assert r["T_final"][0] == pytest.approx((1 - a) ** 3, rel=1e-12)


def test_single_isotropic_gaussian_whole_image_closed_form():
    """C(p) = alpha(p) c + (1 - alpha(p)) bg with alpha = o exp(-|p-(u,v)|^2 / (2 var)),
    var = (f s / z)^2 + dilation, where q <= 9 and alpha >= 1/255; bg elsewhere."""
    cam = gv_synth.make_camera(40, 30, 40.0, bg=(0.05, 0.1, 0.2))
    z, sc, o = 3.0, 0.2, 0.8
    c = np.array([0.7, 0.4, 0.2])
    # on the optical axis, so that the projected covariance is isotropic
    s = scene_of([0.0, 0.0, z], [np.log(sc)] * 3, [0.3, 0.1, 0.5, -0.2], [logit(o)], c)
    img = oracle.render_image(s, cam, ID)["image"]
    u, v = cam.cx, cam.cy
    var = (40.0 * sc / z) ** 2 + cam.dilation
    ys, xs = np.mgrid[0:30, 0:40]
    q = ((xs + 0.5 - u) ** 2 + (ys + 0.5 - v) ** 2) / var
    alpha = np.minimum(0.99, o * np.exp(-0.5 * q))
    use = (q <= 9) & (alpha >= 1 / 255)
    bg = np.array(cam.bg)[:, None, None]
    expect = np.where(use[None], alpha[None] * c[:, None, None] + (1 - alpha[None]) * bg, bg)
    np.testing.assert_allclose(img, expect, atol=1e-12)


def test_alpha_clamp_and_thresholds():
    cam = gv_synth.make_camera(16, 16, 16.0, bg=(0.5, 0.5, 0.5))
    pix = [8 * 16 + 8]
    mu = at_pixel_centre(8, 8, 2.0, cam)
    c = [1.0, 0.0, 0.25]
    # clamp: opacity ~ 1 gives alpha = 0.99
    r = oracle.render_frame(scene_of(mu, [-3] * 3, [1, 0, 0, 0], [40.0], c), cam, ID, pixels=pix)
    np.testing.assert_allclose(r["color"][0], 0.99 * np.array(c) + 0.01 * 0.5, atol=1e-12)
    # alpha just below / above 1/255 at the centre
    for o, used in [(1 / 255 * (1 - 1e-6), False), (1 / 255 * (1 + 1e-6), True)]:
        r = oracle.render_frame(scene_of(mu, [-3] * 3, [1, 0, 0, 0], [logit(o)], c), cam, ID, pixels=pix)
        expect = (o * np.array(c) + (1 - o) * 0.5) if used else np.full(3, 0.5)
        np.testing.assert_allclose(r["color"][0], expect, atol=1e-12)
        assert r["n_contrib"][0] == int(used)


def test_three_sigma_cutoff():
    """A pixel just outside q = 9 gets nothing, just inside gets o e^{-q/2}.
    The Gaussian sits on the optical axis (isotropic footprint) and its scale
    is chosen so that the pixel centre (40.5, 32.5) lies at q = 9 (1 +- 1e-7)."""
    cam = gv_synth.make_camera(64, 64, 64.0)
    z, o = 4.0, 0.9
    r2 = (40.5 - cam.cx) ** 2 + (32.5 - cam.cy) ** 2
    for eps, used in [(1e-7, False), (-1e-7, True)]:
        var = r2 / (9.0 * (1 + eps))
        sc = np.sqrt(var - cam.dilation) * z / 64.0
        s = scene_of([0.0, 0.0, z], [np.log(sc)] * 3, [1, 0, 0, 0], [logit(o)], [1, 1, 1])
        r = oracle.render_frame(s, cam, ID, pixels=[32 * 64 + 40])
        if used:
            np.testing.assert_allclose(r["color"][0], o * np.exp(-0.5 * 9 * (1 - 1e-7)), rtol=1e-6)
        else:
            assert np.all(r["color"][0] == 0.0)


def test_zero_opacity_gives_background_exactly():
    rng = np.random.default_rng(7)
    s, cam = gv_synth.adversarial_scene(rng, 200, "zero_opacity")
    cam.bg = (0.25, 0.5, 0.75)
    img = oracle.render_image(s, cam, ID)["image"]
    assert np.all(img == np.array(cam.bg)[:, None, None])


def test_blend_weights_partition_of_unity_and_T_bounds():
    """sum_i alpha_i T_i + T_final = 1: white Gaussians on a white background
    give exactly white; black Gaussians on white give T_final; T_final lies in
    [1e-4, 1] even for a very dense stack."""
    rng = np.random.default_rng(8)
    s, cam = gv_synth.adversarial_scene(rng, 400, "dense")
    d = oracle.scene_f64(s)
    cam.bg = (1.0, 1.0, 1.0)
    d["colors"][:] = 1.0
    r = oracle.render_image(d, cam, ID)
    np.testing.assert_allclose(r["image"], 1.0, atol=1e-12)
    assert r["T_final"].min() >= 1e-4 and r["T_final"].max() <= 1.0
    assert (r["T_final"] < 2e-4).any()  # the stop rule is exercised
    d["colors"][:] = 0.0
    r2 = oracle.render_image(d, cam, ID)
    np.testing.assert_allclose(r2["image"], np.broadcast_to(r2["T_final"], (3,) + r2["T_final"].shape), atol=1e-15)


def test_colour_linearity():
    rng = np.random.default_rng(9)
    cam = gv_synth.make_camera(32, 24, 32.0)
    s = rand_scene(rng, 60)
    c1, c2 = rng.uniform(0, 1, (3, 60)), rng.uniform(0, 1, (3, 60))
    def img(c):
        d = dict(s); d["colors"] = c
        return oracle.render_image(d, cam, ID)["image"]
    np.testing.assert_allclose(img(0.3 * c1 + 1.7 * c2), 0.3 * img(c1) + 1.7 * img(c2), atol=1e-12)


def _stable(r, tol=1e-6):
    return (r["margins"].reshape(-1, 4)[:, :3] > tol).all(axis=1)


def test_rigid_motion_equivariance():
    """Moving the scene by a rigid motion and the camera with it leaves the
    image unchanged."""
    rng = np.random.default_rng(10)
    cam = gv_synth.make_camera(48, 32, 48.0)
    s = rand_scene(rng, 80)
    pose = np.array([0.98, 0.05, -0.1, 0.07, 0.1, -0.2, 0.3])
    Q = Rotation.from_rotvec([0.3, -0.5, 0.8])
    dvec = np.array([0.4, -1.2, 2.0])
    s2 = dict(s)
    s2["means"] = Q.as_matrix() @ s["means"] + dvec[:, None]
    qs = s["quats"]
    R = Rotation.from_quat(np.stack([qs[1], qs[2], qs[3], qs[0]], axis=1))
    q2 = (Q * R).as_quat()  # x y z w
    s2["quats"] = np.stack([q2[:, 3], q2[:, 0], q2[:, 1], q2[:, 2]])
    Rc = Rotation.from_quat([pose[1], pose[2], pose[3], pose[0]])
    Rc2 = Rc * Q.inv()
    qc2 = Rc2.as_quat()
    tc2 = pose[4:] - Rc2.as_matrix() @ dvec
    pose2 = np.array([qc2[3], qc2[0], qc2[1], qc2[2], *tc2])
    a = oracle.render_frame(s, cam, pose)
    b = oracle.render_frame(s2, cam, pose2)
    ok = _stable(a)
    assert ok.mean() > 0.99
    np.testing.assert_allclose(a["color"][ok], b["color"][ok], atol=1e-9)


def test_mirror_symmetry():
    """Reflecting the scene through the plane x = 0 mirrors the image about
    the principal point's column (cx = W/2)."""
    rng = np.random.default_rng(11)
    cam = gv_synth.make_camera(40, 30, 40.0)
    s = rand_scene(rng, 70)
    s2 = dict(s)
    s2["means"] = s["means"] * np.array([[-1.0], [1.0], [1.0]])
    s2["quats"] = s["quats"] * np.array([[1.0], [1.0], [-1.0], [-1.0]])
    a = oracle.render_image(s, cam, ID)
    b = oracle.render_image(s2, cam, ID)
    ok = (a["margins"][..., :3] > 1e-6).all(-1) & (b["margins"][..., :3] > 1e-6).all(-1)[:, ::-1]
    np.testing.assert_allclose(a["image"][:, ok], b["image"][:, :, ::-1][:, ok], atol=1e-10)


def test_storage_order_invariance_bitwise():
    rng = np.random.default_rng(12)
    cam = gv_synth.make_camera(32, 32, 32.0)
    s = rand_scene(rng, 90)
    perm = rng.permutation(90)
    s2 = {k: (None if v is None else v[..., perm]) for k, v in s.items()}
    a = oracle.render_image(s, cam, ID)["image"]
    b = oracle.render_image(s2, cam, ID)["image"]
    assert np.array_equal(a, b)


def test_depth_ties_resolved_by_index():
    """Equal depth keys: the lower Gaussian index is composited first."""
    cam = gv_synth.make_camera(16, 16, 16.0)
    mu = at_pixel_centre(5, 5, 3.0, cam)
    means = np.array([mu, mu]).T
    s = scene_of(means, np.full((3, 2), -3.0), np.tile([[1.0], [0], [0], [0]], 2), [logit(0.5)] * 2,
                 [[1.0, 0.0], [0.0, 1.0], [0.0, 0.0]])
    r = oracle.render_frame(s, cam, ID, pixels=[5 * 16 + 5])
    np.testing.assert_allclose(r["color"][0], [0.5, 0.25, 0.0], atol=1e-12)


def test_pixel_subset_matches_full_render():
    rng = np.random.default_rng(13)
    cam = gv_synth.make_camera(24, 20, 24.0)
    s = rand_scene(rng, 50)
    full = oracle.render_frame(s, cam, ID)
    pix = rng.choice(24 * 20, 37, replace=False)
    sub = oracle.render_frame(s, cam, ID, pixels=pix)
    assert np.array_equal(sub["color"], full["color"][pix])
    assert np.array_equal(sub["T_final"], full["T_final"][pix])
