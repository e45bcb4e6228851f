"""Pins of the visibility counts (Gaussians that appear in a frame, Sec. 4.1)
and of the Gaussian-pyramid targets (Sec. 3.3)."""
import numpy as np
import pytest
from scipy.ndimage import convolve1d

import gv_synth
import oracle
from oracle import pyramid


def test_contributors_equal_positive_colour_gradient():
    """With an all-ones upstream gradient, dL/dc_g = sum over pixels of
    alpha T: positive exactly for the Gaussians that contribute somewhere."""
    for kind, seed in (("dense", 1), ("offscreen", 2), ("zero_opacity", 3), ("huge", 4)):
        rng = np.random.default_rng(seed)
        scene, cam = gv_synth.adversarial_scene(rng, 200, kind)
        pose = [1, 0, 0, 0, 0, 0, 0]
        flags = oracle.contributors(scene, cam, pose)
        g = oracle.render_frame(scene, cam, pose, dL_dC=np.ones((cam.width * cam.height, 3)))["grads"]
        np.testing.assert_array_equal(flags, g["colors"][0] > 0, err_msg=kind)
        if kind == "zero_opacity":
            assert not flags.any()
        if kind == "dense":  # early termination hides Gaussians whose footprints are on screen
            p = oracle.project(scene, cam, pose)
            assert (p["valid"] > 0).sum() > flags.sum()


def test_visibility_counts_sum_frames():
    w = gv_synth.make_workload("frame128_n2k", n=400)
    w["scene"].means[0, 7] = 50.0  # far outside the frustum in every frame
    cam = w["camera"]
    rng = np.random.default_rng(5)
    poses = gv_synth.make_trajectory(rng, 3)
    counts = oracle.visibility_counts(w["scene"], cam, poses, [0.0, 0.5, 1.0])
    ref = sum(oracle.contributors(w["scene"], cam, poses[f]).astype(int) for f in range(3))
    np.testing.assert_array_equal(counts, ref)
    assert counts.max() == 3 and counts[7] == 0


@pytest.mark.parametrize("H,W", [(17, 32), (40, 29), (1, 7), (5, 1), (64, 64)])
def test_reduce_matches_scipy_mirror_convolution(H, W):
    rng = np.random.default_rng(H * 100 + W)
    img = rng.random((2, 3, H, W))
    k = pyramid.KERNEL
    ref = convolve1d(convolve1d(img, k, axis=-1, mode="mirror"), k, axis=-2, mode="mirror")[..., ::2, ::2]
    got = pyramid.reduce_level(img)
    assert got.shape == img.shape[:-2] + ((H + 1) // 2, (W + 1) // 2)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)


def test_constant_and_linear_images():
    c = np.full((3, 20, 26), 0.37)
    for lvl in pyramid.pyramid(c, 4):
        np.testing.assert_allclose(lvl, 0.37, atol=1e-15)
    # the binomial filter reproduces linear functions away from the border
    y, x = np.mgrid[0:24, 0:30]
    ramp = 0.01 * x + 0.02 * y
    out = pyramid.reduce_level(ramp)
    yy, xx = np.mgrid[0:12, 0:15]
    np.testing.assert_allclose(out[1:-1, 1:-1], (0.01 * 2 * xx + 0.02 * 2 * yy)[1:-1, 1:-1], atol=1e-14)
