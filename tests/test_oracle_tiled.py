"""The oracle's tiled form against its per-pixel definition (an exact
acceleration, the binning being conservative): with each pixel visiting only
the Gaussians whose footprint box meets its tile, colours, final
transmittances, contributor counts, stakes and gradients are identical bit
for bit, and decision margins are identical
wherever they are below 1e-3 (the only ones a comparison uses).  Tile sizes
16, 8, 7 and 1, a tile larger than the image, ragged image sizes, adversarial
scenes, dynamics and SH colour."""
import numpy as np
import pytest

import gv_synth
import oracle

TOL = [2e-5, 1e-4, 2e-4]


def both(w, tile, pose=None, t=0.0, grads=False, seed=0):
    cam = w["camera"]
    pose = w["poses"][0].astype(np.float64) if pose is None else pose
    dl = None
    if grads:
        dl = np.random.default_rng(seed).normal(0, 1, (cam.width * cam.height, 3))
    a = oracle.render_frame(w["scene"], cam, pose, t, dL_dC=dl, stake_tol=TOL, threads=4)
    b = oracle.render_frame(w["scene"], cam, pose, t, dL_dC=dl, stake_tol=TOL, threads=4, tile=tile)
    return a, b


def assert_same(a, b):
    for k in ("color", "T_final", "n_contrib", "stake"):
        assert np.array_equal(a[k], b[k]), k
    low = a["margins"] < 1e-3
    assert np.array_equal(a["margins"][low], b["margins"][low])
    assert np.all(b["margins"][~low] >= 1e-3)
    if "grads" in a:
        for k, v in a["grads"].items():
            if v is not None:
                assert np.array_equal(v, b["grads"][k]), k


@pytest.mark.parametrize("tile", [16, 8, 7, 1, 200])
def test_frame128_all_tile_sizes(tile):
    w = gv_synth.make_workload("frame128_n2k")
    pose = np.array([0.995, 0.05, -0.06, 0.04, 0.05, -0.08, 0.2])
    a, b = both(w, tile, pose=pose, grads=tile in (16, 7))
    assert_same(a, b)
    assert a["n_contrib"].sum() > 10_000


@pytest.mark.parametrize("kind", ["huge", "offscreen", "near", "ties", "zero_opacity", "dense", "elongated"])
def test_adversarial_scenes(kind):
    rng = np.random.default_rng(200)
    scene, cam = gv_synth.adversarial_scene(rng, 300, kind, width=45, height=37)
    cam.bg = (0.1, 0.2, 0.3)
    w = dict(scene=scene, camera=cam, poses=gv_synth.identity_poses(1))
    a, b = both(w, 16, grads=True, seed=1)
    assert_same(a, b)


def test_moving_camera_ragged_bf16_cubic():
    rng = np.random.default_rng(201)
    scene = gv_synth.make_scene(rng, 1500, z=(2.0, 10.0), log_scale=(-3.0, 0.5), dtype="bf16", cubic=True)
    cam = gv_synth.make_camera(83, 61, 83.0, bg=(0.2, 0.1, 0.0))
    poses = gv_synth.make_trajectory(rng, 3)
    w = dict(scene=scene, camera=cam, poses=poses[2:])
    a, b = both(w, 16, t=0.7, grads=True, seed=2)
    assert_same(a, b)


def test_dynamics_and_sh():
    rng = np.random.default_rng(202)
    scene = gv_synth.make_scene(rng, 800, z=(2.0, 6.0), log_scale=(-3.0, 0.3), n_ctrl=6, poly_cov=True,
                                sh_degree=2)
    cam = gv_synth.make_camera(64, 48, 64.0)
    w = dict(scene=scene, camera=cam, poses=gv_synth.make_trajectory(rng, 2)[1:])
    a, b = both(w, 16, t=0.4, grads=True, seed=3)
    assert_same(a, b)
