"""GPU parity of the visibility counts and the Gaussian pyramid, through the
C ABI, against the FP64 oracle."""
import numpy as np
import pytest
import torch

import gv_synth
import oracle
from oracle import pyramid as pyr_ref
from parity_util import device_inputs, workspace_for
from test_gpu_parity import say, small_workload

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2501_04782_amd import raster


def marginal(scene, cam, pose, t, g):
    """True if the oracle's contribution decision for Gaussian g flips under a
    1e-4 change of its opacity logit (a decision within rounding of a
    threshold, which FP32 and FP64 may take differently)."""
    flags = []
    for d in (-1e-4, 1e-4):
        s = oracle.scene_f64(scene)
        s["opacity_logits"] = s["opacity_logits"].copy()
        s["opacity_logits"][g] += d
        flags.append(bool(oracle.contributors(s, cam, pose, t)[g]))
    return flags[0] != flags[1]


@pytest.mark.parametrize("kind,compact", [("clip", 0), ("dense", 0), ("clip", 4)])
def test_visibility_counts_match_oracle(kind, compact):
    """compact 0: the 4x4-block forward flags contributors; 4: the quadrant forward."""
    old = raster.get_tuning()
    raster.set_tuning(old["batch"], old["sort_cap"], compact, old["bwd_batch"])
    try:
        check_visibility(kind)
    finally:
        raster.set_tuning(old["batch"], old["sort_cap"], old["compact"], old["bwd_batch"])


def check_visibility(kind):
    if kind == "clip":
        w = small_workload(80, 128, 96, 3000, 4, trajectory=True, z=(2.0, 10.0), ls=(-3.2, 0.5))
        w["scene"].means[0, :40] += 30.0  # some Gaussians never on screen
    else:
        rng = np.random.default_rng(81)
        scene, cam = gv_synth.adversarial_scene(rng, 400, "dense")
        w = dict(scene=scene, camera=cam, poses=gv_synth.identity_poses(2), times=gv_synth.make_times(2), frames=2,
                 n=400)
    scene, cam, poses, times = device_inputs(w)
    ws = workspace_for(scene, cam, poses, times)
    counts = raster.visibility_counts(scene, cam, poses, times, ws).cpu().numpy()
    assert ws.status()["overflow"] == 0
    per_frame = [oracle.contributors(w["scene"], w["camera"], w["poses"][f].astype(np.float64), float(w["times"][f]))
                 for f in range(w["frames"])]
    ref = np.sum(per_frame, axis=0)
    bad = np.nonzero(counts != ref)[0]
    say(f"visibility {kind}: {len(bad)} of {w['n']} differ; zero-count {int((ref == 0).sum())}")
    assert len(bad) <= max(1, w["n"] // 1000)
    for g in bad:  # only decisions at a threshold may differ
        assert any(marginal(w["scene"], w["camera"], w["poses"][f].astype(np.float64), float(w["times"][f]), g)
                   for f in range(w["frames"])), g
    if kind == "clip":
        assert np.all(ref[:40] == 0) and np.all(counts[:40] == 0)


@pytest.mark.parametrize("H,W,levels", [(540, 960, 5), (33, 17, 4), (1, 9, 3), (64, 64, 7)])
def test_gaussian_pyramid_matches_oracle(H, W, levels):
    rng = np.random.default_rng(H + W)
    img = rng.random((2, 3, H, W)).astype(np.float32)
    got = raster.gaussian_pyramid(torch.from_numpy(img).cuda(), levels)
    torch.cuda.synchronize()
    if H * W > 100000:  # full size: level 1 at sampled output pixels (borders included)
        assert [tuple(g.shape[-2:]) for g in got] == [(540, 960), (270, 480), (135, 240), (68, 120), (34, 60)]
        lvl1 = got[1].cpu().numpy()
        pts = [(0, 0), (0, 479), (269, 0), (269, 479), (1, 1)] + [tuple(p) for p in
                                                                  rng.integers(0, [270, 480], (300, 2))]
        src = img.astype(np.float64)
        for y, x in pts:
            np.testing.assert_allclose(lvl1[..., y, x], pyr_ref.reduce_at(src, y, x), rtol=0, atol=2e-6)
        return
    ref = pyr_ref.pyramid(img.astype(np.float64), levels)
    for lvl, (a, b) in enumerate(zip(got, ref)):
        assert a.shape == b.shape, lvl
        np.testing.assert_allclose(a.cpu().numpy(), b, rtol=0, atol=1e-6 * (lvl + 1), err_msg=str(lvl))
