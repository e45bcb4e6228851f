"""GPU parity of the Eq. 2-3 dynamics (B-spline means, cubic log-scales and
quaternions) against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import gv_synth
import oracle
from parity_util import (GRAD_TOL, colour_range, compare_grads, compare_image, compare_poses, device_inputs,
                         knife_edge, oracle_frame, planar_to_pixels, rel_err, workspace_for)
from test_gpu_parity import check_clip_against_oracle, run_clip, say, upstream_for

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2501_04782_amd import raster


def dyn_workload(seed, W, H, n, F, n_ctrl=6, poly_cov=True, times=None, ctrl_std=0.08, coeff_std=0.2):
    rng = np.random.default_rng(seed)
    scene = gv_synth.make_scene(rng, n, z=(2.0, 10.0), log_scale=(-3.2, 0.5), n_ctrl=n_ctrl, poly_cov=poly_cov,
                                ctrl_std=ctrl_std, coeff_std=coeff_std)
    cam = gv_synth.make_camera(W, H, float(W), bg=(0.1, 0.2, 0.3))
    poses = gv_synth.make_trajectory(rng, F)
    t = gv_synth.make_times(F) if times is None else np.asarray(times, np.float32)
    return dict(scene=scene, camera=cam, poses=poses, times=t, frames=F, n=n)


def test_dynamic_projection_depth_keys_bit_exact():
    """The FP64 span-restricted Cox-de Boor gives the oracle's basis values bit
    for bit, so the depth keys (fp32 rounding of the FP64 depth) agree exactly."""
    w = dyn_workload(40, 128, 96, 3000, 1, n_ctrl=7)
    pose = w["poses"][0]
    scene, cam, _, _ = device_inputs(w)
    ws = raster.Workspace(cam, scene.n, 1, 0)
    for t in (0.0, 0.25, 0.37, 0.75, 1.0):
        t = float(np.float32(t))  # the C ABI takes the frame time as a float: give the oracle the same value
        rec, cnt = raster.project_fwd(scene, cam, torch.from_numpy(pose).cuda(), t, ws)
        rec, cnt = rec.cpu().numpy(), cnt.cpu().numpy()
        ref = oracle.project(w["scene"], w["camera"], pose.astype(np.float64), t)
        vis = cnt > 0
        assert vis.sum() > 1000
        assert np.all(ref["valid"][vis] == 1)
        np.testing.assert_allclose(rec[vis, 0], ref["u"][vis], rtol=1e-6, atol=1e-4)
        np.testing.assert_allclose(rec[vis, 2], ref["A00"][vis], rtol=1e-6, atol=1e-7)
        assert np.array_equal(rec[vis, 5].astype(np.float32), ref["key"][vis].astype(np.float32)), t


@pytest.mark.parametrize("n_ctrl,poly_cov", [(6, True), (4, False), (9, True)])
def test_dynamic_clip_matches_oracle(n_ctrl, poly_cov):
    """Batched fwd+bwd over frames in several knot spans (the control-point
    gradient window is flushed between spans)."""
    w = dyn_workload(41 + n_ctrl, 160, 96, 3000, 5, n_ctrl=n_ctrl, poly_cov=poly_cov)
    check_clip_against_oracle(w, f"dynamic clip M={n_ctrl} poly={poly_cov}")


def test_dynamic_unsorted_times_and_accumulate():
    """Frame times out of order (the window moves back and forth) and
    GV_ACCUMULATE (a second call adds the same gradients)."""
    w = dyn_workload(50, 128, 80, 2000, 4, n_ctrl=7, times=[0.9, 0.05, 0.55, 0.3])
    out = check_clip_against_oracle(w, "dynamic unsorted times")
    refs = [oracle_frame(w, f) for f in range(w["frames"])]
    dl = upstream_for(w, refs, 0)
    scene, cam, poses, times = device_inputs(w)
    ws = workspace_for(scene, cam, poses, times)
    g1 = raster.render_batch(scene, cam, poses, times, ws, dL_dimages=torch.from_numpy(dl).cuda())["grads"]
    g2 = {k: (None if v is None else v.clone()) for k, v in g1.items()}
    raster.render_batch(scene, cam, poses, times, ws, dL_dimages=torch.from_numpy(dl).cuda(), grads=g2,
                        accumulate=True)
    torch.cuda.synchronize()
    for k in ("ctrl", "scale_coeffs", "quat_coeffs", "log_scales", "colors"):
        e = rel_err(g2[k].cpu().numpy(), 2.0 * g1[k].cpu().numpy())
        assert e < 1e-6, (k, e)
    assert torch.all(g1["means"] == 0)  # not written with control points


def test_dynamic_per_frame_path():
    w = dyn_workload(52, 96, 64, 1500, 1, n_ctrl=5, times=[0.62])
    ref = oracle_frame(w, 0)
    scene, cam, poses, times = device_inputs(w)
    ws = workspace_for(scene, cam, poses, times)
    img = raster.render_fwd(scene, cam, poses[0].contiguous(), 0.62, ws)
    torch.cuda.synchronize()
    compare_image(img.cpu().numpy(), ref, "dynamic per-frame fwd", colour_range(w))
    dl = upstream_for(w, [ref], 3)[0]
    g, dpose = raster.render_bwd(scene, cam, poses[0].contiguous(), 0.62, ws, img,
                                 dL_dimage=torch.from_numpy(dl).cuda())
    torch.cuda.synchronize()
    gref = oracle_frame(w, 0, dL_dC=planar_to_pixels(dl))["grads"]
    ge = compare_grads(g, gref, "dynamic per-frame bwd")
    pe = compare_poses(dpose, gref["pose"], "dynamic per-frame bwd")
    say(f"dynamic per-frame: grads {ge} pose {pe:.2e}")


def test_spline_time_outside_domain_drops_gaussians():
    w = dyn_workload(53, 48, 32, 300, 2, n_ctrl=5, times=[1.5, -0.25])
    scene, cam, poses, times = device_inputs(w)
    ws = raster.Workspace(cam, scene.n, 2, 4096)
    out = raster.render_batch(scene, cam, poses, times, ws, dL_dimages=torch.ones(2, 3, 32, 48, device="cuda"))
    torch.cuda.synchronize()
    bg = torch.tensor([0.1, 0.2, 0.3], device="cuda")[:, None, None]
    assert torch.allclose(out["images"], bg.expand(2, 3, 32, 48).contiguous())
    for k in ("ctrl", "scale_coeffs", "quat_coeffs", "colors"):
        assert torch.all(out["grads"][k] == 0), k
    for f in range(2):  # the oracle drops them too
        ref = oracle_frame(w, f)
        assert np.allclose(ref["color"], [0.1, 0.2, 0.3])
