"""GPU parity of the view-dependent (spherical-harmonics) colour against the
FP64 oracle, through the C ABI: colour, its coefficient gradients, and the
view-direction terms of the mean and pose gradients."""
import numpy as np
import pytest
import torch

import gv_synth
from parity_util import (GRAD_TOL, colour_range, compare_grads, compare_image, compare_poses, device_inputs,
                         oracle_frame, planar_to_pixels, rel_err, workspace_for)
from test_gpu_parity import check_clip_against_oracle, say, upstream_for

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2501_04782_amd import raster


def sh_workload(seed, W, H, n, F, degree, n_ctrl=0, sh_std=0.25):
    rng = np.random.default_rng(seed)
    scene = gv_synth.make_scene(rng, n, z=(2.0, 10.0), log_scale=(-3.2, 0.5), sh_degree=degree, sh_std=sh_std,
                                n_ctrl=n_ctrl, poly_cov=n_ctrl > 0, ctrl_std=0.08, coeff_std=0.2)
    cam = gv_synth.make_camera(W, H, float(W), bg=(0.1, 0.2, 0.3))
    return dict(scene=scene, camera=cam, poses=gv_synth.make_trajectory(rng, F), times=gv_synth.make_times(F),
                frames=F, n=n)


@pytest.mark.parametrize("degree", [1, 2, 3])
def test_sh_clip_matches_oracle(degree):
    w = sh_workload(60 + degree, 160, 96, 3000, 4, degree)
    check_clip_against_oracle(w, f"SH degree {degree} clip")


def test_sh_with_spline_dynamics_matches_oracle():
    w = sh_workload(64, 128, 80, 2000, 4, 3, n_ctrl=6)
    check_clip_against_oracle(w, "SH degree 3 + B-spline clip")


def test_sh_per_frame_path():
    w = sh_workload(65, 96, 64, 1500, 1, 2)
    ref = oracle_frame(w, 0)
    scene, cam, poses, times = device_inputs(w)
    ws = workspace_for(scene, cam, poses, times)
    img = raster.render_fwd(scene, cam, poses[0].contiguous(), 0.0, ws)
    torch.cuda.synchronize()
    compare_image(img.cpu().numpy(), ref, "SH per-frame fwd", colour_range(w))
    dl = upstream_for(w, [ref], 3)[0]
    g, dpose = raster.render_bwd(scene, cam, poses[0].contiguous(), 0.0, ws, img,
                                 dL_dimage=torch.from_numpy(dl).cuda())
    torch.cuda.synchronize()
    gref = oracle_frame(w, 0, dL_dC=planar_to_pixels(dl))["grads"]
    ge = compare_grads(g, gref, "SH per-frame bwd")
    pe = compare_poses(dpose, gref["pose"], "SH per-frame bwd")
    say(f"SH per-frame: grads {ge} pose {pe:.2e}")
