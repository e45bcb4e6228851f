"""Full-size parity of the two remaining benchmark configurations, in the
launch configuration bench.py times, on sampled pixels the oracle computes one
by one: the 1920x1080, 500k-Gaussian bf16 clip with cubic means (32 frames),
and the camera-ODE fitting step (100 frames at 960x540, 200k Gaussians:
ODE forward -> batched raster fwd+bwd -> ODE adjoint in one graph)."""
import numpy as np
import pytest
import torch

import gv_synth
import oracle
from oracle import camera_ode as ode_ref
from parity_util import GRAD_TOL, PIXEL_TOL, compare_grads, device_inputs, knife_edge, oracle_frame, \
    planar_to_pixels, rel_err, workspace_for
from test_gpu_parity import run_clip, say, small_workload

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2501_04782_amd import camera as gvcam


def sampled_upstream(w, frames, npix, seed, widen=1.0):
    """Oracle results on `npix` random pixels of each listed frame and a random
    upstream gradient supported on those pixels (zero at knife-edge pixels)."""
    H, W = w["camera"].height, w["camera"].width
    rng = np.random.default_rng(seed)
    pix = [np.sort(rng.choice(H * W, npix, replace=False)) for _ in frames]
    refs, dls = [], []
    for f, p in zip(frames, pix):
        say(f"[{w.get('name', 'clip')}] oracle frame {f}")
        r = oracle_frame(w, f, pixels=p)
        refs.append(r)
        d = rng.normal(0, 1, (p.size, 3))
        d[knife_edge(r["margins"], grads=True, widen=widen)] = 0.0
        dls.append(d)
    dl = np.zeros((w["frames"], 3, H * W), np.float32)
    for f, p, d in zip(frames, pix, dls):
        dl[f][:, p] = d.T
    return pix, refs, dls, dl.reshape(w["frames"], 3, H, W)


def check_pixels(imgs, frames, pix, refs, label, widen=1.0):
    for f, p, r in zip(frames, pix, refs):
        got = planar_to_pixels(imgs[f])[p]
        d = np.abs(got - r["color"]).max(axis=1)
        ke = knife_edge(r["margins"], widen=widen)
        assert d[~ke].max() <= PIXEL_TOL, (label, f, d[~ke].max())
        say(f"[{label}] frame {f}: max|d|={d[~ke].max():.2e} knife-edge={ke.sum()}/{p.size}")


def test_clip1080p_bf16_cubic_full_size_sampled():
    w = gv_synth.make_workload("clip1080p_f32_n500k_bf16", targets=False)
    frames = [0, 15, 31]
    pix, refs, dls, dl = sampled_upstream(w, frames, 512, 40)
    say("[clip1080p] gpu batch")
    out, ws, _ = run_clip(w, dl=dl)
    check_pixels(out["images"].cpu().numpy(), frames, pix, refs, "clip1080p")
    say("[clip1080p] oracle backward")
    g_ref, dposes_ref, _ = oracle.render_clip_grads(w["scene"], w["camera"], w["poses"].astype(np.float64),
                                                    w["times"], frames, pix, dls)
    ge = compare_grads(out["grads"], g_ref, "clip1080p")
    pe = rel_err(out["dL_dposes"].cpu().numpy()[frames], dposes_ref[frames])
    assert pe <= GRAD_TOL, pe
    say(f"[clip1080p] grads={ge} pose={pe:.2e} intersections={ws.status()['intersections']}")


def test_camera_ode_fitting_step_full_size_sampled():
    w = gv_synth.make_workload("clip540p_f100_n200k", targets=False)
    F, S = w["frames"], 4
    theta = gv_synth.init_mlp_theta(np.random.default_rng(7)).astype(np.float32)
    z0 = w["poses"][0].astype(np.float32)
    scene, cam, _, times = device_inputs(w)
    th, z = torch.from_numpy(theta).cuda(), torch.from_numpy(z0).cuda()
    # poses from the GPU ODE, then the raster inputs the oracle sees are the same poses
    ows = gvcam.OdeWorkspace(F, S)
    poses_gpu = gvcam.camera_ode_fwd(th, z, F, S, ows)
    torch.cuda.synchronize()
    poses_ref = ode_ref.camera_ode_fwd(theta.astype(np.float64), z0.astype(np.float64), F, S)
    ep = rel_err(poses_gpu.cpu().numpy(), poses_ref)
    assert ep < 1e-5, ep
    w["poses"] = poses_gpu.cpu().numpy()
    frames = [0, 50, 99]
    pix, refs, dls, dl = sampled_upstream(w, frames, 512, 41)
    ws = workspace_for(scene, cam, poses_gpu, times)
    say("[fit step] gpu graph")
    fit = gvcam.FitGraph(scene, cam, th, z, F, S, times, ws, dL_dimages=torch.from_numpy(dl).cuda())
    fit.launch()
    torch.cuda.synchronize()
    assert ws.status()["overflow"] == 0
    assert torch.equal(fit.poses, poses_gpu)
    check_pixels(fit.images.cpu().numpy(), frames, pix, refs, "fit step")
    say("[fit step] oracle backward + discrete adjoint")
    g_ref, dposes_ref, _ = oracle.render_clip_grads(w["scene"], w["camera"], w["poses"].astype(np.float64),
                                                    w["times"], frames, pix, dls)
    compare_grads(fit.grads, g_ref, "fit step")
    dth_ref, dz_ref = ode_ref.camera_ode_bwd(theta.astype(np.float64), z0.astype(np.float64), F, S, dposes_ref)
    e1, e2 = rel_err(fit.dtheta.cpu().numpy(), dth_ref), rel_err(fit.dz0.cpu().numpy(), dz_ref)
    assert e1 <= GRAD_TOL and e2 <= GRAD_TOL, (e1, e2)
    fit.close()
    say(f"[fit step] poses err {ep:.2e} dtheta err {e1:.2e} dz0 err {e2:.2e}")


def test_tile_grid_beyond_lds_histogram_sampled():
    """A 4128x1056 frame has 258 x 66 = 17,028 tiles, more than the 16,384 an
    LDS tile histogram holds, so binning takes the count and scatter kernels
    with one global atomic per intersection.  Images and gradients on sampled
    pixels against the oracle."""
    W, H = 4128, 1056
    assert ((W + 15) // 16) * ((H + 15) // 16) > 16384
    w = small_workload(43, W, H, 4000, 2, trajectory=True, ls=(-4.5, 0.5))
    w["name"] = "large grid"
    frames = [0, 1]
    pix, refs, dls, dl = sampled_upstream(w, frames, 1024, 44)
    say("[large grid] gpu batch")
    out, ws, _ = run_clip(w, dl=dl)
    check_pixels(out["images"].cpu().numpy(), frames, pix, refs, "large grid")
    say("[large grid] oracle backward")
    g_ref, dposes_ref, _ = oracle.render_clip_grads(w["scene"], w["camera"], w["poses"].astype(np.float64),
                                                    w["times"], frames, pix, dls)
    ge = compare_grads(out["grads"], g_ref, "large grid")
    pe = rel_err(out["dL_dposes"].cpu().numpy()[frames], dposes_ref[frames])
    assert pe <= GRAD_TOL, pe
    say(f"[large grid] grads={ge} pose={pe:.2e} intersections={ws.status()['intersections']}")
