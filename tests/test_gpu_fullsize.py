"""Full-size parity of the benchmark configurations, in the launch
configuration bench.py times, on every pixel of every frame: the oracle's
tiled form (results identical to its per-pixel definition, see
test_oracle_tiled.py) renders each whole frame in about a second, so images,
final transmittance, losses and all gradients are compared at full size.

* the 960x540 frame of 100k Gaussians through the plain per-frame path;
* the benchmark clip (50 frames at 960x540, 200k Gaussians) through the
  captured graph with the fused L2 loss (Sec. 4.1), and again at sort
  capacity 512, where every bucket above 1024 entries takes the global-merge
  path of the per-tile sort;
* the 32-frame 1920x1080 clip of 500k bf16 Gaussians with cubic means;
* the B-spline dynamics and SH-colour clips (50 frames at 960x540), on five
  whole frames each;
* the camera-ODE fitting step (100 frames: ODE forward -> batched raster
  fwd+bwd -> ODE adjoint in one graph), with the trajectory error of the
  learned camera against the ground-truth pose table;
* a 4128x1056 clip whose tile grid exceeds the LDS tile histogram.
"""
import numpy as np
import pytest
import torch

import gv_synth
import oracle
from oracle import camera_ode as ode_ref
from parity_util import (GRAD_TOL, PIXEL_TOL, PixelTally, colour_range, compare_grads, compare_poses, device_inputs,
                         knife_edge, oracle_clip_grads, oracle_frame, planar_to_pixels, rel_err, tile_buckets,
                         workspace_for)
from test_gpu_parity import run_clip, say, small_workload

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2501_04782_amd import camera as gvcam
    from paper_2501_04782_amd import raster

TILE = 16  # tile edge of the oracle's tiled form


def whole_frames(w, label, widen=1.0):
    """The oracle's forward results on every frame of the clip."""
    refs = []
    for f in range(w["frames"]):
        refs.append(oracle_frame(w, f, widen=widen, tile=TILE))
    sizes = tile_buckets(w, 0)
    say(f"[{label}] oracle forward on {w['frames']} whole frames; frame 0: longest bucket {int(sizes.max())}, "
        f"{int((sizes > 1024).sum())} buckets above 1024 entries")
    return refs


def held(r, widen=1.0):
    """Pixels whose upstream gradient is zeroed: a decision within rounding."""
    return knife_edge(r["margins"], grads=True, widen=widen) | (r["stake"] > 0)


def whole_upstream(w, refs, seed, widen=1.0):
    """A random upstream gradient on every frame (zero at set-aside pixels):
    per frame [P][3] and dense [F][3][H][W]."""
    H, W = w["camera"].height, w["camera"].width
    rng = np.random.default_rng(seed)
    dls = []
    dl = np.zeros((w["frames"], 3, H * W), np.float32)
    for f, r in enumerate(refs):
        d = rng.normal(0, 1, (H * W, 3)).astype(np.float32).astype(np.float64)
        d[held(r, widen)] = 0.0
        dls.append(d)
        dl[f] = d.T
    return dls, dl.reshape(w["frames"], 3, H, W)


def check_frames(imgs, refs, w, label, widen=1.0):
    tally = PixelTally(label)
    crange = colour_range(w)
    for f, r in enumerate(refs):
        tally.add(planar_to_pixels(imgs[f]), r, crange, widen=widen, where=f" frame {f}")
    stats = tally.finish()
    say(f"[{label}] pixels {stats}")
    return stats


def clip_grads(w, dls):
    """Oracle gradients over every frame, with the per-element magnitude sums
    that bound the rounding of a sum over frames."""
    return oracle_clip_grads(w, dls, tile=TILE)


def test_frame540p_n100k_full_size():
    """960x540, 100k Gaussians, the plain per-frame path: every pixel, its
    final transmittance, and the gradients for an upstream gradient on every
    pixel."""
    w = gv_synth.make_workload("frame540p_n100k", targets=False)
    refs = whole_frames(w, "540p n100k")
    dls, dl = whole_upstream(w, refs, 20)
    scene, cam, poses, times = device_inputs(w)
    ws = workspace_for(scene, cam, poses, times)
    Tf = torch.empty(w["camera"].height, w["camera"].width, device="cuda")
    img = raster.render_fwd(scene, cam, poses[0].contiguous(), 0.0, ws, T_final=Tf)
    g, dpose = raster.render_bwd(scene, cam, poses[0].contiguous(), 0.0, ws, img,
                                 dL_dimage=torch.from_numpy(dl[0]).cuda())
    torch.cuda.synchronize()
    check_frames(img.cpu().numpy()[None], refs, w, "540p n100k")
    # final transmittance: the relative error the stop decision sees
    r = refs[0]
    free = ~(knife_edge(r["margins"]) | (r["stake"] > 0))
    t_rel = np.abs(Tf.cpu().numpy().reshape(-1) - r["T_final"]) / r["T_final"]
    assert t_rel[free].max() <= 1e-3, t_rel[free].max()  # well inside the stop margin
    say(f"[540p n100k] T_final relative error: max {t_rel[free].max():.2e}, "
        f"99.99th percentile {np.percentile(t_rel[free], 99.99):.2e}")
    gref, dposes_ref, _ = clip_grads(w, dls)
    ge = compare_grads(g, gref, "540p n100k")  # one frame: no sum over frames
    pe = compare_poses(dpose, dposes_ref[0], "540p n100k")
    say(f"[540p n100k] grads={ge} pose={pe:.2e}")


def test_clip540p_f50_n200k_fused_l2_full_size():
    """The benchmark clip in the benchmark's launch configuration (captured
    graph, fused L2 loss), all 50 frames whole.  The targets are seeded
    U[0, 1], except at set-aside pixels, where they are the GPU's own image so
    that the residual there is zero on both sides.  Per-frame losses, all
    parameter gradients and the pose gradients are compared with the oracle's
    L2 loss (Sec. 4.1) and adjoint."""
    w = gv_synth.make_workload("clip540p_f50_n200k", targets=False)
    F, H, W = w["frames"], w["camera"].height, w["camera"].width
    assert max(int(tile_buckets(w, f).max()) for f in (0, F // 2, F - 1)) > 1024
    refs = whole_frames(w, "clip540p")
    scene, cam, poses, times = device_inputs(w)
    ws = workspace_for(scene, cam, poses, times, margin=1.3)
    say("[clip540p] gpu forward (images the set-aside targets are taken from)")
    fwd = raster.render_batch(scene, cam, poses, times, ws, forward=True, backward=False)
    torch.cuda.synchronize()
    assert ws.status()["overflow"] == 0
    base = fwd["images"].clone()
    tg = base.cpu().numpy().reshape(F, 3, H * W)
    rng = np.random.default_rng(22)
    img_ref = np.empty((F, 3, H * W))
    for f, r in enumerate(refs):
        free = ~held(r)
        tg[f][:, free] = rng.random((3, int(free.sum()))).astype(np.float32)
        img_ref[f] = np.where(free[None, :], r["color"].T, tg[f])  # zero residual where held
    targets = torch.from_numpy(tg.reshape(F, 3, H, W)).cuda()
    say("[clip540p] gpu graph (fwd+bwd, fused L2)")
    g = raster.BatchGraph(scene, cam, poses, times, ws, targets=targets)
    g.launch()
    torch.cuda.synchronize()
    assert ws.status()["overflow"] == 0
    assert torch.equal(g.images, base)
    check_frames(g.images.cpu().numpy(), refs, w, "clip540p")
    tgt_ref = tg.astype(np.float64)
    loss_ref, grad = oracle.l2_loss_and_grad(img_ref, tgt_ref, per_frame=True)
    dls = [grad[f].T for f in range(F)]
    loss_gpu = g.loss.cpu().numpy().astype(np.float64)
    n_full = F * 3 * H * W
    bound = np.sum(2 * np.abs(img_ref - tgt_ref) * PIXEL_TOL + PIXEL_TOL ** 2, axis=(1, 2)) / n_full
    bound += 1e-5 * loss_ref
    assert np.all(np.abs(loss_gpu - loss_ref) <= bound), (loss_gpu, loss_ref, bound)
    say(f"[clip540p] loss: max relative error per frame {np.max(np.abs(loss_gpu - loss_ref) / loss_ref):.2e}")
    say("[clip540p] oracle backward")
    g_ref, dposes_ref, mag = clip_grads(w, dls)
    ge = compare_grads(g.grads, g_ref, "clip540p", mag=mag)
    pe = compare_poses(g.dL_dposes, dposes_ref, "clip540p")
    say(f"[clip540p] grads={ge} pose={pe:.2e} intersections={ws.status()['intersections']}")
    # the same step at sort capacity 512: buckets above 1024 entries are sorted
    # in LDS chunks and merged in global memory; the order is fully determined,
    # so every image and gradient is bitwise the same
    old = raster.get_tuning()
    raster.set_tuning(old["batch"], 512, old["compact"], old["bwd_batch"])
    try:
        g2 = raster.BatchGraph(scene, cam, poses, times, ws, targets=targets)
        g2.launch()
        torch.cuda.synchronize()
        assert torch.equal(g2.images, base)
        assert torch.equal(g2.loss, g.loss)
        for k, v in g.grads.items():
            if v is not None:
                assert torch.equal(g2.grads[k], v), k
        assert torch.equal(g2.dL_dposes, g.dL_dposes)
        g2.close()
    finally:
        raster.set_tuning(old["batch"], old["sort_cap"], old["compact"], old["bwd_batch"])
    g.close()


def test_clip1080p_bf16_cubic_full_size():
    w = gv_synth.make_workload("clip1080p_f32_n500k_bf16", targets=False)
    refs = whole_frames(w, "clip1080p")
    dls, dl = whole_upstream(w, refs, 40)
    say("[clip1080p] gpu batch")
    out, ws, _ = run_clip(w, dl=dl)
    check_frames(out["images"].cpu().numpy(), refs, w, "clip1080p")
    say("[clip1080p] oracle backward")
    g_ref, dposes_ref, mag = clip_grads(w, dls)
    ge = compare_grads(out["grads"], g_ref, "clip1080p", mag=mag)
    pe = compare_poses(out["dL_dposes"], dposes_ref, "clip1080p")
    say(f"[clip1080p] grads={ge} pose={pe:.2e} intersections={ws.status()['intersections']}")


@pytest.mark.parametrize("name", ["clip540p_f50_n200k_dyn", "clip540p_f50_n200k_sh3"])
def test_dynamics_and_sh_clips_full_size(name):
    """The clips of the B-spline dynamics (Eq. 2-3: cubic B-spline means over
    8 control points, polynomial log-scales and quaternions) and of SH colour
    of degree 3 at full size (50 frames at 960x540, 200k Gaussians), in the
    launch configuration bench.py times: every pixel of five whole frames
    spread over the clip against the oracle, and every gradient for an
    upstream gradient on those frames (zero on the others, so the sums over
    frames cover exactly them)."""
    w = gv_synth.make_workload(name, targets=False)
    frames = (0, 12, 24, 37, w["frames"] - 1)
    refs = [oracle_frame(w, f, tile=TILE) for f in frames]
    H, W = w["camera"].height, w["camera"].width
    rng = np.random.default_rng(50)
    dls = []
    dl = np.zeros((w["frames"], 3, H * W), np.float32)
    for f, r in zip(frames, refs):
        d = rng.normal(0, 1, (H * W, 3)).astype(np.float32).astype(np.float64)
        d[held(r)] = 0.0
        dls.append(d)
        dl[f] = d.T
    say(f"[{name}] gpu batch")
    out, ws, _ = run_clip(w, dl=dl.reshape(w["frames"], 3, H, W))
    check_frames(out["images"].cpu().numpy()[list(frames)], refs, w, name)
    say(f"[{name}] oracle backward on frames {frames}")
    g_ref, dposes_ref, mag = oracle_clip_grads(w, dls, frames=frames, tile=TILE)
    ge = compare_grads(out["grads"], g_ref, name, mag=mag)
    pe = compare_poses(out["dL_dposes"], dposes_ref, name)
    say(f"[{name}] grads={ge} pose={pe:.2e} intersections={ws.status()['intersections']}")


def test_camera_ode_fitting_step_full_size():
    w = gv_synth.make_workload("clip540p_f100_n200k", targets=False)
    F, S = w["frames"], 4
    gt_poses = w["poses"].copy()
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
    # trajectory error of the learned camera against the ground-truth pose
    # table: the GPU's poses and the FP64 RK4 poses are judged alike
    e_gpu = oracle.trajectory_error(poses_gpu.cpu().numpy(), gt_poses)
    e_ref = oracle.trajectory_error(poses_ref, gt_poses)
    assert abs(e_gpu["translation_rmse"] - e_ref["translation_rmse"]) <= 1e-5 * max(e_ref["translation_rmse"], 1.0)
    assert abs(e_gpu["mean_angle"] - e_ref["mean_angle"]) <= 1e-5
    assert e_ref["translation"][0] < 1e-6 and e_ref["angle"][0] < 1e-6  # z0 is the frame-0 pose
    judged = gvcam.pose_error(poses_gpu, torch.from_numpy(gt_poses).cuda())
    assert judged["translation_rmse"] == pytest.approx(e_gpu["translation_rmse"], rel=1e-5, abs=1e-7)
    assert judged["mean_angle"] == pytest.approx(e_gpu["mean_angle"], rel=1e-5, abs=1e-6)
    say(f"[fit step] trajectory error: rmse {e_ref['translation_rmse']:.4e} angle {e_ref['mean_angle']:.4e} rad")
    w["poses"] = poses_gpu.cpu().numpy()
    refs = whole_frames(w, "fit step")
    dls, dl = whole_upstream(w, refs, 41)
    ws = workspace_for(scene, cam, poses_gpu, times)
    say("[fit step] gpu graph")
    fit = gvcam.FitGraph(scene, cam, th, z, F, S, times, ws, dL_dimages=torch.from_numpy(dl).cuda())
    fit.launch()
    torch.cuda.synchronize()
    assert ws.status()["overflow"] == 0
    assert torch.equal(fit.poses, poses_gpu)
    check_frames(fit.images.cpu().numpy(), refs, w, "fit step")
    say("[fit step] oracle backward + discrete adjoint")
    g_ref, dposes_ref, mag = clip_grads(w, dls)
    compare_grads(fit.grads, g_ref, "fit step", mag=mag)
    dth_ref, dz_ref = ode_ref.camera_ode_bwd(theta.astype(np.float64), z0.astype(np.float64), F, S, dposes_ref)
    e1, e2 = rel_err(fit.dtheta.cpu().numpy(), dth_ref), rel_err(fit.dz0.cpu().numpy(), dz_ref)
    assert e1 <= GRAD_TOL and e2 <= GRAD_TOL, (e1, e2)
    fit.close()
    say(f"[fit step] poses err {ep:.2e} dtheta err {e1:.2e} dz0 err {e2:.2e}")


def test_tile_grid_beyond_lds_histogram():
    """A 4128x1056 frame has 258 x 66 = 17,028 tiles, more than the 16,384 an
    LDS tile histogram holds, so binning takes the count and scatter kernels
    with one global atomic per intersection.  Whole frames against the
    oracle."""
    W, H = 4128, 1056
    assert ((W + 15) // 16) * ((H + 15) // 16) > 16384
    w = small_workload(43, W, H, 4000, 2, trajectory=True, ls=(-4.5, 0.5))
    refs = whole_frames(w, "large grid")
    dls, dl = whole_upstream(w, refs, 44)
    say("[large grid] gpu batch")
    out, ws, _ = run_clip(w, dl=dl)
    check_frames(out["images"].cpu().numpy(), refs, w, "large grid")
    say("[large grid] oracle backward")
    g_ref, dposes_ref, mag = clip_grads(w, dls)
    ge = compare_grads(out["grads"], g_ref, "large grid", mag=mag)
    pe = compare_poses(out["dL_dposes"], dposes_ref, "large grid")
    say(f"[large grid] grads={ge} pose={pe:.2e} intersections={ws.status()['intersections']}")


def test_every_tuning_matches_default_full_size():
    """Every setting the autotuner can choose, one axis at a time from the
    default, on the benchmark clip with the fused L2 loss: images bitwise equal
    to the default's (which the test above checks against the oracle on every
    pixel), per-frame losses and all gradients equal up to the order of
    summation.  The compacted backward, which the autotuner leaves out, is run
    once as well."""
    w = gv_synth.make_workload("clip540p_f50_n200k", targets=True)
    scene, cam, poses, times = device_inputs(w)
    targets = torch.from_numpy(w["targets"]).cuda()
    ws = workspace_for(scene, cam, poses, times, margin=1.3)
    base = dict(batch=128, sort_cap=1024, compact=52, bwd_batch=64)
    settings = [dict(base, batch=b, compact=c | 16) for c in (0, 4, 1, 36) for b in (64, 128, 256)]
    settings += [dict(base, compact=c, bwd_batch=bb)
                 for c, bb in ((36, 64), (36, 128), (36, 256), (44, 64), (44, 128), (38, 128))]
    settings += [dict(base, sort_cap=cap) for cap in (512, 2048, 4096)]
    old = raster.get_tuning()

    def run(t):
        raster.set_tuning(t["batch"], t["sort_cap"], t["compact"], t["bwd_batch"])
        out = raster.render_batch(scene, cam, poses, times, ws, targets=targets)
        torch.cuda.synchronize()
        assert ws.status()["overflow"] == 0, t
        return out

    try:
        ref = run(base)
        ref_images = ref["images"].clone()
        ref_loss = ref["loss"].cpu().numpy().astype(np.float64)
        ref_grads = {k: v.cpu().numpy() for k, v in ref["grads"].items() if v is not None}
        ref_dposes = ref["dL_dposes"].cpu().numpy()
        for t in settings:
            out = run(t)
            assert torch.equal(out["images"], ref_images), t
            dl = np.abs(out["loss"].cpu().numpy() - ref_loss) / ref_loss
            assert dl.max() <= 1e-6, (t, dl.max())
            ge = compare_grads(out["grads"], ref_grads, f"tuning {t}")
            pe = compare_poses(out["dL_dposes"], ref_dposes, f"tuning {t}")
            say(f"[tunings] {t}: images equal, loss {dl.max():.1e}, "
                f"grads max rel {max(e for e, _ in ge.values()):.1e}, pose {pe:.1e}")
    finally:
        raster.set_tuning(old["batch"], old["sort_cap"], old["compact"], old["bwd_batch"])
