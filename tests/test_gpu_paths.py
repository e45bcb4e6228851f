"""GPU parity of the paths around the core renderer, through the C ABI:

* the fused L2 loss of Sec. 4.1 (per-frame loss and every gradient) against
  the oracle's loss and adjoint on whole reduced clips;
* non-finite parameters: such Gaussians are dropped (images and gradients as
  the oracle's, their gradients exactly zero) and counted in the status word;
* the autograd wrappers (RasterizeFrame, RasterizeClip, RasterizeDynamicClip):
  a torch loss back-propagated through them against the oracle adjoint, and
  an undersized workspace that must raise;
* the trajectory-error judge of the learned camera (gv_pose_error) against
  the oracle's;
* the autotuner's cache: a tuned choice is written, read back for the same
  problem key, and a hand-written line is installed as written.
"""
import numpy as np
import pytest
import torch

import gv_synth
import oracle
from parity_util import (PIXEL_TOL, PixelTally, colour_range, compare_grads, compare_image, compare_poses,
                         device_inputs, knife_edge, oracle_frame, planar_to_pixels, workspace_for)
from test_gpu_parity import say, small_workload, upstream_for

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2501_04782_amd import _lib as L
    from paper_2501_04782_amd import camera as gvcam
    from paper_2501_04782_amd import raster


# ------------------------------------------------------------- fused L2 loss


def check_fused_l2(w, label, seed):
    """Whole frames: the GPU's fused loss and gradients against the oracle's
    L2 loss of its own images and the oracle adjoint fed that loss gradient.
    At set-aside pixels the target is the GPU's image, so the residual there
    is zero on both sides."""
    F, H, W = w["frames"], w["camera"].height, w["camera"].width
    say(f"[{label}] oracle forward")
    refs = [oracle_frame(w, f) for f in range(F)]
    scene, cam, poses, times = device_inputs(w)
    ws = workspace_for(scene, cam, poses, times)
    fwd = raster.render_batch(scene, cam, poses, times, ws, forward=True, backward=False)
    torch.cuda.synchronize()
    base = fwd["images"].cpu().numpy()
    rng = np.random.default_rng(seed)
    tg = rng.random((F, 3, H, W)).astype(np.float32)
    img_ref = np.empty((F, 3, H, W))
    for f, r in enumerate(refs):
        held = (knife_edge(r["margins"], grads=True) | (r["stake"] > 0)).reshape(H, W)
        tg[f][:, held] = base[f][:, held]
        img_ref[f] = r["color"].T.reshape(3, H, W)
        img_ref[f][:, held] = tg[f][:, held]
    targets = torch.from_numpy(tg).cuda()
    say(f"[{label}] gpu batch fwd+bwd with fused L2")
    out = raster.render_batch(scene, cam, poses, times, ws, targets=targets)
    torch.cuda.synchronize()
    assert ws.status()["overflow"] == 0
    imgs = out["images"].cpu().numpy()
    assert np.array_equal(imgs, base)
    tally = PixelTally(label)
    for f in range(F):
        compare_image(imgs[f], refs[f], f"{label} frame {f}", colour_range(w), tally)
    stats = tally.finish()
    loss_ref, dldc = oracle.l2_loss_and_grad(img_ref, tg.astype(np.float64), per_frame=True)
    loss_gpu = out["loss"].cpu().numpy().astype(np.float64)
    # what the pixel bar allows (|dC| <= PIXEL_TOL) plus FP32 summation
    n = img_ref.size
    resid = np.abs(img_ref - tg)
    bound = (2 * resid * PIXEL_TOL + PIXEL_TOL ** 2).reshape(F, -1).sum(axis=1) / n + 1e-5 * loss_ref
    assert np.all(np.abs(loss_gpu - loss_ref) <= bound), (loss_gpu, loss_ref, bound)
    say(f"[{label}] oracle backward")
    g_ref, dposes_ref, _ = oracle.render_clip_grads(w["scene"], w["camera"], w["poses"].astype(np.float64),
                                                    w["times"], range(F), [None] * F,
                                                    [planar_to_pixels(dldc[f]) for f in range(F)])
    ge = compare_grads(out["grads"], g_ref, label)
    pe = compare_poses(out["dL_dposes"], dposes_ref, label)
    say(f"[{label}] pixels {stats} loss rel err {np.abs(loss_gpu - loss_ref) / loss_ref} grads={ge} pose={pe:.2e}")


def test_fused_l2_moving_camera_clip():
    w = small_workload(60, 160, 96, 3000, 4, trajectory=True, z=(2.0, 10.0), ls=(-3.2, 0.5), bg=(0.1, 0.3, 0.2))
    check_fused_l2(w, "fused L2 160x96 F=4", 61)


def test_fused_l2_bf16_cubic_clip():
    w = small_workload(62, 192, 108, 4000, 3, dtype="bf16", cubic=True, z=(2.0, 10.0), ls=(-3.0, 0.5))
    check_fused_l2(w, "fused L2 bf16 cubic 192x108 F=3", 63)


# -------------------------------------------------------- non-finite inputs


def test_nonfinite_parameters_are_dropped_and_counted():
    """Gaussians with a NaN or infinite parameter (mean, log-scale, quaternion,
    opacity logit, colour) render as if absent, their gradients are exactly
    zero, and status word 1 counts them once per frame."""
    F = 2
    w = small_workload(64, 64, 48, 500, F, trajectory=True, bg=(0.2, 0.2, 0.4))
    s = w["scene"]
    bad = {0: ("means", 0, np.nan), 1: ("log_scales", 1, np.inf), 2: ("quats", 2, np.nan),
           3: ("opacity_logits", None, -np.inf), 4: ("colors", 0, np.nan), 5: ("means", 2, -np.inf)}
    # make the poisoned Gaussians large and central, so they would matter
    for g in bad:
        s.means[:, g] = [0.0, 0.0, 3.0]
        s.log_scales[:, g] = -1.5
        s.opacity_logits[g] = 2.0
    clean = gv_synth.Scene("f32", s.means.copy(), s.log_scales.copy(), s.quats.copy(), s.opacity_logits.copy(),
                           s.colors.copy())
    for g, (field, row, val) in bad.items():
        arr = getattr(s, field)
        if row is None:
            arr[g] = val
        else:
            arr[row, g] = val
    keep = np.setdiff1d(np.arange(w["n"]), list(bad))
    dropped = dict(w, scene=gv_synth.Scene("f32", clean.means[:, keep].copy(), clean.log_scales[:, keep].copy(),
                                           clean.quats[:, keep].copy(), clean.opacity_logits[keep].copy(),
                                           clean.colors[:, keep].copy()), n=keep.size)
    refs = [oracle_frame(dropped, f) for f in range(F)]
    refs_nan = [oracle_frame(w, f) for f in range(F)]
    for r, rn in zip(refs, refs_nan):  # the oracle itself drops them
        assert np.array_equal(r["color"], rn["color"])
    dl = upstream_for(w, refs, 65)
    scene, cam, poses, times = device_inputs(w)
    ws = workspace_for(scene, cam, poses, times)
    out = raster.render_batch(scene, cam, poses, times, ws, dL_dimages=torch.from_numpy(dl).cuda())
    torch.cuda.synchronize()
    st = ws.status()
    assert st["overflow"] == 0
    assert st["nonfinite"] == F * len(bad), st
    imgs = out["images"].cpu().numpy()
    assert np.all(np.isfinite(imgs))
    tally = PixelTally("non-finite")
    for f in range(F):
        compare_image(imgs[f], refs[f], f"non-finite frame {f}", colour_range(dropped), tally)
    tally.finish()
    g_ref, dposes_ref, _ = oracle.render_clip_grads(dropped["scene"], w["camera"], w["poses"].astype(np.float64),
                                                    w["times"], range(F), [None] * F,
                                                    [planar_to_pixels(dl[f]) for f in range(F)])
    got = {k: v.cpu().numpy() for k, v in out["grads"].items() if v is not None}
    for k in ("means", "log_scales", "quats", "opacity_logits", "colors"):
        assert np.all(got[k][..., list(bad)] == 0.0), k
        got[k] = got[k][..., keep]
    got["intrinsics"] = out["grads"]["intrinsics"].cpu().numpy()
    ge = compare_grads(got, g_ref, "non-finite")
    compare_poses(out["dL_dposes"], dposes_ref, "non-finite")
    say(f"[non-finite] status {st} grads {ge}")


# ----------------------------------------------------------------- autograd


def _leaves(scene, names):
    return [getattr(scene, k).detach().clone().requires_grad_(True) for k in names]


def test_autograd_rasterize_frame():
    w = small_workload(66, 96, 64, 1500, 1, trajectory=True)
    ref = oracle_frame(w, 0)
    R = upstream_for(w, [ref], 67)[0]
    scene, cam, poses, times = device_inputs(w)
    ws = workspace_for(scene, cam, poses, times)
    params = _leaves(scene, ("means", "log_scales", "quats", "opacity_logits", "colors"))
    pose = poses[0].clone().requires_grad_(True)
    img = raster.RasterizeFrame.apply(*params, pose, cam, ws, float(w["times"][0]))
    loss = (img * torch.from_numpy(R).cuda()).sum()
    loss.backward()
    torch.cuda.synchronize()
    compare_image(img.detach().cpu().numpy(), ref, "autograd frame", colour_range(w))
    g_ref = oracle_frame(w, 0, dL_dC=planar_to_pixels(R))["grads"]
    got = dict(zip(("means", "log_scales", "quats", "opacity_logits", "colors"), [p.grad for p in params]))
    ge = compare_grads(got, g_ref, "autograd frame", names=list(got))
    compare_poses(pose.grad, g_ref["pose"], "autograd frame")
    say(f"[autograd frame] grads {ge}")


def test_autograd_rasterize_clip_and_overflow():
    F = 3
    w = small_workload(68, 96, 64, 1500, F, trajectory=True, bg=(0.3, 0.1, 0.2))
    refs = [oracle_frame(w, f) for f in range(F)]
    R = upstream_for(w, refs, 69)
    scene, cam, poses, times = device_inputs(w)
    ws = workspace_for(scene, cam, poses, times)
    params = _leaves(scene, ("means", "log_scales", "quats", "opacity_logits", "colors"))
    P = poses.clone().requires_grad_(True)
    imgs = raster.RasterizeClip.apply(*params, None, None, P, times, cam, ws)
    loss = (imgs * torch.from_numpy(R).cuda()).sum()
    loss.backward()
    torch.cuda.synchronize()
    tally = PixelTally("autograd clip")
    for f in range(F):
        compare_image(imgs[f].detach().cpu().numpy(), refs[f], f"autograd clip frame {f}", colour_range(w), tally)
    tally.finish()
    g_ref, dposes_ref, _ = oracle.render_clip_grads(w["scene"], w["camera"], w["poses"].astype(np.float64),
                                                    w["times"], range(F), [None] * F,
                                                    [planar_to_pixels(R[f]) for f in range(F)])
    got = dict(zip(("means", "log_scales", "quats", "opacity_logits", "colors"), [p.grad for p in params]))
    ge = compare_grads(got, g_ref, "autograd clip", names=list(got))
    compare_poses(P.grad, dposes_ref, "autograd clip")
    say(f"[autograd clip] grads {ge}")
    # an intersection capacity far too small raises in the forward
    small = raster.Workspace(cam, scene.n, F, 10)
    with pytest.raises(L.GvError) as ei:
        raster.RasterizeClip.apply(*params, None, None, P, times, cam, small)
    assert ei.value.status == L.GV_ERR_CAPACITY


def test_autograd_rasterize_dynamic_clip():
    F = 3
    rng = np.random.default_rng(70)
    s = gv_synth.make_scene(rng, 1500, z=(2.0, 6.0), log_scale=(-3.5, 0.3), n_ctrl=6, poly_cov=True)
    cam_np = gv_synth.make_camera(96, 64, 96.0, bg=(0.1, 0.1, 0.1))
    w = dict(scene=s, camera=cam_np, poses=gv_synth.make_trajectory(rng, F), times=gv_synth.make_times(F),
             frames=F, n=1500)
    refs = [oracle_frame(w, f) for f in range(F)]
    R = upstream_for(w, refs, 71)
    scene, cam, poses, times = device_inputs(w)
    ws = workspace_for(scene, cam, poses, times)
    names = ("ctrl", "log_scales", "quats", "opacity_logits", "colors", "scale_coeffs", "quat_coeffs")
    params = _leaves(scene, names)
    P = poses.clone().requires_grad_(True)
    imgs = raster.RasterizeDynamicClip.apply(*params, P, times, cam, ws)
    loss = (imgs * torch.from_numpy(R).cuda()).sum()
    loss.backward()
    torch.cuda.synchronize()
    tally = PixelTally("autograd dynamic clip")
    for f in range(F):
        compare_image(imgs[f].detach().cpu().numpy(), refs[f], f"autograd dynamic frame {f}", colour_range(w),
                      tally)
    tally.finish()
    g_ref, dposes_ref, _ = oracle.render_clip_grads(w["scene"], w["camera"], w["poses"].astype(np.float64),
                                                    w["times"], range(F), [None] * F,
                                                    [planar_to_pixels(R[f]) for f in range(F)])
    got = dict(zip(names, [p.grad for p in params]))
    ge = compare_grads(got, g_ref, "autograd dynamic clip", names=list(got))
    compare_poses(P.grad, dposes_ref, "autograd dynamic clip")
    say(f"[autograd dynamic clip] grads {ge}")


# -------------------------------------------------------- trajectory judge


def test_pose_error_matches_oracle():
    """gv_pose_error against the oracle's trajectory error on 300 frames (more
    than one workgroup's lanes): random poses with non-unit quaternions, plus
    frames that are identical, differ by the quaternion's sign, by a tiny
    rotation, and by nearly half a turn."""
    rng = np.random.default_rng(72)
    F = 300
    ref = np.concatenate([rng.normal(0, 1, (F, 4)) * rng.uniform(0.5, 2.0, (F, 1)), rng.normal(0, 1, (F, 3))], 1)
    got = np.concatenate([rng.normal(0, 1, (F, 4)), rng.normal(0, 1, (F, 3))], 1)
    got[0] = ref[0]
    got[1] = ref[1] * np.array([-2.0] * 4 + [1.0] * 3)
    # frame 2: a rotation of 1e-3 rad about x composed with frame 2's reference
    q = ref[2, :4] / np.linalg.norm(ref[2, :4])
    h = 0.5e-3
    dq = np.array([np.cos(h), np.sin(h), 0.0, 0.0])
    w1, x1, y1, z1 = dq
    w2, x2, y2, z2 = q
    got[2, :4] = [w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                  w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2]
    got[3, :4] = [0.0, 1.0, 0.0, 0.0]
    ref[3, :4] = [1e-3, 0.0, 1.0, 0.0]  # nearly half a turn apart
    got32, ref32 = got.astype(np.float32), ref.astype(np.float32)
    e = oracle.trajectory_error(got32.astype(np.float64), ref32.astype(np.float64))
    j = gvcam.pose_error(torch.from_numpy(got32).cuda(), torch.from_numpy(ref32).cuda())
    np.testing.assert_allclose(j["translation"], e["translation"], rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(j["angle"], e["angle"], rtol=1e-6, atol=1e-6)
    assert j["translation"][0] == 0.0 and j["angle"][0] == 0.0
    assert j["angle"][1] < 1e-6 and j["translation"][1] < 1e-5
    assert j["angle"][2] == pytest.approx(1e-3, rel=1e-3)
    assert j["angle"][3] == pytest.approx(np.pi, abs=3e-3)
    assert j["translation_rmse"] == pytest.approx(e["translation_rmse"], rel=1e-6)
    assert j["mean_angle"] == pytest.approx(e["mean_angle"], rel=1e-6)


# ---------------------------------------------------------------- autotuner


def test_autotune_cache_read_back(tmp_path):
    """gv_autotune times the options and appends its choice to the cache; the
    same problem is then served from the cache without timing, and a cache
    line written by hand for the problem's key is installed as written."""
    w = small_workload(74, 96, 64, 1500, 3, trajectory=True)
    scene, cam, poses, times = device_inputs(w)
    ws = workspace_for(scene, cam, poses, times)
    targets = torch.rand(3, 3, 64, 96, device="cuda")
    old = raster.get_tuning()
    cache = tmp_path / "tune.jsonl"
    try:
        t1 = raster.autotune(scene, cam, poses, times, ws, targets, cache_path=str(cache))
        lines = cache.read_text().splitlines()
        assert len(lines) == 1 and raster.get_tuning() == t1
        assert t1["batch"] in (64, 128, 256) and t1["bwd_batch"] in (64, 128, 256)
        assert t1["sort_cap"] in (512, 1024, 2048, 4096) and t1["compact"] & ~(8 | 16) in (0, 1, 4, 36)
        assert not (t1["compact"] & 8 and t1["bwd_batch"] == 256)  # the paired backward runs batches <= 128
        t2 = raster.autotune(scene, cam, poses, times, ws, targets, cache_path=str(cache))
        assert t2 == t1 and len(cache.read_text().splitlines()) == 1
        # a hand-written line for the same key wins if it comes first
        forced = lines[0]
        for k, v in (("batch", 64), ("bwd_batch", 256), ("sort_cap", 2048), ("compact", 0)):
            forced = forced.replace(f'"{k}": {t1[k]}', f'"{k}": {v}')
        cache.write_text(forced + "\n" + lines[0] + "\n")
        t3 = raster.autotune(scene, cam, poses, times, ws, targets, cache_path=str(cache))
        assert t3 == dict(batch=64, sort_cap=2048, compact=0, bwd_batch=256), t3
        # another problem (different frame count) is tuned anew and appended
        ws2 = workspace_for(scene, cam, poses[:2].contiguous(), times[:2].contiguous())
        raster.autotune(scene, cam, poses[:2].contiguous(), times[:2].contiguous(), ws2, targets[:2].contiguous(),
                        cache_path=str(cache))
        assert len(cache.read_text().splitlines()) == 3
        say(f"[autotune] chose {t1}; cache lines {len(cache.read_text().splitlines())}")
    finally:
        raster.set_tuning(old["batch"], old["sort_cap"], old["compact"], old["bwd_batch"])
