"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Run on an MI355X: ``python -u -m pytest tests -m gpu -x -v``.  Tolerances and
the knife-edge rule are in parity_util.py.
"""
import numpy as np
import pytest
import torch

import gv_synth
import oracle
from oracle import camera_ode as ode_ref
from parity_util import (GRAD_TOL, PIXEL_TOL, PixelTally, colour_range, compare_grads, compare_image, compare_poses,
                         device_inputs, tile_buckets, knife_edge, oracle_frame, planar_to_pixels, rel_err, workspace_for)

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2501_04782_amd import _lib as L
    from paper_2501_04782_amd import camera as gvcam
    from paper_2501_04782_amd import raster


def say(*a):
    print(*a, flush=True)


def small_workload(seed, W, H, n, F, trajectory=False, dtype="f32", cubic=False, z=(2.0, 6.0), ls=(-3.5, 0.3),
                   bg=(0.0, 0.0, 0.0)):
    rng = np.random.default_rng(seed)
    scene = gv_synth.make_scene(rng, n, z=z, log_scale=ls, dtype=dtype, cubic=cubic)
    cam = gv_synth.make_camera(W, H, float(W), bg=bg)
    poses = gv_synth.make_trajectory(rng, F) if trajectory else gv_synth.identity_poses(F)
    return dict(scene=scene, camera=cam, poses=poses, times=gv_synth.make_times(F), frames=F, n=n)


def upstream_for(w, refs, seed, widen=1.0):
    """Random upstream gradient per frame [F][3][H][W], zero at knife-edge pixels."""
    rng = np.random.default_rng(seed)
    H, W = w["camera"].height, w["camera"].width
    dl = rng.normal(0, 1, (w["frames"], 3, H, W)).astype(np.float32)
    for f, r in enumerate(refs):
        ke = knife_edge(r["margins"], grads=True, widen=widen).reshape(H, W)
        dl[f][:, ke] = 0.0
    return dl


def run_clip(w, dl=None, targets=None, forward=True, backward=True):
    scene, cam, poses, times = device_inputs(w)
    ws = workspace_for(scene, cam, poses, times)
    dlt = None if dl is None else torch.from_numpy(dl).cuda()
    tg = None if targets is None else torch.from_numpy(targets).cuda()
    out = raster.render_batch(scene, cam, poses, times, ws, targets=tg, dL_dimages=dlt, forward=forward,
                              backward=backward)
    torch.cuda.synchronize()
    st = ws.status()
    assert st["overflow"] == 0, st
    return out, ws, (scene, cam, poses, times)


def check_clip_against_oracle(w, label, seed=0):
    say(f"[{label}] oracle forward")
    refs = [oracle_frame(w, f) for f in range(w["frames"])]
    dl = upstream_for(w, refs, seed)
    say(f"[{label}] gpu batch fwd+bwd: F={w['frames']} N={w['n']} {w['camera'].width}x{w['camera'].height}")
    out, ws, _ = run_clip(w, dl=dl)
    imgs = out["images"].cpu().numpy()
    tally = PixelTally(label)
    crange = colour_range(w)
    for f in range(w["frames"]):
        compare_image(imgs[f], refs[f], f"{label} frame {f}", crange, tally)
    stats = tally.finish()
    say(f"[{label}] oracle backward")
    g_ref, dposes_ref, _ = oracle.render_clip_grads(w["scene"], w["camera"], w["poses"].astype(np.float64),
                                                    w["times"], range(w["frames"]), [None] * w["frames"],
                                                    [planar_to_pixels(dl[f]) for f in range(w["frames"])])
    ge = compare_grads(out["grads"], g_ref, label)
    pe = compare_poses(out["dL_dposes"], dposes_ref, label)
    say(f"[{label}] pixels {stats} grads={ge} pose={pe:.2e}")
    return out


# ---------------------------------------------------------------------------


def test_project_records_match_oracle():
    w = gv_synth.make_workload("frame128_n2k")
    pose = np.array([0.995, 0.05, -0.06, 0.04, 0.05, -0.08, 0.2], np.float32)
    scene, cam, _, _ = device_inputs(w)
    ws = raster.Workspace(cam, scene.n, 1, 0)
    rec, cnt = raster.project_fwd(scene, cam, torch.from_numpy(pose).cuda(), 0.0, ws)
    rec, cnt = rec.cpu().numpy(), cnt.cpu().numpy()
    ref = oracle.project(w["scene"], w["camera"], pose.astype(np.float64))
    vis = cnt > 0
    assert vis.sum() > 1500
    assert np.all(ref["valid"][vis] == 1)
    np.testing.assert_allclose(rec[vis, 0], ref["u"][vis], rtol=1e-6, atol=1e-4)
    np.testing.assert_allclose(rec[vis, 1], ref["v"][vis], rtol=1e-6, atol=1e-4)
    for k, name in [(2, "A00"), (3, "A01"), (4, "A11")]:
        np.testing.assert_allclose(rec[vis, k], ref[name][vis], rtol=1e-6, atol=1e-7)
    # the depth key is the fp32 rounding of the FP64 depth: bit-exact
    assert np.array_equal(rec[vis, 5].astype(np.float32), ref["key"][vis].astype(np.float32))
    np.testing.assert_allclose(rec[vis, 6], ref["opacity"][vis], rtol=1e-6)


def test_frame128_forward_backward_per_frame_path():
    """The plain per-frame path (render_fwd / render_bwd) on the 128x128, 2k
    Gaussian frame with a rotated camera."""
    w = gv_synth.make_workload("frame128_n2k")
    w["poses"] = np.array([[0.995, 0.05, -0.06, 0.04, 0.05, -0.08, 0.2]], np.float32)
    ref = oracle_frame(w, 0)
    scene, cam, poses, times = device_inputs(w)
    ws = workspace_for(scene, cam, poses, times)
    Tf = torch.empty(128, 128, device="cuda")
    img = raster.render_fwd(scene, cam, poses[0].contiguous(), 0.0, ws, T_final=Tf)
    torch.cuda.synchronize()
    s = compare_image(img.cpu().numpy(), ref, "frame128 fwd", colour_range(w))
    ke = knife_edge(ref["margins"]) | (ref["stake"] > 0)
    np.testing.assert_allclose(Tf.cpu().numpy().reshape(-1)[~ke], ref["T_final"][~ke], atol=PIXEL_TOL)
    t_rel = np.abs(Tf.cpu().numpy().reshape(-1) - ref["T_final"])[~ke] / ref["T_final"][~ke]
    say(f"frame128: T_final relative error max {t_rel.max():.2e}")
    dl = upstream_for(w, [ref], 5)[0]
    g, dpose = raster.render_bwd(scene, cam, poses[0].contiguous(), 0.0, ws, img,
                                 dL_dimage=torch.from_numpy(dl).cuda())
    torch.cuda.synchronize()
    gref = oracle_frame(w, 0, dL_dC=planar_to_pixels(dl))["grads"]
    ge = compare_grads(g, gref, "frame128 bwd")
    pe = compare_poses(dpose, gref["pose"], "frame128 bwd")
    say(f"frame128: {s} grads {ge} pose {pe:.2e}")


@pytest.mark.parametrize("W,H", [(100, 75), (17, 33), (64, 16)])
def test_ragged_image_sizes(W, H):
    w = small_workload(1, W, H, 600, 2, trajectory=True, bg=(0.2, 0.1, 0.3))
    check_clip_against_oracle(w, f"ragged {W}x{H}")


ADVERSARIAL = ["huge", "offscreen", "near", "ties", "zero_opacity", "dense", "elongated"]


@pytest.mark.parametrize("kind", ADVERSARIAL)
def test_adversarial_scenes(kind):
    rng = np.random.default_rng(100 + ADVERSARIAL.index(kind))
    scene, cam = gv_synth.adversarial_scene(rng, 300, kind)
    cam.bg = (0.1, 0.2, 0.3)
    w = dict(scene=scene, camera=cam, poses=gv_synth.identity_poses(1), times=gv_synth.make_times(1), frames=1,
             n=300)
    check_clip_against_oracle(w, f"adversarial {kind}")


def test_empty_and_single_gaussian():
    for n in (0, 1):
        w = small_workload(2, 40, 30, max(n, 1), 1, bg=(0.3, 0.5, 0.7))
        if n == 0:
            s = w["scene"]
            w["scene"] = gv_synth.Scene("f32", s.means[:, :0].copy(), s.log_scales[:, :0].copy(),
                                        s.quats[:, :0].copy(), s.opacity_logits[:0].copy(), s.colors[:, :0].copy())
            w["n"] = 0
            scene, cam, poses, times = device_inputs(w)
            ws = raster.Workspace(cam, 0, 1, 16)
            dl = torch.ones(1, 3, 30, 40, device="cuda")
            out = raster.render_batch(scene, cam, poses, times, ws, dL_dimages=dl)
            torch.cuda.synchronize()
            img = out["images"][0].cpu().numpy()
            assert np.all(img == np.array([0.3, 0.5, 0.7], np.float32)[:, None, None])
            assert torch.all(out["dL_dposes"] == 0)
        else:
            w["scene"].means[:, 0] = [0.0, 0.0, 3.0]
            # anisotropic, so that every parameter has a non-zero gradient
            w["scene"].log_scales[:, 0] = [-1.5, -2.2, -1.8]
            check_clip_against_oracle(w, "single Gaussian")


def test_rectangles_beyond_the_tile_mask():
    """Gaussians whose tile rectangle exceeds 64 tiles have no tile mask: the
    count pass and the scatter re-test their rectangles cell by cell.  Four
    large Gaussians near the centre of the 12 x 10-tile image (3-sigma half
    widths of 67-99 px, rectangles of about 90-120 tiles) lie among 500
    ordinary ones in front of and behind them, over two frames of a moving
    camera."""
    w = small_workload(31, 192, 160, 504, 2, trajectory=True, bg=(0.1, 0.3, 0.2))
    s = w["scene"]
    for k, (x, y, z) in enumerate([(0.0, 0.0, 3.0), (0.2, -0.1, 3.5), (-0.3, 0.2, 4.0), (0.1, 0.3, 4.5)]):
        s.means[:, k] = [x, y, z]
        s.log_scales[:, k] = [np.log(0.5 + 0.1 * k), np.log(0.45), np.log(0.4 + 0.05 * k)]
        s.opacity_logits[k] = -1.0  # opacity 0.27: what lies behind still shows
    check_clip_against_oracle(w, "rectangles beyond the tile mask")


# compact: 0 sub-block forward, 4 quadrant forward, 1 compacted forward, + 32
# one-wave-per-tile forward;
# + 2 compacted backward, + 16 one-wave-per-tile backward, + 8 paired-quadrant
# backward (else the quadrant backward)
@pytest.mark.parametrize("compact,batch,sort_cap", [(0, 256, 4096), (0, 128, 2048), (0, 64, 1024),
                                                    (4, 256, 4096), (4, 128, 2048), (4, 64, 1024),
                                                    (3, 256, 4096), (3, 128, 2048), (3, 64, 1024),
                                                    (1, 128, 2048), (2, 256, 2048), (6, 64, 1024),
                                                    (4, 64, 512), (12, 64, 1024), (12, 128, 2048),
                                                    (12, 256, 4096), (8, 128, 512), (20, 64, 1024),
                                                    (20, 256, 2048), (16, 128, 512), (17, 64, 1024),
                                                    (52, 64, 1024), (52, 128, 2048), (36, 256, 4096)])
def test_clip_reduced_batch_matches_oracle(compact, batch, sort_cap):
    """Batched path on a reduced clip (moving camera, several frames) under
    every setting the autotuner can choose."""
    w = small_workload(3, 160, 96, 3000, 4, trajectory=True, z=(2.0, 10.0), ls=(-3.2, 0.5))
    old = raster.get_tuning()
    raster.set_tuning(batch, sort_cap, compact)
    try:
        check_clip_against_oracle(w, f"clip 160x96 F=4 compact={compact} batch={batch} cap={sort_cap}")
    finally:
        raster.set_tuning(old["batch"], old["sort_cap"], old["compact"], old["bwd_batch"])


def test_poisoned_workspace_dense_scene():
    """A dense, mostly opaque scene, where pixels stop early and most of a
    tile's entries lie behind its last contributor: the adjoint writes partial
    records only up to that point and the projection adjoint adds only the
    records marked as written.  The workspace is filled with 0xFF bytes (NaN
    floats, all-ones counters) before the call, so a stale record or any value
    read before it is written would show in the images or the gradients."""
    w = small_workload(52, 128, 96, 6000, 3, trajectory=True, z=(2.0, 8.0), ls=(-2.6, 0.2))
    w["scene"].opacity_logits[:] += 3.0
    refs = [oracle_frame(w, f) for f in range(w["frames"])]
    sizes = np.concatenate([tile_buckets(w, f) for f in range(w["frames"])])
    contrib = np.mean([r["n_contrib"].mean() for r in refs])
    say(f"[poisoned ws] mean bucket {sizes.mean():.0f}, mean contributors per pixel {contrib:.1f}")
    assert contrib < 0.3 * sizes.mean()
    dl = upstream_for(w, refs, 5)
    scene, cam, poses, times = device_inputs(w)
    ws = workspace_for(scene, cam, poses, times)
    ws.buf.fill_(255)
    out = raster.render_batch(scene, cam, poses, times, ws, dL_dimages=torch.from_numpy(dl).cuda())
    torch.cuda.synchronize()
    assert ws.status()["overflow"] == 0
    imgs = out["images"].cpu().numpy()
    tally = PixelTally("poisoned ws")
    crange = colour_range(w)
    for f in range(w["frames"]):
        compare_image(imgs[f], refs[f], f"poisoned ws frame {f}", crange, tally)
    tally.finish()
    g_ref, dposes_ref, _ = oracle.render_clip_grads(w["scene"], w["camera"], w["poses"].astype(np.float64),
                                                    w["times"], range(w["frames"]), [None] * w["frames"],
                                                    [planar_to_pixels(dl[f]) for f in range(w["frames"])])
    for k, v in out["grads"].items():
        if v is not None:
            assert torch.isfinite(v).all(), k
    compare_grads(out["grads"], g_ref, "poisoned ws")
    compare_poses(out["dL_dposes"], dposes_ref, "poisoned ws")


@pytest.mark.parametrize("compact", [12, 4, 8, 0, 20, 52])
def test_alpha_clamp_paths(compact):
    """Opaque Gaussians (opacity above 0.99) on the left half of the scene:
    tiles there composite with the alpha clamp (alpha = 0.99, no opacity or
    footprint gradient), tiles on the right without it, where the kernels drop
    the clamp once no entry of a batch can reach it.  Both against the oracle,
    under the one-, two- and four-quadrants-per-wave adjoints and the quadrant
    and 4x4-block forwards."""
    w = small_workload(51, 160, 96, 3000, 3, trajectory=True, z=(2.0, 10.0), ls=(-3.2, 0.5))
    s = w["scene"]
    left = s.means[0] < 0
    s.opacity_logits[left] += 6.0
    o = 1.0 / (1.0 + np.exp(-s.opacity_logits.astype(np.float64)))
    assert (o[left] > 0.99).mean() > 0.5 and (o[~left] < 0.98).mean() > 0.99
    # Gaussians whose alpha at the pixel centre nearest their centre is clamped
    p = oracle.project(w["scene"], w["camera"], w["poses"][0].astype(np.float64), float(w["times"][0]))
    vis = p["valid"] > 0
    dx = np.floor(p["u"][vis]) + 0.5 - p["u"][vis]
    dy = np.floor(p["v"][vis]) + 0.5 - p["v"][vis]
    q = p["A00"][vis] * dx * dx + 2 * p["A01"][vis] * dx * dy + p["A11"][vis] * dy * dy
    n_clamped = int((p["opacity"][vis] * np.exp(-0.5 * q) > 0.99).sum())
    say(f"[alpha clamp] {n_clamped} Gaussians clamped at a pixel in frame 0")
    assert n_clamped > 50
    old = raster.get_tuning()
    raster.set_tuning(256, 1024, compact, 128)
    try:
        check_clip_against_oracle(w, f"alpha clamp compact={compact}")
    finally:
        raster.set_tuning(old["batch"], old["sort_cap"], old["compact"], old["bwd_batch"])


# (Gaussians, sort capacity, regime of the largest bucket): chunked LDS sort +
# global merges; two runs merged in LDS; one LDS pass at the largest capacity
@pytest.mark.parametrize("n,cap,regime,compact", [(5000, 1024, "global", 4), (1600, 1024, "two runs", 4),
                                                  (3000, 4096, "one pass", 4), (1600, 512, "global", 4),
                                                  (5000, 1024, "global", 6), (5000, 1024, "global", 12),
                                                  (1600, 512, "global", 12), (5000, 1024, "global", 20),
                                                  (3000, 2048, "two runs", 52), (5000, 2048, "global", 52),
                                                  (5000, 4096, "two runs", 52), (9000, 4096, "global", 52)])
def test_long_tile_buckets(n, cap, regime, compact):
    """Many large Gaussians over a small image: buckets beyond the LDS sort
    capacity, between one and two capacities, and within the largest one."""
    w = small_workload(14, 48, 32, n, 1, z=(2.0, 6.0), ls=(-1.2, 0.3))
    sizes = tile_buckets(w, 0)
    say(f"[long buckets n={n} cap={cap}] bucket sizes {sorted(sizes.tolist())}")
    big = sizes.max()
    assert {"global": big > 2 * cap, "two runs": cap < big <= 2 * cap, "one pass": 2048 < big <= cap}[regime], big
    old = raster.get_tuning()
    raster.set_tuning(old["batch"], cap, compact, old["bwd_batch"])
    try:
        check_clip_against_oracle(w, f"long buckets n={n} cap={cap} compact={compact}")
    finally:
        raster.set_tuning(old["batch"], old["sort_cap"], old["compact"], old["bwd_batch"])


def test_batch_equals_per_frame_path():
    w = small_workload(4, 128, 80, 2000, 3, trajectory=True)
    rng = np.random.default_rng(9)
    targets = rng.random((3, 3, 80, 128)).astype(np.float32)
    out, ws, (scene, cam, poses, times) = run_clip(w, targets=targets)
    F, H, W = 3, 80, 128
    ws1 = raster.Workspace(cam, scene.n, 1, ws.k_capacity)
    grads = raster.grad_buffers(scene)
    scale = 2.0 / (3 * H * W * F)
    for f in range(F):
        img = raster.render_fwd(scene, cam, poses[f].contiguous(), float(times[f]), ws1)
        raster.render_bwd(scene, cam, poses[f].contiguous(), float(times[f]), ws1, img,
                          target=torch.from_numpy(targets[f]).cuda(), loss_scale=scale, grads=grads,
                          accumulate=f > 0)
        torch.cuda.synchronize()
        assert torch.equal(img, out["images"][f]), f"frame {f} image differs"
    for k in ("means", "log_scales", "quats", "opacity_logits", "colors"):
        e = rel_err(grads[k].cpu().numpy(), out["grads"][k].cpu().numpy())
        assert e < 1e-6, (k, e)
    # the fused loss equals the mean squared error of the returned images
    mse = float(((out["images"] - torch.from_numpy(targets).cuda()) ** 2).double().mean())
    assert float(out["loss"].double().sum()) == pytest.approx(mse, rel=1e-5)


def test_fused_l2_equals_explicit_upstream():
    w = small_workload(5, 96, 64, 1500, 2, trajectory=True)
    rng = np.random.default_rng(10)
    targets = rng.random((2, 3, 64, 96)).astype(np.float32)
    out, _, _ = run_clip(w, targets=targets)
    dl = (2.0 * (out["images"] - torch.from_numpy(targets).cuda()) / out["images"].numel()).cpu().numpy()
    out2, _, _ = run_clip(w, dl=dl)
    for k in ("means", "log_scales", "quats", "opacity_logits", "colors"):
        e = rel_err(out["grads"][k].cpu().numpy(), out2["grads"][k].cpu().numpy())
        assert e < 1e-5, (k, e)


def test_graph_replay_matches_eager():
    w = small_workload(6, 96, 64, 1500, 3, trajectory=True)
    rng = np.random.default_rng(11)
    targets = torch.from_numpy(rng.random((3, 3, 64, 96)).astype(np.float32)).cuda()
    scene, cam, poses, times = device_inputs(w)
    ws = workspace_for(scene, cam, poses, times)
    eager = raster.render_batch(scene, cam, poses, times, ws, targets=targets)
    torch.cuda.synchronize()
    ref = {k: (v.clone() if isinstance(v, torch.Tensor) else {kk: vv.clone() for kk, vv in v.items() if vv is not None})
           for k, v in eager.items() if v is not None}
    ws2 = workspace_for(scene, cam, poses, times)
    g = raster.BatchGraph(scene, cam, poses, times, ws2, targets=targets)
    junk = torch.randn(1 << 20, device="cuda")
    for rep in range(3):
        g.launch()
        junk = junk * 1.0001 + 1.0  # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(g.images, ref["images"]), rep
        assert torch.equal(g.loss, ref["loss"]), rep
        for k, v in ref["grads"].items():
            assert torch.equal(g.grads[k], v), (rep, k)
        assert torch.equal(g.dL_dposes, ref["dL_dposes"]), rep
    g.close()


def test_capacity_overflow_is_reported_and_recoverable():
    w = small_workload(7, 96, 64, 1500, 2, trajectory=True)
    scene, cam, poses, times = device_inputs(w)
    ws = raster.Workspace(cam, scene.n, 1, 10)
    with pytest.raises(L.GvError) as ei:
        raster.render_fwd(scene, cam, poses[0].contiguous(), 0.0, ws)
    assert ei.value.status == L.GV_ERR_CAPACITY
    wsb = raster.Workspace(cam, scene.n, 2, 10)
    dl = torch.ones(2, 3, 64, 96, device="cuda")
    raster.render_batch(scene, cam, poses, times, wsb, dL_dimages=dl)
    st = wsb.status()
    assert st["overflow"] == 1 and st["intersections"] > 10
    wsb = raster.Workspace(cam, scene.n, 2, st["intersections"])
    raster.render_batch(scene, cam, poses, times, wsb, dL_dimages=dl)
    assert wsb.status()["overflow"] == 0


def test_determinism_bitwise():
    w = small_workload(8, 128, 96, 3000, 2, trajectory=True)
    rng = np.random.default_rng(12)
    targets = rng.random((2, 3, 96, 128)).astype(np.float32)
    a, _, _ = run_clip(w, targets=targets)
    b, _, _ = run_clip(w, targets=targets)
    assert torch.equal(a["images"], b["images"])
    for k, v in a["grads"].items():
        if v is not None:
            assert torch.equal(v, b["grads"][k]), k
    assert torch.equal(a["dL_dposes"], b["dL_dposes"])


def test_bf16_cubic_means_reduced():
    w = small_workload(13, 192, 108, 4000, 3, dtype="bf16", cubic=True, z=(2.0, 10.0), ls=(-3.0, 0.5))
    check_clip_against_oracle(w, "bf16 cubic 192x108 F=3")


@pytest.mark.parametrize("frames,substeps", [(1, 4), (12, 4), (100, 4)])
def test_camera_ode_matches_oracle(frames, substeps):
    rng = np.random.default_rng(frames)
    theta = gv_synth.init_mlp_theta(rng, last_layer_scale=0.5).astype(np.float32)
    q = rng.normal(0, 1, 4)
    z0 = np.concatenate([q / np.linalg.norm(q), rng.normal(0, 0.2, 3)]).astype(np.float32)
    ref = ode_ref.camera_ode_fwd(theta.astype(np.float64), z0.astype(np.float64), frames, substeps)
    th, z = torch.from_numpy(theta).cuda(), torch.from_numpy(z0).cuda()
    ws = gvcam.OdeWorkspace(frames, substeps)
    poses = gvcam.camera_ode_fwd(th, z, frames, substeps, ws)
    torch.cuda.synchronize()
    np.testing.assert_allclose(poses.cpu().numpy(), ref, atol=2e-5)
    dp = rng.normal(0, 1, (frames, 7)).astype(np.float32)
    dth_ref, dz_ref = ode_ref.camera_ode_bwd(theta.astype(np.float64), z0.astype(np.float64), frames, substeps,
                                             dp.astype(np.float64))
    dth, dz = gvcam.camera_ode_bwd(th, z, frames, substeps, torch.from_numpy(dp).cuda(), ws)
    torch.cuda.synchronize()
    if frames > 1:
        assert rel_err(dth.cpu().numpy(), dth_ref) <= GRAD_TOL
    else:
        assert float(dth.abs().max()) == 0.0
    assert rel_err(dz.cpu().numpy(), dz_ref) <= GRAD_TOL


def test_fit_graph_chains_ode_and_raster():
    """The learned-camera fitting step (ODE forward -> batched raster fwd+bwd ->
    ODE adjoint) as one graph equals the separate calls, and its parameter
    gradient matches the oracle chain (FP64 ODE -> FP64 renderer adjoint ->
    FP64 discrete adjoint) on a reduced clip."""
    F, S = 6, 4
    rng = np.random.default_rng(30)
    w = small_workload(31, 96, 64, 1500, F)
    theta = gv_synth.init_mlp_theta(rng, last_layer_scale=0.3).astype(np.float32)
    z0 = np.array([1.0, 0.02, -0.03, 0.01, 0.05, -0.02, 0.1], np.float32)
    poses_ref = ode_ref.camera_ode_fwd(theta.astype(np.float64), z0.astype(np.float64), F, S)
    w["poses"] = poses_ref.astype(np.float32)
    refs = [oracle_frame(w, f) for f in range(F)]
    # the GPU integrates the poses in FP32: set aside pixels within 50x the usual margins
    dl = upstream_for(w, refs, 31, widen=50.0)
    scene, cam, _, times = device_inputs(w)
    th, z = torch.from_numpy(theta).cuda(), torch.from_numpy(z0).cuda()
    ws = workspace_for(scene, cam, torch.from_numpy(w["poses"]).cuda(), times)
    fit = gvcam.FitGraph(scene, cam, th, z, F, S, times, ws, dL_dimages=torch.from_numpy(dl).cuda())
    fit.launch()
    fit.launch()
    torch.cuda.synchronize()
    # same as the separate calls
    ows = gvcam.OdeWorkspace(F, S)
    poses = gvcam.camera_ode_fwd(th, z, F, S, ows)
    out = raster.render_batch(scene, cam, poses, times, ws, dL_dimages=torch.from_numpy(dl).cuda())
    dth, dz = gvcam.camera_ode_bwd(th, z, F, S, out["dL_dposes"], ows)
    torch.cuda.synchronize()
    assert torch.equal(fit.poses, poses) and torch.equal(fit.images, out["images"])
    assert torch.equal(fit.dtheta, dth) and torch.equal(fit.dz0, dz)
    # against the FP64 chain
    g_ref, dposes_ref, _ = oracle.render_clip_grads(w["scene"], w["camera"], poses_ref, w["times"], range(F),
                                                    [None] * F, [planar_to_pixels(dl[f]) for f in range(F)])
    dth_ref, dz_ref = ode_ref.camera_ode_bwd(theta.astype(np.float64), z0.astype(np.float64), F, S, dposes_ref)
    compare_grads(fit.grads, g_ref, "fit graph")
    e1, e2 = rel_err(fit.dtheta.cpu().numpy(), dth_ref), rel_err(fit.dz0.cpu().numpy(), dz_ref)
    assert e1 <= GRAD_TOL and e2 <= GRAD_TOL, (e1, e2)
    fit.close()
    say(f"[fit graph] dtheta err {e1:.2e} dz0 err {e2:.2e}")
