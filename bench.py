#!/usr/bin/env python3
"""Benchmark of the batched differentiable Gaussian rasterizer on one MI355X.

One step = one forward+backward pass of the whole hot path (projection,
binning, per-tile sort, compositing, fused L2 loss, compositing adjoint,
projection adjoint with per-frame pose gradients) over one clip of synthetic
input: 50 frames at 960x540, 200k Gaussians shared by all frames, a smooth
camera trajectory (the clip540p_f50_n200k workload).  The step is a single
HIP-graph launch; inputs are resident in HBM before timing starts.

Prints ONE JSON line.  Besides the headline frames/s it reports the plain
per-frame GPU path on the same clip, per-stage times from HIP events, the
roofline of the dominant kernel and the FP64 CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

METRIC = "fwd+bwd frames/s at 960×540, 200k Gaussians (batched vs per-frame), % HBM roof"
ODE_WORKLOAD = "clip540p_f100_n200k"
HBM_PEAK = 8.0e12          # B/s, MI355X HBM3E
# FP32 vector peaks: the published 157.3 TFLOP/s counts packed FP32 (two
# operations per lane and instruction); the library is compiled without
# packed FP32 instructions, so what it can issue is the non-packed rate,
# 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz = 78.6 TFLOP/s.
ALU_PEAK = 157.3e12
ALU_PEAK_NONPACKED = 256 * 4 * 16 * 2 * 2.4e9
# LDS: 128 bytes per clock per CU
LDS_PEAK = 256 * 128 * 2.4e9
# Algorithmic FP32 operations per contributing (pixel, Gaussian) pair, the
# hot-path scope table's per-pair estimates: about 25 in the forward
# compositing and 70 in its adjoint.
FLOPS_FWD_PER_PAIR = 25
FLOPS_BWD_PER_PAIR = 70
PARAM_BYTES = 56           # fp32: means 3, log-scales 3, quats 4, opacity 1, colour 3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(N, V, K, P, F, p=PARAM_BYTES, pg=PARAM_BYTES):
    """Compulsory HBM bytes of one fwd+bwd step over F frames (each input read
    once, each output written once), with p stored parameter bytes and pg FP32
    gradient bytes per Gaussian (56 and 56 for the static fp32 scene).  Per
    frame: forward N*p + V*40 + K*64 + P*20; backward P*20 + K*112 + N*(p + pg)."""
    per_frame_fwd = N * p + V * 40 + (K / F) * 64 + P * 20
    per_frame_bwd = P * 20 + (K / F) * 112 + N * (p + pg)
    return F * (per_frame_fwd + per_frame_bwd)


def stage_bytes(stage, N, V, K, P, F, p=PARAM_BYTES):
    """Algorithmic bytes of one launch of a stage over the whole clip, from the
    hot-path table's per-unit figures (K intersections, V visible Gaussians
    per frame, P pixels per frame, F frames)."""
    if stage == "composite_fwd":
        # per entry: sorted index 4 + gathered record 36; per pixel: RGB 12,
        # final transmittance 4, last index 4 written, target 12 read (fused L2)
        return K * 40 + F * P * (20 + 12)
    if stage == "composite_bwd":
        # per pixel: upstream gradient (or target) 12, T_final 4, last index 4;
        # per entry: sorted index 4 + gathered record 36 read, 9-float partial 36 written
        return F * P * 20 + K * 76
    if stage == "project_bwd":
        # partials read once, parameters read once, gradients written once
        return K * 36 + N * (p + 56)
    if stage == "project":
        return F * N * p + F * V * 40
    if stage == "sort":
        return K * 12 * 2
    if stage == "scatter":
        return K * 12 + F * V * 8
    return 0


def host_info() -> dict:
    """Host cores the CPU baseline could use."""
    try:
        aff = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        aff = None
    return dict(nproc=os.cpu_count(), affinity=aff, omp_num_threads=os.environ.get("OMP_NUM_THREADS"))


def counters_summary(c: dict, pairs) -> dict:
    """Per-launch counter figures of the dominant kernel from its committed
    rocprofv3 summary (SQ counters summed over the chip per dispatch):
    VALU lane-instructions per contributing pair, VALU issue share and lane
    utilisation, LDS utilisation (cycles the LDS serves indexed accesses) and
    LDS bandwidth against its peak, and the profile's own kernel time."""
    ms = c["avg_ms"]
    sec = ms * 1e-3
    # cycles the kernel ran: GRBM_GUI_ACTIVE is counted per XCC (8 summed)
    cycles = c["GRBM_GUI_ACTIVE"] / 8 if "GRBM_GUI_ACTIVE" in c else sec * 2.4e9
    out = dict(avg_ms=round(ms, 4), valu_insts=c["SQ_INSTS_VALU"],
               valu_issue_share=round(c["SQ_INSTS_VALU"] * 4 / (cycles * 1024), 3),
               clock_ghz=round(cycles / sec / 1e9, 3))
    if pairs:
        out["valu_lane_insts_per_pair"] = round(c["SQ_INSTS_VALU"] * 64 / pairs, 1)
    if "SQ_THREAD_CYCLES_VALU" in c and c.get("SQ_ACTIVE_INST_VALU"):
        out["valu_lane_util"] = round(c["SQ_THREAD_CYCLES_VALU"] / (c["SQ_ACTIVE_INST_VALU"] * 64), 3)
    if "SQ_LDS_IDX_ACTIVE" in c:
        out["lds_util"] = round(c["SQ_LDS_IDX_ACTIVE"] / (cycles * 256), 3)
    if "SQ_LDS_BANK_CONFLICT" in c:
        out["lds_bank_conflict_share"] = round(c["SQ_LDS_BANK_CONFLICT"] / (cycles * 256), 3)
    if "SQ_INSTS_LDS_LOAD_BANDWIDTH" in c and "SQ_INSTS_LDS_STORE_BANDWIDTH" in c:
        lds_bytes = 64 * (c["SQ_INSTS_LDS_LOAD_BANDWIDTH"] + c["SQ_INSTS_LDS_STORE_BANDWIDTH"])
        out["lds_bytes"] = lds_bytes
        out["lds_bw_frac"] = round(lds_bytes / sec / LDS_PEAK, 3)
    return out


def quick_clip(name, dev, steps=3):
    """Frames/s of one batched fwd+bwd step (one HIP graph) on another
    workload, with the installed tuning; for the camera-ODE workload the step
    is the fitting graph (ODE forward -> batch -> ODE adjoint)."""
    import torch
    import gv_synth
    from paper_2501_04782_amd import camera, raster
    w = gv_synth.make_workload(name, seed=0, targets=True)
    F, N = w["frames"], w["n"]
    scene = raster.Scene.from_synth(w["scene"], dev)
    cam = raster.Camera.of(w["camera"])
    poses = torch.from_numpy(w["poses"]).to(dev)
    times = torch.from_numpy(w["times"]).to(dev)
    targets = torch.from_numpy(w["targets"]).to(dev)
    cap = raster.estimate_capacity(scene, cam, poses, times, margin=1.3)
    ws = raster.Workspace(cam, N, F, cap, device=dev)
    info = dict(workload=name, frames=F, gaussians=N, width=cam.width, height=cam.height)
    if name == ODE_WORKLOAD:
        gt = raster.render_batch(scene, cam, poses, times, ws, forward=True, backward=False)
        targets = gt["images"].clone()
        theta = torch.from_numpy(gv_synth.init_mlp_theta(np.random.default_rng(7)).astype(np.float32)).to(dev)
        graph = camera.FitGraph(scene, cam, theta, poses[0].clone(), F, 4, times, ws, targets=targets)
        info["step"] = "camera ODE forward (RK4, 4 substeps) -> batched fwd+bwd -> ODE adjoint, one graph"
    else:
        graph = raster.BatchGraph(scene, cam, poses, times, ws, targets=targets)
        info["step"] = "batched fwd+bwd with fused L2, one graph"
    graph.launch()
    torch.cuda.synchronize()
    st = ws.status()
    if st["overflow"]:
        raise RuntimeError(f"{name}: intersection capacity overflow")
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.launch()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    info.update(ms_per_step=round(1e3 * dt, 3), frames_per_s=round(F / dt, 1),
                intersections_per_frame=int(st["intersections"] / F))
    if name == ODE_WORKLOAD:
        # the learned camera's trajectory against the ground-truth pose table
        te = camera.pose_error(graph.poses, poses)
        info["trajectory_error"] = dict(translation_rmse=round(te["translation_rmse"], 6),
                                        mean_angle_rad=round(te["mean_angle"], 6), of="ODE poses at the initial theta")
        ows = camera.OdeWorkspace(F, 4, device=dev)
        th = torch.from_numpy(gv_synth.init_mlp_theta(np.random.default_rng(7)).astype(np.float32)).to(dev)
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        p = camera.camera_ode_fwd(th, poses[0].clone(), F, 4, ows)
        torch.cuda.synchronize()
        e[0].record()
        p = camera.camera_ode_fwd(th, poses[0].clone(), F, 4, ows)
        e[1].record()
        camera.camera_ode_bwd(th, poses[0].clone(), F, 4, torch.ones_like(p), ows)
        e[2].record()
        torch.cuda.synchronize()
        info.update(ode_fwd_ms=round(e[0].elapsed_time(e[1]), 4), ode_bwd_ms=round(e[1].elapsed_time(e[2]), 4))
    del graph, ws
    torch.cuda.empty_cache()
    return info


def cpu_protocol(dev) -> dict:
    """The FP64 oracle's per-frame forward and forward+backward times on this
    host, in its per-pixel definition and in its tiled form, next to the GPU's
    plain per-frame path on the same frames: the 128x128 frame of 2k Gaussians
    in full (all threads and one thread), one full 960x540 frame of 100k
    Gaussians, and the first two frames of the benchmark clip and of the
    1920x1080 clip of 500k Gaussians (for these two the per-pixel definition
    on a stated pixel sample, extrapolated by pixel count; the tiled form
    always on whole frames)."""
    import torch
    import gv_synth
    import oracle
    from paper_2501_04782_amd import raster
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    out = dict(host=host_info(), threads=threads, configs=[])

    def gpu_per_frame(w, frames):
        scene = raster.Scene.from_synth(w["scene"], dev)
        cam = raster.Camera.of(w["camera"])
        poses = torch.from_numpy(np.ascontiguousarray(w["poses"], np.float32)).to(dev)
        times = [float(x) for x in w["times"]]
        F, H, W = w["frames"], cam.height, cam.width
        ws1 = raster.Workspace(cam, scene.n, 1, 0, device=dev)
        kmax = max(int(raster.project_fwd(scene, cam, poses[f].contiguous(), times[f], ws1)[1].sum().item())
                   for f in frames)
        ws = raster.Workspace(cam, scene.n, 1, int(kmax * 1.25) + 4096, device=dev)
        tg = torch.rand(3, H, W, device=dev)
        img = torch.empty(3, H, W, device=dev)
        grads = raster.grad_buffers(scene)

        def step(f):
            raster.render_fwd(scene, cam, poses[f].contiguous(), times[f], ws, image=img)
            raster.render_bwd(scene, cam, poses[f].contiguous(), times[f], ws, img, target=tg,
                              loss_scale=2.0 / (3 * H * W), grads=grads)
        for f in frames:
            step(f)
        torch.cuda.synchronize()
        reps = 5
        t = time.perf_counter()
        for _ in range(reps):
            for f in frames:
                step(f)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / (reps * len(frames))

    def oracle_frame_times(w, f, nthreads, npx=None, seed=0, tile=0):
        H, W = w["camera"].height, w["camera"].width
        P = H * W
        rng = np.random.default_rng(seed)
        pix = None if npx is None else np.sort(rng.choice(P, npx, replace=False))
        n = P if npx is None else npx
        dl = rng.normal(0, 1, (n, 3)) * (2.0 / (3.0 * P))
        pose = w["poses"][f].astype(np.float64)
        t0 = time.perf_counter()
        oracle.render_frame(w["scene"], w["camera"], pose, float(w["times"][f]), pixels=pix, threads=nthreads,
                            tile=tile)
        t1 = time.perf_counter()
        oracle.render_frame(w["scene"], w["camera"], pose, float(w["times"][f]), pixels=pix, dL_dC=dl,
                            threads=nthreads, tile=tile)
        t2 = time.perf_counter()
        scale = P / n
        return (t1 - t0) * scale, (t2 - t1) * scale

    plan = [("frame128_n2k", [0], None, [threads, 1]), ("frame540p_n100k", [0], None, [threads]),
            ("clip540p_f50_n200k", [0, 1], 51840, [threads]), ("clip1080p_f32_n500k_bf16", [0, 1], 20736, [threads])]
    for name, frames, npx, thread_list in plan:
        w = gv_synth.make_workload(name, seed=0, targets=False)
        gpu_s = gpu_per_frame(w, frames)
        # the per-pixel definition (every pixel over every Gaussian), then the
        # tiled form (whole frames always)
        for form, tile, sample in (("per-pixel", 0, npx), ("tiled", 16, None)):
            for nt in thread_list:
                fw, fb = [], []
                for f in frames:
                    a, b = oracle_frame_times(w, f, nt, sample, tile=tile)
                    fw.append(a)
                    fb.append(b)
                    log(f"[cpu protocol] {name} {form} frame {f} threads {nt}: fwd {a:.2f} s, fwd+bwd {b:.2f} s")
                rec = dict(workload=name, form=form, frames=frames, threads=nt,
                           cpu_fwd_s_per_frame=round(float(np.mean(fw)), 4),
                           cpu_fwd_bwd_s_per_frame=round(float(np.mean(fb)), 4),
                           gpu_per_frame_fwd_bwd_ms=round(1e3 * gpu_s, 4),
                           gpu_over_cpu=round(float(np.mean(fb)) / gpu_s, 1))
                if sample is not None:
                    rec["sample"] = (f"{sample} random pixels per frame, times scaled by pixel count "
                                     f"({w['camera'].width * w['camera'].height} per frame)")
                out["configs"].append(rec)
    return out


def micro_benchmarks(scene_np, targets, dev):
    """HBM-bound helpers of the fitting loop: the fused Adan step over all
    parameters of the benchmark scene, the Gaussian pyramid of the clip's
    targets, and the visibility-count pass."""
    import torch
    from paper_2501_04782_amd import optim, raster
    out = {}
    params = [torch.from_numpy(np.ascontiguousarray(getattr(scene_np, k), dtype=np.float32)).to(dev)
              for k in scene_np.fields()]
    grads = [torch.randn_like(p) for p in params]
    opt = optim.Adan(params)
    opt.step(grads)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        opt.step(grads)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    n = sum(p.numel() for p in params)
    out["adan"] = dict(params=n, ms=round(ms, 4), bytes_per_param=44, gb_per_s=round(44 * n / ms / 1e6, 1),
                       hbm_frac=round(44 * n / (ms * 1e-3) / HBM_PEAK, 3))
    levels = 4
    raster.gaussian_pyramid(targets, levels)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(5):
        pyr = raster.gaussian_pyramid(targets, levels)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    moved = sum(4 * t.numel() for t in pyr[:-1]) + sum(4 * t.numel() for t in pyr[1:])
    out["pyramid"] = dict(levels=levels, frames=int(targets.shape[0]), ms=round(ms, 4),
                          gb_per_s=round(moved / ms / 1e6, 1), hbm_frac=round(moved / (ms * 1e-3) / HBM_PEAK, 3))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clip540p_f50_n200k")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-frame", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tuning", default=None,
                    help="batch,sort_cap,compact[,bwd_batch]: fixed tuning (skips the autotuner)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="target CPU time of the oracle sample")
    ap.add_argument("--stage-reps", type=int, default=5)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the secondary measurements (ODE fitting step, 1080p bf16 clip, dynamics, SH, "
                         "Adan, pyramid, visibility)")
    ap.add_argument("--cpu-protocol", action="store_true",
                    help="only time the FP64 oracle per frame on the host (four workloads, see cpu_protocol) next "
                         "to the GPU's per-frame path, print one JSON line and exit (several minutes)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (counter calibration) and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); the clip "
              "would shard by frames across GPUs with one gradient all-reduce, which this library does not run.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    ROOT = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, ROOT)
    import gv_synth
    from paper_2501_04782_amd import _lib, raster

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.rand(nbytes // 4, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "reps": 3}))
        return

    if args.cpu_protocol:
        print(json.dumps(cpu_protocol(dev)), flush=True)
        return

    log(f"[bench] building inputs: {args.workload}")
    w = gv_synth.make_workload(args.workload, seed=0, targets=True)
    F, N = w["frames"], w["n"]
    H, W = w["camera"].height, w["camera"].width
    P = H * W
    scene = raster.Scene.from_synth(w["scene"], dev)
    cam = raster.Camera.of(w["camera"])
    poses = torch.from_numpy(w["poses"]).to(dev)
    times = torch.from_numpy(w["times"]).to(dev)
    targets = torch.from_numpy(w["targets"]).to(dev)
    dtype_name = "bf16-params/f32" if w["scene"].dtype == "bf16" else "f32"
    # stored parameter bytes per Gaussian (static fields plus any dynamics / SH coefficients)
    read_fields = [k for k in w["scene"].fields() if not (k == "means" and w["scene"].ctrl is not None)]
    param_bytes = sum(getattr(w["scene"], k).nbytes for k in read_fields) / N
    grad_bytes = 4 * sum(getattr(w["scene"], k).size for k in read_fields) / N

    # capacity from the exact tile counts of three frames, and visible counts
    ws1 = raster.Workspace(cam, N, 1, 0, device=dev)
    vis, kf = [], []
    for f in sorted({0, F // 2, F - 1}):
        _, cnt = raster.project_fwd(scene, cam, poses[f].contiguous(), float(w["times"][f]), ws1)
        vis.append(int((cnt > 0).sum().item()))
        kf.append(int(cnt.sum().item()))
    cap = int(max(kf) * F * 1.25) + 4096
    ws = raster.Workspace(cam, N, F, cap, device=dev)
    log(f"[bench] workspace {ws.nbytes / 1e9:.2f} GB, capacity {cap}")

    tuning = raster.get_tuning()
    if args.tuning:
        raster.set_tuning(*(int(x) for x in args.tuning.split(",")))
        tuning = raster.get_tuning()
    elif not args.no_autotune:
        log("[bench] autotuning")
        tuning = raster.autotune(scene, cam, poses, times, ws, targets)
    log(f"[bench] tuning {tuning}")

    ode_info = None
    if args.workload == ODE_WORKLOAD:
        # learned camera (Eq. 1): targets are renders at the ground-truth
        # trajectory; one step integrates the ODE from (theta, z0 = frame-0
        # pose), renders all frames, back-propagates the L2 loss and runs the
        # ODE adjoint, captured in one graph
        from paper_2501_04782_amd import camera
        gt = raster.render_batch(scene, cam, poses, times, ws, forward=True, backward=False)
        targets = gt["images"].clone()
        rng_t = np.random.default_rng(7)
        theta = torch.from_numpy(gv_synth.init_mlp_theta(rng_t).astype(np.float32)).to(dev)
        z0 = poses[0].clone()
        ode_substeps = 4
        graph = camera.FitGraph(scene, cam, theta, z0, F, ode_substeps, times, ws, targets=targets)
        ows = camera.OdeWorkspace(F, ode_substeps, device=dev)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        camera.camera_ode_fwd(theta, z0, F, ode_substeps, ows)
        torch.cuda.synchronize()
        e0.record()
        p = camera.camera_ode_fwd(theta, z0, F, ode_substeps, ows)
        e1.record()
        camera.camera_ode_bwd(theta, z0, F, ode_substeps, torch.ones_like(p), ows)
        e2.record()
        torch.cuda.synchronize()
        ode_info = dict(fwd_ms=round(e0.elapsed_time(e1), 4), bwd_ms=round(e1.elapsed_time(e2), 4),
                        substeps=ode_substeps, mlp_evals=4 * ode_substeps * (F - 1))
        te = camera.pose_error(p, poses)
        ode_info["trajectory_error"] = dict(translation_rmse=round(te["translation_rmse"], 6),
                                            mean_angle_rad=round(te["mean_angle"], 6),
                                            of="ODE poses at the initial theta vs the ground-truth pose table")
        log(f"[bench] camera ODE: {ode_info}")
    else:
        graph = raster.BatchGraph(scene, cam, poses, times, ws, targets=targets)
    for _ in range(args.warmup):
        graph.launch()
    torch.cuda.synchronize()
    st = ws.status()
    if st["overflow"]:
        raise RuntimeError(f"intersection capacity overflow: {st}")
    K = st["intersections"]
    V = float(np.mean(vis))
    log(f"[bench] intersections per step {K} ({K / F:.0f} per frame), visible ~{V:.0f}")

    # timed region: K graph launches, one fwd+bwd step each
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.launch()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = 1e3 * elapsed / args.steps
    fps = F * args.steps / elapsed
    log(f"[bench] batched: {ms_step:.3f} ms/step, {fps:.1f} frames/s")
    loss_val = float(graph.loss.double().sum())

    # per-stage durations (HIP events on the launch stream, eager sequence)
    stage_ms = {}
    out = dict(images=graph.images, loss=graph.loss, grads=graph.grads, dL_dposes=graph.dL_dposes)
    for r in range(args.stage_reps + 1):
        res = raster.render_batch_timed(scene, cam, poses, times, ws, targets=targets, out=out)
        if r == 0:
            continue  # warm
        for k, v in res["stage_ms"].items():
            stage_ms[k] = stage_ms.get(k, 0.0) + v / args.stage_reps
    log(f"[bench] stages (ms): " + ", ".join(f"{k}={v:.3f}" for k, v in stage_ms.items()))

    # plain per-frame path on the same clip (render_fwd reads K back each frame)
    per_frame = None
    if not args.no_per_frame and ode_info is None:
        wsf = raster.Workspace(cam, N, 1, int(max(kf) * 1.25) + 4096, device=dev)
        grads = raster.grad_buffers(scene)
        scale = 2.0 / (3.0 * P * F)
        img = torch.empty(3, H, W, device=dev)
        tms = [float(x) for x in w["times"]]

        def per_frame_clip():
            for f in range(F):
                raster.render_fwd(scene, cam, poses[f], tms[f], wsf, image=img)
                raster.render_bwd(scene, cam, poses[f], tms[f], wsf, img, target=targets[f], loss_scale=scale,
                                  grads=grads, accumulate=f > 0)

        per_frame_clip()
        torch.cuda.synchronize()
        reps = 2
        t0 = time.perf_counter()
        for _ in range(reps):
            per_frame_clip()
        torch.cuda.synchronize()
        pf_elapsed = time.perf_counter() - t0
        pf_fps = F * reps / pf_elapsed
        per_frame = dict(value=round(pf_fps, 2), unit="frames/s", ms_per_clip=round(1e3 * pf_elapsed / reps, 3),
                         batched_speedup=round(fps / pf_fps, 3))
        log(f"[bench] per-frame path: {pf_fps:.1f} frames/s (batched x{fps / pf_fps:.2f})")

    # CPU baseline: the FP64 oracle in its tiled form (results identical to
    # its per-pixel definition) on whole frames of the clip, forward and
    # backward, as many as fit in the time budget (at least five, spread over
    # the clip).  Its contributor counts give the number of contributing
    # (pixel, Gaussian) pairs the compositing kernels' operations are priced on.
    cpu = None
    mean_contrib = None
    if not args.no_cpu_baseline:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
        host = host_info()
        spread = [0, F - 1, F // 2, F // 4, (3 * F) // 4]
        order = list(dict.fromkeys(spread + list(range(F))))
        rng = np.random.default_rng(1)
        dl = rng.normal(0, 1, (P, 3)) * (2.0 / (3.0 * P * F))
        t_cpu, done, nc = 0.0, [], []
        log("[bench] CPU oracle (tiled form, whole frames)")
        for f in order:
            t = time.perf_counter()
            r = oracle.render_frame(w["scene"], w["camera"], w["poses"][f].astype(np.float64), float(w["times"][f]),
                                    dL_dC=dl, threads=threads, tile=16)
            t_cpu += time.perf_counter() - t
            done.append(f)
            nc.append(float(np.mean(r["n_contrib"])))
            if len(done) >= len(spread) and t_cpu >= args.cpu_seconds:
                break
        mean_contrib = float(np.mean(nc))
        cpu_fps = len(done) / t_cpu
        cpu = dict(value=cpu_fps, unit="frames/s", cores=threads, kind="oracle",
                   sample=f"{len(done)} whole frames of the clip (first frames {done[:5]}), forward+backward incl. "
                          f"projection, binning and depth sort of all {N} Gaussians per frame, {t_cpu:.1f} s; "
                          "the oracle's tiled form (each pixel visits its 16x16 tile's candidates; results "
                          "identical to the per-pixel definition)", host=host)
        log(f"[bench] CPU oracle: {cpu_fps:.3f} frames/s on {threads} threads ({host})")

    # roofline of the dominant kernel, priced on the hot-path table's
    # per-unit figures: bytes per pixel and per intersection, operations per
    # contributing pair (E = the oracle's mean contributors per pixel x P x F)
    dom = max(stage_ms, key=stage_ms.get)
    t_dom = stage_ms[dom] / 1e3
    from paper_2501_04782_amd import rocprof_summary
    key = rocprof_summary.stage_key(dom, tuning)
    traffic = rocprof_summary.read_traffic(
        os.path.join(ROOT, "profiles", f"{dom}_{args.workload}_{key}_hbm_traffic.txt"), dom, args.workload, key)
    counters = rocprof_summary.read_counters(
        os.path.join(ROOT, "profiles", f"{dom}_{args.workload}_{key}_sq.txt"), dom, args.workload, key)
    bytes_dom = stage_bytes(dom, N, V, K, P, F, param_bytes)
    hbm_ach = bytes_dom / t_dom if bytes_dom else 0.0
    roof = dict(bound="hbm", achieved=round(hbm_ach / 1e9, 2), peak=HBM_PEAK / 1e9, unit="GB/s",
                frac=round(hbm_ach / HBM_PEAK, 4), traffic=traffic, kernel=dom,
                avg_ms=round(stage_ms[dom], 4), algorithmic_bytes=int(bytes_dom))
    if mean_contrib is not None and dom in ("composite_fwd", "composite_bwd"):
        pairs = mean_contrib * P * F
        per_pair = FLOPS_FWD_PER_PAIR if dom == "composite_fwd" else FLOPS_BWD_PER_PAIR
        alu_ach = pairs * per_pair / t_dom
        alu = dict(alu_frac=round(alu_ach / ALU_PEAK, 4), alu_frac_nonpacked=round(alu_ach / ALU_PEAK_NONPACKED, 4),
                   alu_peak_nonpacked=round(ALU_PEAK_NONPACKED / 1e12, 2), flops_per_pair=per_pair,
                   contributing_pairs=int(pairs))
        if alu_ach / ALU_PEAK > hbm_ach / HBM_PEAK:
            roof = dict(bound="alu", achieved=round(alu_ach / 1e12, 3), peak=round(ALU_PEAK / 1e12, 2),
                        unit="TFLOP/s", frac=round(alu_ach / ALU_PEAK, 4), traffic=traffic, kernel=dom,
                        avg_ms=round(stage_ms[dom], 4), algorithmic_bytes=int(bytes_dom),
                        hbm_frac=round(hbm_ach / HBM_PEAK, 4))
        roof.update(alu)
        if counters is not None:
            roof["profile"] = counters_summary(counters, pairs)
    elif counters is not None:
        roof["profile"] = counters_summary(counters, None)
    b_alg = algorithmic_bytes(N, V, K, P, F, param_bytes, grad_bytes)

    extras = None
    if not args.no_extras and ode_info is None and args.workload == "clip540p_f50_n200k":
        log("[bench] secondary measurements")
        extras = micro_benchmarks(w["scene"], targets, dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        raster.visibility_counts(scene, cam, poses, times, ws)
        torch.cuda.synchronize()
        e0.record()
        raster.visibility_counts(scene, cam, poses, times, ws)
        e1.record()
        torch.cuda.synchronize()
        extras["visibility_counts"] = dict(frames=F, ms=round(e0.elapsed_time(e1), 3),
                                           note="projection + binning + sort + flagging forward + count")
        graph.close()
        graph = None
        torch.cuda.empty_cache()
        extras["workloads"] = []
        for name in (ODE_WORKLOAD, "clip1080p_f32_n500k_bf16", "clip540p_f50_n200k_dyn", "clip540p_f50_n200k_sh3"):
            log(f"[bench] {name}")
            extras["workloads"].append(quick_clip(name, dev))
        log(f"[bench] extras: {extras}")
    step_hbm_frac = b_alg / (ms_step / 1e3) / HBM_PEAK

    line = {
        "metric": METRIC,
        "value": round(fps, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "width": W, "height": H, "gaussians": N, "frames_per_step": F,
                   "loss": "l2", "path": "batched, one HIP graph per step", "param_dtype": dtype_name},
        "gaussians_per_s": round(fps * N, 1),
        "hbm_roof_frac_step": round(step_hbm_frac, 4),
        "algorithmic_bytes_per_frame": int(b_alg / F),
        "per_frame_path": per_frame,
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "intersections_per_frame": int(K / F),
        "tuning": tuning,
        "loss": loss_val,
        "roofline": roof,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    if mean_contrib is not None:
        line["mean_contributors_per_pixel"] = round(mean_contrib, 3)
    if ode_info is not None:
        line["camera_ode"] = ode_info
        line["config"]["path"] = "camera ODE fwd -> batched raster fwd+bwd -> ODE adjoint, one HIP graph per step"
    print(json.dumps(line), flush=True)
    if graph is not None:
        graph.close()


if __name__ == "__main__":
    main()
