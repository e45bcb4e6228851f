/*
 * gv.h -- C ABI of the MI355X (gfx950) differentiable Gaussian rasterizer.
 *
 * The library renders 3D Gaussians (paper Sec. 3.1: mean mu, covariance
 * Sigma = (R S)(R S)^T from a rotation quaternion and per-axis scales, colour c,
 * opacity o) through a pinhole camera with constant intrinsics and per-frame
 * extrinsics (Sec. 3.4), fits them with the L2 reconstruction loss (Sec. 4.1),
 * and returns gradients through a hand-written adjoint.  The rasterizer is the
 * tile-based one of 3D Gaussian Splatting that Sec. 3.1 cites: EWA projection,
 * 16x16 tile binning with a per-tile depth sort, front-to-back alpha
 * compositing (alpha <= 0.99, entries with alpha < 1/255 skipped, a pixel stops
 * before its transmittance drops below 1e-4, footprint cut at q = 9, i.e. 3
 * sigma).  The camera extrinsics may come from the camera-motion Neural ODE of
 * Eq. 1 (gv_camera_ode_*).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Memory: every array argument is a DEVICE pointer owned by the caller,
 *   except the gv_camera / gv_scene / gv_grads / gv_tuning structs themselves
 *   and explicitly marked host outputs.  The library never allocates device
 *   memory for rendering; scratch space is the caller's workspace `ws`, sized
 *   by gv_workspace_bytes.  Arrays are planar: parameters [C][N], images
 *   [F][3][H][W] (row-major), poses [F][7].
 * - Poses are world->camera: (qw, qx, qy, qz, tx, ty, tz); the quaternion need
 *   not be normalised (it is normalised inside, and its gradient is that of
 *   the unnormalised input).  Pixel (x, y) has its centre at (x+1/2, y+1/2).
 * - Streams: `stream` is a hipStream_t (NULL = the null stream).  All work is
 *   enqueued on it; calls return after enqueueing.  Only gv_render_fwd (one
 *   blocking read of the intersection count), gv_device_status and
 *   gv_autotune synchronise.
 * - Errors: a gv_status return code, never an abort or exception.  Arguments
 *   are validated on the host before anything is enqueued.  Device-side
 *   conditions (intersection capacity exceeded, non-finite parameters) are
 *   recorded in a status word inside the workspace (gv_device_status).
 * - Reentrancy: calls with distinct workspaces may run concurrently on
 *   different streams.  Two calls sharing one workspace must be ordered.
 */
#ifndef GV_H
#define GV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GV_OK = 0,
    GV_ERR_INVALID_ARG = 1, /* a null pointer, a non-positive size, an unknown flag or dtype */
    GV_ERR_WORKSPACE = 2,   /* the workspace is smaller than gv_workspace_bytes requires */
    GV_ERR_CAPACITY = 3,    /* more (Gaussian, tile) intersections than the workspace holds */
    GV_ERR_HIP = 4,         /* a HIP runtime call failed (the HIP error is in gv_last_hip_error) */
    GV_ERR_UNSUPPORTED = 5  /* e.g. no gfx950 device */
} gv_status;

typedef enum { GV_F32 = 0, GV_BF16 = 1 } gv_dtype;

/* Pinhole intrinsics shared by all frames of a clip (Sec. 3.4), plus the
 * rasterizer constants: near-plane depth below which a Gaussian is dropped,
 * the low-pass term added to the diagonal of every projected 2D covariance,
 * and the background colour composited behind the last Gaussian. */
typedef struct {
    int32_t width, height;  /* pixels, 1 .. 16384 each */
    float fx, fy, cx, cy;   /* focal lengths and principal point, in pixels */
    float near_plane;       /* > 0; default 0.01 */
    float dilation;         /* >= 0; default 0.3 (pixel^2) */
    float bg[3];            /* background RGB */
} gv_camera;

/* Gaussian parameters in their stored parameterisation, planar [C][N]
 * (Sec. 3.1 and Eq. 3): means [3][N] (mu0 when mean_coeffs is set),
 * log-scales [3][N] (s = exp), quaternions [4][N] (w, x, y, z; normalised
 * inside), opacity logits [N] (o = sigmoid), RGB colours [3][N] (constant in
 * time, Eq. 3).  dtype GV_F32: float arrays; GV_BF16: bfloat16 bit patterns
 * (uint16), widened to FP32/FP64 on load.
 *
 * Optional time dependence, evaluated at each frame's time t (Sec. 3.2):
 * - mean_coeffs [3 coeff][3 xyz][N]: the cubic mean
 *   mu(t) = mu0 + a1 t + a2 t^2 + a3 t^3 (the polynomial motion basis);
 * - n_ctrl = M (4 .. GV_MAX_CTRL) and ctrl [M][3 xyz][N]: the clamped cubic
 *   B-spline mean of Eq. 2, mu(t) = sum_i N_{i,3}(t) P_i, with four knots at
 *   0, four at 1 and M - 4 evenly spaced between; `means` is then ignored
 *   (may be NULL) and every frame time must lie in [0, 1] (a Gaussian is
 *   dropped in a frame whose time does not);
 * - scale_coeffs [3 coeff][3][N] and quat_coeffs [3 coeff][4][N]: cubic
 *   polynomials for the log-scales and the quaternion (Eq. 3),
 *   l(t) = l0 + b1 t + b2 t^2 + b3 t^3 and q(t) = q0 + r1 t + r2 t^2 + r3 t^3
 *   (normalised after evaluation).
 * mean_coeffs and ctrl exclude each other.  NULL / 0 = absent.
 *
 * Optional view-dependent colour (Sec. 3.1: colour as spherical harmonics of
 * degree d_c): sh_degree D in 1..3 and sh [(D+1)^2 - 1][3 rgb][N], the real
 * SH coefficients k_lm of degrees 1..D in (l, m) ascending order; the colour
 * seen from a frame's camera is colors + sum_lm k_lm Y_lm(d), d the unit
 * vector from the camera centre (-Rc^T tc) to the mean; `colors` is the
 * degree-0 term (raw RGB, no offset, no clamp). */
#define GV_MAX_CTRL 64
#define GV_MAX_SH_DEGREE 3
typedef struct {
    int64_t n;              /* number of Gaussians, 0 .. 2^31-1 */
    int32_t dtype;          /* gv_dtype */
    const void *means;
    const void *log_scales;
    const void *quats;
    const void *opacity_logits;
    const void *colors;
    const void *mean_coeffs; /* may be NULL */
    int32_t n_ctrl;          /* 0, or 4 .. GV_MAX_CTRL */
    const void *ctrl;        /* NULL, or [n_ctrl][3][N] */
    const void *scale_coeffs;/* may be NULL */
    const void *quat_coeffs; /* may be NULL */
    int32_t sh_degree;       /* 0 (RGB only) .. GV_MAX_SH_DEGREE */
    const void *sh;          /* NULL, or [(sh_degree+1)^2 - 1][3][N] */
} gv_scene;

/* FP32 gradient outputs, same layouts as gv_scene (always FP32, even for bf16
 * parameters).  A NULL member skips that output; members for parameters the
 * scene does not have are ignored.  With control points, `means` receives
 * nothing (the gradient goes to `ctrl`). */
typedef struct {
    float *means;
    float *log_scales;
    float *quats;
    float *opacity_logits;
    float *colors;
    float *mean_coeffs;
    float *ctrl;
    float *scale_coeffs;
    float *quat_coeffs;
    float *sh;
    float *intrinsics;  /* [4]: dL/d(fx, fy, cx, cy), shared by all frames (Sec. 3.4) */
} gv_grads;

/* Flags for gv_render_batch / gv_render_bwd. */
#define GV_FWD 1u        /* forward: images (+ loss with GV_LOSS_L2) */
#define GV_BWD 2u        /* backward: gradients */
#define GV_LOSS_L2 4u    /* loss = mean over (F,3,H,W) of (image - target)^2 (Sec. 4.1), fused */
#define GV_ACCUMULATE 8u /* add gradients into `grads` instead of overwriting them */

/* Tunables of the rasterizer kernels (chosen by gv_autotune, or set directly).
 * batch: entries staged in LDS per round of a tile's compositing loop
 * (64, 128 or 256); sort_cap: longest per-tile list sorted in one LDS pass
 * (512, 1024, 2048 or 4096; lists up to twice that merge two LDS-sorted
 * runs, longer lists are sorted in chunks and merged in global memory);
 * compact: compositing kernel choice, 0..63.  With bit 2 set the forward lets
 * each wave walk the entries meeting its 8x8 quadrant; with it clear each
 * 16-lane row of a wave walks the entries meeting its 4x4 pixel block; with
 * bit 5 set, which takes precedence over bit 2, one wave owns the tile and
 * each 16-lane row walks one quadrant's entries (four pixels per lane;
 * batches of 64 or 128, a batch of 256 runs as 128).  The
 * backward lets each wave walk one quadrant's entries (one pixel per lane),
 * with bit 3 set two quadrants' entries, one per half-wave (two pixels per
 * lane; batches of 64 or 128, a bwd_batch of 256 runs as 128), or with bit
 * 4 set, which takes precedence over bit 3, all four quadrants' entries,
 * one per 16-lane row (one wave per tile, four pixels per lane; batches of
 * 64 whatever bwd_batch says).  Bit 0 (forward) / bit 1 (backward), which
 * take precedence, select kernels that first build per-pixel entry lists
 * from closed-form coverage masks;
 * bwd_batch: the backward's LDS batch (0 = same as batch).
 * Defaults: batch 128, sort_cap 1024, compact 52, bwd_batch 64.  Images are
 * identical under every setting and gradients equal up to floating-point
 * rounding (order of summation, and the compacted backward's arithmetic);
 * only the speed differs. */
typedef struct {
    int32_t batch;
    int32_t sort_cap;
    int32_t compact;
    int32_t bwd_batch;
    int32_t reserved[4];
} gv_tuning;

/* Bytes of workspace for up to `frames` frames of `n` Gaussians at the
 * camera's resolution, with room for `k_capacity` (Gaussian, tile)
 * intersections over all frames (a 16x16 tile grid; a typical random scene
 * at 960x540 has about 4 intersections per visible Gaussian per frame). */
gv_status gv_workspace_bytes(const gv_camera *cam, int64_t n, int32_t frames, int64_t k_capacity,
                             size_t *out_bytes);

/* Largest intersection capacity a workspace of ws_bytes offers. */
gv_status gv_workspace_capacity(const gv_camera *cam, int64_t n, int32_t frames, size_t ws_bytes,
                                int64_t *out_k_capacity);

/* Projection only (EWA step of Sec. 3.1 as in 3DGS), for inspection: per
 * Gaussian, records[g][8] = (u, v, A00, A01, A11, depth, opacity, 0) where
 * (u, v) is the projected mean in pixels, A the conic (inverse of the dilated
 * 2D covariance), depth the camera-space z; tile_counts[g] = number of 16x16
 * tiles its 3-sigma ellipse meets (0 = culled).  pose7: device [7]; t: the
 * frame time of the cubic mean.  Needs a workspace for frames = 1. */
gv_status gv_project_fwd(const gv_scene *scene, const gv_camera *cam, const float *pose7, float t,
                         float *records, int32_t *tile_counts, void *ws, size_t ws_bytes, void *stream);

/* Forward render of one frame (the plain per-frame path).  image [3][H][W];
 * T_final [H][W] (final transmittance) may be NULL.  Reads the intersection
 * count back to the host once (synchronises `stream`) and returns
 * GV_ERR_CAPACITY, with nothing rendered, if it exceeds the workspace.
 * The workspace then holds what gv_render_bwd needs. */
gv_status gv_render_fwd(const gv_scene *scene, const gv_camera *cam, const float *pose7, float t,
                        float *image, float *T_final, void *ws, size_t ws_bytes, void *stream);

/* gv_render_fwd without a workspace argument, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation.  The call allocates nothing: its scratch
 * space is a fixed device array of GV_NOALLOC_SCRATCH_BYTES (64 MiB) inside
 * the library, one per GPU (each device holds its own copy until the process
 * ends).  Arguments, outputs, the one synchronisation and the error codes are
 * those of gv_render_fwd, plus: GV_ERR_WORKSPACE (nothing enqueued) when the
 * frame's fixed arrays exceed the scratch (about 141 B per Gaussian, 8 B per
 * pixel and 12 B per 16x16 tile), GV_ERR_CAPACITY when its (Gaussian, tile)
 * intersections do not fit in the rest (76 B and one bit each).  All calls on one GPU
 * share that GPU's array: calls that overlap on one GPU (from different
 * streams or host threads) race and must be ordered by the caller.  The
 * array keeps the last call's contents; every value a call reads is written
 * by that call first (counters are cleared by fill kernels). */
#define GV_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
gv_status gv_render_fwd_noalloc(const gv_scene *scene, const gv_camera *cam, const float *pose7, float t,
                                float *image, float *T_final, void *stream);

/* Backward of the last gv_render_fwd on this workspace (same scene, camera,
 * pose, t and image buffer).  Upstream gradient: dL_dimage [3][H][W], or,
 * with GV_LOSS_L2 in flags, the gradient of the L2 loss against `target`
 * [3][H][W] scaled by loss_scale (2/(3HW) for the mean over one frame).
 * Gradients are written to `grads` (added with GV_ACCUMULATE); dL_dpose7 [7]
 * may be NULL.  Transmittances are recomputed back to front from the stored
 * final transmittance; nothing else per pixel is kept from the forward pass. */
gv_status gv_render_bwd(const gv_scene *scene, const gv_camera *cam, const float *pose7, float t,
                        const float *image, const float *dL_dimage, const float *target, float loss_scale,
                        uint32_t flags, gv_grads *grads, float *dL_dpose7, void *ws, size_t ws_bytes,
                        void *stream);

/* All frames of a clip in one launch sequence, without host synchronisation
 * (batched form; capturable into a HIP graph).  poses [F][7] and times [F]
 * (cubic-mean time of each frame; NULL = all 0) are device arrays.
 * flags: GV_FWD and/or GV_BWD.  GV_FWD renders images [F][3][H][W]; with
 * GV_LOSS_L2 it also writes loss[F], each frame's share of the mean over all
 * F*3*H*W values of (image - target)^2 (targets [F][3][H][W]).  GV_BWD
 * back-propagates either that loss (GV_LOSS_L2) or an explicit upstream
 * gradient dL_dimages [F][3][H][W]; without GV_FWD in the same call it is the
 * backward of the last forward on this workspace (same arguments, `images`
 * holding its output).  grads: SUM over frames of the shared parameters'
 * gradients (overwritten, or added with GV_ACCUMULATE); dL_dposes [F][7] per
 * frame (may be NULL).  An intersection overflow is reported through
 * gv_device_status; outputs are then undefined and the call must be repeated
 * with a larger workspace. */
gv_status gv_render_batch(const gv_scene *scene, const gv_camera *cam, const float *poses, const float *times,
                          int32_t frames, const float *targets, const float *dL_dimages, uint32_t flags,
                          float *images, float *loss, gv_grads *grads, float *dL_dposes, void *ws,
                          size_t ws_bytes, void *stream);

/* gv_render_batch with HIP events recorded on `stream` between its stages,
 * for measurement.  Synchronises; stage_ms[GV_STAGES] (host) receives each
 * stage's elapsed time in ms: 0 projection (+ clearing the counters),
 * 1 prefix sums, 2 key scatter, 3 per-tile sort, 4 forward compositing,
 * 5 loss reduction, 6 backward compositing, 7 projection adjoint (+ pose
 * reduction).  Stages a call does not run read 0. */
#define GV_STAGES 8
gv_status gv_render_batch_timed(const gv_scene *scene, const gv_camera *cam, const float *poses, const float *times,
                                int32_t frames, const float *targets, const float *dL_dimages, uint32_t flags,
                                float *images, float *loss, gv_grads *grads, float *dL_dposes, void *ws,
                                size_t ws_bytes, void *stream, float *stage_ms);

/* Capture one gv_render_batch call (same arguments; every pointer is baked
 * in) into an executable HIP graph; launch it any number of times; destroy
 * it.  Capture happens on a private stream; nothing runs at creation. */
typedef struct gv_graph gv_graph;
gv_status gv_batch_graph_create(const gv_scene *scene, const gv_camera *cam, const float *poses,
                                const float *times, int32_t frames, const float *targets,
                                const float *dL_dimages, uint32_t flags, float *images, float *loss,
                                gv_grads *grads, float *dL_dposes, void *ws, size_t ws_bytes, gv_graph **out);
gv_status gv_batch_graph_launch(gv_graph *graph, void *stream);
gv_status gv_batch_graph_destroy(gv_graph *graph);

/* Camera-motion Neural ODE (Eq. 1, Sec. 3.4): state z = (qw,qx,qy,qz,tx,ty,tz),
 * dz/dt = W3 tanh(W2 tanh(W1 [z; t] + b1) + b2) + b3 with an 8->64->64->7
 * MLP; theta [5191] = W1[64][8], b1[64], W2[64][64], b2[64], W3[7][64], b3[7]
 * (device, fp32).  Classic RK4 with `substeps` steps per frame interval over
 * t in [0, 1] (frame f at t = f/(F-1)); poses [F][7] = (q/|q|, t) of the state
 * at each frame.  gv_camera_ode_bwd is the discrete adjoint (the exact
 * gradient of the computed RK4 trajectory) given dL_dposes [F][7]; it writes
 * dtheta [5191] and dz0 [7] (overwritten) and needs the workspace of the
 * matching forward call. */
gv_status gv_camera_ode_workspace_bytes(int32_t frames, int32_t substeps, size_t *out_bytes);
gv_status gv_camera_ode_fwd(const float *theta, const float *z0, int32_t frames, int32_t substeps, float *poses,
                            void *ws, size_t ws_bytes, void *stream);
gv_status gv_camera_ode_bwd(const float *theta, const float *z0, int32_t frames, int32_t substeps,
                            const float *dL_dposes, float *dtheta, float *dz0, void *ws, size_t ws_bytes,
                            void *stream);

/* Trajectory error of a camera path against a reference pose table (Sec. 3.4:
 * the learned camera of Eq. 1 judged by per-frame poses).  poses and
 * ref_poses: device [frames][7] world->camera (qw, qx, qy, qz, tx, ty, tz),
 * quaternions need not be unit.  Per frame f (device, [frames][2], fp32):
 * per_frame[2f] = distance between the camera centres -R^T t, per_frame[2f+1]
 * = angle (radians, in [0, pi]) of the relative rotation R R_ref^T.
 * summary (device, [2]): root mean square of the centre distances and mean
 * angle.  Computed in FP64; stream-ordered, no synchronisation.
 * GV_ERR_INVALID_ARG for null pointers or frames outside [1, 100000]. */
gv_status gv_pose_error(const float *poses, const float *ref_poses, int32_t frames, float *per_frame,
                        float *summary, void *stream);

/* One fitting step of the learned-camera form, captured into one HIP graph
 * (launch/destroy with gv_batch_graph_launch / gv_batch_graph_destroy):
 * gv_camera_ode_fwd (theta, z0 -> poses [F][7]), then gv_render_batch with
 * GV_FWD | GV_BWD on those poses (GV_LOSS_L2 with targets, or an explicit
 * dL_dimages: exactly one of the two is given), then gv_camera_ode_bwd
 * (dL_dposes -> dtheta [5191], dz0 [7]).  Everything stays on the device
 * (Sec. 3.4: camera and renderer are integrated to avoid transfers). */
gv_status gv_fit_graph_create(const gv_scene *scene, const gv_camera *cam, const float *theta, const float *z0,
                              int32_t substeps, void *ode_ws, size_t ode_ws_bytes, const float *times, int32_t frames,
                              const float *targets, const float *dL_dimages, float *poses, float *images, float *loss,
                              gv_grads *grads, float *dL_dposes, float *dtheta, float *dz0, void *ws, size_t ws_bytes,
                              gv_graph **out);

/* Tunables: read/set the process-wide table.  gv_autotune installs the
 * fastest setting for the given batch problem.  With cache_path, it first
 * looks there for a line with this problem's key (device architecture,
 * width, height, N to a quarter octave, frames, parameter dtype, dynamics,
 * SH degree) and installs that line's setting without timing anything;
 * otherwise it times the options of each stage (forward kernel x LDS batch,
 * backward LDS batch, sort capacity: nine runs per round, three timed rounds
 * after a warm-up round, each stage keeping its own fastest option since no
 * stage's output depends on another's kernel) by running gv_render_batch on
 * the caller's buffers (overwriting its outputs; synchronises) and, with
 * cache_path, appends the choice as one JSON line.  `chosen` (host, or NULL)
 * receives the installed setting. */
gv_status gv_get_tuning(gv_tuning *out);
gv_status gv_set_tuning(const gv_tuning *t);
gv_status gv_autotune(const gv_scene *scene, const gv_camera *cam, const float *poses, const float *times,
                      int32_t frames, const float *targets, float *images, float *loss, gv_grads *grads,
                      float *dL_dposes, void *ws, size_t ws_bytes, const char *cache_path, gv_tuning *chosen);

/* Device status word of a workspace (host outputs; synchronises the device):
 * out[0] = 1 if the intersection capacity overflowed (2: internal binning
 * inconsistency; outputs invalid), out[1] = number of (frame, Gaussian)
 * pairs skipped for non-finite parameters in the last call's projection (a
 * Gaussian with a NaN or infinite parameter is dropped and counted once per
 * frame; its gradients are zero), out[2..3] =
 * low/high 32 bits of the intersection count of the last projection. */
gv_status gv_device_status(const void *ws, uint32_t out[4]);

/* Per-Gaussian visibility counts (Sec. 4.1: Gaussians that appear in no
 * frame are periodically moved): renders the frames like gv_render_batch with
 * GV_FWD (images [F][3][H][W] are written) and sets counts[g] (device, [N])
 * to the number of frames in which Gaussian g contributes to at least one
 * pixel (alpha >= 1/255 inside its 3-sigma ellipse, before the pixel's
 * termination).  Same workspace and argument rules as gv_render_batch. */
gv_status gv_visibility_counts(const gv_scene *scene, const gv_camera *cam, const float *poses, const float *times,
                               int32_t frames, float *images, uint32_t *counts, void *ws, size_t ws_bytes,
                               void *stream);

/* Gaussian pyramid of target frames for the spatial hierarchy (Sec. 3.3):
 * level 0 is `images` ([planes][H][W] FP32, e.g. planes = 3F); level l+1 is
 * level l convolved with the separable binomial filter [1 4 6 4 1]/16
 * (borders mirrored without repeating the edge sample) and decimated to its
 * even rows and columns, size ceil(H/2) x ceil(W/2).  `out` (device) receives
 * levels 1 .. levels-1 one after the other, each [planes][H_l][W_l];
 * gv_pyramid_floats gives its length.  levels 1..16. */
gv_status gv_pyramid_floats(int64_t planes, int32_t height, int32_t width, int32_t levels, int64_t *out_count);
gv_status gv_gaussian_pyramid(const float *images, int64_t planes, int32_t height, int32_t width, int32_t levels,
                              float *out, void *stream);

/* Fused Adan step (Sec. 4.1 trains with Adan: learning rate 0.01, decayed
 * by 0.99995 per step; the schedule is the caller's, who passes this step's
 * lr).  Per element, with g the gradient and (m, v, n, g_prev) the state:
 *   step 0:  m = g, v = 0, n = g^2
 *   step k:  m = (1-b1) m + b1 g;  v = (1-b2) v + b2 (g - g_prev) (step 1:
 *            v = g - g_prev);  n = (1-b3) n + b3 (g + (1-b2)(g - g_prev))^2
 *   theta = (theta - lr / sqrt(n + eps) * (m + (1-b2) v)) / (1 + wd * lr)
 * and g_prev = g.  Up to GV_ADAN_MAX_TENSORS tensors in one launch: the
 * pointer and count arrays are HOST arrays of n_tensors entries; params[t]
 * (FP32, updated in place), grads[t] (FP32) and states[t] ([4][counts[t]]
 * FP32, contents ignored at step 0) are device arrays.  Enqueued on `stream`;
 * GV_ERR_INVALID_ARG for a bad count, pointer or hyper-parameter. */
#define GV_ADAN_MAX_TENSORS 16
typedef struct {
    float lr, beta1, beta2, beta3, eps, weight_decay;
    int32_t step;     /* 0-based iteration */
    int32_t reserved;
} gv_adan_params;
gv_status gv_adan_step(int32_t n_tensors, float *const *params, const float *const *grads, float *const *states,
                       const int64_t *counts, const gv_adan_params *hp, void *stream);

const char *gv_status_str(gv_status s);
int32_t gv_last_hip_error(void);
/* Version of this interface: 5 (2: B-spline / polynomial dynamics and
 * bwd_batch; 3: spherical-harmonics colour; 4: intrinsics gradient, Adan;
 * 5: visibility counts, Gaussian pyramid). */
int32_t gv_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GV_H */
