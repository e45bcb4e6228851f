// Internal declarations of the gfx950 rasterizer: workspace layout, kernel
// argument block, device helpers.  Not part of the public ABI (include/gv.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "gv.h"

namespace gv {

// 16x16 pixel tiles; a 256-thread workgroup owns one tile, each of its four
// waves one 8x8 quadrant, each lane one pixel.
constexpr int TILE = 16;
constexpr int WG = 256;

// Compositing constants of the 3DGS forward model.
constexpr float ALPHA_MAX = 0.99f;
constexpr float ALPHA_MIN = 1.0f / 255.0f;
constexpr float T_MIN = 1e-4f;
constexpr float Q_MAX = 9.0f;
// -0.5 * log2(e): exp(-q/2) = exp2(q * K_EXP)
constexpr float K_EXP = -0.72134752044448170368f;

// Conservative slack of the binning tests relative to the per-pixel test
// (which runs in fp32 on the same rounded conic).
constexpr double BIN_Q_SLACK = 9.0 * (1.0 + 1e-5) + 1e-6;
constexpr float SUB_Q_SLACK = 9.0f * (1.0f + 1e-4f) + 1e-4f;

// Gaussians per workgroup of the LDS-histogram binning kernels, and the
// largest tile grid whose histogram fits in LDS (64 KiB).
constexpr int BIN_GROUP = 1024;
constexpr int LDS_TILE_LIMIT = 16384;

// Per (frame, Gaussian) projected record, 32 bytes (one aligned half-line).
// (u, v) stays in fp64 so that the tile-local offsets formed at staging time
// are exact to fp32 rounding of a small number.
// Partials of one (Gaussian, tile) pair, stored contiguously per pre-sort
// slot so that a Gaussian's tiles share cache lines.
constexpr int PART = 9;

__device__ __forceinline__ void store_partials(float* part, uint32_t slot, const float (&v)[PART]) {
    float* p = part + static_cast<int64_t>(slot) * PART;
#pragma unroll
    for (int k = 0; k < PART; ++k) p[k] = v[k];
}

// A binned intersection: 64-bit sort key (fp32 depth bits << 32 | Gaussian
// index) and the pre-sort slot of its partial gradients, written by the
// scatter as one 16-byte store.
struct __align__(16) KeySlot {
    uint64_t key;
    uint32_t slot;
    uint32_t pad;
};

struct __align__(32) Record {
    double u, v;
    float a, b, c;   // conic A = [[a, b], [b, c]]
    float depth;     // camera-space z rounded to fp32 (the sort key)
};

// Per Gaussian, shared by all frames: RGB + opacity.
struct __align__(16) ColorOp {
    float r, g, b, o;
};

// Status word at the start of every workspace.
enum : int { ST_OVERFLOW = 0, ST_NONFINITE = 1, ST_K_LO = 2, ST_K_HI = 3, ST_WORDS = 16 };

struct Tuning {
    int batch;      // 64 / 128 / 256 entries per LDS round of the forward compositing kernel
    int sort_cap;   // 512 / 1024 / 2048 / 4096
    int bwd_batch;  // the same for the backward compositing kernel
    int compact;    // bit 0 / bit 1: compacted forward / backward compositing (coverage masks + per-lane entry
                    // walks); else bit 2: quadrant forward (clear: 4x4-block forward); bit 4 / bit 3: the
                    // backward walks four / two quadrant lists per wave (clear: one)
};

// Byte offsets of the workspace regions (host-computed).
struct Layout {
    int64_t n;
    int frames, width, height, tiles_x, tiles_y, tiles;
    int64_t pixels;        // width * height
    int64_t k_cap;
    int64_t scan_blocks;   // for the (frames*n) scan
    int64_t pose_blocks;   // workgroups of the projection adjoint (upper bound)
    int64_t bin_blocks;    // workgroups per frame of the LDS-histogram binning (0: global atomics)
    size_t status, col4, rec, dkey, rect, tmask, gcnt, goff, tcnt, toff, tcur, bhist, scan_tmp, tfin, nlast, loss_part, pose_part,
        intr_part, vis, shapes,
        kv, sgid, sslot, part, pused, tkv;
    size_t total;
};

Layout make_layout(const gv_camera& cam, int64_t n, int frames, int64_t k_cap);

// Everything a kernel needs, passed by value.
// Frame-independent part of a static Gaussian's projection, computed once
// per call (k_static_shapes) with the very operations project_gaussian would
// repeat in every frame: 3D covariance and opacity, whether the shape's
// parameters (log-scales, quaternion, opacity logit, colour) are finite, and
// whether the quaternion has a nonzero norm.
struct ShapeD {
    double Sig[6];
    double o;
    uint32_t fin, qn_ok;
};
static_assert(sizeof(ShapeD) == 64, "one 64-byte record per Gaussian");

struct Args {
    // scene
    int64_t n;
    int dtype;
    const void* means;
    const void* log_scales;
    const void* quats;
    const void* opacity_logits;
    const void* colors;
    const void* mean_coeffs;
    int n_ctrl;                // B-spline control points (0 = none)
    const void* ctrl;          // [n_ctrl][3][N]
    const void* scale_coeffs;  // [3][3][N] or nullptr
    const void* quat_coeffs;   // [3][4][N] or nullptr
    int sh_degree;             // 0 .. 3
    const void* sh;            // [(D+1)^2 - 1][3][N] or nullptr
    // camera
    int width, height, tiles_x, tiles_y, tiles;
    float fx, fy, cx, cy, near_plane, dilation, bg[3];
    // frames
    int frames;
    const float* poses;   // [F][7]
    const float* times;   // [F] or nullptr (then every frame uses t0)
    float t0;
    // workspace
    uint32_t* status;
    ColorOp* col4;        // [F][N] (colour seen from each frame's camera) when view-dependent, else [N]
    int64_t col_stride;   // N with view-dependent colour, else 0: frame f reads col4[f * col_stride + g]
    Record* rec;          // [F][N]
    float* dkey;          // [F][N]: the record's depth alone, for the scatter's keys
    uint2* rect;          // [F][N]: (x0 | x1 << 16, y0 | y1 << 16) in tiles
    uint64_t* tmask;      // [F][N]: tiles that passed the ellipse test, row-major bits over the rectangle
                          // (rectangles of at most 64 tiles; larger ones are tested again by the scatter)
    uint32_t* gcnt;       // [F*N]
    uint32_t* goff;       // [F*N + 1]
    uint32_t* tcnt;       // [F*T]
    uint32_t* toff;       // [F*T + 1]
    uint32_t* tcur;       // [F*T]
    uint32_t* bhist;      // [F][bin_blocks][T] workgroup tile histograms, or nullptr (global-atomic binning)
    int bin_blocks;
    float* tfin;          // [F][P]
    uint32_t* nlast;      // [F][P]
    float* loss_part;     // [F*T]
    double* pose_part;    // [blocks][F][12]
    double* intr_part;    // [blocks][4] intrinsics-gradient partials of the projection adjoint
    uint8_t* vis;         // [F][N] contribution flags, or nullptr (not requested)
    KeySlot* kv;          // [K] binned (depth | index) keys with their pre-sort slots
    uint32_t* sgid;       // [K]
    uint32_t* sslot;      // [K]
    float* part;          // [K][PART] (du, dv, dA00, dA01, dA11, do, dr, dg, db) per pre-sort slot
    uint32_t* pused;      // [K/32 + 2] bit per pre-sort slot: its partial record was written this pass
    ShapeD* shapes;       // [N] static shapes of this call (scenes without dynamics or SH), or nullptr
    KeySlot* tkv;         // [K] merge scratch of the sort
    int64_t k_cap;
    // image-space inputs/outputs
    float* images;            // [F][3][H][W]
    const float* targets;     // [F][3][H][W] or nullptr
    const float* dl_dimages;  // [F][3][H][W] or nullptr
    float loss_scale;         // d(loss)/d(C) = loss_scale * (C - target)
    float loss_norm;          // loss = loss_norm * sum (C - target)^2
    float* loss;              // [F] or nullptr
    float* tfin_out;          // optional copy of T_final (single frame)
    // gradients
    float* g_means;
    float* g_log_scales;
    float* g_quats;
    float* g_opacity;
    float* g_colors;
    float* g_coeffs;
    float* g_ctrl;
    float* g_scale_coeffs;
    float* g_quat_coeffs;
    float* g_sh;
    float* g_intr;            // [4] fx, fy, cx, cy
    float* g_poses;           // [F][7]
    int accumulate;
    Tuning tune;
};

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

__device__ __forceinline__ double load_param(const void* base, int dtype, int64_t i) {
    if (dtype == GV_BF16) return static_cast<double>(bf16_to_f32(static_cast<const uint16_t*>(base)[i]));
    return static_cast<double>(static_cast<const float*>(base)[i]);
}

// Rotation matrix (row-major) of the unit quaternion (w, x, y, z).
__device__ __forceinline__ void rot_from_quat(double w, double x, double y, double z, double R[9]) {
    const double xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z, wx = w * x,
                 wy = w * y, wz = w * z;
    R[0] = 1.0 - 2.0 * (yy + zz); R[1] = 2.0 * (xy - wz);       R[2] = 2.0 * (xz + wy);
    R[3] = 2.0 * (xy + wz);       R[4] = 1.0 - 2.0 * (xx + zz); R[5] = 2.0 * (yz - wx);
    R[6] = 2.0 * (xz - wy);       R[7] = 2.0 * (yz + wx);       R[8] = 1.0 - 2.0 * (xx + yy);
}

// Gradient w.r.t. an unnormalised quaternion q (norm qn, unit qh) given the
// gradient G (row-major 3x3) w.r.t. R(qh).
__device__ __forceinline__ void quat_grad(const double qh[4], double qn, const double G[9], double dq[4]) {
    const double w = qh[0], x = qh[1], y = qh[2], z = qh[3];
    const double gw = 2.0 * (-z * G[1] + y * G[2] + z * G[3] - x * G[5] - y * G[6] + x * G[7]);
    const double gx = 2.0 * (y * G[1] + z * G[2] + y * G[3] - 2.0 * x * G[4] - w * G[5] + z * G[6] + w * G[7] -
                             2.0 * x * G[8]);
    const double gy = 2.0 * (-2.0 * y * G[0] + x * G[1] + w * G[2] + x * G[3] + z * G[5] - w * G[6] + z * G[7] -
                             2.0 * y * G[8]);
    const double gz = 2.0 * (-2.0 * z * G[0] - w * G[1] + x * G[2] + w * G[3] - 2.0 * z * G[4] + y * G[5] +
                             x * G[6] + y * G[7]);
    const double dot = w * gw + x * gx + y * gy + z * gz;
    dq[0] = (gw - w * dot) / qn;
    dq[1] = (gx - x * dot) / qn;
    dq[2] = (gy - y * dot) / qn;
    dq[3] = (gz - z * dot) / qn;
}

// Camera of frame f: rotation (row-major), translation, normalised quaternion.
struct CamD {
    double R[9], t[3], qh[4], qn;
    bool ok;
};

__device__ __forceinline__ CamD load_camera(const float* pose7) {
    CamD c;
    const double w = pose7[0], x = pose7[1], y = pose7[2], z = pose7[3];
    c.qn = sqrt(w * w + x * x + y * y + z * z);
    c.ok = c.qn > 0.0 && isfinite(c.qn);
    const double qn = c.ok ? c.qn : 1.0;
    c.qh[0] = w / qn; c.qh[1] = x / qn; c.qh[2] = y / qn; c.qh[3] = z / qn;
    rot_from_quat(c.qh[0], c.qh[1], c.qh[2], c.qh[3], c.R);
    c.t[0] = pose7[4]; c.t[1] = pose7[5]; c.t[2] = pose7[6];
    c.ok = c.ok && isfinite(c.t[0]) && isfinite(c.t[1]) && isfinite(c.t[2]);
    return c;
}

// Clamped cubic B-spline of Eq. 2 with M control points: knot u_j = 0 for
// j <= 3, 1 for j >= M, (j - 3) / (M - 3) between.
__device__ __forceinline__ double spline_knot(int j, int M) {
    if (j <= 3) return 0.0;
    if (j >= M) return 1.0;
    return static_cast<double>(j - 3) / static_cast<double>(M - 3);
}

// The four basis functions N_{b..b+3, 3}(t) that can be non-zero at t in
// [0, 1]; returns b (the first control point they weight).  Runs the
// Cox-de Boor recurrence only over the triangle of non-zero terms, each in
// the form ((t - u_i) / d) * N + ((u - t) / d') * N': the terms left out are
// exact zeros, so the values equal those of the full recurrence bit for bit.
template <typename R>
__device__ __forceinline__ int spline_basis(int M, R t, R N[4]) {
    int j = M - 1;  // knot span u_j <= t < u_{j+1}; t = 1 closes the last one
    if (t < R(1)) {
        j = 3 + static_cast<int>(t * static_cast<R>(M - 3));
        j = j < 3 ? 3 : (j > M - 1 ? M - 1 : j);
        while (j > 3 && t < static_cast<R>(spline_knot(j, M))) --j;
        while (j < M - 1 && t >= static_cast<R>(spline_knot(j + 1, M))) ++j;
    }
    R B[4] = {R(1), R(0), R(0), R(0)};  // B[r] = N_{j-p+r, p}
#pragma unroll
    for (int p = 1; p <= 3; ++p) {
        R nb[4] = {R(0), R(0), R(0), R(0)};
#pragma unroll
        for (int r = 0; r <= p; ++r) {
            const int i = j - p + r;
            R v = R(0);
            bool any = false;
            if (r >= 1) {  // (t - u_i) / (u_{i+p} - u_i) * N_{i, p-1}
                const R ui = static_cast<R>(spline_knot(i, M));
                const R d1 = static_cast<R>(spline_knot(i + p, M)) - ui;
                v = (t - ui) / d1 * B[r - 1];
                any = true;
            }
            if (r <= p - 1) {  // (u_{i+p+1} - t) / (u_{i+p+1} - u_{i+1}) * N_{i+1, p-1}
                const R ue = static_cast<R>(spline_knot(i + p + 1, M));
                const R d2 = ue - static_cast<R>(spline_knot(i + 1, M));
                const R w = (ue - t) / d2 * B[r];
                v = any ? v + w : w;
            }
            nb[r] = v;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) B[r] = nb[r];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) N[r] = B[r];
    return j - 3;
}

// Real spherical harmonics of degrees 1..3 at the unit vector (x, y, z), in
// (l, m) ascending order: the harmonic polynomials of degree l normalised to
// unit L2 norm on the sphere, with the (-1)^m sign for m > 0.  If G is given,
// G[k][j] = d Y_k / d(x, y, z)_j of the polynomial.
template <typename R>
__device__ __forceinline__ void sh_eval(int degree, R x, R y, R z, R Y[15], R (*G)[3]) {
    const R k1 = R(0.48860251190291992);                                   // sqrt(3 / 4pi)
    const R k2a = R(1.0925484305920792), k2b = R(0.31539156525252005);    // sqrt(15 / 4pi), sqrt(5 / 16pi)
    const R k2c = R(0.54627421529603959);                                  // sqrt(15 / 16pi)
    const R k3a = R(-0.59004358992664352), k3b = R(2.8906114426405538);   // -sqrt(35 / 32pi), sqrt(105 / 4pi)
    const R k3c = R(-0.45704579946446572), k3d = R(0.3731763325901154);   // -sqrt(21 / 32pi), sqrt(7 / 16pi)
    const R k3e = R(1.4453057213202769);                                   // sqrt(105 / 16pi)
    const R xx = x * x, yy = y * y, zz = z * z;
    Y[0] = -k1 * y;
    Y[1] = k1 * z;
    Y[2] = -k1 * x;
    if (G) {
        G[0][0] = R(0); G[0][1] = -k1; G[0][2] = R(0);
        G[1][0] = R(0); G[1][1] = R(0); G[1][2] = k1;
        G[2][0] = -k1; G[2][1] = R(0); G[2][2] = R(0);
    }
    if (degree < 2) return;
    Y[3] = k2a * x * y;
    Y[4] = -k2a * y * z;
    Y[5] = k2b * (R(2) * zz - xx - yy);
    Y[6] = -k2a * x * z;
    Y[7] = k2c * (xx - yy);
    if (G) {
        G[3][0] = k2a * y; G[3][1] = k2a * x; G[3][2] = R(0);
        G[4][0] = R(0); G[4][1] = -k2a * z; G[4][2] = -k2a * y;
        G[5][0] = R(-2) * k2b * x; G[5][1] = R(-2) * k2b * y; G[5][2] = R(4) * k2b * z;
        G[6][0] = -k2a * z; G[6][1] = R(0); G[6][2] = -k2a * x;
        G[7][0] = R(2) * k2c * x; G[7][1] = R(-2) * k2c * y; G[7][2] = R(0);
    }
    if (degree < 3) return;
    Y[8] = k3a * y * (R(3) * xx - yy);
    Y[9] = k3b * x * y * z;
    Y[10] = k3c * y * (R(4) * zz - xx - yy);
    Y[11] = k3d * z * (R(2) * zz - R(3) * xx - R(3) * yy);
    Y[12] = k3c * x * (R(4) * zz - xx - yy);
    Y[13] = k3e * z * (xx - yy);
    Y[14] = k3a * x * (xx - R(3) * yy);
    if (G) {
        G[8][0] = k3a * R(6) * x * y; G[8][1] = k3a * R(3) * (xx - yy); G[8][2] = R(0);
        G[9][0] = k3b * y * z; G[9][1] = k3b * x * z; G[9][2] = k3b * x * y;
        G[10][0] = k3c * R(-2) * x * y; G[10][1] = k3c * (R(4) * zz - xx - R(3) * yy); G[10][2] = k3c * R(8) * y * z;
        G[11][0] = k3d * R(-6) * x * z; G[11][1] = k3d * R(-6) * y * z;
        G[11][2] = k3d * (R(6) * zz - R(3) * xx - R(3) * yy);
        G[12][0] = k3c * (R(4) * zz - R(3) * xx - yy); G[12][1] = k3c * R(-2) * x * y; G[12][2] = k3c * R(8) * x * z;
        G[13][0] = k3e * R(2) * x * z; G[13][1] = k3e * R(-2) * y * z; G[13][2] = k3e * (xx - yy);
        G[14][0] = k3a * R(3) * (xx - yy); G[14][1] = k3a * R(-6) * x * y; G[14][2] = R(0);
    }
}

__device__ __forceinline__ int sh_count(int degree) { return (degree + 1) * (degree + 1) - 1; }

// FP64 projection state of one Gaussian in one frame (EWA splatting).
struct ProjD {
    double mu[3], s[3], qh[4], qn, R[9];
    double Sig[6];        // xx xy xz yy yz zz
    double m[3];
    double u, v;
    double T[6];          // J Rc, 2x3 row-major
    double cov[3];        // 00 01 11 (dilated)
    double A[3];          // conic 00 01 11
    double o;
    double eta;
    double col[3];        // colour seen from this frame's camera (view-dependent with SH)
    bool nonfinite;
};

// q-norm, unit quaternion, scales, opacity, R and Sigma = (R S)(R S)^T
// (Sec. 3.1) of a Gaussian from its raw parameters (raw[3..5] log-scales,
// raw[6..9] quaternion, raw[10] opacity logit); false if the quaternion's
// norm is not positive.  The per-frame projection and the once-per-call
// static shapes share it, so both give the same values.
__device__ __forceinline__ bool shape_from_params(const double* raw, ProjD& P) {
    P.qn = sqrt(raw[6] * raw[6] + raw[7] * raw[7] + raw[8] * raw[8] + raw[9] * raw[9]);
    if (!(P.qn > 0.0)) return false;
    for (int k = 0; k < 4; ++k) P.qh[k] = raw[6 + k] / P.qn;
    for (int k = 0; k < 3; ++k) P.s[k] = exp(raw[3 + k]);
    P.eta = raw[10];
    P.o = 1.0 / (1.0 + exp(-raw[10]));
    rot_from_quat(P.qh[0], P.qh[1], P.qh[2], P.qh[3], P.R);
    // Sigma = M M^T with M = R diag(s)
    double M[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[i * 3 + j] = P.R[i * 3 + j] * P.s[j];
    P.Sig[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
    P.Sig[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
    P.Sig[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
    P.Sig[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
    P.Sig[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
    P.Sig[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
    return true;
}

__device__ __forceinline__ bool project_shaped(const Args& a, const CamD& cam, ProjD& P);

// Returns true if the Gaussian is in front of the near plane with a valid
// footprint.  P.nonfinite marks non-finite inputs.  EXT compiles in the
// optional B-spline / polynomial dynamics and the SH colour; the projection
// kernel takes project_gaussian_shaped instead for scenes without them, whose
// frame-independent shape is precomputed once per call.
template <bool EXT>
__device__ __forceinline__ bool project_gaussian(const Args& a, int64_t g, const CamD& cam, double t, ProjD& P) {
    const int64_t n = a.n;
    double raw[14];
    for (int k = 0; k < 3; ++k) raw[k] = EXT && a.n_ctrl > 0 ? 0.0 : load_param(a.means, a.dtype, k * n + g);
    for (int k = 0; k < 3; ++k) raw[3 + k] = load_param(a.log_scales, a.dtype, k * n + g);
    for (int k = 0; k < 4; ++k) raw[6 + k] = load_param(a.quats, a.dtype, k * n + g);
    raw[10] = load_param(a.opacity_logits, a.dtype, g);
    for (int k = 0; k < 3; ++k) raw[11 + k] = load_param(a.colors, a.dtype, k * n + g);
    bool fin = true;
    for (int k = 0; k < 14; ++k) fin = fin && isfinite(raw[k]);
    bool in_domain = true;
    if (EXT && a.n_ctrl > 0) {
        // B-spline mean (Eq. 2): sum over the span's four control points in
        // index order (the other basis functions are exact zeros)
        in_domain = t >= 0.0 && t <= 1.0;
        double N[4];
        const int b = spline_basis<double>(a.n_ctrl, in_domain ? t : 0.0, N);
        for (int k = 0; k < 3; ++k) {
            double mu = 0.0;
            for (int r = 0; r < 4; ++r) {
                if (N[r] == 0.0) continue;  // local support: zero weight, no part in mu
                const double c = load_param(a.ctrl, a.dtype, (static_cast<int64_t>(b + r) * 3 + k) * n + g);
                fin = fin && isfinite(c);
                mu = mu + N[r] * c;
            }
            P.mu[k] = mu;
        }
    } else {
        for (int k = 0; k < 3; ++k) {
            double mu = raw[k];
            if (a.mean_coeffs) {
                const double c1 = load_param(a.mean_coeffs, a.dtype, (0 * 3 + k) * n + g);
                const double c2 = load_param(a.mean_coeffs, a.dtype, (1 * 3 + k) * n + g);
                const double c3 = load_param(a.mean_coeffs, a.dtype, (2 * 3 + k) * n + g);
                fin = fin && isfinite(c1) && isfinite(c2) && isfinite(c3);
                // same left-to-right order as mu0 + a1 t + a2 t t + a3 t t t
                mu = mu + c1 * t + c2 * t * t + c3 * t * t * t;
            }
            P.mu[k] = mu;
        }
    }
    if (EXT && a.scale_coeffs)
        for (int k = 0; k < 3; ++k) {
            const double b1 = load_param(a.scale_coeffs, a.dtype, (0 * 3 + k) * n + g);
            const double b2 = load_param(a.scale_coeffs, a.dtype, (1 * 3 + k) * n + g);
            const double b3 = load_param(a.scale_coeffs, a.dtype, (2 * 3 + k) * n + g);
            fin = fin && isfinite(b1) && isfinite(b2) && isfinite(b3);
            raw[3 + k] = raw[3 + k] + b1 * t + b2 * t * t + b3 * t * t * t;
        }
    if (EXT && a.quat_coeffs)
        for (int k = 0; k < 4; ++k) {
            const double r1 = load_param(a.quat_coeffs, a.dtype, (0 * 4 + k) * n + g);
            const double r2 = load_param(a.quat_coeffs, a.dtype, (1 * 4 + k) * n + g);
            const double r3 = load_param(a.quat_coeffs, a.dtype, (2 * 4 + k) * n + g);
            fin = fin && isfinite(r1) && isfinite(r2) && isfinite(r3);
            raw[6 + k] = raw[6 + k] + r1 * t + r2 * t * t + r3 * t * t * t;
        }
    for (int c = 0; c < 3; ++c) P.col[c] = raw[11 + c];
    if (EXT && a.sh_degree > 0) {
        // view-dependent colour: SH at the unit direction camera centre -> mean
        double v[3];
        for (int i = 0; i < 3; ++i)
            v[i] = P.mu[i] + (cam.R[0 * 3 + i] * cam.t[0] + cam.R[1 * 3 + i] * cam.t[1] + cam.R[2 * 3 + i] * cam.t[2]);
        const double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        const double iv = vn > 0.0 ? 1.0 / vn : 0.0;
        double Y[15];
        sh_eval<double>(a.sh_degree, v[0] * iv, v[1] * iv, v[2] * iv, Y, nullptr);
        const int nb = sh_count(a.sh_degree);
        for (int c = 0; c < 3; ++c) {
            double acc = P.col[c];
            for (int k = 0; k < nb; ++k) {
                const double kc = load_param(a.sh, a.dtype, (static_cast<int64_t>(k) * 3 + c) * n + g);
                fin = fin && isfinite(kc);
                acc = acc + Y[k] * kc;
            }
            P.col[c] = acc;
        }
    }
    P.nonfinite = !fin;
    if (!fin || !cam.ok || !in_domain) return false;
    if (!shape_from_params(raw, P)) return false;
    return project_shaped(a, cam, P);
}

// The static path with the frame-independent shape precomputed (a.shapes):
// only the mean (and its cubic in t) is read per frame.
__device__ __forceinline__ bool project_gaussian_shaped(const Args& a, int64_t g, const CamD& cam, double t,
                                                        ProjD& P) {
    const int64_t n = a.n;
    const ShapeD& S = a.shapes[g];
    bool fin = S.fin != 0u;
    for (int k = 0; k < 3; ++k) {
        double mu = load_param(a.means, a.dtype, k * n + g);
        fin = fin && isfinite(mu);
        if (a.mean_coeffs) {
            const double c1 = load_param(a.mean_coeffs, a.dtype, (0 * 3 + k) * n + g);
            const double c2 = load_param(a.mean_coeffs, a.dtype, (1 * 3 + k) * n + g);
            const double c3 = load_param(a.mean_coeffs, a.dtype, (2 * 3 + k) * n + g);
            fin = fin && isfinite(c1) && isfinite(c2) && isfinite(c3);
            // same left-to-right order as mu0 + a1 t + a2 t t + a3 t t t
            mu = mu + c1 * t + c2 * t * t + c3 * t * t * t;
        }
        P.mu[k] = mu;
    }
    P.nonfinite = !fin;
    if (!fin || !cam.ok) return false;
    if (!S.qn_ok) return false;
    for (int k = 0; k < 6; ++k) P.Sig[k] = S.Sig[k];
    P.o = S.o;
    return project_shaped(a, cam, P);
}

// Camera-space mean, perspective projection, 2D covariance and conic of a
// Gaussian whose mean (P.mu) and 3D covariance (P.Sig) are set.
__device__ __forceinline__ bool project_shaped(const Args& a, const CamD& cam, ProjD& P) {
    const double* Rc = cam.R;
    // m = tc + Rc mu, summed in this order (with no contraction the fp32
    // rounding of m_z, the depth sort key, is then reproducible bit for bit)
    for (int i = 0; i < 3; ++i)
        P.m[i] = ((cam.t[i] + Rc[i * 3 + 0] * P.mu[0]) + Rc[i * 3 + 1] * P.mu[1]) + Rc[i * 3 + 2] * P.mu[2];
    if (!(P.m[2] > static_cast<double>(a.near_plane))) return false;
    const double iz = 1.0 / P.m[2];
    const double fx = a.fx, fy = a.fy;
    P.u = fx * P.m[0] * iz + static_cast<double>(a.cx);
    P.v = fy * P.m[1] * iz + static_cast<double>(a.cy);
    // J = [[fx/z, 0, -fx x/z^2], [0, fy/z, -fy y/z^2]];  T = J Rc
    const double j00 = fx * iz, j02 = -fx * P.m[0] * iz * iz;
    const double j11 = fy * iz, j12 = -fy * P.m[1] * iz * iz;
    for (int j = 0; j < 3; ++j) {
        P.T[j] = j00 * Rc[0 * 3 + j] + j02 * Rc[2 * 3 + j];
        P.T[3 + j] = j11 * Rc[1 * 3 + j] + j12 * Rc[2 * 3 + j];
    }
    // cov = T Sig T^T + dil I
    double TS[6];
    for (int i = 0; i < 2; ++i) {
        const double t0 = P.T[i * 3 + 0], t1 = P.T[i * 3 + 1], t2 = P.T[i * 3 + 2];
        TS[i * 3 + 0] = t0 * P.Sig[0] + t1 * P.Sig[1] + t2 * P.Sig[2];
        TS[i * 3 + 1] = t0 * P.Sig[1] + t1 * P.Sig[3] + t2 * P.Sig[4];
        TS[i * 3 + 2] = t0 * P.Sig[2] + t1 * P.Sig[4] + t2 * P.Sig[5];
    }
    const double dil = a.dilation;
    P.cov[0] = TS[0] * P.T[0] + TS[1] * P.T[1] + TS[2] * P.T[2] + dil;
    P.cov[1] = TS[0] * P.T[3] + TS[1] * P.T[4] + TS[2] * P.T[5];
    P.cov[2] = TS[3] * P.T[3] + TS[4] * P.T[4] + TS[5] * P.T[5] + dil;
    const double det = P.cov[0] * P.cov[2] - P.cov[1] * P.cov[1];
    if (!(det > 0.0) || !isfinite(det)) return false;
    const double idet = 1.0 / det;
    P.A[0] = P.cov[2] * idet;
    P.A[1] = -P.cov[1] * idet;
    P.A[2] = P.cov[0] * idet;
    return true;
}

// Does the ellipse {p : (p-c)^T A (p-c) <= thr} meet the axis-aligned box
// [x0,x1] x [y0,y1]?  Exact minimum of the quadratic over the box: zero when
// the centre is inside, else the smallest of the four edge minima.
template <typename F>
__device__ __forceinline__ bool ellipse_meets_box(F u, F v, F a, F b, F c, F x0, F x1, F y0, F y1, F thr) {
    const F dx0 = x0 - u, dx1 = x1 - u, dy0 = y0 - v, dy1 = y1 - v;
    if (dx0 <= F(0) && dx1 >= F(0) && dy0 <= F(0) && dy1 >= F(0)) return true;
    auto on_x_edge = [&](F dx) {
        F dy = -b * dx / c;
        dy = dy < dy0 ? dy0 : (dy > dy1 ? dy1 : dy);
        return a * dx * dx + F(2) * b * dx * dy + c * dy * dy;
    };
    auto on_y_edge = [&](F dy) {
        F dx = -b * dy / a;
        dx = dx < dx0 ? dx0 : (dx > dx1 ? dx1 : dx);
        return a * dx * dx + F(2) * b * dx * dy + c * dy * dy;
    };
    F m = on_x_edge(dx0);
    F t1 = on_x_edge(dx1);
    m = t1 < m ? t1 : m;
    t1 = on_y_edge(dy0);
    m = t1 < m ? t1 : m;
    t1 = on_y_edge(dy1);
    m = t1 < m ? t1 : m;
    return m <= thr;
}

// The same test without divisions: rbc = -b / c and rba = -b / a, the slopes
// of the edge minimisers, computed once per ellipse.  A minimiser off by an
// ulp changes the edge minimum only in second order.
template <typename F>
__device__ __forceinline__ bool ellipse_meets_box_r(F u, F v, F a, F b, F c, F rbc, F rba, F x0, F x1, F y0, F y1,
                                                    F thr) {
    const F dx0 = x0 - u, dx1 = x1 - u, dy0 = y0 - v, dy1 = y1 - v;
    if (dx0 <= F(0) && dx1 >= F(0) && dy0 <= F(0) && dy1 >= F(0)) return true;
    auto on_x_edge = [&](F dx) {
        F dy = rbc * dx;
        dy = dy < dy0 ? dy0 : (dy > dy1 ? dy1 : dy);
        return a * dx * dx + F(2) * b * dx * dy + c * dy * dy;
    };
    auto on_y_edge = [&](F dy) {
        F dx = rba * dy;
        dx = dx < dx0 ? dx0 : (dx > dx1 ? dx1 : dx);
        return a * dx * dx + F(2) * b * dx * dy + c * dy * dy;
    };
    F m = on_x_edge(dx0);
    F t1 = on_x_edge(dx1);
    m = t1 < m ? t1 : m;
    t1 = on_y_edge(dy0);
    m = t1 < m ? t1 : m;
    t1 = on_y_edge(dy1);
    m = t1 < m ? t1 : m;
    return m <= thr;
}

// Pixel-centre box of tile (tx, ty), clipped to the image.
__device__ __forceinline__ void tile_box(int tx, int ty, int W, int H, double& x0, double& x1, double& y0,
                                         double& y1) {
    x0 = tx * TILE + 0.5;
    x1 = fmin(tx * TILE + (TILE - 0.5), W - 0.5);
    y0 = ty * TILE + 0.5;
    y1 = fmin(ty * TILE + (TILE - 0.5), H - 0.5);
}

// Sum of v over the 64 lanes of a wave, valid in lane 63 (DPP row shifts
// within each row of 16, then row broadcasts across rows).
__device__ __forceinline__ float wave_sum_to_lane63(float v) {
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x111, 0xf, 0xf, true));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x112, 0xf, 0xf, true));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x114, 0xf, 0xf, true));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x118, 0xf, 0xf, true));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x142, 0xa, 0xf, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x143, 0xc, 0xf, false));
    return v;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Value of lane (lane ^ 8) (row rotate by 8), lane 7 - (lane mod 8) (row
// half-mirror), lane ^ 2 or lane ^ 1 (quad permutations): the DPP moves the
// reductions below use.
__device__ __forceinline__ float dpp_f(float x, int ctrl) {
    switch (ctrl) {  // constant after inlining
        case 0x128: return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x128, 0xf, 0xf, true));
        case 0x141: return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x141, 0xf, 0xf, true));
        case 0x4E: return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x4E, 0xf, 0xf, true));
        default: return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0xB1, 0xf, 0xf, true));
    }
}

// Sum of 16 values over the 64 lanes: four halving stages (cross-half swaps
// for 32 and 16 lanes, DPP for 8 and 4) and two quad additions.  Afterwards
// the four lanes of quad q hold the wave total of value
// 8 b5 + 4 b4 + 2 b3 + b2 (b_i the lane's address bits).
__device__ __forceinline__ float reduce_scatter16(float (&v)[16], int lane) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 8]), false, false);
        v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 4]), false, false);
        v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    const bool b3 = lane & 8, b2 = lane & 4;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const float keep = b3 ? v[i + 2] : v[i], send = b3 ? v[i] : v[i + 2];
        v[i] = keep + dpp_f(send, 0x128);
    }
    {
        const float keep = b2 ? v[1] : v[0], send = b2 ? v[0] : v[1];
        v[0] = keep + dpp_f(send, 0x141);
    }
    float x = v[0] + dpp_f(v[0], 0x4E);
    return x + dpp_f(x, 0xB1);
}

__device__ __forceinline__ int reduce_scatter16_index(int lane) {
    return ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 + ((lane >> 2) & 1);
}

// Entry range [s, e) of bucket `seg`, clamped to the intersection capacity.
// Partial record of pre-sort slot `slot`, and its bit in pused.  The
// adjoint writes records only for the entries up to each tile's last
// contributor; the projection adjoint adds only the marked slots, so the
// entries behind (about half of them on dense scenes) need no zero records.
// The bits are cleared before the adjoint; OR is order-independent.
__device__ __forceinline__ void store_partials_marked(const Args& a, uint32_t slot, const float (&v)[PART]) {
    store_partials(a.part, slot, v);
    atomicOr(&a.pused[slot >> 5], 1u << (slot & 31u));
}

__device__ __forceinline__ void bucket_range(const Args& a, int64_t seg, uint32_t& s, uint32_t& e) {
    const uint32_t cap = static_cast<uint32_t>(a.k_cap);
    e = min(a.toff[seg + 1], cap);
    s = min(a.toff[seg], e);
}

__device__ __forceinline__ bool overflowed(const uint32_t* status) {
    return status[ST_OVERFLOW] != 0u;
}

}  // namespace gv
