// Adjoint of the EWA projection.  One thread per Gaussian loops over the
// frames: it sums the per-(Gaussian, tile) partials left by the compositing
// adjoint (contiguous slots of this Gaussian, in FP64), takes the conic of the
// forward record, re-derives the rest of the frame's projection and applies
// the chain rule down to the stored parameters in FP32, accumulating the
// shared parameters over frames in FP64 (in LDS, which keeps the chain rule's
// registers free for occupancy).
// Each frame's pose gradient (dL/dRc, dL/dtc) is reduced per workgroup in a
// fixed order; a second kernel sums the workgroups and maps it to the 7-vector
// pose.  Everything is deterministic (no floating-point atomics).
#include "gv_internal.h"

namespace gv {

// dR_e * dR_e/dq for the e-th entry (row-major) of the rotation matrix of the
// unit quaternion (w, x, y, z); e is a compile-time constant after unrolling.
__device__ __forceinline__ void add_rot_partial(int e, float v, const float q[4], float g[4]) {
    const float w = q[0], x = q[1], y = q[2], z = q[3];
    switch (e) {
        case 0: g[2] += -4.0f * y * v; g[3] += -4.0f * z * v; break;
        case 1: g[0] += -2.0f * z * v; g[1] += 2.0f * y * v; g[2] += 2.0f * x * v; g[3] += -2.0f * w * v; break;
        case 2: g[0] += 2.0f * y * v; g[1] += 2.0f * z * v; g[2] += 2.0f * w * v; g[3] += 2.0f * x * v; break;
        case 3: g[0] += 2.0f * z * v; g[1] += 2.0f * y * v; g[2] += 2.0f * x * v; g[3] += 2.0f * w * v; break;
        case 4: g[1] += -4.0f * x * v; g[3] += -4.0f * z * v; break;
        case 5: g[0] += -2.0f * x * v; g[1] += -2.0f * w * v; g[2] += 2.0f * z * v; g[3] += 2.0f * y * v; break;
        case 6: g[0] += -2.0f * y * v; g[1] += 2.0f * z * v; g[2] += -2.0f * w * v; g[3] += 2.0f * x * v; break;
        case 7: g[0] += 2.0f * x * v; g[1] += 2.0f * w * v; g[2] += 2.0f * z * v; g[3] += 2.0f * y * v; break;
        default: g[1] += -4.0f * x * v; g[2] += -4.0f * y * v; break;
    }
}

// FP32 quantities of the projection of (f, g) that the adjoint needs.  The
// conic is read from the forward record (the FP64 value rounded once: exactly
// the one the compositing kernels used); the rest is recomputed.
struct AdjIn {
    float mu[3], s[3], qh[4], iqn, R[9], Sig[6], m[3], iz, T[6], A[3], o;
    float N[4];  // B-spline weights of control points span .. span + 3
    int span;
};

// Cubic polynomial in t without a constant term: c1 t + c2 t^2 + c3 t^3.
__device__ __forceinline__ float cubic_in_t(const Args& a, const void* coeffs, int rows, int k, int64_t g, float t) {
    const int64_t n = a.n;
    const float c1 = static_cast<float>(load_param(coeffs, a.dtype, (0 * rows + k) * n + g));
    const float c2 = static_cast<float>(load_param(coeffs, a.dtype, (1 * rows + k) * n + g));
    const float c3 = static_cast<float>(load_param(coeffs, a.dtype, (2 * rows + k) * n + g));
    return t * (c1 + t * (c2 + t * c3));
}

// Shape part of the adjoint inputs at time t: scales, normalised quaternion
// (and 1/|q|), rotation, 3D covariance and opacity.  Static Gaussians (DYN
// false) compute it once; t enters only through Eq. 3's polynomials.
template <bool DYN>
__device__ __forceinline__ void shape_inputs(const Args& a, int64_t g, float t, AdjIn& P) {
    const int64_t n = a.n;
    float q[4];
    for (int k = 0; k < 3; ++k) {
        float ls = static_cast<float>(load_param(a.log_scales, a.dtype, k * n + g));
        if (DYN && a.scale_coeffs) ls = ls + cubic_in_t(a, a.scale_coeffs, 3, k, g, t);
        P.s[k] = expf(ls);
    }
    for (int k = 0; k < 4; ++k) {
        q[k] = static_cast<float>(load_param(a.quats, a.dtype, k * n + g));
        if (DYN && a.quat_coeffs) q[k] = q[k] + cubic_in_t(a, a.quat_coeffs, 4, k, g, t);
    }
    P.iqn = 1.0f / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; ++k) P.qh[k] = q[k] * P.iqn;
    const float eta = static_cast<float>(load_param(a.opacity_logits, a.dtype, g));
    P.o = 1.0f / (1.0f + expf(-eta));
    {
        const float w = P.qh[0], x = P.qh[1], y = P.qh[2], z = P.qh[3];
        float* R = P.R;
        R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z);       R[2] = 2.f * (x * z + w * y);
        R[3] = 2.f * (x * y + w * z);       R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
        R[6] = 2.f * (x * z - w * y);       R[7] = 2.f * (y * z + w * x);       R[8] = 1.f - 2.f * (x * x + y * y);
    }
    {
        float M[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) M[i * 3 + j] = P.R[i * 3 + j] * P.s[j];
        P.Sig[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
        P.Sig[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
        P.Sig[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
        P.Sig[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
        P.Sig[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
        P.Sig[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
    }
}

// Frame part: the mean at time t (B-spline, cubic or static), its camera-space
// position, the projection Jacobian times the camera rotation, and the conic
// of the forward record (the FP64 value rounded once: exactly the one the
// compositing kernels used).
template <bool DYN>
__device__ __forceinline__ void frame_inputs(const Args& a, int64_t g, const Record& rec, const float* Rc,
                                             const float* tc, float t, AdjIn& P) {
    const int64_t n = a.n;
    P.span = 0;
    if (DYN && a.n_ctrl > 0) {
        P.span = spline_basis<float>(a.n_ctrl, fminf(fmaxf(t, 0.0f), 1.0f), P.N);
        for (int k = 0; k < 3; ++k) {
            float mu = 0.0f;
            for (int r = 0; r < 4; ++r)
                if (P.N[r] != 0.0f)
                    mu += P.N[r] * static_cast<float>(
                                       load_param(a.ctrl, a.dtype, (static_cast<int64_t>(P.span + r) * 3 + k) * n + g));
            P.mu[k] = mu;
        }
    } else {
        for (int k = 0; k < 3; ++k) {
            float mu = static_cast<float>(load_param(a.means, a.dtype, k * n + g));
            if (a.mean_coeffs) mu = mu + cubic_in_t(a, a.mean_coeffs, 3, k, g, t);
            P.mu[k] = mu;
        }
    }
    for (int i = 0; i < 3; ++i)
        P.m[i] = tc[i] + Rc[i * 3 + 0] * P.mu[0] + Rc[i * 3 + 1] * P.mu[1] + Rc[i * 3 + 2] * P.mu[2];
    P.iz = 1.0f / P.m[2];
    const float iz = P.iz;
    const float j00 = a.fx * iz, j02 = -a.fx * P.m[0] * iz * iz;
    const float j11 = a.fy * iz, j12 = -a.fy * P.m[1] * iz * iz;
    for (int j = 0; j < 3; ++j) {
        P.T[j] = j00 * Rc[0 * 3 + j] + j02 * Rc[2 * 3 + j];
        P.T[3 + j] = j11 * Rc[1 * 3 + j] + j12 * Rc[2 * 3 + j];
    }
    P.A[0] = rec.a;
    P.A[1] = rec.b;
    P.A[2] = rec.c;
}

// dL/dSig (symmetric, stored xx xy xz yy yz zz) -> gradients of the stored
// log-scales (out 0-2) and the unnormalised quaternion (out 3-6), through
// Sig = M M^T, M = R diag(s): dM = 2 G M, dR = dM diag(s), ds_j = sum_i dM_ij R_ij.
__device__ __forceinline__ void sigma_adjoint(const float G[6], const AdjIn& P, float out[7]) {
    const float Gm[9] = {G[0], G[1], G[2], G[1], G[3], G[4], G[2], G[4], G[5]};
    float ds[3] = {0.f, 0.f, 0.f};
    float gq[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const float V = Gm[i * 3 + 0] * P.R[0 * 3 + j] + Gm[i * 3 + 1] * P.R[1 * 3 + j] +
                            Gm[i * 3 + 2] * P.R[2 * 3 + j];
            const float dM = 2.0f * P.s[j] * V;
            ds[j] += dM * P.R[i * 3 + j];
            add_rot_partial(i * 3 + j, dM * P.s[j], P.qh, gq);
        }
    for (int k = 0; k < 3; ++k) out[k] = ds[k] * P.s[k];
    // q_hat = q / |q|
    const float dot = P.qh[0] * gq[0] + P.qh[1] * gq[1] + P.qh[2] * gq[2] + P.qh[3] * gq[3];
    for (int k = 0; k < 4; ++k) out[3 + k] = (gq[k] - P.qh[k] * dot) * P.iqn;
}

// Chain rule for one (frame, Gaussian).  d: dL/d(u, v, A00, A01, A11, o, r, g,
// b) with A01 the single off-diagonal conic parameter (it enters q twice).
// Writes the gradients w.r.t. the frame's parameter values to gout (mean 0-2,
// log-scales 3-5, quaternion 6-9, opacity logit 10, colour 11-13; with
// SIGMA_OUT, dL/dSig at 3-8 instead of 3-9) and adds the pose gradient
// (dL/dRc row-major 0-8, dL/dtc 9-11) to pose.
template <bool SIGMA_OUT>
__device__ __forceinline__ void projection_adjoint(const Args& a, const float* Rc, const AdjIn& P,
                                                   const float d[9], float gout[14], float (&pose)[12],
                                                   float gintr[4]) {
    const float A0 = P.A[0], A1 = P.A[1], A2 = P.A[2];
    // gradient w.r.t. the symmetric conic matrix
    const float G00 = d[2], G01 = 0.5f * d[3], G11 = d[4];
    // A = cov^-1  =>  dL/dcov = -A G A
    const float AG00 = A0 * G00 + A1 * G01, AG01 = A0 * G01 + A1 * G11;
    const float AG10 = A1 * G00 + A2 * G01, AG11 = A1 * G01 + A2 * G11;
    const float C00 = -(AG00 * A0 + AG01 * A1);
    const float C01 = -0.5f * ((AG00 * A1 + AG01 * A2) + (AG10 * A0 + AG11 * A1));
    const float C11 = -(AG10 * A1 + AG11 * A2);
    // cov = T Sig T^T + dil I with T = J Rc (2x3); CT = C T
    const float* Tm = P.T;
    float CT[6];
    for (int j = 0; j < 3; ++j) {
        CT[j] = C00 * Tm[j] + C01 * Tm[3 + j];
        CT[3 + j] = C01 * Tm[j] + C11 * Tm[3 + j];
    }
    // dT = 2 C T Sig  (Sig symmetric, stored xx xy xz yy yz zz)
    const float* S = P.Sig;
    float dT[6];
    for (int i = 0; i < 2; ++i) {
        const float c0 = CT[i * 3 + 0], c1 = CT[i * 3 + 1], c2 = CT[i * 3 + 2];
        dT[i * 3 + 0] = 2.0f * (c0 * S[0] + c1 * S[1] + c2 * S[2]);
        dT[i * 3 + 1] = 2.0f * (c0 * S[1] + c1 * S[3] + c2 * S[4]);
        dT[i * 3 + 2] = 2.0f * (c0 * S[2] + c1 * S[4] + c2 * S[5]);
    }
    // T = J Rc with J = [[j00, 0, j02], [0, j11, j12]]
    const float mx = P.m[0], my = P.m[1];
    const float iz = P.iz, iz2 = iz * iz, iz3 = iz2 * iz;
    const float fx = a.fx, fy = a.fy;
    const float j00 = fx * iz, j02 = -fx * mx * iz2, j11 = fy * iz, j12 = -fy * my * iz2;
    float dJ00 = 0.f, dJ02 = 0.f, dJ11 = 0.f, dJ12 = 0.f;
    for (int j = 0; j < 3; ++j) {
        dJ00 += dT[j] * Rc[0 * 3 + j];
        dJ02 += dT[j] * Rc[2 * 3 + j];
        dJ11 += dT[3 + j] * Rc[1 * 3 + j];
        dJ12 += dT[3 + j] * Rc[2 * 3 + j];
        pose[0 * 3 + j] += j00 * dT[j];
        pose[1 * 3 + j] += j11 * dT[3 + j];
        pose[2 * 3 + j] += j02 * dT[j] + j12 * dT[3 + j];
    }
    // intrinsics: u = fx mx/mz + cx, v = fy my/mz + cy, J00 = fx/mz,
    // J02 = -fx mx/mz^2, J11 = fy/mz, J12 = -fy my/mz^2
    gintr[0] = d[0] * mx * iz + dJ00 * iz - dJ02 * mx * iz2;
    gintr[1] = d[1] * my * iz + dJ11 * iz - dJ12 * my * iz2;
    gintr[2] = d[0];
    gintr[3] = d[1];
    // J(m) and (u, v)(m)
    float dm[3];
    dm[0] = -dJ02 * fx * iz2 + d[0] * fx * iz;
    dm[1] = -dJ12 * fy * iz2 + d[1] * fy * iz;
    dm[2] = -dJ00 * fx * iz2 + dJ02 * 2.0f * fx * mx * iz3 - dJ11 * fy * iz2 + dJ12 * 2.0f * fy * my * iz3 -
            d[0] * fx * mx * iz2 - d[1] * fy * my * iz2;
    // m = Rc mu + tc
    for (int k = 0; k < 3; ++k) {
        gout[k] = Rc[0 * 3 + k] * dm[0] + Rc[1 * 3 + k] * dm[1] + Rc[2 * 3 + k] * dm[2];
        pose[9 + k] += dm[k];
    }
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) pose[i * 3 + k] += dm[i] * P.mu[k];
    // dL/dSig = T^T C T; static Gaussians return it (summed over frames and
    // taken through sigma_adjoint once), the others apply sigma_adjoint per frame
    float G[6];
    G[0] = Tm[0] * CT[0] + Tm[3] * CT[3];
    G[1] = Tm[0] * CT[1] + Tm[3] * CT[4];
    G[2] = Tm[0] * CT[2] + Tm[3] * CT[5];
    G[3] = Tm[1] * CT[1] + Tm[4] * CT[4];
    G[4] = Tm[1] * CT[2] + Tm[4] * CT[5];
    G[5] = Tm[2] * CT[2] + Tm[5] * CT[5];
    if (SIGMA_OUT) {
        for (int k = 0; k < 6; ++k) gout[3 + k] = G[k];
        gout[9] = 0.0f;
    } else {
        sigma_adjoint(G, P, gout + 3);
    }
    gout[10] = d[5] * P.o * (1.0f - P.o);
    gout[11] = d[6];
    gout[12] = d[7];
    gout[13] = d[8];
}

// Accumulator slots (FP64, in LDS) of the projection adjoint kernel.  The
// static layout holds the per-frame gradients of the mean (0-2), dL/dSig
// (3-8; slot 9 unused), opacity (10) and colour (11-13), and the cubic mean
// coefficients 14-22.  The dynamic layout (B-spline means and/or polynomial
// log-scales and quaternions, Eq. 2-3) holds the 14 at 0-13, a window of four
// control points 14-25 (point span + r, axis k at 14 + 3 r + k), the
// log-scale coefficients 26-34 and the quaternion coefficients 35-46.
template <bool DYN>
struct AccLayout {
    static constexpr int N = DYN ? 47 : 23;
    static constexpr int CUBIC = 14, WIN = 14, SCALE = 26, QUAT = 35;
};

// View-dependent colour (SH, Sec. 3.1): given dL/d(colour) of one frame,
// add Y_k(d) dL/dc to the coefficient accumulators and return, through the
// unit direction d = v / |v|, v = mu - C, dL/dv (it adds to dL/dmu, and
// -dL/dv is the gradient of the camera centre C = -Rc^T tc).
template <int NT>
__device__ __forceinline__ void sh_adjoint(const Args& a, int64_t g, const AdjIn& P, const float* camC,
                                           const float dc[3], float (*acc_sh)[NT], int tid, float dv[3]) {
    const int64_t n = a.n;
    float v[3];
    for (int i = 0; i < 3; ++i) v[i] = P.mu[i] - camC[i];
    const float vn = sqrtf(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    const float iv = vn > 0.0f ? 1.0f / vn : 0.0f;
    const float d[3] = {v[0] * iv, v[1] * iv, v[2] * iv};
    float Y[15], G[15][3];
    sh_eval<float>(3, d[0], d[1], d[2], Y, G);  // all degrees (static indexing); unused ones are skipped
    const int nb = sh_count(a.sh_degree);
    float dd[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 15; ++k) {  // static indices keep Y and G in registers
        if (k < nb) {
            float w = 0.f;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                acc_sh[k * 3 + c][tid] += Y[k] * dc[c];
                w += dc[c] * static_cast<float>(load_param(a.sh, a.dtype, (static_cast<int64_t>(k) * 3 + c) * n + g));
            }
#pragma unroll
            for (int j = 0; j < 3; ++j) dd[j] += w * G[k][j];
        }
    }
    const float dot = d[0] * dd[0] + d[1] * dd[1] + d[2] * dd[2];
    for (int j = 0; j < 3; ++j) dv[j] = (dd[j] - d[j] * dot) * iv;
}

// SPLIT waves share each Gaussian: wave h of a workgroup takes the h-th
// contiguous part of the frames for the workgroup's 64 Gaussians, and the
// parts' accumulators are added in a fixed order at the end.  Shorter parts
// keep more waves in flight for this latency-bound kernel and leave a shorter
// tail when the last workgroups run alone.  The dynamic variant keeps one
// wave per Gaussian (its control-point window adds to memory as it moves) and
// the SH variant two parts (its coefficient accumulators take LDS).
template <bool DYN, bool SH>
constexpr int pb_split() { return DYN ? 1 : SH ? 2 : 4; }
template <bool DYN, bool SH>
constexpr int pb_threads() { return DYN ? 128 : 64 * pb_split<DYN, SH>(); }

template <bool DYN, bool SH>
__global__ __launch_bounds__((pb_threads<DYN, SH>())) void k_project_bwd(Args a) {
    if (overflowed(a.status)) return;
    using LA = AccLayout<DYN>;
    constexpr int PB_THREADS = pb_threads<DYN, SH>();
    constexpr int SPLIT = pb_split<DYN, SH>();
    constexpr int GPB = PB_THREADS / SPLIT;  // Gaussians per workgroup
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int h = tid / GPB;                 // which part of the frames
    const int64_t g = static_cast<int64_t>(blockIdx.x) * GPB + (tid % GPB);
    const bool live = g < a.n;
    const int64_t n = a.n;
    const int fpart = (a.frames + SPLIT - 1) / SPLIT;
    const int fb = h * fpart < a.frames ? h * fpart : a.frames;
    const int fe = fb + fpart < a.frames ? fb + fpart : a.frames;
    __shared__ double red[PB_THREADS / 64][4];
    // per-thread gradient accumulators (FP64) live in LDS, see AccLayout
    __shared__ double acc[LA::N][PB_THREADS];
    // cameras of a chunk of frames (R 0-8, t 9-11, centre 12-14) and the
    // per-wave pose sums of each of its frames
    constexpr int FC = SPLIT >= 4 ? 16 : 32;
    __shared__ float cam[SPLIT][FC][15];
    __shared__ float wpose[SPLIT][FC][PB_THREADS / 64 / SPLIT][12];
    __shared__ double iacc[4][PB_THREADS];  // intrinsics gradient, summed over frames
    for (int k = 0; k < 4; ++k) iacc[k][tid] = 0.0;
    // SH coefficient gradients (FP32: at most a few hundred frames are summed)
    __shared__ float acc_sh[SH ? 45 : 1][PB_THREADS];
    for (int k = 0; k < LA::N; ++k) acc[k][tid] = 0.0;
    if (SH)
        for (int k = 0; k < 3 * sh_count(a.sh_degree); ++k) acc_sh[k][tid] = 0.0f;
    // control-point window: gradients of points win .. win + 3, flushed to
    // memory (added) when a frame falls in another knot span
    int win = -1;
    const bool spline = DYN && a.n_ctrl > 0 && a.g_ctrl != nullptr;
    auto flush_window = [&]() {
        if (win < 0) return;
        for (int r = 0; r < 4; ++r)
            for (int k = 0; k < 3; ++k) {
                float* dst = a.g_ctrl + (static_cast<int64_t>(win + r) * 3 + k) * n + g;
                *dst += static_cast<float>(acc[LA::WIN + 3 * r + k][tid]);
                acc[LA::WIN + 3 * r + k][tid] = 0.0;
            }
    };
    if (spline && live && !a.accumulate)
        for (int64_t i = 0; i < static_cast<int64_t>(a.n_ctrl) * 3; ++i) a.g_ctrl[i * n + g] = 0.0f;

    // a static Gaussian's shape (scales, rotation, 3D covariance, opacity) is
    // the same in every frame
    AdjIn Pstatic = {};
    if (!DYN && live) shape_inputs<false>(a, g, 0.0f, Pstatic);
    // the next frame's count, slot offset and record are loaded one frame ahead
    uint32_t cnt_n = 0u, base_n = 0u;
    Record rec_n = {};
    // (unconditional loads: no wait on the count before the record is requested)
    auto fetch = [&](int f) {
        const int64_t i = static_cast<int64_t>(f) * a.n + (live ? g : 0);
        cnt_n = live ? a.gcnt[i] : 0u;
        base_n = live ? a.goff[i] : 0u;
        rec_n = a.rec[i];
    };
    if (fb < fe) fetch(fb);
#pragma unroll 1
    for (int c0 = 0; c0 < fpart; c0 += FC) {  // the same chunk count in every wave (uniform barriers)
        const int f0 = fb + c0;
        const int nf = fe - f0 < FC ? (fe - f0 > 0 ? fe - f0 : 0) : FC;
        __syncthreads();  // the previous chunk's cameras and pose sums are consumed
        for (int q = tid; q < SPLIT * FC; q += PB_THREADS) {
            const int hh = q / FC, fi = q % FC;
            const int ff = hh * fpart + c0 + fi;
            const int fend = (hh + 1) * fpart < a.frames ? (hh + 1) * fpart : a.frames;
            if (ff < fend) {
                const CamD c = load_camera(a.poses + 7 * ff);
                for (int k = 0; k < 9; ++k) cam[hh][fi][k] = c.ok ? static_cast<float>(c.R[k]) : 0.0f;
                for (int k = 0; k < 3; ++k) cam[hh][fi][9 + k] = c.ok ? static_cast<float>(c.t[k]) : 0.0f;
                for (int i = 0; i < 3; ++i)
                    cam[hh][fi][12 + i] = c.ok ? static_cast<float>(-(c.R[0 * 3 + i] * c.t[0] +
                                                                      c.R[1 * 3 + i] * c.t[1] + c.R[2 * 3 + i] * c.t[2]))
                                               : 0.0f;
            }
        }
        __syncthreads();
#pragma unroll 1
        for (int fi = 0; fi < nf; ++fi) {
            const int f = f0 + fi;
            uint32_t cnt = cnt_n;
            const uint32_t base = base_n;
            const Record rec = rec_n;
            if (f + 1 < fe) fetch(f + 1);
            if (static_cast<int64_t>(base) + cnt > a.k_cap) cnt = 0u;  // only after an internal error
            const float* camR = cam[h][fi];
            const float* camT = cam[h][fi] + 9;
            const float* camC = cam[h][fi] + 12;
            float pose[12];
            for (int k = 0; k < 12; ++k) pose[k] = 0.0f;
            if (cnt) {
                // PU records per round, loads issued together (past the end
                // they repeat a valid record and are not added), summed in
                // order k = 0, 1, ...; the first round is requested before the
                // frame's projection inputs are computed, which do not need it.
                // Only the records the adjoint wrote this pass (bit set in
                // pused) are added: the others belong to entries behind their
                // tile's last contributor and hold stale values.
                constexpr uint32_t PU = 8;
                float r[PU][PART];
                uint32_t w0 = 0u, w1 = 0u;  // pused words holding the round's bits
                auto load_round = [&](uint32_t k0) {
                    const uint32_t wi = (base + k0) >> 5;
                    w0 = a.pused[wi];
                    w1 = a.pused[wi + 1];
#pragma unroll
                    for (uint32_t u = 0; u < PU; ++u) {
                        const uint32_t k = k0 + u < cnt ? k0 + u : k0;
                        const float* pp = a.part + static_cast<int64_t>(base + k) * PART;
#pragma unroll
                        for (int m = 0; m < PART; ++m) r[u][m] = pp[m];
                    }
                };
                load_round(0);
                const float t = a.times ? a.times[f] : a.t0;
                AdjIn P = Pstatic;
                if (DYN) shape_inputs<DYN>(a, g, t, P);
                frame_inputs<DYN>(a, g, rec, camR, camT, t, P);
                double dd[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
                for (uint32_t k0 = 0;;) {
                    const uint32_t bits = static_cast<uint32_t>(
                        ((static_cast<uint64_t>(w1) << 32) | w0) >> ((base + k0) & 31u));
#pragma unroll
                    for (uint32_t u = 0; u < PU; ++u)
                        if (k0 + u < cnt && ((bits >> u) & 1u))
#pragma unroll
                            for (int m = 0; m < PART; ++m) dd[m] += r[u][m];
                    k0 += PU;
                    if (k0 >= cnt) break;
                    load_round(k0);
                }
                float d[9];
                for (int k = 0; k < 9; ++k) d[k] = static_cast<float>(dd[k]);
                float go[14], gi[4];
                projection_adjoint<!DYN>(a, camR, P, d, go, pose, gi);
                if (a.g_intr)
                    for (int k = 0; k < 4; ++k) iacc[k][tid] += gi[k];
                if (SH) {
                    float dv[3];
                    const float dc[3] = {go[11], go[12], go[13]};
                    sh_adjoint<PB_THREADS>(a, g, P, camC, dc, acc_sh, tid, dv);
                    for (int j = 0; j < 3; ++j) {
                        go[j] += dv[j];
                        // C = -Rc^T tc, dL/dC = -dv: dL/dtc = Rc dv, dL/dRc[j][i] = tc[j] dv[i]
                        pose[9 + j] += camR[j * 3 + 0] * dv[0] + camR[j * 3 + 1] * dv[1] + camR[j * 3 + 2] * dv[2];
                        for (int i = 0; i < 3; ++i) pose[j * 3 + i] += camT[j] * dv[i];
                    }
                }
                for (int k = 0; k < 14; ++k) acc[k][tid] += go[k];
                const double t1 = t, t2 = t1 * t1, t3 = t2 * t1;
                if (!DYN && a.mean_coeffs)
                    for (int k = 0; k < 3; ++k) {
                        acc[LA::CUBIC + k][tid] += go[k] * t1;
                        acc[LA::CUBIC + 3 + k][tid] += go[k] * t2;
                        acc[LA::CUBIC + 6 + k][tid] += go[k] * t3;
                    }
                if (DYN) {
                    if (spline) {
                        if (P.span != win) {
                            flush_window();
                            win = P.span;
                        }
                        for (int r = 0; r < 4; ++r)
                            for (int k = 0; k < 3; ++k) acc[LA::WIN + 3 * r + k][tid] += P.N[r] * go[k];
                    }
                    if (a.scale_coeffs)
                        for (int k = 0; k < 3; ++k) {
                            acc[LA::SCALE + k][tid] += go[3 + k] * t1;
                            acc[LA::SCALE + 3 + k][tid] += go[3 + k] * t2;
                            acc[LA::SCALE + 6 + k][tid] += go[3 + k] * t3;
                        }
                    if (a.quat_coeffs)
                        for (int k = 0; k < 4; ++k) {
                            acc[LA::QUAT + k][tid] += go[6 + k] * t1;
                            acc[LA::QUAT + 4 + k][tid] += go[6 + k] * t2;
                            acc[LA::QUAT + 8 + k][tid] += go[6 + k] * t3;
                        }
                }
            }
            if (a.g_poses) {  // wave sums of this frame's pose contributions
                float v[16];
#pragma unroll
                for (int k = 0; k < 12; ++k) v[k] = pose[k];
#pragma unroll
                for (int k = 12; k < 16; ++k) v[k] = 0.0f;
                const float x = reduce_scatter16(v, lane);
                const int idx = reduce_scatter16_index(lane);
                if ((lane & 3) == 0 && idx < 12) wpose[h][fi][w % (PB_THREADS / 64 / SPLIT)][idx] = x;
            }
        }
        if (a.g_poses) {
            __syncthreads();
            constexpr int WPH = PB_THREADS / 64 / SPLIT;  // waves per part
            for (int q = tid; q < SPLIT * FC * 12; q += PB_THREADS) {
                const int hh = q / (FC * 12), r = q % (FC * 12), fi = r / 12, k = r % 12;
                const int ff = hh * fpart + c0 + fi;
                const int fend = (hh + 1) * fpart < a.frames ? (hh + 1) * fpart : a.frames;
                if (ff >= fend) continue;
                double v = 0.0;
                for (int ww = 0; ww < WPH; ++ww) v += static_cast<double>(wpose[hh][fi][ww][k]);
                a.pose_part[(static_cast<int64_t>(blockIdx.x) * a.frames + ff) * 12 + k] = v;
            }
        }
    }
    if (a.g_intr) {  // uniform: every thread takes part in the block reduction
        __syncthreads();
        for (int k = 0; k < 4; ++k) {
            const double v = wave_sum_f64(iacc[k][tid]);
            if (lane == 0) red[w][k] = v;
        }
        __syncthreads();
        if (tid < 4) {
            double v = 0.0;
            for (int ww = 0; ww < PB_THREADS / 64; ++ww) v += red[ww][tid];
            a.intr_part[static_cast<int64_t>(blockIdx.x) * 4 + tid] = v;
        }
    }
    if (SPLIT > 1) {  // add the later parts' accumulators to part 0's, in order
        __syncthreads();
        if (h == 0) {
            for (int k = 0; k < LA::N; ++k) {
                double v = acc[k][tid];
                for (int hh = 1; hh < SPLIT; ++hh) v += acc[k][tid + hh * GPB];
                acc[k][tid] = v;
            }
            if (SH)
                for (int k = 0; k < 3 * sh_count(a.sh_degree); ++k) {
                    float v = acc_sh[k][tid];
                    for (int hh = 1; hh < SPLIT; ++hh) v += acc_sh[k][tid + hh * GPB];
                    acc_sh[k][tid] = v;
                }
        }
    }
    if (!live || h != 0) return;
    if (spline) flush_window();
    auto put = [&](float* dst, int64_t idx, double v) {
        if (!dst) return;
        if (a.accumulate) dst[idx] += static_cast<float>(v);
        else dst[idx] = static_cast<float>(v);
    };
    double gsq[7];  // log-scales, quaternion
    if (DYN) {
        for (int k = 0; k < 7; ++k) gsq[k] = acc[3 + k][tid];
    } else {  // dL/dSig summed over the frames, through the shape once
        // a Gaussian culled in every frame (e.g. for non-finite parameters)
        // has dL/dSig = 0 exactly; its shape may hold NaN, so it is not taken
        // through the chain (0 * NaN would poison its gradient)
        float Gs[6], o7[7];
        bool touched = false;
        for (int k = 0; k < 6; ++k) {
            Gs[k] = static_cast<float>(acc[3 + k][tid]);
            touched = touched || Gs[k] != 0.0f;
        }
        if (touched) sigma_adjoint(Gs, Pstatic, o7);
        for (int k = 0; k < 7; ++k) gsq[k] = touched ? o7[k] : 0.0;
    }
    for (int k = 0; k < 3; ++k) {
        if (a.n_ctrl == 0) put(a.g_means, k * n + g, acc[k][tid]);
        put(a.g_log_scales, k * n + g, gsq[k]);
        put(a.g_colors, k * n + g, acc[11 + k][tid]);
    }
    for (int k = 0; k < 4; ++k) put(a.g_quats, k * n + g, gsq[3 + k]);
    put(a.g_opacity, g, acc[10][tid]);
    if (!DYN && a.mean_coeffs)
        for (int c = 0; c < 3; ++c)
            for (int k = 0; k < 3; ++k) put(a.g_coeffs, (c * 3 + k) * n + g, acc[LA::CUBIC + c * 3 + k][tid]);
    if (DYN && a.scale_coeffs)
        for (int c = 0; c < 3; ++c)
            for (int k = 0; k < 3; ++k) put(a.g_scale_coeffs, (c * 3 + k) * n + g, acc[LA::SCALE + c * 3 + k][tid]);
    if (DYN && a.quat_coeffs)
        for (int c = 0; c < 3; ++c)
            for (int k = 0; k < 4; ++k) put(a.g_quat_coeffs, (c * 4 + k) * n + g, acc[LA::QUAT + c * 4 + k][tid]);
    if (SH)
        for (int k = 0; k < 3 * sh_count(a.sh_degree); ++k) put(a.g_sh, static_cast<int64_t>(k) * n + g, acc_sh[k][tid]);
}

// Per frame: sum the workgroups' pose partials (each of the 256 threads takes
// a strided subset of workgroups, then a fixed-order tree over threads), then
// map dL/dRc and dL/dtc to the unnormalised pose quaternion and translation.
__global__ __launch_bounds__(256) void k_pose_finalize(Args a, int64_t n_blocks) {
    const int f = blockIdx.x;
    __shared__ double red[256][13];
    double v[12];
    for (int k = 0; k < 12; ++k) v[k] = 0.0;
    for (int64_t b = threadIdx.x; b < n_blocks; b += 256) {
        const double* p = a.pose_part + (b * a.frames + f) * 12;
        for (int k = 0; k < 12; ++k) v[k] += p[k];
    }
    for (int k = 0; k < 12; ++k) red[threadIdx.x][k] = v[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int k = 0; k < 12; ++k) red[threadIdx.x][k] += red[threadIdx.x + s][k];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double acc[12];
        for (int k = 0; k < 12; ++k) acc[k] = red[0][k];
        const CamD cam = load_camera(a.poses + 7 * f);
        double dq[4] = {0, 0, 0, 0};
        if (cam.ok) quat_grad(cam.qh, cam.qn, acc, dq);
        float* out = a.g_poses + 7 * f;
        const bool bad = overflowed(a.status);
        for (int k = 0; k < 4; ++k) out[k] = bad ? 0.0f : static_cast<float>(dq[k]);
        for (int k = 0; k < 3; ++k) out[4 + k] = bad ? 0.0f : static_cast<float>(acc[9 + k]);
    }
}

// Intrinsics gradient: fixed-order sum of the workgroups' partials.
__global__ __launch_bounds__(256) void k_intr_finalize(Args a, int64_t n_blocks) {
    __shared__ double red[256][4];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t b = threadIdx.x; b < n_blocks; b += 256)
        for (int k = 0; k < 4; ++k) v[k] += a.intr_part[b * 4 + k];
    for (int k = 0; k < 4; ++k) red[threadIdx.x][k] = v[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int k = 0; k < 4; ++k) red[threadIdx.x][k] += red[threadIdx.x + s][k];
        __syncthreads();
    }
    if (threadIdx.x < 4) {
        const float g = overflowed(a.status) ? 0.0f : static_cast<float>(red[0][threadIdx.x]);
        if (a.accumulate) a.g_intr[threadIdx.x] += g;
        else a.g_intr[threadIdx.x] = g;
    }
}

// Gaussians per workgroup of each variant.
template <bool DYN, bool SH>
constexpr int pb_gaussians() { return pb_threads<DYN, SH>() / pb_split<DYN, SH>(); }
static_assert(pb_gaussians<false, false>() == 64 && pb_gaussians<false, true>() == 64 &&
                  pb_gaussians<true, false>() >= 64 && pb_gaussians<true, true>() >= 64,
              "the static variants have the most workgroups");

// Upper bound over the variants.
int64_t project_bwd_blocks(int64_t n) {
    constexpr int gpb = pb_gaussians<false, false>();
    return (n + gpb - 1) / gpb;
}

static int64_t blocks_for(int64_t n, bool dyn, bool sh) {
    const int gpb = dyn ? (sh ? pb_gaussians<true, true>() : pb_gaussians<true, false>())
                        : (sh ? pb_gaussians<false, true>() : pb_gaussians<false, false>());
    return (n + gpb - 1) / gpb;
}

hipError_t launch_project_bwd(const Args& a, hipStream_t stream) {
    const bool dyn = a.n_ctrl > 0 || a.scale_coeffs || a.quat_coeffs;
    const bool sh = a.sh_degree > 0;
    const int64_t nb = blocks_for(a.n, dyn, sh);
    const dim3 grid(static_cast<uint32_t>(nb > 0 ? nb : 1));
    if (nb > 0) {
        if (dyn && sh)
            hipLaunchKernelGGL((k_project_bwd<true, true>), grid, dim3(pb_threads<true, true>()), 0, stream, a);
        else if (dyn)
            hipLaunchKernelGGL((k_project_bwd<true, false>), grid, dim3(pb_threads<true, false>()), 0, stream, a);
        else if (sh)
            hipLaunchKernelGGL((k_project_bwd<false, true>), grid, dim3(pb_threads<false, true>()), 0, stream, a);
        else
            hipLaunchKernelGGL((k_project_bwd<false, false>), grid, dim3(pb_threads<false, false>()), 0, stream, a);
    }
    if (a.g_poses)
        hipLaunchKernelGGL(k_pose_finalize, dim3(static_cast<uint32_t>(a.frames)), dim3(256), 0, stream, a, nb);
    if (a.g_intr) {
        if (nb > 0) hipLaunchKernelGGL(k_intr_finalize, dim3(1), dim3(256), 0, stream, a, nb);
        else hipLaunchKernelGGL(k_intr_finalize, dim3(1), dim3(256), 0, stream, a, int64_t(0));
    }
    return hipGetLastError();
}

}  // namespace gv
