// Adjoint of the EWA projection.  One thread per Gaussian loops over the
// frames: it sums the per-(Gaussian, tile) partials left by the compositing
// adjoint (contiguous slots of this Gaussian), re-derives the frame's
// projection in FP64 and applies the chain rule down to the stored
// parameters, accumulating the shared parameters over frames in registers.
// Each frame's pose gradient (dL/dRc, dL/dtc) is reduced per workgroup in a
// fixed order; a second kernel sums the workgroups and maps it to the 7-vector
// pose.  Everything is deterministic (no floating-point atomics).
#include "gv_internal.h"

namespace gv {

constexpr int PB_THREADS = 128;

// Chain rule for one (frame, Gaussian).  d: dL/d(u, v, A00, A01, A11, o, r, g,
// b) with A01 the single off-diagonal conic parameter (it enters q twice).
__device__ __forceinline__ void projection_adjoint(const Args& a, const CamD& cam, const ProjD& P, double t,
                                                   const double d[9], double dmu[3], double dls[3], double dq[4],
                                                   double& deta, double dcol[3], double dRc[9], double dtc[3]) {
    const double A0 = P.A[0], A1 = P.A[1], A2 = P.A[2];
    // gradient w.r.t. the symmetric conic matrix
    const double G00 = d[2], G01 = 0.5 * d[3], G11 = d[4];
    // A = cov^-1  =>  dL/dcov = -A G A
    const double AG00 = A0 * G00 + A1 * G01, AG01 = A0 * G01 + A1 * G11;
    const double AG10 = A1 * G00 + A2 * G01, AG11 = A1 * G01 + A2 * G11;
    const double C00 = -(AG00 * A0 + AG01 * A1);
    const double C01 = -0.5 * ((AG00 * A1 + AG01 * A2) + (AG10 * A0 + AG11 * A1));
    const double C11 = -(AG10 * A1 + AG11 * A2);
    // cov = T Sig T^T + dil I with T = J Rc (2x3)
    const double* Tm = P.T;
    // dSig = T^T C T (3x3 symmetric)
    double CT[6];  // C T, 2x3
    for (int j = 0; j < 3; ++j) {
        CT[j] = C00 * Tm[j] + C01 * Tm[3 + j];
        CT[3 + j] = C01 * Tm[j] + C11 * Tm[3 + j];
    }
    double GS[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) GS[i * 3 + j] = Tm[i] * CT[j] + Tm[3 + i] * CT[3 + j];
    // dT = 2 C T Sig
    const double* S = P.Sig;  // xx xy xz yy yz zz
    const double Sm[9] = {S[0], S[1], S[2], S[1], S[3], S[4], S[2], S[4], S[5]};
    double dT[6];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j)
            dT[i * 3 + j] = 2.0 * (CT[i * 3 + 0] * Sm[0 * 3 + j] + CT[i * 3 + 1] * Sm[1 * 3 + j] +
                                   CT[i * 3 + 2] * Sm[2 * 3 + j]);
    // T = J Rc with J = [[j00, 0, j02], [0, j11, j12]]
    const double* Rc = cam.R;
    const double mx = P.m[0], my = P.m[1], mz = P.m[2];
    const double iz = 1.0 / mz, iz2 = iz * iz, iz3 = iz2 * iz;
    const double fx = a.fx, fy = a.fy;
    const double j00 = fx * iz, j02 = -fx * mx * iz2, j11 = fy * iz, j12 = -fy * my * iz2;
    double dJ00 = 0, dJ02 = 0, dJ11 = 0, dJ12 = 0;
    for (int j = 0; j < 3; ++j) {
        dJ00 += dT[j] * Rc[0 * 3 + j];
        dJ02 += dT[j] * Rc[2 * 3 + j];
        dJ11 += dT[3 + j] * Rc[1 * 3 + j];
        dJ12 += dT[3 + j] * Rc[2 * 3 + j];
        dRc[0 * 3 + j] += j00 * dT[j];
        dRc[1 * 3 + j] += j11 * dT[3 + j];
        dRc[2 * 3 + j] += j02 * dT[j] + j12 * dT[3 + j];
    }
    // J(m) and (u, v)(m)
    double dm[3];
    dm[0] = -dJ02 * fx * iz2 + d[0] * fx * iz;
    dm[1] = -dJ12 * fy * iz2 + d[1] * fy * iz;
    dm[2] = -dJ00 * fx * iz2 + dJ02 * 2.0 * fx * mx * iz3 - dJ11 * fy * iz2 + dJ12 * 2.0 * fy * my * iz3 -
            d[0] * fx * mx * iz2 - d[1] * fy * my * iz2;
    // m = Rc mu + tc
    for (int k = 0; k < 3; ++k) {
        dmu[k] = Rc[0 * 3 + k] * dm[0] + Rc[1 * 3 + k] * dm[1] + Rc[2 * 3 + k] * dm[2];
        dtc[k] += dm[k];
    }
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) dRc[i * 3 + k] += dm[i] * P.mu[k];
    // Sig = M M^T, M = R diag(s)
    double dR[9];
    double ds[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double dM = 2.0 * (GS[i * 3 + 0] * P.M[0 * 3 + j] + GS[i * 3 + 1] * P.M[1 * 3 + j] +
                                     GS[i * 3 + 2] * P.M[2 * 3 + j]);
            dR[i * 3 + j] = dM * P.s[j];
            ds[j] += dM * P.R[i * 3 + j];
        }
    for (int k = 0; k < 3; ++k) dls[k] = ds[k] * P.s[k];
    quat_grad(P.qh, P.qn, dR, dq);
    deta = d[5] * P.o * (1.0 - P.o);
    dcol[0] = d[6];
    dcol[1] = d[7];
    dcol[2] = d[8];
    (void)t;
}

__global__ __launch_bounds__(PB_THREADS) void k_project_bwd(Args a) {
    if (overflowed(a.status)) return;
    const int64_t g = static_cast<int64_t>(blockIdx.x) * PB_THREADS + threadIdx.x;
    const bool live = g < a.n;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __shared__ double red[PB_THREADS / 64][12];

    double gmu[3] = {0, 0, 0}, gls[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, geta = 0, gcol[3] = {0, 0, 0};
    double gco[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int f = 0; f < a.frames; ++f) {
        double pr[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        const int64_t i = static_cast<int64_t>(f) * a.n + g;
        uint32_t cnt = live ? a.gcnt[i] : 0u;
        const uint32_t base = live ? a.goff[i] : 0u;
        if (static_cast<int64_t>(base) + cnt > a.k_cap) cnt = 0u;  // only after an internal error
        if (cnt) {
            double d[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            for (uint32_t k = 0; k < cnt; ++k) {
                const float4 pa = a.partA[base + k];
                const float4 pb = a.partB[base + k];
                const float pc = a.partC[base + k];
                d[0] += pa.x; d[1] += pa.y; d[2] += pa.z; d[3] += pa.w;
                d[4] += pb.x; d[5] += pb.y; d[6] += pb.z; d[7] += pb.w; d[8] += pc;
            }
            const CamD cam = load_camera(a.poses + 7 * f);
            const double t = a.times ? static_cast<double>(a.times[f]) : static_cast<double>(a.t0);
            ProjD P;
            if (project_gaussian(a, g, cam, t, P)) {
                double dmu[3], dls[3], dq[4], deta, dcol[3];
                projection_adjoint(a, cam, P, t, d, dmu, dls, dq, deta, dcol, pr, pr + 9);
                for (int k = 0; k < 3; ++k) {
                    gmu[k] += dmu[k];
                    gls[k] += dls[k];
                    gcol[k] += dcol[k];
                    gco[k] += dmu[k] * t;
                    gco[3 + k] += dmu[k] * t * t;
                    gco[6 + k] += dmu[k] * t * t * t;
                }
                for (int k = 0; k < 4; ++k) gq[k] += dq[k];
                geta += deta;
            }
        }
        if (a.g_poses) {
            for (int k = 0; k < 12; ++k) {
                const double v = wave_sum_f64(pr[k]);
                if (lane == 0) red[w][k] = v;
            }
            __syncthreads();
            if (threadIdx.x < 12) {
                double v = 0.0;
                for (int ww = 0; ww < PB_THREADS / 64; ++ww) v += red[ww][threadIdx.x];
                a.pose_part[(static_cast<int64_t>(blockIdx.x) * a.frames + f) * 12 + threadIdx.x] = v;
            }
            __syncthreads();
        }
    }
    if (!live) return;
    const int64_t n = a.n;
    auto put = [&](float* dst, int64_t idx, double v) {
        if (!dst) return;
        if (a.accumulate) dst[idx] += static_cast<float>(v);
        else dst[idx] = static_cast<float>(v);
    };
    for (int k = 0; k < 3; ++k) {
        put(a.g_means, k * n + g, gmu[k]);
        put(a.g_log_scales, k * n + g, gls[k]);
        put(a.g_colors, k * n + g, gcol[k]);
    }
    for (int k = 0; k < 4; ++k) put(a.g_quats, k * n + g, gq[k]);
    put(a.g_opacity, g, geta);
    if (a.mean_coeffs)
        for (int c = 0; c < 3; ++c)
            for (int k = 0; k < 3; ++k) put(a.g_coeffs, (c * 3 + k) * n + g, gco[c * 3 + k]);
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

int64_t project_bwd_blocks(int64_t n) { return (n + PB_THREADS - 1) / PB_THREADS; }

hipError_t launch_project_bwd(const Args& a, hipStream_t stream) {
    const int64_t nb = project_bwd_blocks(a.n);
    if (nb > 0) hipLaunchKernelGGL(k_project_bwd, dim3(static_cast<uint32_t>(nb)), dim3(PB_THREADS), 0, stream, a);
    if (a.g_poses)
        hipLaunchKernelGGL(k_pose_finalize, dim3(static_cast<uint32_t>(a.frames)), dim3(256), 0, stream, a, nb);
    return hipGetLastError();
}

}  // namespace gv
