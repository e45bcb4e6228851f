// Camera-motion Neural ODE (Eq. 1, Sec. 3.4): fused MLP + RK4 forward and its
// discrete adjoint, each in one single-wave workgroup.
//
// The integration is a serial chain of (F-1) * S * 4 evaluations of the
// 8 -> 64 -> 64 -> 7 tanh MLP, so latency, not throughput, is what matters:
// lane j owns hidden unit j and keeps its weights in VGPRs (row j of W1 and W2,
// column j of W3, and for the adjoint also column j of W2); the hidden layer
// is exchanged through LDS (broadcast reads) and the 7 outputs are summed over
// the lanes by one reduce-scatter.  The state z is carried in FP64, the MLP runs in FP32.
// The forward pass records every evaluation's input and both hidden
// activations so that the adjoint needs no recomputation; the adjoint's
// serial chain records each evaluation's cotangents, and the parameter
// gradient (outer products summed over the evaluations) is formed from those
// records by parallel kernels afterwards.
#include "gv_internal.h"

namespace gv {

constexpr int ODE_H = 64;
constexpr int ODE_S = 7;
constexpr int ODE_REC = 8 + ODE_H + ODE_H;  // x, h1, h2 of one evaluation
static_assert(ODE_REC % 4 == 0, "records start on 16-byte boundaries");
// offsets of the parameter blocks in theta
constexpr int OFF_W1 = 0, OFF_B1 = 512, OFF_W2 = 576, OFF_B2 = 4672, OFF_W3 = 4736, OFF_B3 = 5184, N_THETA = 5191;

constexpr int ODE_ADJ = ODE_H + ODE_H + 8;  // da1, da2, dy (+ pad) of one evaluation
constexpr int ODE_CHUNKS = 64;              // partial sums of the parameter gradient

struct OdeLayout {
    size_t evals, chunks, chunk;
    size_t acts, zf, adj, part, total;
};

static inline size_t ode_align(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

OdeLayout ode_layout(int frames, int substeps) {
    OdeLayout L;
    L.evals = static_cast<size_t>(frames - 1) * substeps * 4;
    L.chunks = L.evals < ODE_CHUNKS ? (L.evals > 0 ? L.evals : 1) : ODE_CHUNKS;
    L.chunk = (L.evals + L.chunks - 1) / L.chunks;
    L.acts = 0;
    L.zf = ode_align(L.evals * ODE_REC * sizeof(float));
    L.adj = L.zf + ode_align(static_cast<size_t>(frames) * ODE_S * sizeof(double));
    L.part = L.adj + ode_align(L.evals * ODE_ADJ * sizeof(float));
    L.total = L.part + ode_align(L.chunks * N_THETA * sizeof(float));
    return L;
}

__device__ __forceinline__ float ode_tanh(float x) { return tanhf(x); }

// Sum of 8 values over the 64 lanes at once: cross-half and cross-row swaps,
// then DPP within rows; afterwards lanes 8 i .. 8 i + 7 hold the wave total of
// value i.  The order of the additions is fixed.
__device__ __forceinline__ float reduce_scatter8(float (&v)[8], int lane) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 4]), false, false);
        v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 2]), false, false);
        v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    const bool b3 = lane & 8;
    const float keep = b3 ? v[1] : v[0], send = b3 ? v[0] : v[1];
    float x = keep + dpp_f(send, 0x128);
    x = x + dpp_f(x, 0x141);
    x = x + dpp_f(x, 0x4E);
    return x + dpp_f(x, 0xB1);
}

// Copy a 64-float LDS row into registers: every read is issued, then a
// scheduling barrier keeps the arithmetic that uses them after the reads.
__device__ __forceinline__ void lds_row(const float* row, float (&r)[ODE_H]) {
    const float4* q = reinterpret_cast<const float4*>(row);
#pragma unroll
    for (int k = 0; k < ODE_H / 4; ++k) {
        const float4 v = q[k];
        r[4 * k] = v.x;
        r[4 * k + 1] = v.y;
        r[4 * k + 2] = v.z;
        r[4 * k + 3] = v.w;
    }
    __builtin_amdgcn_sched_barrier(0);
}

// One MLP evaluation at (y, t); lanes hold hidden unit j = lane.  Returns the
// 7 outputs (uniform).  If rec != nullptr, stores x, h1, h2 there.
__device__ __forceinline__ void mlp_eval(const double y[ODE_S], double t, const float w1[8], float b1,
                                         const float w2[ODE_H], float b2, const float w3[ODE_S],
                                         const float* b3, float* h1s, float* rec, float out[ODE_S]) {
    const int j = threadIdx.x;
    float x[8];
    for (int k = 0; k < ODE_S; ++k) x[k] = static_cast<float>(y[k]);
    x[7] = static_cast<float>(t);
    float a1 = b1;
    for (int k = 0; k < 8; ++k) a1 = __builtin_fmaf(w1[k], x[k], a1);
    const float h1 = ode_tanh(a1);
    h1s[j] = h1;
    __syncthreads();
    // the single wave cannot hide LDS latency behind other waves: all of the
    // hidden layer's reads are issued before the first product
    float hv[ODE_H];
    lds_row(h1s, hv);
    float a2 = b2;
    for (int k = 0; k < ODE_H; ++k) a2 = __builtin_fmaf(w2[k], hv[k], a2);
    const float h2 = ode_tanh(a2);
    float v[8];
    for (int i = 0; i < ODE_S; ++i) v[i] = w3[i] * h2;
    v[7] = 0.0f;
    const float sum = reduce_scatter8(v, j);
    for (int i = 0; i < ODE_S; ++i) out[i] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sum), 8 * i)) + b3[i];
    if (rec) {
        if (j == 0) {  // x is uniform: one lane writes it (records are 16-byte aligned)
            reinterpret_cast<float4*>(rec)[0] = make_float4(x[0], x[1], x[2], x[3]);
            reinterpret_cast<float4*>(rec)[1] = make_float4(x[4], x[5], x[6], x[7]);
        }
        rec[8 + j] = h1;
        rec[8 + ODE_H + j] = h2;
    }
    __syncthreads();
}

__device__ __forceinline__ void write_pose(const double z[ODE_S], float* pose) {
    if (threadIdx.x != 0) return;
    const double n = sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2] + z[3] * z[3]);
    for (int k = 0; k < 4; ++k) pose[k] = static_cast<float>(z[k] / n);
    for (int k = 4; k < ODE_S; ++k) pose[k] = static_cast<float>(z[k]);
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_ode_fwd(const float* __restrict__ theta, const float* __restrict__ z0,
                                                int frames, int substeps, float* __restrict__ poses,
                                                float* __restrict__ acts, double* __restrict__ zf) {
    const int j = threadIdx.x;
    __shared__ __align__(16) float h1s[ODE_H];
    float w1[8], w2[ODE_H], w3[ODE_S], b3[ODE_S];
    for (int k = 0; k < 8; ++k) w1[k] = theta[OFF_W1 + j * 8 + k];
    const float b1 = theta[OFF_B1 + j];
    for (int k = 0; k < ODE_H; ++k) w2[k] = theta[OFF_W2 + j * ODE_H + k];
    const float b2 = theta[OFF_B2 + j];
    for (int i = 0; i < ODE_S; ++i) w3[i] = theta[OFF_W3 + i * ODE_H + j];
    for (int i = 0; i < ODE_S; ++i) b3[i] = theta[OFF_B3 + i];
    double z[ODE_S];
    for (int k = 0; k < ODE_S; ++k) z[k] = z0[k];
    write_pose(z, poses);
    if (j < ODE_S) zf[j] = z[j];
    if (frames < 2) return;
    const double h = 1.0 / (static_cast<double>(substeps) * (frames - 1));
    int e = 0;
    for (int f = 1; f < frames; ++f) {
        for (int s = 0; s < substeps; ++s) {
            const double t = (static_cast<double>(f - 1) * substeps + s) * h;
            float k1[ODE_S], k2[ODE_S], k3[ODE_S], k4[ODE_S];
            double y[ODE_S];
            mlp_eval(z, t, w1, b1, w2, b2, w3, b3, h1s, acts + static_cast<size_t>(e++) * ODE_REC, k1);
            for (int k = 0; k < ODE_S; ++k) y[k] = z[k] + 0.5 * h * k1[k];
            mlp_eval(y, t + 0.5 * h, w1, b1, w2, b2, w3, b3, h1s, acts + static_cast<size_t>(e++) * ODE_REC, k2);
            for (int k = 0; k < ODE_S; ++k) y[k] = z[k] + 0.5 * h * k2[k];
            mlp_eval(y, t + 0.5 * h, w1, b1, w2, b2, w3, b3, h1s, acts + static_cast<size_t>(e++) * ODE_REC, k3);
            for (int k = 0; k < ODE_S; ++k) y[k] = z[k] + h * k3[k];
            mlp_eval(y, t + h, w1, b1, w2, b2, w3, b3, h1s, acts + static_cast<size_t>(e++) * ODE_REC, k4);
            for (int k = 0; k < ODE_S; ++k)
                z[k] = z[k] + (h / 6.0) * (static_cast<double>(k1[k]) + 2.0 * k2[k] + 2.0 * k3[k] + k4[k]);
        }
        write_pose(z, poses + ODE_S * f);
        if (j < ODE_S) zf[ODE_S * f + j] = z[j];
    }
}

// Cotangent of the state from the cotangent of the pose (q/|q|, t).
// The value lane k holds (wave-uniform result).
__device__ __forceinline__ double lane_value(double v, int k) {
    const uint64_t b = __double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(b), k);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(b >> 32), k);
    return __longlong_as_double((static_cast<uint64_t>(hi) << 32) | lo);
}

__device__ __forceinline__ void pose_cotangent(const double* z, const float* dp, double out[ODE_S]) {
    const double n = sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2] + z[3] * z[3]);
    double qh[4], dot = 0.0;
    for (int k = 0; k < 4; ++k) {
        qh[k] = z[k] / n;
        dot += qh[k] * static_cast<double>(dp[k]);
    }
    for (int k = 0; k < 4; ++k) out[k] = (static_cast<double>(dp[k]) - qh[k] * dot) / n;
    for (int k = 4; k < ODE_S; ++k) out[k] = dp[k];
}

// Vector-Jacobian product of one recorded evaluation with upstream dy: returns
// dL/dy (state part) and records the evaluation's cotangents (da1, da2 of the
// hidden pre-activations, dy) in adj; the parameter gradient is summed from
// these records afterwards, off the serial chain.
__device__ __forceinline__ void mlp_vjp(float h1, float h2, const double dy[ODE_S], const float w1[8],
                                        const float w2c[ODE_H], const float w3[ODE_S], float* da2s, float* adj,
                                        double gx[ODE_S]) {
    const int j = threadIdx.x;
    float dyf[ODE_S];
    for (int i = 0; i < ODE_S; ++i) dyf[i] = static_cast<float>(dy[i]);
    float dh2 = 0.0f;
    for (int i = 0; i < ODE_S; ++i) dh2 = __builtin_fmaf(w3[i], dyf[i], dh2);
    const float da2 = dh2 * (1.0f - h2 * h2);
    da2s[j] = da2;
    __syncthreads();
    float dv[ODE_H];
    lds_row(da2s, dv);
    float dh1 = 0.0f;
    for (int k = 0; k < ODE_H; ++k) dh1 = __builtin_fmaf(w2c[k], dv[k], dh1);
    const float da1 = dh1 * (1.0f - h1 * h1);
    adj[j] = da1;
    adj[ODE_H + j] = da2;
    if (j == 0)
        for (int i = 0; i < ODE_S; ++i) adj[2 * ODE_H + i] = dyf[i];
    float v[8];
    for (int m = 0; m < ODE_S; ++m) v[m] = w1[m] * da1;
    v[7] = 0.0f;
    const float sum = reduce_scatter8(v, j);
    for (int m = 0; m < ODE_S; ++m)
        gx[m] = static_cast<double>(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(sum), 8 * m)));
    __syncthreads();
}

__global__ __launch_bounds__(64) void k_ode_bwd(const float* __restrict__ theta, int frames, int substeps,
                                                const float* __restrict__ dposes, const float* __restrict__ acts,
                                                const double* __restrict__ zf, float* __restrict__ adj,
                                                float* __restrict__ dz0) {
    const int j = threadIdx.x;
    __shared__ __align__(16) float da2s[ODE_H];
    float w1[8], w2c[ODE_H], w3[ODE_S];
    for (int k = 0; k < 8; ++k) w1[k] = theta[OFF_W1 + j * 8 + k];
    for (int k = 0; k < ODE_H; ++k) w2c[k] = theta[OFF_W2 + k * ODE_H + j];
    for (int i = 0; i < ODE_S; ++i) w3[i] = theta[OFF_W3 + i * ODE_H + j];

    double lam[ODE_S];
    pose_cotangent(zf + ODE_S * (frames - 1), dposes + ODE_S * (frames - 1), lam);
    if (frames > 1) {
        const double h = 1.0 / (static_cast<double>(substeps) * (frames - 1));
        // The evaluations are taken in descending order; this lane's hidden
        // activations of the next one are requested while the current one is
        // differentiated (one wave: nothing else hides their latency).
        const size_t elast = static_cast<size_t>(frames - 1) * substeps * 4 - 1;
        float nh1 = acts[elast * ODE_REC + 8 + j], nh2 = acts[elast * ODE_REC + 8 + ODE_H + j];
        for (int f = frames - 1; f >= 1; --f) {
            // frame f - 1's state and pose cotangent, needed after this
            // frame's substeps: requested now, one component per lane (vector
            // loads, which the LDS waits of the substeps do not wait for)
            const double zl = j < ODE_S ? zf[ODE_S * (f - 1) + j] : 0.0;
            const float dl = j < ODE_S ? dposes[ODE_S * (f - 1) + j] : 0.0f;
            for (int s = substeps - 1; s >= 0; --s) {
                const size_t e0 = (static_cast<size_t>(f - 1) * substeps + s) * 4;
                double dz[ODE_S], dk[4][ODE_S], gx[ODE_S];
                for (int k = 0; k < ODE_S; ++k) {
                    dz[k] = lam[k];
                    dk[0][k] = (h / 6.0) * lam[k];
                    dk[1][k] = (h / 3.0) * lam[k];
                    dk[2][k] = (h / 3.0) * lam[k];
                    dk[3][k] = (h / 6.0) * lam[k];
                }
                auto vjp = [&](size_t e, const double dy[ODE_S]) {
                    const float h1 = nh1, h2 = nh2;
                    if (e > 0) {
                        nh1 = acts[(e - 1) * ODE_REC + 8 + j];
                        nh2 = acts[(e - 1) * ODE_REC + 8 + ODE_H + j];
                    }
                    mlp_vjp(h1, h2, dy, w1, w2c, w3, da2s, adj + e * ODE_ADJ, gx);
                };
                vjp(e0 + 3, dk[3]);
                for (int k = 0; k < ODE_S; ++k) { dz[k] += gx[k]; dk[2][k] += h * gx[k]; }
                vjp(e0 + 2, dk[2]);
                for (int k = 0; k < ODE_S; ++k) { dz[k] += gx[k]; dk[1][k] += 0.5 * h * gx[k]; }
                vjp(e0 + 1, dk[1]);
                for (int k = 0; k < ODE_S; ++k) { dz[k] += gx[k]; dk[0][k] += 0.5 * h * gx[k]; }
                vjp(e0, dk[0]);
                for (int k = 0; k < ODE_S; ++k) lam[k] = dz[k] + gx[k];
            }
            double zk[ODE_S], c[ODE_S];
            float dp[ODE_S];
            for (int k = 0; k < ODE_S; ++k) {
                zk[k] = lane_value(zl, k);
                dp[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(dl), k));
            }
            pose_cotangent(zk, dp, c);
            for (int k = 0; k < ODE_S; ++k) lam[k] += c[k];
        }
    }
    if (j == 0)
        for (int k = 0; k < ODE_S; ++k) dz0[k] = static_cast<float>(lam[k]);
}

// Parameter gradient from the recorded evaluations (x, h1, h2 in acts; da1,
// da2, dy in adj): dW1 = sum da1 x^T, db1 = sum da1, dW2 = sum da2 h1^T,
// db2 = sum da2, dW3 = sum dy h2^T, db3 = sum dy.  Thread p of chunk c sums
// parameter p over the evaluations [c chunk, (c + 1) chunk) in order; the
// chunks are then added in order, so the result is reproducible.
__global__ __launch_bounds__(256) void k_ode_grad_part(const float* __restrict__ acts, const float* __restrict__ adj,
                                                       int64_t evals, int64_t chunk, float* __restrict__ part) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= N_THETA) return;
    const int64_t e0 = blockIdx.y * chunk;
    const int64_t e1 = e0 + chunk < evals ? e0 + chunk : evals;
    // parameter p as (cotangent index in adj, activation index in acts or -1)
    int ia, ix;
    if (p < OFF_B1) ia = p / 8, ix = p % 8;                                          // W1[j][k]
    else if (p < OFF_W2) ia = p - OFF_B1, ix = -1;                                   // b1[j]
    else if (p < OFF_B2) ia = ODE_H + (p - OFF_W2) / ODE_H, ix = 8 + (p - OFF_W2) % ODE_H;  // W2[j][k]
    else if (p < OFF_W3) ia = ODE_H + (p - OFF_B2), ix = -1;                         // b2[j]
    else if (p < OFF_B3) ia = 2 * ODE_H + (p - OFF_W3) / ODE_H, ix = 8 + ODE_H + (p - OFF_W3) % ODE_H;  // W3[i][j]
    else ia = 2 * ODE_H + (p - OFF_B3), ix = -1;                                     // b3[i]
    float acc = 0.0f;
    for (int64_t e = e0; e < e1; ++e) {
        const float g = adj[e * ODE_ADJ + ia];
        acc = ix >= 0 ? __builtin_fmaf(g, acts[e * ODE_REC + ix], acc) : acc + g;
    }
    part[blockIdx.y * static_cast<int64_t>(N_THETA) + p] = acc;
}

__global__ __launch_bounds__(256) void k_ode_grad_final(const float* __restrict__ part, int64_t chunks,
                                                        float* __restrict__ dtheta) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= N_THETA) return;
    float acc = 0.0f;
    for (int64_t c = 0; c < chunks; ++c) acc += part[c * N_THETA + p];
    dtheta[p] = acc;
}

// Trajectory error of a camera path against a reference pose table (the
// per-frame poses judging the learned camera of Sec. 3.4).  Per frame, in
// FP64: the camera centre c = -R(q)^T t of each pose and the distance between
// the two centres; the rotation error is the angle of the relative rotation
// R(q) R(q_ref)^T, taken from the relative quaternion q (x) conj(q_ref) as
// 2 atan2(|vector part|, |scalar part|) (both quaternions normalised first).
// One workgroup; the two sums are reduced in a fixed order.
constexpr int PE_WG = 256;

__device__ __forceinline__ void pose_centre(const float* p, double qn[4], double c[3]) {
    double q[4] = {p[0], p[1], p[2], p[3]};
    const double r = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; ++k) qn[k] = q[k] / r;
    const double w = qn[0], x = qn[1], y = qn[2], z = qn[3];
    const double R[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                            {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                            {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
    for (int i = 0; i < 3; ++i) c[i] = -(R[0][i] * p[4] + R[1][i] * p[5] + R[2][i] * p[6]);
}

__global__ __launch_bounds__(PE_WG) void k_pose_error(const float* __restrict__ poses, const float* __restrict__ ref,
                                                      int32_t frames, float* __restrict__ per_frame,
                                                      float* __restrict__ summary) {
    __shared__ double s_t[PE_WG], s_a[PE_WG];
    double st = 0.0, sa = 0.0;
    for (int f = threadIdx.x; f < frames; f += PE_WG) {
        double q1[4], c1[3], q2[4], c2[3];
        pose_centre(poses + 7 * f, q1, c1);
        pose_centre(ref + 7 * f, q2, c2);
        const double dx = c1[0] - c2[0], dy = c1[1] - c2[1], dz = c1[2] - c2[2];
        const double te = sqrt(dx * dx + dy * dy + dz * dz);
        // relative quaternion q1 (x) conj(q2)
        const double w = q1[0] * q2[0] + q1[1] * q2[1] + q1[2] * q2[2] + q1[3] * q2[3];
        const double vx = q2[0] * q1[1] - q1[0] * q2[1] - (q1[2] * q2[3] - q1[3] * q2[2]);
        const double vy = q2[0] * q1[2] - q1[0] * q2[2] - (q1[3] * q2[1] - q1[1] * q2[3]);
        const double vz = q2[0] * q1[3] - q1[0] * q2[3] - (q1[1] * q2[2] - q1[2] * q2[1]);
        const double ang = 2.0 * atan2(sqrt(vx * vx + vy * vy + vz * vz), fabs(w));
        per_frame[2 * f] = static_cast<float>(te);
        per_frame[2 * f + 1] = static_cast<float>(ang);
        st += te * te;
        sa += ang;
    }
    s_t[threadIdx.x] = st;
    s_a[threadIdx.x] = sa;
    __syncthreads();
    for (int h = PE_WG / 2; h > 0; h >>= 1) {
        if (static_cast<int>(threadIdx.x) < h) {
            s_t[threadIdx.x] += s_t[threadIdx.x + h];
            s_a[threadIdx.x] += s_a[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        summary[0] = static_cast<float>(sqrt(s_t[0] / frames));
        summary[1] = static_cast<float>(s_a[0] / frames);
    }
}

}  // namespace gv

using namespace gv;

extern "C" {

gv_status gv_camera_ode_workspace_bytes(int32_t frames, int32_t substeps, size_t* out) {
    if (frames < 1 || frames > 100000 || substeps < 1 || substeps > 64 || !out) return GV_ERR_INVALID_ARG;
    *out = ode_layout(frames, substeps).total;
    return GV_OK;
}

gv_status gv_camera_ode_fwd(const float* theta, const float* z0, int32_t frames, int32_t substeps, float* poses,
                            void* ws, size_t ws_bytes, void* stream) {
    if (!theta || !z0 || !poses || frames < 1 || frames > 100000 || substeps < 1 || substeps > 64)
        return GV_ERR_INVALID_ARG;
    const OdeLayout L = ode_layout(frames, substeps);
    if (!ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255u)) return GV_ERR_WORKSPACE;
    char* b = static_cast<char*>(ws);
    hipLaunchKernelGGL(k_ode_fwd, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream), theta, z0, frames, substeps,
                       poses, reinterpret_cast<float*>(b + L.acts), reinterpret_cast<double*>(b + L.zf));
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? GV_OK : GV_ERR_HIP;
}

gv_status gv_camera_ode_bwd(const float* theta, const float* z0, int32_t frames, int32_t substeps,
                            const float* dL_dposes, float* dtheta, float* dz0, void* ws, size_t ws_bytes,
                            void* stream) {
    if (!theta || !z0 || !dL_dposes || !dtheta || !dz0 || frames < 1 || frames > 100000 || substeps < 1 ||
        substeps > 64)
        return GV_ERR_INVALID_ARG;
    const OdeLayout L = ode_layout(frames, substeps);
    if (!ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255u)) return GV_ERR_WORKSPACE;
    char* b = static_cast<char*>(ws);
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const float* acts = reinterpret_cast<const float*>(b + L.acts);
    float* adj = reinterpret_cast<float*>(b + L.adj);
    float* part = reinterpret_cast<float*>(b + L.part);
    hipLaunchKernelGGL(k_ode_bwd, dim3(1), dim3(64), 0, st, theta, frames, substeps, dL_dposes, acts,
                       reinterpret_cast<const double*>(b + L.zf), adj, dz0);
    const dim3 pg((N_THETA + 255) / 256, static_cast<uint32_t>(L.chunks));
    hipLaunchKernelGGL(k_ode_grad_part, pg, dim3(256), 0, st, acts, adj, static_cast<int64_t>(L.evals),
                       static_cast<int64_t>(L.chunk), part);
    hipLaunchKernelGGL(k_ode_grad_final, dim3((N_THETA + 255) / 256), dim3(256), 0, st, part,
                       static_cast<int64_t>(L.chunks), dtheta);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? GV_OK : GV_ERR_HIP;
}

gv_status gv_pose_error(const float* poses, const float* ref_poses, int32_t frames, float* per_frame, float* summary,
                        void* stream) {
    if (!poses || !ref_poses || !per_frame || !summary || frames < 1 || frames > 100000) return GV_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_pose_error, dim3(1), dim3(PE_WG), 0, static_cast<hipStream_t>(stream), poses, ref_poses,
                       frames, per_frame, summary);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? GV_OK : GV_ERR_HIP;
}

}  // extern "C"
