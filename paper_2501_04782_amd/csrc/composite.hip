// Front-to-back alpha compositing of each 16x16 tile (forward) and its adjoint
// (back to front, transmittance recomputed by division from the stored final
// value).  One workgroup per (frame, tile).  The tile's depth-sorted entries
// are staged through LDS in batches of B, each with a mask of the parts of the
// tile its 3-sigma ellipse meets, and each part of the tile walks the list of
// the entries meeting it:
//  - quadrant kernels (256 threads): wave w owns the 8x8 quadrant
//    (w & 1, w >> 1), lane l its pixel (l & 7, l >> 3);
//  - sub-block forward (256 threads): each 16-lane row owns a 4x4 block;
//  - paired adjoint (128 threads): each half-wave owns a quadrant, two pixels
//    per lane;
//  - per-tile kernels (64 threads, the defaults): each 16-lane row of the one
//    wave owns a quadrant, four pixels of one column per lane.
// A workgroup stops staging once every pixel has terminated.
#include "gv_internal.h"

#include <type_traits>

namespace gv {

// One staged entry, 48 bytes.  The conic is stored pre-multiplied by
// K_EXP = -log2(e)/2 and the exponent carries log2 of the opacity, so the
// per-pixel exponent q' = K_EXP q + log2 o is the quadratic form plus a
// constant and the unclamped alpha o exp(-q/2) is one exp2.  `thr` folds the
// 3-sigma cut (q <= 9) and the opacity floor (alpha >= 1/255) into a single
// test q' >= thr; the inert padding entry has thr = +inf.
struct Staged {
    float4 p0;  // (u, v) in tile-local pixel-centre coordinates, K a, K 2b
    float4 p1;  // K c, log2 o, r, g
    float4 p2;  // b, thr, Gaussian index (bits), opacity
};
constexpr uint32_t STAGED_BYTES = sizeof(Staged);
static_assert(STAGED_BYTES == 48, "three 16-byte LDS reads per entry");
constexpr float INV_K_EXP = 1.0f / K_EXP;

// Exponent q' = K_EXP d^T A d + log2 o with d = pixel - centre (2^q' is the
// unclamped alpha), and the entry's threshold.  Shared by every compositing
// kernel, forward and adjoint, so that all of them re-derive the same values
// and decisions.  Evaluated as dy (K c dy + K 2b dx) + (K a dx dx + log2 o):
// the two terms in dx alone (footprint_row) are shared by the pixels of one
// column.
struct FootRow {
    float t;  // K 2b dx
    float s;  // K a dx dx + log2 o
};

__device__ __forceinline__ FootRow footprint_row(float dx, const float4& p0, const float4& p1) {
    return FootRow{p0.w * dx, __builtin_fmaf(p0.z * dx, dx, p1.y)};
}

__device__ __forceinline__ float footprint_q(float dy, const FootRow& r, const float4& p1) {
    return __builtin_fmaf(dy, __builtin_fmaf(p1.x, dy, r.t), r.s);
}

__device__ __forceinline__ float footprint_q(float dx, float dy, const float4& p0, const float4& p1) {
    return footprint_q(dy, footprint_row(dx, p0, p1), p1);
}

// log2 of the opacity as staged (-inf for o = 0, whose entries never pass)
__device__ __forceinline__ float log2_opacity(float o) { return __builtin_amdgcn_logf(o); }

__device__ __forceinline__ float entry_threshold(float lo) {
    // q <= 9 is q' >= 9 K_EXP + log2 o; alpha >= 1/255 is q' >= -log2 255
    return fmaxf(__builtin_fmaf(Q_MAX, K_EXP, lo), -7.99435343685885793773f);
}

// Stage entry `gid` of the tile: gather its record and colour and move the
// centre to tile-local coordinates (exact subtraction in FP64, then one
// rounding).  `conic` returns the unscaled conic (a, b, c).
__device__ __forceinline__ void stage_entry(const Args& a, int f, uint32_t gid, double ox, double oy, Staged& st,
                                            float3& conic) {
    if (gid >= static_cast<uint64_t>(a.n)) {  // only after an internal error: stage an inert entry
        st.p0 = make_float4(0.f, 0.f, 0.f, 0.f);
        st.p1 = make_float4(0.f, 0.f, 0.f, 0.f);
        st.p2 = make_float4(0.f, __builtin_inff(), 0.f, 0.f);
        conic = make_float3(0.f, 0.f, 0.f);
        return;
    }
    const Record r = a.rec[static_cast<int64_t>(f) * a.n + gid];
    const ColorOp co = a.col4[static_cast<int64_t>(f) * a.col_stride + gid];
    const float lu = static_cast<float>(r.u - ox);
    const float lv = static_cast<float>(r.v - oy);
    const float lo = log2_opacity(co.o);
    st.p0 = make_float4(lu, lv, K_EXP * r.a, K_EXP * (2.0f * r.b));
    st.p1 = make_float4(K_EXP * r.c, lo, co.r, co.g);
    st.p2 = make_float4(co.b, entry_threshold(lo), __uint_as_float(gid), co.o);
    conic = make_float3(r.a, r.b, r.c);
}

// Mask of the S x S pixel blocks of the tile that the entry's slightly
// inflated 3-sigma ellipse meets: S = 8, the four quadrants (bit q); S = 4,
// the 16 blocks (bit 4 q + r: block r of quadrant q).  Per band of S pixel
// rows, the ellipse restricted to the band is convex, so its x-extent is an
// interval whose ends lie at the ellipse's right- and leftmost points clamped
// into the band; a block is kept if its columns meet that interval (widened
// by a rounding margin).
template <int S>
__device__ __forceinline__ uint32_t band_mask(const Staged& st, float3 cn, int xlim, int ylim) {
    constexpr int NB = TILE / S;
    auto bit = [](int by, int bx) {
        return S == 8 ? 2 * by + bx : 4 * (2 * (by >> 1) + (bx >> 1)) + 2 * (by & 1) + (bx & 1);
    };
    const float a = cn.x, b = cn.y, c = cn.z;
    if (a == 0.f && b == 0.f && c == 0.f) return 0u;  // inert
    const float lu = st.p0.x, lv = st.p0.y;
    const float det = static_cast<float>(static_cast<double>(a) * c - static_cast<double>(b) * b);
    uint32_t all = 0;
    for (int by = 0; by < NB; ++by)
        for (int bx = 0; bx < NB; ++bx)
            if (S * bx <= xlim && S * by <= ylim) all |= 1u << bit(by, bx);
    if (!(det > 0.0f) || !(a > 0.0f) || !(c > 0.0f)) return all;  // degenerate conic: the exact test decides
    // hardware sqrt and reciprocals (about 1 ulp): far inside the margins below
    const float rdet = __builtin_amdgcn_rcpf(det);
    const float hy = __builtin_amdgcn_sqrtf(SUB_Q_SLACK * a * rdet);  // half-extent in y
    const float hx = __builtin_amdgcn_sqrtf(SUB_Q_SLACK * c * rdet);  // half-extent in x
    const float dyr = -b * hx * __builtin_amdgcn_rcpf(c);             // dy of the rightmost point
    const float aq = a * SUB_Q_SLACK;
    const float inva = __builtin_amdgcn_rcpf(a);
    const float tol = 1e-3f + 1e-4f * hy;
    uint32_t m = 0;
    for (int by = 0; by < NB; ++by) {
        const int y0 = S * by;
        if (y0 > ylim) break;
        const int y1 = min(y0 + S - 1, ylim);
        const float d0 = static_cast<float>(y0) - lv, d1 = static_cast<float>(y1) - lv;
        if (d0 > hy + tol || d1 < -hy - tol) continue;
        float lo = fmaxf(d0, -hy), hi = fminf(d1, hy);
        if (lo > hi) lo = hi = fminf(fmaxf(0.5f * (d0 + d1), -hy), hy);  // within the tolerance of a tip
        const float dr = fminf(fmaxf(dyr, lo), hi);
        const float dl = fminf(fmaxf(-dyr, lo), hi);
        const float sr = __builtin_amdgcn_sqrtf(fmaxf(0.0f, aq - det * dr * dr));
        const float sl = __builtin_amdgcn_sqrtf(fmaxf(0.0f, aq - det * dl * dl));
        const float xr = (-b * dr + sr) * inva;
        const float xl = (-b * dl - sl) * inva;
        const float eps = 0.01f + 1e-4f * (fabsf(xl) + fabsf(xr));
        const float xlo = lu + xl - eps, xhi = lu + xr + eps;
        for (int bx = 0; bx < NB; ++bx) {
            const int x0 = S * bx;
            if (x0 > xlim) break;
            const int x1 = min(x0 + S - 1, xlim);
            if (static_cast<float>(x0) <= xhi && static_cast<float>(x1) >= xlo) m |= 1u << bit(by, bx);
        }
    }
    return m;
}

__device__ __forceinline__ uint32_t quadrant_mask(const Staged& st, float3 cn, int xlim, int ylim) {
    return band_mask<8>(st, cn, xlim, ylim);
}

__device__ __forceinline__ uint32_t block_mask(const Staged& st, float3 cn, int xlim, int ylim) {
    return band_mask<4>(st, cn, xlim, ylim);
}

// Whether the entry's alpha can reach the clamp ALPHA_MAX at some pixel of
// the tile.  For a positive-definite conic the exact exponent
// K_EXP q + log2 o never exceeds log2 o.  footprint_q evaluates it with five
// roundings of terms bounded by M = |K a| dx^2 + |2 K b| |dx dy| + |K c| dy^2
// + |log2 o| over the tile's pixel offsets, so it errs by less than
// 6 u M < 1e-6 M (u = 2^-24), and exp2 by about one ulp: alpha stays below
// ALPHA_MAX at every pixel of the tile when log2 o + 1e-6 M is below
// log2(ALPHA_MAX) - 1e-5.  A conic that is not clearly positive definite
// after rounding may clamp.  The paired adjoint drops the clamp from its
// per-pixel loop for a batch in which no entry of a wave's lists can reach
// it, with identical results.
constexpr uint32_t MAY_CLAMP_BIT = 0x80000000u;  // in the staged block masks
constexpr float LOG2_ALPHA_MAX = -0.014499569695115091f;  // log2(0.99)

__device__ __forceinline__ bool may_clamp(const Staged& st, float3 cn) {
    const double a = cn.x, b = cn.y, c = cn.z;
    if (!(a > 0.0) || !(a * c - b * b > 1e-6 * a * c)) return true;
    const float lu = st.p0.x, lv = st.p0.y;
    const float dx = fmaxf(fabsf(lu), fabsf(static_cast<float>(TILE - 1) - lu));
    const float dy = fmaxf(fabsf(lv), fabsf(static_cast<float>(TILE - 1) - lv));
    const float m = fabsf(st.p0.z) * dx * dx + fabsf(st.p0.w) * dx * dy + fabsf(st.p1.x) * dy * dy + fabsf(st.p1.y);
    return !(st.p1.y + 1e-6f * m < LOG2_ALPHA_MAX - 1e-5f);
}

// Inert entry that pads the wave lists to whole groups (never reaches a pixel).
__device__ __forceinline__ void stage_inert(Staged& st) {
    st.p0 = make_float4(0.f, 0.f, 0.f, 0.f);
    st.p1 = make_float4(0.f, 0.f, 0.f, 0.f);
    st.p2 = make_float4(0.f, __builtin_inff(), 0.f, 0.f);
}

__device__ __forceinline__ const Staged& staged_at(const Staged* sh, uint32_t off) {
    return *reinterpret_cast<const Staged*>(reinterpret_cast<const char*>(sh) + off);
}

// Per-entry partials from the wave-summed moments of D = alpha dL/dalpha
// (sum D dx, sum D dy, sum D dx^2, sum D dx dy, sum D dy^2, sum D) and the
// colour sums, with the unscaled conic (a, b, c) and opacity o:
// (dL/du, dL/dv, dL/dA00, dL/dA01, dL/dA11, dL/do, dL/dr, dL/dg, dL/db).
__device__ __forceinline__ void finish_partials(float (&v)[PART], float ca, float cb, float cc, float o) {
    const float X = v[0], Y = v[1];
    v[0] = ca * X + cb * Y;
    v[1] = cb * X + cc * Y;
    v[2] = -0.5f * v[2];
    v[3] = -v[3];
    v[4] = -0.5f * v[4];
    v[5] = o > 0.0f ? v[5] * __builtin_amdgcn_rcpf(o) : 0.0f;
}

// Entries per unrolled group of the quadrant forward loop.
constexpr int FWD_GROUP = 8;

// VIS: also flag every (frame, Gaussian) that contributes to a pixel of the
// tile (vis[f * N + g] = 1), for the per-Gaussian visibility counts.
template <int B, bool VIS>
__global__ __launch_bounds__(WG) void k_composite_fwd(Args a) {
    if (overflowed(a.status)) return;
    const int f = blockIdx.y;
    const int tile = blockIdx.x;
    const int txi = tile % a.tiles_x, tyi = tile / a.tiles_x;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lx = ((w & 1) << 3) | (lane & 7), ly = ((w >> 1) << 3) | (lane >> 3);
    const int px = txi * TILE + lx, py = tyi * TILE + ly;
    const bool inside = px < a.width && py < a.height;
    const int64_t seg = static_cast<int64_t>(f) * a.tiles + tile;
    uint32_t s, e;
    bucket_range(a, seg, s, e);
    const double ox = txi * TILE + 0.5, oy = tyi * TILE + 0.5;
    const int xlim = a.width - 1 - txi * TILE, ylim = a.height - 1 - tyi * TILE;

    // sh[B] is an inert entry that pads the wave lists to whole groups; the
    // lists hold byte offsets into sh
    __shared__ Staged sh[B + 1];
    __shared__ uint32_t shm[B];
    __shared__ float red[WG / 64];
    __shared__ __align__(16) uint32_t wl[WG / 64][B + FWD_GROUP];
    if (tid == 0) stage_inert(sh[B]);

    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    uint32_t last = 0;
    bool done = !inside;
    const float fx = static_cast<float>(lx), fy = static_cast<float>(ly);

    // each batch's entry ids are requested during the previous batch's loop
    uint32_t gnext = tid < static_cast<int>(min(static_cast<uint32_t>(B), e - s)) ? a.sgid[s + tid] : 0u;
    for (uint32_t b0 = s; b0 < e; b0 += B) {
        if (__syncthreads_count(!done) == 0) break;
        const uint32_t nb = min(static_cast<uint32_t>(B), e - b0);
        if (tid < static_cast<int>(nb)) {
            Staged st;
            float3 conic;
            stage_entry(a, f, gnext, ox, oy, st, conic);
            sh[tid] = st;
            shm[tid] = quadrant_mask(st, conic, xlim, ylim);
        }
        __syncthreads();
        if (e - b0 > B && tid < static_cast<int>(min(static_cast<uint32_t>(B), e - b0 - B))) gnext = a.sgid[b0 + B + tid];
        if (__ballot(!done) == 0) continue;  // wave-uniform; the barriers are outside
        // this wave's entries, front to back (ballot compaction)
        int cnt = 0;
        for (int j0 = 0; j0 < static_cast<int>(nb); j0 += 64) {
            const int j = j0 + lane;
            const bool on = j < static_cast<int>(nb) && ((shm[j] >> w) & 1u);
            const uint64_t bal = __ballot(on);
            if (on) wl[w][cnt + __popcll(bal & ((1ull << lane) - 1ull))] = static_cast<uint32_t>(j) * STAGED_BYTES;
            cnt += __popcll(bal);
        }
        if (lane < FWD_GROUP) wl[w][cnt + lane] = static_cast<uint32_t>(B) * STAGED_BYTES;
        __builtin_amdgcn_wave_barrier();
        // Branch-free groups: an entry that misses the pixel, or reaches it
        // after it terminated, adds a zero weight and leaves T unchanged.
        // loff: byte offset of this lane's last entry taken in this batch.
        int loff = -1;
        for (int g = 0; g < cnt; g += FWD_GROUP) {
            static_assert(FWD_GROUP == 8, "two 16-byte reads of the wave list per group");
            const uint4 ja = *reinterpret_cast<const uint4*>(&wl[w][g]);
            const uint4 jb = *reinterpret_cast<const uint4*>(&wl[w][g + 4]);
            const uint32_t jo[FWD_GROUP] = {ja.x, ja.y, ja.z, ja.w, jb.x, jb.y, jb.z, jb.w};
            float4 P0[FWD_GROUP], P1[FWD_GROUP];
            float2 P2[FWD_GROUP];
#pragma unroll
            for (int r = 0; r < FWD_GROUP; ++r) {
                const Staged& st = staged_at(sh, jo[r]);
                P0[r] = st.p0;
                P1[r] = st.p1;
                P2[r] = make_float2(st.p2.x, st.p2.y);
            }
#pragma unroll
            for (int r = 0; r < FWD_GROUP; ++r) {
                const float4 p0 = P0[r];
                const float4 p1 = P1[r];
                const float dx = fx - p0.x, dy = fy - p0.y;
                const float q = footprint_q(dx, dy, p0, p1);
                const bool hit = !done && q >= P2[r].y;
                const float al = fminf(ALPHA_MAX, __builtin_amdgcn_exp2f(q));
                const float tn = __builtin_fmaf(-al, T, T);
                const bool take = hit && tn >= T_MIN;  // else stop before this entry
                done = done || (hit != take);
                const float Tn = take ? tn : T;
                const float wgt = T - Tn;  // alpha T to rounding; 0 when not taken
                c0 = __builtin_fmaf(p1.z, wgt, c0);
                c1 = __builtin_fmaf(p1.w, wgt, c1);
                c2 = __builtin_fmaf(P2[r].x, wgt, c2);
                T = Tn;
                loff = take ? static_cast<int>(jo[r]) : loff;
                if (VIS && __ballot(take) != 0 && lane == 0) {
                    const uint32_t gid = __float_as_uint(staged_at(sh, jo[r]).p2.z);
                    if (gid < static_cast<uint64_t>(a.n)) a.vis[static_cast<int64_t>(f) * a.n + gid] = 1;
                }
            }
            if (__ballot(!done) == 0) break;
        }
        if (loff >= 0) last = b0 - s + static_cast<uint32_t>(loff) / STAGED_BYTES + 1;
    }

    float sq = 0.0f;
    if (inside) {
        const int64_t P = static_cast<int64_t>(a.width) * a.height;
        const int64_t pix = static_cast<int64_t>(py) * a.width + px;
        c0 = __builtin_fmaf(T, a.bg[0], c0);
        c1 = __builtin_fmaf(T, a.bg[1], c1);
        c2 = __builtin_fmaf(T, a.bg[2], c2);
        float* img = a.images + static_cast<int64_t>(f) * 3 * P + pix;
        img[0] = c0;
        img[P] = c1;
        img[2 * P] = c2;
        a.tfin[static_cast<int64_t>(f) * P + pix] = T;
        a.nlast[static_cast<int64_t>(f) * P + pix] = last;
        if (a.tfin_out) a.tfin_out[static_cast<int64_t>(f) * P + pix] = T;
        if (a.targets && a.loss) {
            const float* tg = a.targets + static_cast<int64_t>(f) * 3 * P + pix;
            const float d0 = c0 - tg[0], d1 = c1 - tg[P], d2 = c2 - tg[2 * P];
            sq = d0 * d0 + d1 * d1 + d2 * d2;
        }
    }
    if (a.targets && a.loss) {
        sq = wave_sum_to_lane63(sq);
        if (lane == 63) red[w] = sq;
        __syncthreads();
        if (tid == 0) a.loss_part[seg] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// Forward with one wave per tile: lanes 16q .. 16q + 15 take quadrant q, each
// lane four pixels of one column of it (rows r, r + 2, r + 4, r + 6), and each
// 16-lane row walks its own quadrant's list front to back (the four lists
// padded with the inert entry to a common length).  The per-pixel arithmetic
// and decisions are those of the quadrant forward (the pixels share the
// exponent's terms in dx), so images, final transmittances and last indices
// are identical; a lane reads each entry's staged data once for its four
// pixels.
constexpr int WGF4 = 64;
constexpr int FWD4_GROUP = 4;

template <int B>
__global__ __launch_bounds__(WGF4) __attribute__((amdgpu_waves_per_eu(4))) void k_composite_fwd4(Args a) {
    constexpr int SPT = B / WGF4;  // entries staged per thread
    static_assert(SPT * WGF4 == B, "whole entries per thread");
    if (overflowed(a.status)) return;
    const int f = blockIdx.y;
    const int tile = blockIdx.x;
    const int txi = tile % a.tiles_x, tyi = tile / a.tiles_x;
    const int lane = threadIdx.x;
    const int quad = lane >> 4, rl = lane & 15;
    const int lx = ((quad & 1) << 3) | (rl & 7), ly0 = ((quad >> 1) << 3) | (rl >> 3);
    const int px = txi * TILE + lx;
    const int64_t seg = static_cast<int64_t>(f) * a.tiles + tile;
    uint32_t s, e;
    bucket_range(a, seg, s, e);
    const double ox = txi * TILE + 0.5, oy = tyi * TILE + 0.5;
    const int xlim = a.width - 1 - txi * TILE, ylim = a.height - 1 - tyi * TILE;

    __shared__ Staged sh[B + 1];
    __shared__ uint32_t shm[B];
    __shared__ uint32_t wl[4][B + FWD4_GROUP];
    if (lane == 0) stage_inert(sh[B]);

    float T[4], c0[4], c1[4], c2[4], fy[4];
    uint32_t last[4];
    bool done[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        T[k] = 1.0f;
        c0[k] = c1[k] = c2[k] = 0.0f;
        last[k] = 0u;
        done[k] = !(px < a.width && tyi * TILE + ly0 + 2 * k < a.height);
        fy[k] = static_cast<float>(ly0 + 2 * k);
    }
    const float fx = static_cast<float>(lx);
    constexpr uint32_t INERT = static_cast<uint32_t>(B) * STAGED_BYTES;
    const uint64_t below = (1ull << lane) - 1ull;

    // each batch's entry ids are requested during the previous batch's loop
    uint32_t gn[SPT];
#pragma unroll
    for (int i = 0; i < SPT; ++i) {
        const uint32_t t = static_cast<uint32_t>(lane + WGF4 * i);
        gn[i] = t < min(static_cast<uint32_t>(B), e - s) ? a.sgid[s + t] : 0u;
    }
    for (uint32_t b0 = s; b0 < e; b0 += B) {
        const bool alive = !(done[0] && done[1] && done[2] && done[3]);
        const uint64_t alive_bal = __ballot(alive);
        if (alive_bal == 0ull) break;  // every pixel of the tile has terminated
        const uint32_t nb = min(static_cast<uint32_t>(B), e - b0);
#pragma unroll
        for (int i = 0; i < SPT; ++i) {
            const uint32_t t = static_cast<uint32_t>(lane + WGF4 * i);
            if (t < nb) {
                Staged st;
                float3 conic;
                stage_entry(a, f, gn[i], ox, oy, st, conic);
                sh[t] = st;
                shm[t] = quadrant_mask(st, conic, xlim, ylim);
            }
        }
        __syncthreads();
        if (e - b0 > B) {
#pragma unroll
            for (int i = 0; i < SPT; ++i) {
                const uint32_t t = static_cast<uint32_t>(lane + WGF4 * i);
                if (t < min(static_cast<uint32_t>(B), e - b0 - B)) gn[i] = a.sgid[b0 + B + t];
            }
        }
        // the four quadrants' lists, front to back; a quadrant whose pixels
        // have all terminated takes none
        int cnt[4] = {0, 0, 0, 0};
        for (int j0 = 0; j0 < static_cast<int>(nb); j0 += 64) {
            const int j = j0 + lane;
            const uint32_t m = j < static_cast<int>(nb) ? shm[j] : 0u;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool on = ((m >> q) & 1u) && ((alive_bal >> (16 * q)) & 0xFFFFull) != 0ull;
                const uint64_t bal = __ballot(on);
                if (on) wl[q][cnt[q] + __popcll(bal & below)] = static_cast<uint32_t>(j) * STAGED_BYTES;
                cnt[q] += __popcll(bal);
            }
        }
        const int cmax = max(max(cnt[0], cnt[1]), max(cnt[2], cnt[3]));
        const int npad = (cmax + FWD4_GROUP - 1) / FWD4_GROUP * FWD4_GROUP;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            for (int k = cnt[q] + lane; k < npad; k += 64) wl[q][k] = INERT;
        const uint32_t* mylist = wl[quad];
        __builtin_amdgcn_wave_barrier();
        // Branch-free groups, as in the quadrant forward; loff: byte offset of
        // each pixel's last entry taken in this batch
        int loff[4] = {-1, -1, -1, -1};
        for (int g = 0; g < npad; g += FWD4_GROUP) {
            uint32_t J[FWD4_GROUP];
            float4 P0[FWD4_GROUP], P1[FWD4_GROUP];
            float2 P2[FWD4_GROUP];
#pragma unroll
            for (int r = 0; r < FWD4_GROUP; ++r) J[r] = mylist[g + r];
#pragma unroll
            for (int r = 0; r < FWD4_GROUP; ++r) {
                const Staged& st = staged_at(sh, J[r]);
                P0[r] = st.p0;
                P1[r] = st.p1;
                P2[r] = make_float2(st.p2.x, st.p2.y);
            }
#pragma unroll
            for (int r = 0; r < FWD4_GROUP; ++r) {
                const float4 p0 = P0[r];
                const float4 p1 = P1[r];
                const float dx = fx - p0.x;
                const FootRow fr = footprint_row(dx, p0, p1);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float dy = fy[k] - p0.y;
                    const float q = footprint_q(dy, fr, p1);
                    const bool hit = !done[k] && q >= P2[r].y;
                    const float al = fminf(ALPHA_MAX, __builtin_amdgcn_exp2f(q));
                    const float tn = __builtin_fmaf(-al, T[k], T[k]);
                    const bool take = hit && tn >= T_MIN;  // else stop before this entry
                    done[k] = done[k] || (hit != take);
                    const float Tn = take ? tn : T[k];
                    const float wgt = T[k] - Tn;  // alpha T to rounding; 0 when not taken
                    c0[k] = __builtin_fmaf(p1.z, wgt, c0[k]);
                    c1[k] = __builtin_fmaf(p1.w, wgt, c1[k]);
                    c2[k] = __builtin_fmaf(P2[r].x, wgt, c2[k]);
                    T[k] = Tn;
                    loff[k] = take ? static_cast<int>(J[r]) : loff[k];
                }
            }
            if (__ballot(!(done[0] && done[1] && done[2] && done[3])) == 0ull) break;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (loff[k] >= 0) last[k] = b0 - s + static_cast<uint32_t>(loff[k]) / STAGED_BYTES + 1;
        __syncthreads();  // the next batch overwrites the staged entries and lists
    }

    float sq = 0.0f;
    const int64_t P = static_cast<int64_t>(a.width) * a.height;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int py = tyi * TILE + ly0 + 2 * k;
        if (!(px < a.width && py < a.height)) continue;
        const int64_t pix = static_cast<int64_t>(py) * a.width + px;
        const float r0 = __builtin_fmaf(T[k], a.bg[0], c0[k]);
        const float r1 = __builtin_fmaf(T[k], a.bg[1], c1[k]);
        const float r2 = __builtin_fmaf(T[k], a.bg[2], c2[k]);
        float* img = a.images + static_cast<int64_t>(f) * 3 * P + pix;
        img[0] = r0;
        img[P] = r1;
        img[2 * P] = r2;
        a.tfin[static_cast<int64_t>(f) * P + pix] = T[k];
        a.nlast[static_cast<int64_t>(f) * P + pix] = last[k];
        if (a.tfin_out) a.tfin_out[static_cast<int64_t>(f) * P + pix] = T[k];
        if (a.targets && a.loss) {
            const float* tg = a.targets + static_cast<int64_t>(f) * 3 * P + pix;
            const float d0 = r0 - tg[0], d1 = r1 - tg[P], d2 = r2 - tg[2 * P];
            sq += d0 * d0 + d1 * d1 + d2 * d2;
        }
    }
    if (a.targets && a.loss) {
        sq = wave_sum_to_lane63(sq);
        if (lane == 63) a.loss_part[seg] = sq;
    }
}

// Per-frame loss: fixed-order sum of the tiles' partial sums.
__global__ __launch_bounds__(WG) void k_loss_finalize(Args a) {
    const int f = blockIdx.x;
    __shared__ float red[WG];
    float s = 0.0f;
    for (int t = threadIdx.x; t < a.tiles; t += WG) s += a.loss_part[static_cast<int64_t>(f) * a.tiles + t];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = WG / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.loss[f] = overflowed(a.status) ? 0.0f : red[0] * a.loss_norm;
}

// One halving step of the reduce-scatter below for lane pairs that differ in
// lane bit 3 or 2 (the bank bits of a DPP row): lanes with the bit clear
// return a + (a of the partner), the others b + (b of the partner).  Two DPP
// adds whose bank masks split the lanes replace a select-then-add; s_nop 1
// gives the wait states a DPP read of a VGPR needs after a VALU write of it.
// partner lane ^ 8; lane bit 3 clear: banks 0 and 1
__device__ __forceinline__ float dpp_pair_add_ror8(float a, float b) {
    float r;
    asm volatile(
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %1, %1 row_ror:8 row_mask:0xf bank_mask:0x3\n\t"
        "v_add_f32_dpp %0, %2, %2 row_ror:8 row_mask:0xf bank_mask:0xc"
        : "=&v"(r)
        : "v"(a), "v"(b));
    return r;
}
// partner lane 7 - p within each 8 lanes; lane bit 2 clear: banks 0 and 2
__device__ __forceinline__ float dpp_pair_add_mirror(float a, float b) {
    float r;
    asm volatile(
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %1, %1 row_half_mirror row_mask:0xf bank_mask:0x5\n\t"
        "v_add_f32_dpp %0, %2, %2 row_half_mirror row_mask:0xf bank_mask:0xa"
        : "=&v"(r)
        : "v"(a), "v"(b));
    return r;
}

// Sum over the 64 lanes of 64 values at once: after six halving stages
// (cross-half swaps for 32 and 16 lanes, DPP within rows for the rest) lane l holds
// the wave total of value l.  Exact in the order of its additions, which is
// fixed.
__device__ __forceinline__ float reduce_scatter64(float (&v)[64], int lane) {
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 32]), false, false);
        v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 16]), false, false);
        v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    const bool b2 = lane & 2, b1 = lane & 1;
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = dpp_pair_add_ror8(v[i], v[i + 8]);
    // row_half_mirror pairs lane p with 7 - p within each 8 lanes: always
    // across bit 2, and with the later xor-2 / xor-1 stages it still merges
    // all 8 lanes
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = dpp_pair_add_mirror(v[i], v[i + 4]);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const float keep = b2 ? v[i + 2] : v[i], send = b2 ? v[i] : v[i + 2];
        v[i] = keep + dpp_f(send, 0x4E);  // quad_perm [2,3,0,1] (partner lane ^ 2)
    }
    {
        const float keep = b1 ? v[1] : v[0], send = b1 ? v[0] : v[1];
        v[0] = keep + dpp_f(send, 0xB1);  // quad_perm [1,0,3,2] (partner lane ^ 1)
    }
    return v[0];
}

// Adjoint of the quadrant loop.  Each wave first lists, back to front, the
// staged entries whose ellipse meets its quadrant; it then takes them in
// groups of RS_GROUP, keeps every lane's 9 partials of each entry in
// registers, and sums all 9 x RS_GROUP values over the wave with one
// reduce-scatter (lane l ends with partial l % 9 of the group's entry l / 9).
constexpr int RS_GROUP = 7;

template <int B>
__global__ __launch_bounds__(WG) void k_composite_bwd(Args a) {
    if (overflowed(a.status)) return;
    const int f = blockIdx.y;
    const int tile = blockIdx.x;
    const int txi = tile % a.tiles_x, tyi = tile / a.tiles_x;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lx = ((w & 1) << 3) | (lane & 7), ly = ((w >> 1) << 3) | (lane >> 3);
    const int px = txi * TILE + lx, py = tyi * TILE + ly;
    const bool inside = px < a.width && py < a.height;
    const int64_t seg = static_cast<int64_t>(f) * a.tiles + tile;
    uint32_t s, e;
    bucket_range(a, seg, s, e);
    const double ox = txi * TILE + 0.5, oy = tyi * TILE + 0.5;
    const int xlim = a.width - 1 - txi * TILE, ylim = a.height - 1 - tyi * TILE;

    // sh[B] is an inert entry that pads the wave lists to whole groups; the
    // lists hold byte offsets into sh
    __shared__ Staged sh[B + 1];
    __shared__ uint32_t shm[B];
    __shared__ float acc[WG / 64][9][B];
    __shared__ uint32_t wl[WG / 64][B + RS_GROUP];
    if (tid == 0) stage_inert(sh[B]);
    __shared__ uint32_t wlast[WG / 64];

    // per-pixel state: T after the current entry and GS = sum_c g_c S_c, the
    // colour composited behind it (S_c, background included) weighted by the
    // upstream gradient; only this weighted sum enters dL/dalpha
    float T = 1.0f, GS = 0.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
    uint32_t last = 0;
    if (inside) {
        const int64_t P = static_cast<int64_t>(a.width) * a.height;
        const int64_t pix = static_cast<int64_t>(py) * a.width + px;
        T = a.tfin[static_cast<int64_t>(f) * P + pix];
        last = a.nlast[static_cast<int64_t>(f) * P + pix];
        const int64_t o3 = static_cast<int64_t>(f) * 3 * P + pix;
        if (a.targets) {
            g0 = (a.images[o3] - a.targets[o3]) * a.loss_scale;
            g1 = (a.images[o3 + P] - a.targets[o3 + P]) * a.loss_scale;
            g2 = (a.images[o3 + 2 * P] - a.targets[o3 + 2 * P]) * a.loss_scale;
        } else {
            g0 = a.dl_dimages[o3];
            g1 = a.dl_dimages[o3 + P];
            g2 = a.dl_dimages[o3 + 2 * P];
        }
        GS = T * (g0 * a.bg[0] + g1 * a.bg[1] + g2 * a.bg[2]);
    }
    // entries at or past a wave's last contributor need no work in that wave,
    // and entries past the tile's last contributor none at all
    uint32_t wmax = last;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) wmax = max(wmax, static_cast<uint32_t>(__shfl_xor(static_cast<int>(wmax), d)));
    if (lane == 0) wlast[w] = wmax;
    __syncthreads();
    uint32_t used = 0;
#pragma unroll
    for (int ww = 0; ww < WG / 64; ++ww) used = max(used, wlast[ww]);
    // each batch's entry ids are requested during the previous batch's loop
    // (the first batch's before the zero partials)
    uint32_t gnext = 0;
    {
        const uint32_t b0f = used > B ? s + used - B : s;
        if (tid < static_cast<int>(s + used - b0f)) gnext = a.sgid[b0f + tid];
    }
    // entries no pixel reached get zero partials
    const float fx = static_cast<float>(lx), fy = static_cast<float>(ly);

    for (int64_t bend = static_cast<int64_t>(s) + used; bend > s; bend -= B) {
        const uint32_t b0 = static_cast<uint32_t>(bend - B > s ? bend - B : s);
        const uint32_t nb = static_cast<uint32_t>(bend - b0);
        if (tid < static_cast<int>(nb)) {
            Staged st;
            float3 conic;
            stage_entry(a, f, gnext, ox, oy, st, conic);
            sh[tid] = st;
            shm[tid] = quadrant_mask(st, conic, xlim, ylim);
        }
        __syncthreads();
        // this batch's slots (for the flush) and the next batch's ids, in
        // flight during the loop
        const uint32_t slot = tid < static_cast<int>(nb) ? a.sslot[b0 + tid] : 0u;
        if (b0 > s) {
            const uint32_t b0n = b0 - s > B ? b0 - B : s;
            if (tid < static_cast<int>(b0 - b0n)) gnext = a.sgid[b0n + tid];
        }
        // this wave's entries, back to front (ballot compaction; the list is
        // written and read by this wave only)
        int cnt = 0;
        for (int j0 = static_cast<int>(nb) - 1; j0 >= 0; j0 -= 64) {
            const int j = j0 - lane;
            const bool on = j >= 0 && ((shm[j] >> w) & 1u) && b0 + j - s < wmax;
            const uint64_t bal = __ballot(on);
            if (on) wl[w][cnt + __popcll(bal & ((1ull << lane) - 1ull))] = static_cast<uint32_t>(j) * STAGED_BYTES;
            cnt += __popcll(bal);
        }
        if (lane < RS_GROUP) wl[w][cnt + lane] = static_cast<uint32_t>(B) * STAGED_BYTES;
        // this pixel's entries in the batch lie below byte offset lim
        const int64_t rl = static_cast<int64_t>(last) - (static_cast<int64_t>(b0) - s);
        const int lim = static_cast<int>(rl < 0 ? 0 : (rl > B ? B : rl)) * static_cast<int>(STAGED_BYTES);
        __builtin_amdgcn_wave_barrier();
        for (int g = 0; g < cnt; g += RS_GROUP) {
            // Branch-free: an entry that does not reach the pixel (or the inert
            // padding entry) takes alpha = 0, which leaves T and the colour
            // behind it exactly unchanged (1 - 0 and its reciprocal are exact)
            // and gives zero partials.
            float P[64];
            P[63] = 0.0f;
            uint32_t J[RS_GROUP];
            float4 P0[RS_GROUP], P1[RS_GROUP];
            float2 P2[RS_GROUP];
#pragma unroll
            for (int r = 0; r < RS_GROUP; ++r) J[r] = wl[w][g + r];
#pragma unroll
            for (int r = 0; r < RS_GROUP; ++r) {
                const Staged& st = staged_at(sh, J[r]);
                P0[r] = st.p0;
                P1[r] = st.p1;
                P2[r] = make_float2(st.p2.x, st.p2.y);
            }
#pragma unroll
            for (int r = 0; r < RS_GROUP; ++r) {
                const float4 p0 = P0[r];
                const float4 p1 = P1[r];
                const float dx = fx - p0.x, dy = fy - p0.y;
                const float q = footprint_q(dx, dy, p0, p1);
                const bool on = (static_cast<int>(J[r]) < lim) & (q >= P2[r].y);
                const float raw = __builtin_amdgcn_exp2f(q);
                const float al = on ? fminf(ALPHA_MAX, raw) : 0.0f;
                const float inv = __builtin_amdgcn_rcpf(1.0f - al);
                const float ai = al * inv;
                const float Tj = T * inv;  // transmittance in front of this entry
                const float wgt = ai * T;  // alpha T_j
                P[r * 9 + 6] = wgt * g0;
                P[r * 9 + 7] = wgt * g1;
                P[r * 9 + 8] = wgt * g2;
                // dL/dalpha = sum_c g_c (c_c T_j - S_c / (1 - alpha))
                //           = (T gc - GS) / (1 - alpha), gc = sum_c g_c c_c, so
                // alpha dL/dalpha = wgt gc - ai GS, and wgt gc is the colour
                // partials weighted by the colour
                const float wgc = __builtin_fmaf(P2[r].x, P[r * 9 + 8], __builtin_fmaf(p1.w, P[r * 9 + 7], p1.z * P[r * 9 + 6]));
                const float Dal = __builtin_fmaf(-ai, GS, wgc);
                GS = GS + wgc;
                T = Tj;
                // a clamped alpha has no gradient w.r.t. the opacity or footprint
                // (alpha = 0 already zeroes entries that do not reach the pixel);
                // with D = alpha dL/dalpha, dL/dq = -D/2 and dL/do = D/o, and the
                // footprint partials are moments of D over the pixel offsets, to
                // which the conic is applied once per entry after the reduction
                const float D = raw < ALPHA_MAX ? Dal : 0.0f;
                const float X = D * dx, Y = D * dy;
                P[r * 9 + 0] = X;
                P[r * 9 + 1] = Y;
                P[r * 9 + 2] = X * dx;
                P[r * 9 + 3] = X * dy;
                P[r * 9 + 4] = Y * dy;
                P[r * 9 + 5] = D;
            }
            const float tot = reduce_scatter64(P, lane);
            const int r = lane / 9;
            if (lane < 9 * RS_GROUP && g + r < cnt) acc[w][lane - 9 * r][wl[w][g + r] / STAGED_BYTES] = tot;
        }
        __syncthreads();
        if (tid < static_cast<int>(nb)) {
            const uint32_t m = shm[tid];
            const uint32_t rel = b0 + tid - s;
            // a wave's slot holds this entry's sums only if the entry was in
            // its list; the waves are added in a fixed order
            bool in[WG / 64];
#pragma unroll
            for (int ww = 0; ww < WG / 64; ++ww) in[ww] = ((m >> ww) & 1u) && rel < wlast[ww];
            // every slot is read (stale slots are in bounds) and selected, so
            // that the sums compile without branches
            float v[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                float x = 0.0f;
#pragma unroll
                for (int ww = 0; ww < WG / 64; ++ww) {
                    const float r = acc[ww][k][tid];
                    x += in[ww] ? r : 0.0f;
                }
                v[k] = x;
            }
            const Staged st = sh[tid];
            finish_partials(v, st.p0.z * INV_K_EXP, 0.5f * st.p0.w * INV_K_EXP, st.p1.x * INV_K_EXP, st.p2.w);
            if (slot < a.k_cap) {
                store_partials_marked(a, slot, v);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Paired-quadrant adjoint.  A 128-thread workgroup owns a 16x16 tile: wave w
// takes the quadrants 2w (lanes 0-31) and 2w + 1 (lanes 32-63), the top or
// bottom half of the tile, and each lane two pixels of its quadrant, (x, y)
// and (x, y + 4).  Each half-wave walks its own quadrant's list (the two
// lists padded with the inert entry to a common length of whole groups); a
// lane adds its two pixels' partials in registers, and one reduce-scatter
// over the 32 lanes of each half (one instruction stream for both halves)
// leaves lane l of a half with the sums 2l and 2l + 1 of that half's group.
// The reduce-scatter is thus paid once per 128 pixels instead of once per 64.
// The two quadrants of a wave add their sums into one zeroed LDS slot per
// entry and partial: two addends give the same sum in either order, so the
// result does not depend on the order of the LDS additions.
// ---------------------------------------------------------------------------
constexpr int WG2 = 128;

// Sums over the 32 lanes of each half-wave of 64 values at once: lane l
// (l < 32 within its half) ends with the half's totals of values 2l (return
// .x) and 2l + 1 (.y).  Stages: lane bit 4 (cross-row swap), bit 3 (row
// rotate by 8), bit 2 (row half-mirror), bits 1 and 0 (quad permutations);
// the order of additions is fixed.
__device__ __forceinline__ float2 reduce_scatter32x2(float (&v)[64], int lane) {
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 32]), false, false);
        v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = dpp_pair_add_ror8(v[i], v[i + 16]);
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = dpp_pair_add_mirror(v[i], v[i + 8]);
    const bool b1 = lane & 2, b0 = lane & 1;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float keep = b1 ? v[i + 4] : v[i], send = b1 ? v[i] : v[i + 4];
        v[i] = keep + dpp_f(send, 0x4E);  // quad_perm [2,3,0,1] (partner lane ^ 2)
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const float keep = b0 ? v[i + 2] : v[i], send = b0 ? v[i] : v[i + 2];
        v[i] = keep + dpp_f(send, 0xB1);  // quad_perm [1,0,3,2] (partner lane ^ 1)
    }
    return make_float2(v[0], v[1]);
}

template <int B>
__global__ __launch_bounds__(WG2) __attribute__((amdgpu_waves_per_eu(4))) void k_composite_bwd2(Args a) {
    static_assert(B <= WG2, "one staged entry per thread");
    if (overflowed(a.status)) return;
    const int f = blockIdx.y;
    const int tile = blockIdx.x;
    const int txi = tile % a.tiles_x, tyi = tile / a.tiles_x;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int h = lane >> 5, hl = lane & 31;
    const int quad = 2 * w + h;
    const int lx = (h << 3) | (hl & 7), lyA = (w << 3) | (hl >> 3), lyB = lyA + 4;
    const int px = txi * TILE + lx, pyA = tyi * TILE + lyA, pyB = tyi * TILE + lyB;
    const bool inA = px < a.width && pyA < a.height, inB = px < a.width && pyB < a.height;
    const int64_t seg = static_cast<int64_t>(f) * a.tiles + tile;
    uint32_t s, e;
    bucket_range(a, seg, s, e);
    const double ox = txi * TILE + 0.5, oy = tyi * TILE + 0.5;
    const int xlim = a.width - 1 - txi * TILE, ylim = a.height - 1 - tyi * TILE;

    __shared__ Staged sh[B + 1];
    __shared__ uint32_t shm[B];
    __shared__ float acc[WG2 / 64][9][B];
    __shared__ uint32_t wl[WG2 / 64][2][B + RS_GROUP];
    __shared__ uint32_t qlast[4];
    if (tid == 0) stage_inert(sh[B]);
    for (int i = tid; i < (WG2 / 64) * 9 * B; i += WG2) (&acc[0][0][0])[i] = 0.0f;

    // per-pixel state (pixels A and B of this lane), as in the quadrant adjoint
    float TA = 1.0f, GSA = 0.0f, gA0 = 0.0f, gA1 = 0.0f, gA2 = 0.0f;
    float TB = 1.0f, GSB = 0.0f, gB0 = 0.0f, gB1 = 0.0f, gB2 = 0.0f;
    uint32_t lastA = 0, lastB = 0;
    {
        const int64_t P = static_cast<int64_t>(a.width) * a.height;
        auto load = [&](int py, float& T, float& GS, float& g0, float& g1, float& g2, uint32_t& last) {
            const int64_t pix = static_cast<int64_t>(py) * a.width + px;
            T = a.tfin[static_cast<int64_t>(f) * P + pix];
            last = a.nlast[static_cast<int64_t>(f) * P + pix];
            const int64_t o3 = static_cast<int64_t>(f) * 3 * P + pix;
            if (a.targets) {
                g0 = (a.images[o3] - a.targets[o3]) * a.loss_scale;
                g1 = (a.images[o3 + P] - a.targets[o3 + P]) * a.loss_scale;
                g2 = (a.images[o3 + 2 * P] - a.targets[o3 + 2 * P]) * a.loss_scale;
            } else {
                g0 = a.dl_dimages[o3];
                g1 = a.dl_dimages[o3 + P];
                g2 = a.dl_dimages[o3 + 2 * P];
            }
            GS = T * (g0 * a.bg[0] + g1 * a.bg[1] + g2 * a.bg[2]);
        };
        if (inA) load(pyA, TA, GSA, gA0, gA1, gA2, lastA);
        if (inB) load(pyB, TB, GSB, gB0, gB1, gB2, lastB);
    }
    // last contributor of each quadrant (maximum over its 64 pixels)
    uint32_t qmax = max(lastA, lastB);
#pragma unroll
    for (int d = 1; d < 32; d <<= 1) qmax = max(qmax, static_cast<uint32_t>(__shfl_xor(static_cast<int>(qmax), d)));
    if (hl == 0) qlast[quad] = qmax;
    __syncthreads();
    const uint32_t used = max(max(qlast[0], qlast[1]), max(qlast[2], qlast[3]));
    const uint32_t wq0 = qlast[2 * w], wq1 = qlast[2 * w + 1];
    uint32_t gnext = 0;
    {
        const uint32_t b0f = used > B ? s + used - B : s;
        if (tid < static_cast<int>(s + used - b0f)) gnext = a.sgid[b0f + tid];
    }
    const float fx = static_cast<float>(lx), fyA = static_cast<float>(lyA), fyB = static_cast<float>(lyB);
    constexpr uint32_t INERT = static_cast<uint32_t>(B) * STAGED_BYTES;

    for (int64_t bend = static_cast<int64_t>(s) + used; bend > s; bend -= B) {
        const uint32_t b0 = static_cast<uint32_t>(bend - B > s ? bend - B : s);
        const uint32_t nb = static_cast<uint32_t>(bend - b0);
        if (tid < static_cast<int>(nb)) {
            Staged st;
            float3 conic;
            stage_entry(a, f, gnext, ox, oy, st, conic);
            sh[tid] = st;
            shm[tid] = quadrant_mask(st, conic, xlim, ylim) | (may_clamp(st, conic) ? MAY_CLAMP_BIT : 0u);
        }
        __syncthreads();
        const uint32_t slot = tid < static_cast<int>(nb) ? a.sslot[b0 + tid] : 0u;
        if (b0 > s) {
            const uint32_t b0n = b0 - s > B ? b0 - B : s;
            if (tid < static_cast<int>(b0 - b0n)) gnext = a.sgid[b0n + tid];
        }
        // the two quadrants' lists of this wave, back to front
        int cnt0 = 0, cnt1 = 0;
        bool clamp = false;  // some entry of the two lists may clamp (wave-uniform)
        for (int j0 = static_cast<int>(nb) - 1; j0 >= 0; j0 -= 64) {
            const int j = j0 - lane;
            const uint32_t m = j >= 0 ? shm[j] : 0u;
            const uint32_t rel = b0 + static_cast<uint32_t>(j) - s;
            const bool on0 = ((m >> (2 * w)) & 1u) && rel < wq0;
            const bool on1 = ((m >> (2 * w + 1)) & 1u) && rel < wq1;
            const uint64_t bal0 = __ballot(on0), bal1 = __ballot(on1);
            const uint64_t below = (1ull << lane) - 1ull;
            if (on0) wl[w][0][cnt0 + __popcll(bal0 & below)] = static_cast<uint32_t>(j) * STAGED_BYTES;
            if (on1) wl[w][1][cnt1 + __popcll(bal1 & below)] = static_cast<uint32_t>(j) * STAGED_BYTES;
            cnt0 += __popcll(bal0);
            cnt1 += __popcll(bal1);
            clamp = clamp || __ballot((on0 || on1) && (m & MAY_CLAMP_BIT)) != 0ull;
        }
        const int npad = (max(cnt0, cnt1) + RS_GROUP - 1) / RS_GROUP * RS_GROUP;
        for (int k = cnt0 + lane; k < npad; k += 64) wl[w][0][k] = INERT;
        for (int k = cnt1 + lane; k < npad; k += 64) wl[w][1][k] = INERT;
        const int mycnt = h ? cnt1 : cnt0;
        auto limit = [&](uint32_t last) {
            const int64_t rl = static_cast<int64_t>(last) - (static_cast<int64_t>(b0) - s);
            return static_cast<int>(rl < 0 ? 0 : (rl > B ? B : rl)) * static_cast<int>(STAGED_BYTES);
        };
        const int limA = limit(lastA), limB = limit(lastB);
        const uint32_t* mylist = wl[w][h];
        __builtin_amdgcn_wave_barrier();
        // the group loop, with or without the alpha clamp (identical results
        // when no entry can reach it)
        auto groups = [&](auto clamp_tag) {
        constexpr bool CLAMP = decltype(clamp_tag)::value;
        for (int g = 0; g < npad; g += RS_GROUP) {
            float P[64];
            P[63] = 0.0f;
            uint32_t J[RS_GROUP];
            float4 P0[RS_GROUP], P1[RS_GROUP];
            float2 P2[RS_GROUP];
#pragma unroll
            for (int r = 0; r < RS_GROUP; ++r) J[r] = mylist[g + r];
#pragma unroll
            for (int r = 0; r < RS_GROUP; ++r) {
                const Staged& st = staged_at(sh, J[r]);
                P0[r] = st.p0;
                P1[r] = st.p1;
                P2[r] = make_float2(st.p2.x, st.p2.y);
            }
#pragma unroll
            for (int r = 0; r < RS_GROUP; ++r) {
                const float4 p0 = P0[r];
                const float4 p1 = P1[r];
                const float dx = fx - p0.x, dyA = fyA - p0.y, dyB = fyB - p0.y;
                const float qA = footprint_q(dx, dyA, p0, p1);
                const float qB = footprint_q(dx, dyB, p0, p1);
                const bool onA = (static_cast<int>(J[r]) < limA) & (qA >= P2[r].y);
                const bool onB = (static_cast<int>(J[r]) < limB) & (qB >= P2[r].y);
                const float rawA = __builtin_amdgcn_exp2f(qA), rawB = __builtin_amdgcn_exp2f(qB);
                const float alA = onA ? (CLAMP ? fminf(ALPHA_MAX, rawA) : rawA) : 0.0f;
                const float alB = onB ? (CLAMP ? fminf(ALPHA_MAX, rawB) : rawB) : 0.0f;
                const float invA = __builtin_amdgcn_rcpf(1.0f - alA), invB = __builtin_amdgcn_rcpf(1.0f - alB);
                const float aiA = alA * invA, aiB = alB * invB;
                const float wA = aiA * TA, wB = aiB * TB;  // alpha T_j
                TA = TA * invA;
                TB = TB * invB;
                // colour partials summed over the two pixels; alpha dL/dalpha
                // per pixel as in the quadrant adjoint
                const float cA0 = wA * gA0, cA1 = wA * gA1, cA2 = wA * gA2;
                const float wgcA = __builtin_fmaf(P2[r].x, cA2, __builtin_fmaf(p1.w, cA1, p1.z * cA0));
                const float gcB = __builtin_fmaf(P2[r].x, gB2, __builtin_fmaf(p1.w, gB1, p1.z * gB0));
                const float wgcB = wB * gcB;
                P[r * 9 + 6] = __builtin_fmaf(wB, gB0, cA0);
                P[r * 9 + 7] = __builtin_fmaf(wB, gB1, cA1);
                P[r * 9 + 8] = __builtin_fmaf(wB, gB2, cA2);
                const float DalA = __builtin_fmaf(-aiA, GSA, wgcA), DalB = __builtin_fmaf(-aiB, GSB, wgcB);
                GSA = GSA + wgcA;
                GSB = GSB + wgcB;
                const float DA = !CLAMP || rawA < ALPHA_MAX ? DalA : 0.0f;
                const float DB = !CLAMP || rawB < ALPHA_MAX ? DalB : 0.0f;
                // moments over both pixels (they share dx)
                const float Ds = DA + DB;
                const float X = Ds * dx;
                const float YA = DA * dyA, YB = DB * dyB;
                const float Y = YA + YB;
                P[r * 9 + 0] = X;
                P[r * 9 + 1] = Y;
                P[r * 9 + 2] = X * dx;
                P[r * 9 + 3] = Y * dx;
                P[r * 9 + 4] = __builtin_fmaf(YA, dyA, YB * dyB);
                P[r * 9 + 5] = Ds;
            }
            const float2 tot = reduce_scatter32x2(P, lane);
            const int i0 = 2 * hl, r0 = i0 / 9, r1 = (i0 + 1) / 9;
            if (g + r0 < mycnt) atomicAdd(&acc[w][i0 - 9 * r0][mylist[g + r0] / STAGED_BYTES], tot.x);
            if (i0 + 1 < 9 * RS_GROUP && g + r1 < mycnt)
                atomicAdd(&acc[w][i0 + 1 - 9 * r1][mylist[g + r1] / STAGED_BYTES], tot.y);
        }
        };
        if (clamp)
            groups(std::true_type{});
        else
            groups(std::false_type{});
        __syncthreads();
        if (tid < static_cast<int>(nb)) {
            // the two waves' sums in a fixed order; the slots are cleared for
            // the next batch
            float v[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                v[k] = acc[0][k][tid] + acc[1][k][tid];
                acc[0][k][tid] = 0.0f;
                acc[1][k][tid] = 0.0f;
            }
            const Staged st = sh[tid];
            finish_partials(v, st.p0.z * INV_K_EXP, 0.5f * st.p0.w * INV_K_EXP, st.p1.x * INV_K_EXP, st.p2.w);
            if (slot < a.k_cap) store_partials_marked(a, slot, v);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Adjoint with one wave per tile.  A 64-thread workgroup owns a 16x16 tile:
// lanes 16q .. 16q + 15 take quadrant q, each lane four pixels of one column
// of it, rows r, r + 2, r + 4, r + 6 (r = 0 or 1).  Each 16-lane row walks its
// own quadrant's list (the four lists padded with the inert entry to a common
// length of whole groups); a lane adds its four pixels' partials in registers
// (the pixels share dx and the exponent's terms in dx), and one
// reduce-scatter over the 16 lanes of each row leaves lane l of a row with
// the sums 2l and 2l + 1 of that row's RS4 entries: the reduce-scatter is paid
// once per 256 pixels.  Quadrants 0 and 1 add their sums into one zeroed LDS
// slot per entry and partial, quadrants 2 and 3 into another: two addends
// give the same sum in either order, so the result does not depend on the
// order of the LDS additions.
// ---------------------------------------------------------------------------
constexpr int WG4 = 64;
constexpr int RS4 = 3;  // entries per group: 27 partials (+5 pads) per reduce-scatter

// Sums over the 16 lanes of each row of 32 values at once: lane l (l < 16
// within its row) ends with the row's totals of values 2l (.x) and 2l + 1
// (.y).  Stages: lane bit 3 (row rotate by 8), bit 2 (row half-mirror), bits
// 1 and 0 (quad permutations); the order of additions is fixed.
__device__ __forceinline__ float2 reduce_scatter16x2(float (&v)[32], int lane) {
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = dpp_pair_add_ror8(v[i], v[i + 16]);
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = dpp_pair_add_mirror(v[i], v[i + 8]);
    const bool b1 = lane & 2, b0 = lane & 1;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float keep = b1 ? v[i + 4] : v[i], send = b1 ? v[i] : v[i + 4];
        v[i] = keep + dpp_f(send, 0x4E);  // quad_perm [2,3,0,1] (partner lane ^ 2)
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const float keep = b0 ? v[i + 2] : v[i], send = b0 ? v[i] : v[i + 2];
        v[i] = keep + dpp_f(send, 0xB1);  // quad_perm [1,0,3,2] (partner lane ^ 1)
    }
    return make_float2(v[0], v[1]);
}

template <int B>
__global__ __launch_bounds__(WG4) __attribute__((amdgpu_waves_per_eu(4))) void k_composite_bwd4(Args a) {
    static_assert(B <= WG4, "one staged entry per thread");
    if (overflowed(a.status)) return;
    const int f = blockIdx.y;
    const int tile = blockIdx.x;
    const int txi = tile % a.tiles_x, tyi = tile / a.tiles_x;
    const int lane = threadIdx.x;
    const int quad = lane >> 4, rl = lane & 15;
    const int lx = ((quad & 1) << 3) | (rl & 7), ly0 = ((quad >> 1) << 3) | (rl >> 3);
    const int px = txi * TILE + lx;
    const int64_t seg = static_cast<int64_t>(f) * a.tiles + tile;
    uint32_t s, e;
    bucket_range(a, seg, s, e);
    const double ox = txi * TILE + 0.5, oy = tyi * TILE + 0.5;
    const int xlim = a.width - 1 - txi * TILE, ylim = a.height - 1 - tyi * TILE;

    __shared__ Staged sh[B + 1];
    __shared__ uint32_t shm[B];
    __shared__ float acc[2][9][B];
    __shared__ uint32_t wl[4][B + RS4];
    __shared__ uint32_t qlast[4];
    if (lane == 0) stage_inert(sh[B]);
    for (int i = lane; i < 2 * 9 * B; i += WG4) (&acc[0][0][0])[i] = 0.0f;

    // per-pixel state of the lane's four pixels, as in the quadrant adjoint
    float T[4], GS[4], g0[4], g1[4], g2[4];
    uint32_t last[4];
    const int64_t P = static_cast<int64_t>(a.width) * a.height;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        T[k] = 1.0f;
        GS[k] = g0[k] = g1[k] = g2[k] = 0.0f;
        last[k] = 0u;
        const int py = tyi * TILE + ly0 + 2 * k;
        if (px < a.width && py < a.height) {
            const int64_t pix = static_cast<int64_t>(py) * a.width + px;
            T[k] = a.tfin[static_cast<int64_t>(f) * P + pix];
            last[k] = a.nlast[static_cast<int64_t>(f) * P + pix];
            const int64_t o3 = static_cast<int64_t>(f) * 3 * P + pix;
            if (a.targets) {
                g0[k] = (a.images[o3] - a.targets[o3]) * a.loss_scale;
                g1[k] = (a.images[o3 + P] - a.targets[o3 + P]) * a.loss_scale;
                g2[k] = (a.images[o3 + 2 * P] - a.targets[o3 + 2 * P]) * a.loss_scale;
            } else {
                g0[k] = a.dl_dimages[o3];
                g1[k] = a.dl_dimages[o3 + P];
                g2[k] = a.dl_dimages[o3 + 2 * P];
            }
            GS[k] = T[k] * (g0[k] * a.bg[0] + g1[k] * a.bg[1] + g2[k] * a.bg[2]);
        }
    }
    // last contributor of each quadrant (maximum over its 64 pixels)
    uint32_t qmax = max(max(last[0], last[1]), max(last[2], last[3]));
#pragma unroll
    for (int d = 1; d < 16; d <<= 1) qmax = max(qmax, static_cast<uint32_t>(__shfl_xor(static_cast<int>(qmax), d)));
    if (rl == 0) qlast[quad] = qmax;
    __syncthreads();
    uint32_t wq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) wq[q] = __builtin_amdgcn_readfirstlane(qlast[q]);
    const uint32_t used = max(max(wq[0], wq[1]), max(wq[2], wq[3]));
    uint32_t gnext = 0;
    {
        const uint32_t b0f = used > B ? s + used - B : s;
        if (lane < static_cast<int>(s + used - b0f)) gnext = a.sgid[b0f + lane];
    }
    const float fx = static_cast<float>(lx);
    float fy[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) fy[k] = static_cast<float>(ly0 + 2 * k);
    constexpr uint32_t INERT = static_cast<uint32_t>(B) * STAGED_BYTES;
    const int sl = quad >> 1;  // accumulation slot of this row's quadrant

    for (int64_t bend = static_cast<int64_t>(s) + used; bend > s; bend -= B) {
        const uint32_t b0 = static_cast<uint32_t>(bend - B > s ? bend - B : s);
        const uint32_t nb = static_cast<uint32_t>(bend - b0);
        if (lane < static_cast<int>(nb)) {
            Staged st;
            float3 conic;
            stage_entry(a, f, gnext, ox, oy, st, conic);
            sh[lane] = st;
            shm[lane] = quadrant_mask(st, conic, xlim, ylim) | (may_clamp(st, conic) ? MAY_CLAMP_BIT : 0u);
        }
        __syncthreads();
        const uint32_t slot = lane < static_cast<int>(nb) ? a.sslot[b0 + lane] : 0u;
        if (b0 > s) {
            const uint32_t b0n = b0 - s > B ? b0 - B : s;
            if (lane < static_cast<int>(b0 - b0n)) gnext = a.sgid[b0n + lane];
        }
        // the four quadrants' lists, back to front
        int cnt[4] = {0, 0, 0, 0};
        bool clamp = false;  // some entry of the lists may clamp (uniform)
        {
            const int j = static_cast<int>(nb) - 1 - lane;  // nb <= 64: one pass
            const uint32_t m = j >= 0 ? shm[j] : 0u;
            const uint32_t rel = b0 + static_cast<uint32_t>(j) - s;
            const uint64_t below = (1ull << lane) - 1ull;
            bool any = false;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool on = ((m >> q) & 1u) && rel < wq[q];
                const uint64_t bal = __ballot(on);
                if (on) wl[q][__popcll(bal & below)] = static_cast<uint32_t>(j) * STAGED_BYTES;
                cnt[q] = __popcll(bal);
                any = any || on;
            }
            clamp = __ballot(any && (m & MAY_CLAMP_BIT)) != 0ull;
        }
        const int cmax = max(max(cnt[0], cnt[1]), max(cnt[2], cnt[3]));
        const int npad = (cmax + RS4 - 1) / RS4 * RS4;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            for (int k = cnt[q] + lane; k < npad; k += 64) wl[q][k] = INERT;
        const int mycnt = quad == 0 ? cnt[0] : quad == 1 ? cnt[1] : quad == 2 ? cnt[2] : cnt[3];
        int lim[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t r = static_cast<int64_t>(last[k]) - (static_cast<int64_t>(b0) - s);
            lim[k] = static_cast<int>(r < 0 ? 0 : (r > B ? B : r)) * static_cast<int>(STAGED_BYTES);
        }
        const uint32_t* mylist = wl[quad];
        __builtin_amdgcn_wave_barrier();
        // the group loop, with or without the alpha clamp (identical results
        // when no entry can reach it)
        auto groups = [&](auto clamp_tag) {
        constexpr bool CLAMP = decltype(clamp_tag)::value;
        for (int g = 0; g < npad; g += RS4) {
            float Pv[32];
#pragma unroll
            for (int i = 9 * RS4; i < 32; ++i) Pv[i] = 0.0f;
            uint32_t J[RS4];
            float4 P0[RS4], P1[RS4];
            float2 P2[RS4];
#pragma unroll
            for (int r = 0; r < RS4; ++r) J[r] = mylist[g + r];
#pragma unroll
            for (int r = 0; r < RS4; ++r) {
                const Staged& st = staged_at(sh, J[r]);
                P0[r] = st.p0;
                P1[r] = st.p1;
                P2[r] = make_float2(st.p2.x, st.p2.y);
            }
#pragma unroll
            for (int r = 0; r < RS4; ++r) {
                const float4 p0 = P0[r];
                const float4 p1 = P1[r];
                const float2 p2 = P2[r];  // (b, threshold)
                const float dx = fx - p0.x;
                const FootRow fr = footprint_row(dx, p0, p1);
                float Ds = 0.0f, Y = 0.0f, Ydy = 0.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float dy = fy[k] - p0.y;
                    const float q = footprint_q(dy, fr, p1);
                    const bool on = (static_cast<int>(J[r]) < lim[k]) & (q >= p2.y);
                    const float raw = __builtin_amdgcn_exp2f(q);
                    const float al = on ? (CLAMP ? fminf(ALPHA_MAX, raw) : raw) : 0.0f;
                    const float inv = __builtin_amdgcn_rcpf(1.0f - al);
                    const float ai = al * inv;
                    const float wk = ai * T[k];  // alpha T_j
                    T[k] = T[k] * inv;
                    const float gc = __builtin_fmaf(p2.x, g2[k], __builtin_fmaf(p1.w, g1[k], p1.z * g0[k]));
                    const float wgc = wk * gc;
                    c0 = __builtin_fmaf(wk, g0[k], c0);
                    c1 = __builtin_fmaf(wk, g1[k], c1);
                    c2 = __builtin_fmaf(wk, g2[k], c2);
                    const float Dal = __builtin_fmaf(-ai, GS[k], wgc);
                    GS[k] = GS[k] + wgc;
                    const float D = !CLAMP || raw < ALPHA_MAX ? Dal : 0.0f;
                    const float Yk = D * dy;
                    Ds = Ds + D;
                    Y = Y + Yk;
                    Ydy = __builtin_fmaf(Yk, dy, Ydy);
                }
                const float X = Ds * dx;
                Pv[r * 9 + 0] = X;
                Pv[r * 9 + 1] = Y;
                Pv[r * 9 + 2] = X * dx;
                Pv[r * 9 + 3] = Y * dx;
                Pv[r * 9 + 4] = Ydy;
                Pv[r * 9 + 5] = Ds;
                Pv[r * 9 + 6] = c0;
                Pv[r * 9 + 7] = c1;
                Pv[r * 9 + 8] = c2;
            }
            const float2 tot = reduce_scatter16x2(Pv, lane);
            const int i0 = 2 * rl, r0 = i0 / 9, r1 = (i0 + 1) / 9;
            if (i0 < 9 * RS4 && g + r0 < mycnt) atomicAdd(&acc[sl][i0 - 9 * r0][mylist[g + r0] / STAGED_BYTES], tot.x);
            if (i0 + 1 < 9 * RS4 && g + r1 < mycnt)
                atomicAdd(&acc[sl][i0 + 1 - 9 * r1][mylist[g + r1] / STAGED_BYTES], tot.y);
        }
        };
        if (clamp)
            groups(std::true_type{});
        else
            groups(std::false_type{});
        __syncthreads();
        if (lane < static_cast<int>(nb)) {
            // the two slots' sums in a fixed order; the slots are cleared for
            // the next batch
            float v[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                v[k] = acc[0][k][lane] + acc[1][k][lane];
                acc[0][k][lane] = 0.0f;
                acc[1][k][lane] = 0.0f;
            }
            const Staged st = sh[lane];
            finish_partials(v, st.p0.z * INV_K_EXP, 0.5f * st.p0.w * INV_K_EXP, st.p1.x * INV_K_EXP, st.p2.w);
            if (slot < a.k_cap) store_partials_marked(a, slot, v);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Compacted variant.  The quadrant loop above issues every staged entry to all
// 64 lanes of a wave although a small Gaussian covers only a fraction of the
// 8x8 quadrant.  Here each batch is processed in two phases:
//  1. entry-parallel coverage: the thread that stages entry j solves the
//     3-sigma ellipse row by row in closed form and writes four 64-bit
//     quadrant masks (a conservative superset of the per-pixel test);
//     each wave then transposes its quadrant's masks (64x64 bit matrices,
//     xor shuffles) so that lane l holds the set of entries covering pixel l;
//  2. every lane walks only the entries in its own set, in depth order (back
//     to front in the adjoint), with the per-pixel arithmetic of the quadrant
//     loop (shared helpers, so values and decisions are identical).
// The adjoint accumulates each entry's partials with LDS atomics into one
// slot per wave (one instruction's lanes commit in lane order), and the four
// wave slots are summed in a fixed order.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void coverage_masks(float lu, float lv, float a, float b, float c, int xlim, int ylim,
                                               uint64_t qm[4]) {
    qm[0] = qm[1] = qm[2] = qm[3] = 0ull;
    const float det = static_cast<float>(static_cast<double>(a) * c - static_cast<double>(b) * b);
    if (!(det > 0.0f) || !(a > 0.0f)) {  // degenerate conic: keep every pixel (the exact test decides)
        for (int Y = 0; Y < TILE && Y <= ylim; ++Y) {
            const uint32_t bits = (0xFFFFu >> (15 - min(xlim, 15)));
            qm[(Y >> 3) * 2 + 0] |= static_cast<uint64_t>(bits & 0xFFu) << ((Y & 7) * 8);
            qm[(Y >> 3) * 2 + 1] |= static_cast<uint64_t>(bits >> 8) << ((Y & 7) * 8);
        }
        return;
    }
    const float inva = 1.0f / a;
    const float aq = a * SUB_Q_SLACK;
    for (int Y = 0; Y < TILE; ++Y) {
        if (Y > ylim) break;
        const float dy = static_cast<float>(Y) - lv;
        const float disc = aq - dy * dy * det;
        if (disc < 0.0f) continue;
        const float r = sqrtf(disc) * inva;
        const float cen = lu - b * dy * inva;
        const float eps = 0.01f + 1e-4f * r;
        const float lo = fminf(fmaxf(ceilf(cen - r - eps), 0.0f), 16.0f);
        const float hi = fmaxf(fminf(floorf(cen + r + eps), static_cast<float>(min(xlim, 15))), -1.0f);
        const int x0 = static_cast<int>(lo), x1 = static_cast<int>(hi);
        if (x0 > x1) continue;
        const uint32_t bits = (0xFFFFu >> (15 - (x1 - x0))) << x0;
        qm[(Y >> 3) * 2 + 0] |= static_cast<uint64_t>(bits & 0xFFu) << ((Y & 7) * 8);
        qm[(Y >> 3) * 2 + 1] |= static_cast<uint64_t>(bits >> 8) << ((Y & 7) * 8);
    }
}

// Lane l holds row l of a 64x64 bit matrix; returns column l.
__device__ __forceinline__ uint64_t transpose64(uint64_t x, int lane) {
    const uint64_t masks[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                               0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int sft = 32 >> k;
        const uint64_t m = masks[k];
        const uint32_t ylo = __shfl_xor(static_cast<uint32_t>(x), sft, 64);
        const uint32_t yhi = __shfl_xor(static_cast<uint32_t>(x >> 32), sft, 64);
        const uint64_t y = (static_cast<uint64_t>(yhi) << 32) | ylo;
        x = (lane & sft) ? ((x & ~m) | ((y & ~m) >> sft)) : ((x & m) | ((y & m) << sft));
    }
    return x;
}

// Stage the batch [b0, b0 + nb) and its quadrant masks (threads t < B).  The
// compacted kernels read staged entries at lane-dependent indices, so they are
// staged structure-of-arrays (4-byte stride: lanes reading different entries
// fall into different banks): sv[0..SV - 1][j] = local u, local v, K a, K 2b,
// K c, log2 opacity, r, g, b, threshold (as in Staged), opacity.
constexpr int SV = 11;

template <int B>
__device__ __forceinline__ void stage_batch_masks(const Args& a, int f, uint32_t b0, uint32_t nb, double ox, double oy,
                                                  int xlim, int ylim, float (*sv)[B], uint64_t (*qmask)[B]) {
    const int t = threadIdx.x;
    if (t < B) {
        uint64_t qm[4] = {0ull, 0ull, 0ull, 0ull};
        if (t < static_cast<int>(nb)) {
            Staged st;
            float3 cn;
            stage_entry(a, f, a.sgid[b0 + t], ox, oy, st, cn);
            sv[0][t] = st.p0.x; sv[1][t] = st.p0.y; sv[2][t] = st.p0.z; sv[3][t] = st.p0.w;
            sv[4][t] = st.p1.x; sv[5][t] = st.p1.y; sv[6][t] = st.p1.z; sv[7][t] = st.p1.w;
            sv[8][t] = st.p2.x; sv[9][t] = st.p2.y; sv[10][t] = st.p2.w;
            if (quadrant_mask(st, cn, xlim, ylim)) coverage_masks(st.p0.x, st.p0.y, cn.x, cn.y, cn.z, xlim, ylim, qm);
        }
        for (int q = 0; q < 4; ++q) qmask[q][t] = qm[q];
    }
}

// Lane l's set of staged entries covering its pixel, as NW 64-bit words
// (rounds beyond the staged count are empty and not transposed).
template <int B>
__device__ __forceinline__ void lane_entry_sets(uint64_t (*qmask)[B], int w, int lane, uint32_t nb,
                                                uint64_t wq[B / 64]) {
#pragma unroll
    for (int r = 0; r < B / 64; ++r)
        wq[r] = (static_cast<uint32_t>(r * 64) < nb) ? transpose64(qmask[w][r * 64 + lane], lane) : 0ull;
}

template <int B>
__global__ __launch_bounds__(WG) void k_composite_fwd_c(Args a) {
    if (overflowed(a.status)) return;
    constexpr int NW = B / 64;
    const int f = blockIdx.y;
    const int tile = blockIdx.x;
    const int txi = tile % a.tiles_x, tyi = tile / a.tiles_x;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lx = ((w & 1) << 3) | (lane & 7), ly = ((w >> 1) << 3) | (lane >> 3);
    const int px = txi * TILE + lx, py = tyi * TILE + ly;
    const bool inside = px < a.width && py < a.height;
    const int64_t seg = static_cast<int64_t>(f) * a.tiles + tile;
    uint32_t s, e;
    bucket_range(a, seg, s, e);
    const double ox = txi * TILE + 0.5, oy = tyi * TILE + 0.5;
    const int xlim = a.width - 1 - txi * TILE, ylim = a.height - 1 - tyi * TILE;

    __shared__ float sv[SV][B];
    __shared__ uint64_t qmask[4][B];
    __shared__ float red[WG / 64];

    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    uint32_t last = 0;
    bool done = !inside;
    const float fx = static_cast<float>(lx), fy = static_cast<float>(ly);

    for (uint32_t b0 = s; b0 < e; b0 += B) {
        if (__syncthreads_count(!done) == 0) break;
        const uint32_t nb = min(static_cast<uint32_t>(B), e - b0);
        stage_batch_masks<B>(a, f, b0, nb, ox, oy, xlim, ylim, sv, qmask);
        __syncthreads();
        uint64_t wq[NW];
        lane_entry_sets<B>(qmask, w, lane, nb, wq);
        if (!done) {
            uint64_t cur = wq[0];
            int base = 0;
            for (;;) {
                while (cur == 0ull && base < (NW - 1) * 64) {
#pragma unroll
                    for (int r = 0; r + 1 < NW; ++r) wq[r] = wq[r + 1];
                    wq[NW - 1] = 0ull;
                    cur = wq[0];
                    base += 64;
                }
                if (cur == 0ull) break;
                const int j = base + __builtin_ctzll(cur);
                cur &= cur - 1ull;
                const float4 p0 = make_float4(sv[0][j], sv[1][j], sv[2][j], sv[3][j]);
                const float4 p1 = make_float4(sv[4][j], sv[5][j], 0.0f, 0.0f);
                const float dx = fx - p0.x, dy = fy - p0.y;
                const float q = footprint_q(dx, dy, p0, p1);
                if (!(q >= sv[9][j])) continue;
                const float al = fminf(ALPHA_MAX, __builtin_amdgcn_exp2f(q));
                const float tn = __builtin_fmaf(-al, T, T);
                if (tn < T_MIN) {
                    done = true;
                    break;
                }
                const float wgt = T - tn;  // alpha T to rounding, as in the other forwards
                c0 = __builtin_fmaf(sv[6][j], wgt, c0);
                c1 = __builtin_fmaf(sv[7][j], wgt, c1);
                c2 = __builtin_fmaf(sv[8][j], wgt, c2);
                T = tn;
                last = b0 + j - s + 1;
            }
        }
    }

    float sq = 0.0f;
    if (inside) {
        const int64_t P = static_cast<int64_t>(a.width) * a.height;
        const int64_t pix = static_cast<int64_t>(py) * a.width + px;
        c0 = __builtin_fmaf(T, a.bg[0], c0);
        c1 = __builtin_fmaf(T, a.bg[1], c1);
        c2 = __builtin_fmaf(T, a.bg[2], c2);
        float* img = a.images + static_cast<int64_t>(f) * 3 * P + pix;
        img[0] = c0;
        img[P] = c1;
        img[2 * P] = c2;
        a.tfin[static_cast<int64_t>(f) * P + pix] = T;
        a.nlast[static_cast<int64_t>(f) * P + pix] = last;
        if (a.tfin_out) a.tfin_out[static_cast<int64_t>(f) * P + pix] = T;
        if (a.targets && a.loss) {
            const float* tg = a.targets + static_cast<int64_t>(f) * 3 * P + pix;
            const float d0 = c0 - tg[0], d1 = c1 - tg[P], d2 = c2 - tg[2 * P];
            sq = d0 * d0 + d1 * d1 + d2 * d2;
        }
    }
    if (a.targets && a.loss) {
        sq = wave_sum_to_lane63(sq);
        if (lane == 63) red[w] = sq;
        __syncthreads();
        if (tid == 0) a.loss_part[seg] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

template <int B>
__global__ __launch_bounds__(WG) void k_composite_bwd_c(Args a) {
    if (overflowed(a.status)) return;
    constexpr int NW = B / 64;
    const int f = blockIdx.y;
    const int tile = blockIdx.x;
    const int txi = tile % a.tiles_x, tyi = tile / a.tiles_x;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lx = ((w & 1) << 3) | (lane & 7), ly = ((w >> 1) << 3) | (lane >> 3);
    const int px = txi * TILE + lx, py = tyi * TILE + ly;
    const bool inside = px < a.width && py < a.height;
    const int64_t seg = static_cast<int64_t>(f) * a.tiles + tile;
    uint32_t s, e;
    bucket_range(a, seg, s, e);
    const double ox = txi * TILE + 0.5, oy = tyi * TILE + 0.5;
    const int xlim = a.width - 1 - txi * TILE, ylim = a.height - 1 - tyi * TILE;

    __shared__ float sv[SV][B];
    __shared__ uint64_t qmask[4][B];
    __shared__ float acc[WG / 64][9][B];
    __shared__ uint32_t smax;

    float T = 1.0f, S0 = 0.0f, S1 = 0.0f, S2 = 0.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
    uint32_t last = 0;
    if (inside) {
        const int64_t P = static_cast<int64_t>(a.width) * a.height;
        const int64_t pix = static_cast<int64_t>(py) * a.width + px;
        T = a.tfin[static_cast<int64_t>(f) * P + pix];
        last = a.nlast[static_cast<int64_t>(f) * P + pix];
        const int64_t o3 = static_cast<int64_t>(f) * 3 * P + pix;
        if (a.targets) {
            g0 = (a.images[o3] - a.targets[o3]) * a.loss_scale;
            g1 = (a.images[o3 + P] - a.targets[o3 + P]) * a.loss_scale;
            g2 = (a.images[o3 + 2 * P] - a.targets[o3 + 2 * P]) * a.loss_scale;
        } else {
            g0 = a.dl_dimages[o3];
            g1 = a.dl_dimages[o3 + P];
            g2 = a.dl_dimages[o3 + 2 * P];
        }
        S0 = T * a.bg[0];
        S1 = T * a.bg[1];
        S2 = T * a.bg[2];
    }
    if (tid == 0) smax = 0;
    __syncthreads();
    if (last) atomicMax(&smax, last);
    __syncthreads();
    const uint32_t used = smax;
    const float fx = static_cast<float>(lx), fy = static_cast<float>(ly);

    for (int64_t bend = static_cast<int64_t>(s) + used; bend > s; bend -= B) {
        const uint32_t b0 = static_cast<uint32_t>(bend - B > s ? bend - B : s);
        const uint32_t nb = static_cast<uint32_t>(bend - b0);
        stage_batch_masks<B>(a, f, b0, nb, ox, oy, xlim, ylim, sv, qmask);
        for (int k = tid; k < (WG / 64) * 9 * B; k += WG) (&acc[0][0][0])[k] = 0.0f;
        __syncthreads();
        // entries at or behind this pixel's last contributor are not part of its sum
        const int64_t lim = static_cast<int64_t>(last) - (static_cast<int64_t>(b0) - s);
        uint64_t wq[NW];
        lane_entry_sets<B>(qmask, w, lane, nb, wq);
#pragma unroll
        for (int r = 0; r < NW; ++r) {
            const int64_t keep = lim - 64 * r;
            wq[r] = keep <= 0 ? 0ull : (keep >= 64 ? wq[r] : (wq[r] & ((1ull << keep) - 1ull)));
        }
        {
            uint64_t cur = wq[NW - 1];
            int base = (NW - 1) * 64;
            for (;;) {
                while (cur == 0ull && base > 0) {
#pragma unroll
                    for (int r = NW - 1; r > 0; --r) wq[r] = wq[r - 1];
                    wq[0] = 0ull;
                    cur = wq[NW - 1];
                    base -= 64;
                }
                if (cur == 0ull) break;
                const int bit = 63 - __builtin_clzll(cur);
                cur ^= 1ull << bit;
                const int j = base + bit;
                const float4 p0 = make_float4(sv[0][j], sv[1][j], sv[2][j], sv[3][j]);
                const float4 p1 = make_float4(sv[4][j], sv[5][j], sv[6][j], sv[7][j]);
                const float dx = fx - p0.x, dy = fy - p0.y;
                const float q = footprint_q(dx, dy, p0, p1);
                if (!(q >= sv[9][j])) continue;
                const float raw = __builtin_amdgcn_exp2f(q);
                const float al = fminf(ALPHA_MAX, raw);
                const float inv = 1.0f / (1.0f - al);
                const float Tj = T * inv;
                const float wgt = al * Tj;
                const float cb = sv[8][j];
                const float dal = g0 * (p1.z * Tj - S0 * inv) + g1 * (p1.w * Tj - S1 * inv) + g2 * (cb * Tj - S2 * inv);
                S0 = __builtin_fmaf(p1.z, wgt, S0);
                S1 = __builtin_fmaf(p1.w, wgt, S1);
                S2 = __builtin_fmaf(cb, wgt, S2);
                T = Tj;
                float* ac = &acc[w][0][j];
                atomicAdd(ac + 6 * B, wgt * g0);
                atomicAdd(ac + 7 * B, wgt * g1);
                atomicAdd(ac + 8 * B, wgt * g2);
                if (raw < ALPHA_MAX) {  // moments of D = alpha dL/dalpha, as in the quadrant adjoint
                    const float D = al * dal;
                    const float X = D * dx, Y = D * dy;
                    atomicAdd(ac + 0 * B, X);
                    atomicAdd(ac + 1 * B, Y);
                    atomicAdd(ac + 2 * B, X * dx);
                    atomicAdd(ac + 3 * B, X * dy);
                    atomicAdd(ac + 4 * B, Y * dy);
                    atomicAdd(ac + 5 * B, D);
                }
            }
        }
        __syncthreads();
        if (tid < static_cast<int>(nb)) {
            float v[9];
            for (int k = 0; k < 9; ++k) v[k] = (acc[0][k][tid] + acc[1][k][tid]) + (acc[2][k][tid] + acc[3][k][tid]);
            finish_partials(v, sv[2][tid] * INV_K_EXP, 0.5f * sv[3][tid] * INV_K_EXP, sv[4][tid] * INV_K_EXP,
                            sv[10][tid]);
            const uint32_t slot = a.sslot[b0 + tid];
            if (slot < a.k_cap) {
                store_partials_marked(a, slot, v);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Sub-block forward.  Each 16-lane row of a wave owns a
// 4x4 block of the wave's quadrant (row r: block (r & 1, r >> 1); lane l of
// the row: pixel (l & 3, l >> 2) of the block) and walks its own list of the
// staged entries whose ellipse meets that block.  The rows advance together,
// so a wave takes as many steps as its longest block list rather than the
// length of its quadrant list (0.8x on the 3DGS benchmark clip: the near
// Gaussians, composited first, are large), and each staged read is a
// broadcast within a row.  Per pixel the arithmetic is that of the quadrant
// loop, so images, final transmittances and last indices are identical.
// ---------------------------------------------------------------------------

// Build the four block lists of wave w over the staged batch, front to back,
// each padded with the inert entry to `steps` entries, a multiple of G shared
// by the four lists.  Lists hold byte offsets into the staged array.
template <int B, int G>
__device__ __forceinline__ int build_block_lists(uint32_t (*wl)[B + G], const uint32_t* shm, int w, int lane,
                                                 uint32_t nb) {
    int c[4] = {0, 0, 0, 0};
    for (int j0 = 0; j0 < static_cast<int>(nb); j0 += 64) {
        const int j = j0 + lane;
        const uint32_t m = j < static_cast<int>(nb) ? (shm[j] >> (4 * w)) & 0xFu : 0u;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const bool on = (m >> r) & 1u;
            const uint64_t bal = __ballot(on);
            if (on) wl[r][c[r] + __popcll(bal & ((1ull << lane) - 1ull))] = static_cast<uint32_t>(j) * STAGED_BYTES;
            c[r] += __popcll(bal);
        }
    }
    const int cmax = max(max(c[0], c[1]), max(c[2], c[3]));
    const int steps = (cmax + G - 1) / G * G;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        for (int k = c[r] + lane; k < steps; k += 64) wl[r][k] = static_cast<uint32_t>(B) * STAGED_BYTES;
    return steps;
}

template <int B, bool VIS>
__global__ __launch_bounds__(WG) void k_composite_fwd_sb(Args a) {
    if (overflowed(a.status)) return;
    const int f = blockIdx.y;
    const int tile = blockIdx.x;
    const int txi = tile % a.tiles_x, tyi = tile / a.tiles_x;
    const int tid = threadIdx.x, lane = tid & 63, row = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lx = ((w & 1) << 3) | ((row & 1) << 2) | (lane & 3);
    const int ly = ((w >> 1) << 3) | ((row >> 1) << 2) | ((lane >> 2) & 3);
    const int px = txi * TILE + lx, py = tyi * TILE + ly;
    const bool inside = px < a.width && py < a.height;
    const int64_t seg = static_cast<int64_t>(f) * a.tiles + tile;
    uint32_t s, e;
    bucket_range(a, seg, s, e);
    const double ox = txi * TILE + 0.5, oy = tyi * TILE + 0.5;
    const int xlim = a.width - 1 - txi * TILE, ylim = a.height - 1 - tyi * TILE;

    __shared__ Staged sh[B + 1];
    __shared__ uint32_t shm[B];
    __shared__ float red[WG / 64];
    __shared__ __align__(16) uint32_t wl[WG / 64][4][B + FWD_GROUP];
    if (tid == 0) stage_inert(sh[B]);

    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    uint32_t last = 0;
    bool done = !inside;
    const float fx = static_cast<float>(lx), fy = static_cast<float>(ly);
    const uint32_t* my = wl[w][row];

    // each batch's entry ids are requested during the previous batch's loop
    uint32_t gnext = tid < static_cast<int>(min(static_cast<uint32_t>(B), e - s)) ? a.sgid[s + tid] : 0u;
    for (uint32_t b0 = s; b0 < e; b0 += B) {
        if (__syncthreads_count(!done) == 0) break;
        const uint32_t nb = min(static_cast<uint32_t>(B), e - b0);
        if (tid < static_cast<int>(nb)) {
            Staged st;
            float3 conic;
            stage_entry(a, f, gnext, ox, oy, st, conic);
            sh[tid] = st;
            shm[tid] = block_mask(st, conic, xlim, ylim);
        }
        __syncthreads();
        if (e - b0 > B && tid < static_cast<int>(min(static_cast<uint32_t>(B), e - b0 - B))) gnext = a.sgid[b0 + B + tid];
        if (__ballot(!done) == 0) continue;  // wave-uniform; the barriers are outside
        const int steps = build_block_lists<B, FWD_GROUP>(wl[w], shm, w, lane, nb);
        __builtin_amdgcn_wave_barrier();
        // Branch-free groups, as in the quadrant loop; loff: byte offset of
        // this lane's last entry taken in this batch.
        int loff = -1;
        for (int g = 0; g < steps; g += FWD_GROUP) {
            static_assert(FWD_GROUP == 8, "two 16-byte reads of the block list per group");
            const uint4 ja = *reinterpret_cast<const uint4*>(my + g);
            const uint4 jb = *reinterpret_cast<const uint4*>(my + g + 4);
            const uint32_t jo[FWD_GROUP] = {ja.x, ja.y, ja.z, ja.w, jb.x, jb.y, jb.z, jb.w};
            float4 P0[FWD_GROUP], P1[FWD_GROUP];
            float2 P2[FWD_GROUP];
#pragma unroll
            for (int r = 0; r < FWD_GROUP; ++r) {
                const Staged& st = staged_at(sh, jo[r]);
                P0[r] = st.p0;
                P1[r] = st.p1;
                P2[r] = make_float2(st.p2.x, st.p2.y);
            }
#pragma unroll
            for (int r = 0; r < FWD_GROUP; ++r) {
                const float4 p0 = P0[r];
                const float4 p1 = P1[r];
                const float dx = fx - p0.x, dy = fy - p0.y;
                const float q = footprint_q(dx, dy, p0, p1);
                const bool hit = !done && q >= P2[r].y;
                const float al = fminf(ALPHA_MAX, __builtin_amdgcn_exp2f(q));
                const float tn = __builtin_fmaf(-al, T, T);
                const bool take = hit && tn >= T_MIN;  // else stop before this entry
                done = done || (hit != take);
                const float Tn = take ? tn : T;
                const float wgt = T - Tn;  // alpha T to rounding; 0 when not taken
                c0 = __builtin_fmaf(p1.z, wgt, c0);
                c1 = __builtin_fmaf(p1.w, wgt, c1);
                c2 = __builtin_fmaf(P2[r].x, wgt, c2);
                T = Tn;
                loff = take ? static_cast<int>(jo[r]) : loff;
                if (VIS) {
                    const uint64_t bal = __ballot(take);
                    if (((bal >> (16 * row)) & 0xFFFFull) != 0ull && (lane & 15) == 0) {
                        const uint32_t gid = __float_as_uint(staged_at(sh, jo[r]).p2.z);
                        if (gid < static_cast<uint64_t>(a.n)) a.vis[static_cast<int64_t>(f) * a.n + gid] = 1;
                    }
                }
            }
            if (__ballot(!done) == 0) break;
        }
        if (loff >= 0) last = b0 - s + static_cast<uint32_t>(loff) / STAGED_BYTES + 1;
    }

    float sq = 0.0f;
    if (inside) {
        const int64_t P = static_cast<int64_t>(a.width) * a.height;
        const int64_t pix = static_cast<int64_t>(py) * a.width + px;
        c0 = __builtin_fmaf(T, a.bg[0], c0);
        c1 = __builtin_fmaf(T, a.bg[1], c1);
        c2 = __builtin_fmaf(T, a.bg[2], c2);
        float* img = a.images + static_cast<int64_t>(f) * 3 * P + pix;
        img[0] = c0;
        img[P] = c1;
        img[2 * P] = c2;
        a.tfin[static_cast<int64_t>(f) * P + pix] = T;
        a.nlast[static_cast<int64_t>(f) * P + pix] = last;
        if (a.tfin_out) a.tfin_out[static_cast<int64_t>(f) * P + pix] = T;
        if (a.targets && a.loss) {
            const float* tg = a.targets + static_cast<int64_t>(f) * 3 * P + pix;
            const float d0 = c0 - tg[0], d1 = c1 - tg[P], d2 = c2 - tg[2 * P];
            sq = d0 * d0 + d1 * d1 + d2 * d2;
        }
    }
    if (a.targets && a.loss) {
        sq = wave_sum_to_lane63(sq);
        if (lane == 63) red[w] = sq;
        __syncthreads();
        if (tid == 0) a.loss_part[seg] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// Kernel choice: tune.compact bit 0 selects the compacted forward, else bit 2
// the quadrant forward, else the sub-block forward runs; bit 1 selects the
// compacted adjoint, else the quadrant adjoint runs.  The visibility flags use
// the sub-block or quadrant forward.
hipError_t launch_composite_fwd(const Args& a, hipStream_t stream) {
    const dim3 grid(static_cast<uint32_t>(a.tiles), static_cast<uint32_t>(a.frames)), block(WG);
    const int c = a.tune.compact;
    if ((c & 1) && !a.vis) {
        switch (a.tune.batch) {
            case 64: hipLaunchKernelGGL(k_composite_fwd_c<64>, grid, block, 0, stream, a); break;
            case 128: hipLaunchKernelGGL(k_composite_fwd_c<128>, grid, block, 0, stream, a); break;
            default: hipLaunchKernelGGL(k_composite_fwd_c<256>, grid, block, 0, stream, a); break;
        }
        return hipGetLastError();
    }
    if ((c & 32) && !a.vis) {  // one wave per tile (batches of at most 128)
        if (a.tune.batch == 64)
            hipLaunchKernelGGL(k_composite_fwd4<64>, grid, dim3(WGF4), 0, stream, a);
        else
            hipLaunchKernelGGL(k_composite_fwd4<128>, grid, dim3(WGF4), 0, stream, a);
        return hipGetLastError();
    }
#define GV_FWD_SWITCH(KERNEL, VIS)                                                                       \
    switch (a.tune.batch) {                                                                              \
        case 64: hipLaunchKernelGGL((KERNEL<64, VIS>), grid, block, 0, stream, a); break;                \
        case 128: hipLaunchKernelGGL((KERNEL<128, VIS>), grid, block, 0, stream, a); break;              \
        default: hipLaunchKernelGGL((KERNEL<256, VIS>), grid, block, 0, stream, a); break;               \
    }
    if (c & 4) {
        if (a.vis) {
            GV_FWD_SWITCH(k_composite_fwd, true)
        } else {
            GV_FWD_SWITCH(k_composite_fwd, false)
        }
    } else {
        if (a.vis) {
            GV_FWD_SWITCH(k_composite_fwd_sb, true)
        } else {
            GV_FWD_SWITCH(k_composite_fwd_sb, false)
        }
    }
#undef GV_FWD_SWITCH
    return hipGetLastError();
}

// counts[g] = number of frames whose flag vis[f * N + g] is set.
__global__ __launch_bounds__(256) void k_vis_count(Args a, uint32_t* __restrict__ counts) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (g >= a.n) return;
    uint32_t c = 0;
    for (int f = 0; f < a.frames; ++f) c += a.vis[static_cast<int64_t>(f) * a.n + g];
    counts[g] = overflowed(a.status) ? 0u : c;
}

hipError_t launch_vis_count(const Args& a, uint32_t* counts, hipStream_t stream) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_vis_count, dim3(static_cast<uint32_t>((a.n + 255) / 256)), dim3(256), 0, stream, a, counts);
    return hipGetLastError();
}

hipError_t launch_loss_finalize(const Args& a, hipStream_t stream) {
    hipLaunchKernelGGL(k_loss_finalize, dim3(static_cast<uint32_t>(a.frames)), dim3(WG), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_composite_bwd(const Args& a, hipStream_t stream) {
    const dim3 grid(static_cast<uint32_t>(a.tiles), static_cast<uint32_t>(a.frames)), block(WG);
    if (a.tune.compact & 2) {
        switch (a.tune.bwd_batch) {
            case 64: hipLaunchKernelGGL(k_composite_bwd_c<64>, grid, block, 0, stream, a); break;
            case 128: hipLaunchKernelGGL(k_composite_bwd_c<128>, grid, block, 0, stream, a); break;
            default: hipLaunchKernelGGL(k_composite_bwd_c<256>, grid, block, 0, stream, a); break;
        }
        return hipGetLastError();
    }
    if (a.tune.compact & 16) {  // one wave per tile (batches of 64)
        hipLaunchKernelGGL(k_composite_bwd4<64>, grid, dim3(WG4), 0, stream, a);
        return hipGetLastError();
    }
    if (a.tune.compact & 8) {  // paired quadrants (batches of at most 128)
        if (a.tune.bwd_batch == 64)
            hipLaunchKernelGGL(k_composite_bwd2<64>, grid, dim3(WG2), 0, stream, a);
        else
            hipLaunchKernelGGL(k_composite_bwd2<128>, grid, dim3(WG2), 0, stream, a);
        return hipGetLastError();
    }
    switch (a.tune.bwd_batch) {
        case 64: hipLaunchKernelGGL(k_composite_bwd<64>, grid, block, 0, stream, a); break;
        case 128: hipLaunchKernelGGL(k_composite_bwd<128>, grid, block, 0, stream, a); break;
        default: hipLaunchKernelGGL(k_composite_bwd<256>, grid, block, 0, stream, a); break;
    }
    return hipGetLastError();
}

}  // namespace gv
