// EWA projection of every (frame, Gaussian) pair and the two binning passes
// (count, then scatter of (depth, index) keys into per-tile buckets).
//
// The projection runs in FP64: on CDNA4 the FP64 vector rate equals the
// non-packed FP32 rate, the stage streams 56 bytes per Gaussian from HBM, and
// FP64 keeps the rounded records (centre, conic, depth key) as close to the
// exact values as their storage format allows.  Only the per-pixel loop of the
// compositing kernels runs in FP32.
#include "gv_internal.h"

namespace gv {

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t value, int64_t count) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

// Tile range [t0, t1] along one axis whose pixel-centre span meets [lo, hi].
__device__ __forceinline__ bool tile_span(double lo, double hi, int n_tiles, int& t0, int& t1) {
    double a = ceil((lo - (TILE - 0.5)) / TILE);
    double b = floor((hi - 0.5) / TILE);
    a = fmax(a, 0.0);
    b = fmin(b, static_cast<double>(n_tiles - 1));
    if (!(a <= b)) return false;
    t0 = static_cast<int>(a);
    t1 = static_cast<int>(b);
    return true;
}

// Project Gaussian g in frame f: write its record and tile rectangle and call
// tally(tile) for every 16x16 tile whose pixel-centre box meets its 3-sigma
// ellipse (exact ellipse-box test).  Returns the number of such tiles.  Frame
// 0 also writes the per-Gaussian colour/opacity table shared by all frames.
template <bool EXT, typename Tally>
__device__ __forceinline__ uint32_t project_and_count(const Args& a, int f, int64_t g, const CamD& cam, double t,
                                                      Tally tally) {
    const int64_t i = static_cast<int64_t>(f) * a.n + g;
    if (f == 0 && a.sh_degree == 0) {
        const double eta = load_param(a.opacity_logits, a.dtype, g);
        ColorOp co;
        co.r = static_cast<float>(load_param(a.colors, a.dtype, g));
        co.g = static_cast<float>(load_param(a.colors, a.dtype, a.n + g));
        co.b = static_cast<float>(load_param(a.colors, a.dtype, 2 * a.n + g));
        co.o = static_cast<float>(1.0 / (1.0 + exp(-eta)));
        a.col4[g] = co;
    }
    ProjD P;
    const bool vis = project_gaussian<EXT>(a, g, cam, t, P);
    if (EXT && vis && a.sh_degree > 0) {
        ColorOp co;
        co.r = static_cast<float>(P.col[0]);
        co.g = static_cast<float>(P.col[1]);
        co.b = static_cast<float>(P.col[2]);
        co.o = static_cast<float>(P.o);
        a.col4[i] = co;
    }
    if (P.nonfinite) atomicAdd(&a.status[ST_NONFINITE], 1u);
    uint32_t cnt = 0;
    // o < 1/255 can never pass the per-pixel alpha test (alpha <= o).
    if (vis && P.o >= static_cast<double>(ALPHA_MIN) * (1.0 - 1e-6)) {
        Record r;
        r.u = P.u;
        r.v = P.v;
        r.a = static_cast<float>(P.A[0]);
        r.b = static_cast<float>(P.A[1]);
        r.c = static_cast<float>(P.A[2]);
        r.depth = static_cast<float>(P.m[2]);
        // axis-aligned box of the 3-sigma ellipse, padded for the rounded conic
        const double hx = 3.0 * sqrt(P.cov[0]) * (1.0 + 2e-5) + 1e-4;
        const double hy = 3.0 * sqrt(P.cov[2]) * (1.0 + 2e-5) + 1e-4;
        int tx0, tx1, ty0, ty1;
        if (tile_span(P.u - hx, P.u + hx, a.tiles_x, tx0, tx1) && tile_span(P.v - hy, P.v + hy, a.tiles_y, ty0, ty1)) {
            const double ca = r.a, cb = r.b, cc = r.c;
            const int rw = tx1 - tx0 + 1;
            const bool small = rw * (ty1 - ty0 + 1) <= 64;
            uint64_t mask = 0;
            for (int ty = ty0; ty <= ty1; ++ty)
                for (int tx = tx0; tx <= tx1; ++tx) {
                    double x0, x1, y0, y1;
                    tile_box(tx, ty, a.width, a.height, x0, x1, y0, y1);
                    if (ellipse_meets_box<double>(r.u, r.v, ca, cb, cc, x0, x1, y0, y1, BIN_Q_SLACK)) {
                        ++cnt;
                        tally(ty * a.tiles_x + tx);
                        if (small) mask |= 1ull << ((ty - ty0) * rw + (tx - tx0));
                    }
                }
            a.tmask[i] = mask;
            a.rec[i] = r;
            a.rect[i] = make_uint2(static_cast<uint32_t>(tx0) | (static_cast<uint32_t>(tx1) << 16),
                                   static_cast<uint32_t>(ty0) | (static_cast<uint32_t>(ty1) << 16));
        }
    }
    a.gcnt[i] = cnt;
    return cnt;
}

// Write key = (fp32 depth bits << 32 | Gaussian index) and the pre-sort slot
// (goff + k for the k-th tile of this Gaussian) of every intersection of
// (f, g) at position next(tile) of its tile's bucket.  The decisions repeat
// project_and_count's exactly (same inputs, same test, no contraction).
template <typename Next>
__device__ __forceinline__ void scatter_one(const Args& a, int f, int64_t g, Next next) {
    const int64_t i = static_cast<int64_t>(f) * a.n + g;
    const uint32_t cnt = a.gcnt[i];
    if (cnt == 0) return;
    const Record r = a.rec[i];
    const uint2 rc = a.rect[i];
    const int tx0 = rc.x & 0xffff, tx1 = rc.x >> 16, ty0 = rc.y & 0xffff, ty1 = rc.y >> 16;
    const uint64_t key = (static_cast<uint64_t>(__float_as_uint(r.depth)) << 32) | static_cast<uint64_t>(g);
    const uint32_t base = a.goff[i];
    const int64_t tile0 = static_cast<int64_t>(f) * a.tiles;
    uint32_t k = 0;
    auto emit = [&](int tx, int ty) {
        const int tl = ty * a.tiles_x + tx;
        const uint32_t pos = next(tl);
        // the counts bound every write; a mismatch is an internal error,
        // reported instead of written out of bounds
        if (pos >= a.toff[tile0 + tl + 1] || k >= cnt) {
            a.status[ST_OVERFLOW] = 2u;
            return;
        }
        KeySlot ks;
        ks.key = key;
        ks.slot = base + k;
        ks.pad = 0u;
        a.kv[pos] = ks;
        ++k;
    };
    const int rw = tx1 - tx0 + 1;
    if (rw * (ty1 - ty0 + 1) <= 64) {
        // the count pass left the tiles that passed as a row-major mask over
        // the rectangle: walk its set bits (same order as the loops below)
        uint64_t m = a.tmask[i];
        while (m) {
            const int b = __builtin_ctzll(m);
            m &= m - 1;
            const int ry = b / rw;
            emit(tx0 + (b - ry * rw), ty0 + ry);
        }
        return;
    }
    const double ca = r.a, cb = r.b, cc = r.c;
    for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx) {
            double x0, x1, y0, y1;
            tile_box(tx, ty, a.width, a.height, x0, x1, y0, y1);
            if (ellipse_meets_box<double>(r.u, r.v, ca, cb, cc, x0, x1, y0, y1, BIN_Q_SLACK)) emit(tx, ty);
        }
}

// Binning with workgroup-local tile histograms in LDS: each workgroup
// projects BIN_GROUP Gaussians of one frame, counts their intersections per
// tile with LDS atomics, stores its histogram and adds it to the frame's tile
// counts with one global atomic per non-empty tile.
template <bool EXT>
__global__ __launch_bounds__(256) void k_project_lds(Args a) {
    extern __shared__ uint32_t hist[];
    const int f = blockIdx.y;
    for (int t = threadIdx.x; t < a.tiles; t += 256) hist[t] = 0u;
    __syncthreads();
    const CamD cam = load_camera(a.poses + 7 * f);
    const double tt = a.times ? static_cast<double>(a.times[f]) : static_cast<double>(a.t0);
    const int64_t g0 = static_cast<int64_t>(blockIdx.x) * BIN_GROUP;
#pragma unroll 1
    for (int k = 0; k < BIN_GROUP / 256; ++k) {
        const int64_t g = g0 + k * 256 + threadIdx.x;
        if (g < a.n) project_and_count<EXT>(a, f, g, cam, tt, [&](int tl) { atomicAdd(&hist[tl], 1u); });
    }
    __syncthreads();
    uint32_t* bh = a.bhist + (static_cast<int64_t>(f) * a.bin_blocks + blockIdx.x) * a.tiles;
    uint32_t* tc = a.tcnt + static_cast<int64_t>(f) * a.tiles;
    for (int t = threadIdx.x; t < a.tiles; t += 256) {
        const uint32_t v = hist[t];
        bh[t] = v;
        if (v) atomicAdd(&tc[t], v);
    }
}

// Scatter counterpart: one global atomic per non-empty (workgroup, tile)
// reserves the workgroup's range in the tile's bucket; positions inside it are
// handed out by LDS atomics.
__global__ __launch_bounds__(256) void k_scatter_lds(Args a) {
    if (overflowed(a.status)) return;
    extern __shared__ uint32_t base[];
    const int f = blockIdx.y;
    const uint32_t* bh = a.bhist + (static_cast<int64_t>(f) * a.bin_blocks + blockIdx.x) * a.tiles;
    const int64_t tile0 = static_cast<int64_t>(f) * a.tiles;
    for (int t = threadIdx.x; t < a.tiles; t += 256) {
        const uint32_t v = bh[t];
        base[t] = v ? a.toff[tile0 + t] + atomicAdd(&a.tcur[tile0 + t], v) : 0u;
    }
    __syncthreads();
    const int64_t g0 = static_cast<int64_t>(blockIdx.x) * BIN_GROUP;
#pragma unroll 1
    for (int k = 0; k < BIN_GROUP / 256; ++k) {
        const int64_t g = g0 + k * 256 + threadIdx.x;
        if (g < a.n) scatter_one(a, f, g, [&](int tl) { return atomicAdd(&base[tl], 1u); });
    }
}

// Fallback for tile grids too large for an LDS histogram: global atomics per
// intersection.
template <bool EXT>
__global__ __launch_bounds__(256) void k_project(Args a) {
    const int f = blockIdx.y;
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= a.n) return;
    const CamD cam = load_camera(a.poses + 7 * f);
    const double t = a.times ? static_cast<double>(a.times[f]) : static_cast<double>(a.t0);
    uint32_t* tc = a.tcnt + static_cast<int64_t>(f) * a.tiles;
    project_and_count<EXT>(a, f, g, cam, t, [&](int tl) { atomicAdd(&tc[tl], 1u); });
}

__global__ __launch_bounds__(256) void k_scatter(Args a) {
    if (overflowed(a.status)) return;
    const int f = blockIdx.y;
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= a.n) return;
    const int64_t tile0 = static_cast<int64_t>(f) * a.tiles;
    scatter_one(a, f, g, [&](int tl) { return a.toff[tile0 + tl] + atomicAdd(&a.tcur[tile0 + tl], 1u); });
}

// Copy frame 0's projected records out for inspection: (u, v, A00, A01, A11,
// depth, opacity, 0) and the tile count (0 = culled).
__global__ __launch_bounds__(256) void k_export_records(Args a, float* __restrict__ out, int32_t* __restrict__ counts) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= a.n) return;
    const uint32_t c = a.gcnt[g];
    counts[g] = static_cast<int32_t>(c);
    float* o = out + 8 * g;
    if (c) {
        const Record r = a.rec[g];
        o[0] = static_cast<float>(r.u);
        o[1] = static_cast<float>(r.v);
        o[2] = r.a;
        o[3] = r.b;
        o[4] = r.c;
        o[5] = r.depth;
        o[6] = a.col4[g].o;  // frame 0
    } else {
        for (int k = 0; k < 7; ++k) o[k] = 0.0f;
    }
    o[7] = 0.0f;
}

hipError_t launch_export_records(const Args& a, float* records, int32_t* counts, hipStream_t stream) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_export_records, dim3(static_cast<uint32_t>((a.n + 255) / 256)), dim3(256), 0, stream, a,
                       records, counts);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(static_cast<uint32_t>((count + 255) / 256)), dim3(256), 0, stream, p, value,
                       count);
    return hipGetLastError();
}

int64_t bin_blocks(int64_t n) { return (n + BIN_GROUP - 1) / BIN_GROUP; }

hipError_t launch_project(const Args& a, hipStream_t stream) {
    if (a.n <= 0) return hipSuccess;
    const bool ext = a.n_ctrl > 0 || a.scale_coeffs || a.quat_coeffs || a.sh_degree > 0;
    const dim3 block(256);
    if (a.bhist) {
        const dim3 grid(static_cast<uint32_t>(a.bin_blocks), a.frames);
        const size_t lds = sizeof(uint32_t) * a.tiles;
        if (ext) hipLaunchKernelGGL(k_project_lds<true>, grid, block, lds, stream, a);
        else hipLaunchKernelGGL(k_project_lds<false>, grid, block, lds, stream, a);
    } else {
        const dim3 grid(static_cast<uint32_t>((a.n + 255) / 256), a.frames);
        if (ext) hipLaunchKernelGGL(k_project<true>, grid, block, 0, stream, a);
        else hipLaunchKernelGGL(k_project<false>, grid, block, 0, stream, a);
    }
    return hipGetLastError();
}

hipError_t launch_scatter(const Args& a, hipStream_t stream) {
    if (a.n <= 0) return hipSuccess;
    if (a.bhist) {
        hipLaunchKernelGGL(k_scatter_lds, dim3(static_cast<uint32_t>(a.bin_blocks), a.frames), dim3(256),
                           sizeof(uint32_t) * a.tiles, stream, a);
    } else {
        hipLaunchKernelGGL(k_scatter, dim3(static_cast<uint32_t>((a.n + 255) / 256), a.frames), dim3(256), 0, stream,
                           a);
    }
    return hipGetLastError();
}

}  // namespace gv
