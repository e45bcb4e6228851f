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

// One thread per (frame, Gaussian): projected record, tile rectangle, the
// number of 16x16 tiles whose pixel-centre box meets the 3-sigma ellipse
// (exact ellipse-box test) and the per-tile counts.  Frame 0 also writes the
// per-Gaussian colour/opacity table shared by all frames.
__global__ __launch_bounds__(256) void k_project(Args a) {
    const int f = blockIdx.y;
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= a.n) return;
    const int64_t i = static_cast<int64_t>(f) * a.n + g;
    const CamD cam = load_camera(a.poses + 7 * f);
    const double t = a.times ? static_cast<double>(a.times[f]) : static_cast<double>(a.t0);

    if (f == 0) {
        const double eta = load_param(a.opacity_logits, a.dtype, g);
        ColorOp co;
        co.r = static_cast<float>(load_param(a.colors, a.dtype, g));
        co.g = static_cast<float>(load_param(a.colors, a.dtype, a.n + g));
        co.b = static_cast<float>(load_param(a.colors, a.dtype, 2 * a.n + g));
        co.o = static_cast<float>(1.0 / (1.0 + exp(-eta)));
        a.col4[g] = co;
    }

    ProjD P;
    const bool vis = project_gaussian(a, g, cam, t, P);
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
            uint32_t* tc = a.tcnt + static_cast<int64_t>(f) * a.tiles;
            for (int ty = ty0; ty <= ty1; ++ty)
                for (int tx = tx0; tx <= tx1; ++tx) {
                    double x0, x1, y0, y1;
                    tile_box(tx, ty, a.width, a.height, x0, x1, y0, y1);
                    if (ellipse_meets_box<double>(r.u, r.v, ca, cb, cc, x0, x1, y0, y1, BIN_Q_SLACK)) {
                        ++cnt;
                        atomicAdd(&tc[ty * a.tiles_x + tx], 1u);
                    }
                }
            a.rec[i] = r;
            a.rect[i] = make_uint2(static_cast<uint32_t>(tx0) | (static_cast<uint32_t>(tx1) << 16),
                                   static_cast<uint32_t>(ty0) | (static_cast<uint32_t>(ty1) << 16));
        }
    }
    a.gcnt[i] = cnt;
}

// Second pass: write key = (fp32 depth bits << 32 | Gaussian index) and the
// pre-sort slot (goff + k for the k-th tile of this Gaussian) of every
// intersection into its tile's bucket.  Decisions repeat k_project's exactly
// (same inputs, same test, no contraction).
__global__ __launch_bounds__(256) void k_scatter(Args a) {
    if (overflowed(a.status)) return;
    const int f = blockIdx.y;
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= a.n) return;
    const int64_t i = static_cast<int64_t>(f) * a.n + g;
    const uint32_t cnt = a.gcnt[i];
    if (cnt == 0) return;
    const Record r = a.rec[i];
    const uint2 rc = a.rect[i];
    const int tx0 = rc.x & 0xffff, tx1 = rc.x >> 16, ty0 = rc.y & 0xffff, ty1 = rc.y >> 16;
    const uint64_t key = (static_cast<uint64_t>(__float_as_uint(r.depth)) << 32) | static_cast<uint64_t>(g);
    const uint32_t base = a.goff[i];
    const double ca = r.a, cb = r.b, cc = r.c;
    const int64_t tile0 = static_cast<int64_t>(f) * a.tiles;
    uint32_t k = 0;
    for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx) {
            double x0, x1, y0, y1;
            tile_box(tx, ty, a.width, a.height, x0, x1, y0, y1);
            if (ellipse_meets_box<double>(r.u, r.v, ca, cb, cc, x0, x1, y0, y1, BIN_Q_SLACK)) {
                const int64_t tile = tile0 + ty * a.tiles_x + tx;
                const uint32_t pos = a.toff[tile] + atomicAdd(&a.tcur[tile], 1u);
                // the counts of k_project bound every write; a mismatch is an
                // internal error, reported instead of written out of bounds
                if (pos >= a.toff[tile + 1] || k >= cnt) {
                    a.status[ST_OVERFLOW] = 2u;
                    continue;
                }
                a.keys[pos] = key;
                a.kslot[pos] = base + k;
                ++k;
            }
        }
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
        o[6] = a.col4[g].o;
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

hipError_t launch_project(const Args& a, hipStream_t stream) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_project, dim3(static_cast<uint32_t>((a.n + 255) / 256), a.frames), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_scatter(const Args& a, hipStream_t stream) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3(static_cast<uint32_t>((a.n + 255) / 256), a.frames), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace gv
