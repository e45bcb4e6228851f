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

// The frame-independent shape of every Gaussian of a static scene (no
// dynamics, no SH), once per call instead of once per frame.
__global__ __launch_bounds__(256) void k_static_shapes(Args a) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= a.n) return;
    const int64_t n = a.n;
    double raw[14];
    for (int k = 0; k < 3; ++k) raw[k] = 0.0;
    for (int k = 0; k < 3; ++k) raw[3 + k] = load_param(a.log_scales, a.dtype, k * n + g);
    for (int k = 0; k < 4; ++k) raw[6 + k] = load_param(a.quats, a.dtype, k * n + g);
    raw[10] = load_param(a.opacity_logits, a.dtype, g);
    for (int k = 0; k < 3; ++k) raw[11 + k] = load_param(a.colors, a.dtype, k * n + g);
    bool fin = true;
    for (int k = 3; k < 14; ++k) fin = fin && isfinite(raw[k]);
    ShapeD S;
    ProjD P;
    const bool ok = fin && shape_from_params(raw, P);
    for (int k = 0; k < 6; ++k) S.Sig[k] = ok ? P.Sig[k] : 0.0;
    S.o = ok ? P.o : 0.0;
    S.fin = fin ? 1u : 0u;
    S.qn_ok = ok ? 1u : 0u;
    a.shapes[g] = S;
}

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

// A projected Gaussian's binning data: its ellipse (centre, rounded conic
// and the edge-minimiser slopes of ellipse_meets_box_r) and its tile
// rectangle (tx0, ty0, width rw, height rh).
struct BinShape {
    double u, v, a, b, c, rbc, rba;
    int tx0, ty0, rw, rh;
};

// Project Gaussian g in frame f: write its record, tile rectangle and colour,
// and return true with its binning shape if it can reach a pixel (visible,
// opacity at least 1/255, non-empty tile rectangle).  Frame 0 also writes
// the per-Gaussian colour/opacity table shared by all frames.
template <bool EXT>
__device__ __forceinline__ bool project_one(const Args& a, int f, int64_t g, const CamD& cam, double t, BinShape& S) {
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
    // the static instantiation takes the shapes launch_project computed first
    bool vis;
    if constexpr (EXT) vis = project_gaussian<true>(a, g, cam, t, P);
    else vis = project_gaussian_shaped(a, g, cam, t, P);
    if (EXT && vis && a.sh_degree > 0) {
        ColorOp co;
        co.r = static_cast<float>(P.col[0]);
        co.g = static_cast<float>(P.col[1]);
        co.b = static_cast<float>(P.col[2]);
        co.o = static_cast<float>(P.o);
        a.col4[i] = co;
    }
    if (P.nonfinite) atomicAdd(&a.status[ST_NONFINITE], 1u);
    // o < 1/255 can never pass the per-pixel alpha test (alpha <= o).
    if (!vis || !(P.o >= static_cast<double>(ALPHA_MIN) * (1.0 - 1e-6))) return false;
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
    if (!tile_span(P.u - hx, P.u + hx, a.tiles_x, tx0, tx1) || !tile_span(P.v - hy, P.v + hy, a.tiles_y, ty0, ty1))
        return false;
    a.rec[i] = r;
    a.dkey[i] = r.depth;
    a.rect[i] = make_uint2(static_cast<uint32_t>(tx0) | (static_cast<uint32_t>(tx1) << 16),
                           static_cast<uint32_t>(ty0) | (static_cast<uint32_t>(ty1) << 16));
    S.u = r.u;
    S.v = r.v;
    S.a = r.a;
    S.b = r.b;
    S.c = r.c;
    S.rbc = -S.b / S.c;
    S.rba = -S.b / S.a;
    S.tx0 = tx0;
    S.ty0 = ty0;
    S.rw = tx1 - tx0 + 1;
    S.rh = ty1 - ty0 + 1;
    return true;
}

// Does the ellipse of S meet tile (tx, ty)?  The one test of both binning
// passes (exact ellipse-box minimum, slack for the fp32 per-pixel test).
__device__ __forceinline__ bool shape_meets_tile(const Args& a, const BinShape& S, int tx, int ty) {
    double x0, x1, y0, y1;
    tile_box(tx, ty, a.width, a.height, x0, x1, y0, y1);
    return ellipse_meets_box_r<double>(S.u, S.v, S.a, S.b, S.c, S.rbc, S.rba, x0, x1, y0, y1, BIN_Q_SLACK);
}

__device__ __forceinline__ BinShape shape_from_record(const Record& r, uint2 rc) {
    BinShape S;
    S.u = r.u;
    S.v = r.v;
    S.a = r.a;
    S.b = r.b;
    S.c = r.c;
    S.rbc = -S.b / S.c;
    S.rba = -S.b / S.a;
    S.tx0 = rc.x & 0xffff;
    S.ty0 = rc.y & 0xffff;
    S.rw = static_cast<int>(rc.x >> 16) - S.tx0 + 1;
    S.rh = static_cast<int>(rc.y >> 16) - S.ty0 + 1;
    return S;
}

// Exclusive prefix sum of x over the wave and the wave total.
__device__ __forceinline__ uint32_t wave_exclusive_scan(uint32_t x, int lane, uint32_t& total) {
    uint32_t incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = static_cast<uint32_t>(__shfl_up(static_cast<int>(incl), d, 64));
        if (lane >= d) incl += t;
    }
    total = static_cast<uint32_t>(__shfl(static_cast<int>(incl), 63, 64));
    return incl - x;
}

// Lane owning work item b0 + lane of a wave whose lanes deal out `cnt` items
// each from exclusive starts `start`: the last lane with items whose start is
// at most the item.  Each owner whose first item falls in [b0, b0 + 64) marks
// that position in `own` (64 slots of the wave, in LDS); an item's owner is
// the mark at or below its position, or, before the first mark, the owner of
// item b0 (the last lane with items starting at or before b0).
__device__ __forceinline__ int chunk_owner(uint32_t* own, uint32_t start, uint32_t cnt, uint32_t b0, int lane) {
    own[lane] = 0u;
    __builtin_amdgcn_wave_barrier();
    if (cnt && start >= b0 && start - b0 < 64u) own[start - b0] = static_cast<uint32_t>(lane) + 1u;
    __builtin_amdgcn_wave_barrier();
    const uint32_t mark = own[lane];
    const uint64_t marks = __ballot(mark != 0u);
    const uint64_t before = __ballot(cnt != 0u && start <= b0);
    const int carry = before ? 63 - __builtin_clzll(before) : 0;
    const uint64_t upto = marks & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
    const int src = upto ? 63 - __builtin_clzll(upto) : 0;
    const int m = __shfl(static_cast<int>(mark), src, 64);
    __builtin_amdgcn_wave_barrier();
    return upto ? m - 1 : carry;
}

// Index of the (k+1)-th set bit of m (k < popcount(m)).
__device__ __forceinline__ int kth_set_bit(uint64_t m, uint32_t k) {
    int b = 0;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const uint64_t low = m & ((1ull << w) - 1ull);
        const uint32_t c = static_cast<uint32_t>(__popcll(low));
        if (k >= c) {
            k -= c;
            m >>= w;
            b += w;
        } else {
            m = low;
        }
    }
    return b;
}

// Per-wave LDS staging of the cooperative rectangle walk: the cells of the
// 64 lanes' tile rectangles are dealt out one per lane and step, so a wave
// takes (total cells) / 64 steps instead of its largest rectangle.
struct WaveCells {
    BinShape shape[64];
    uint32_t start[64];
    uint32_t own[64];
    unsigned long long mask[64];
    uint32_t cnt[64];
};

// Binning with workgroup-local tile histograms in LDS: each workgroup
// projects BIN_GROUP Gaussians of one frame, counts their intersections per
// tile with LDS atomics (16-bit counts, two tiles per word: a count never
// exceeds BIN_GROUP), stores its histogram and adds it to the frame's tile
// counts with one global atomic per non-empty tile.  A Gaussian's passing
// tiles are also recorded as a row-major mask over its rectangle (rectangles
// of at most 64 tiles), which the scatter walks.
template <bool EXT>
__global__ __launch_bounds__(256) void k_project_lds(Args a) {
    extern __shared__ uint32_t hist[];
    __shared__ WaveCells wc[4];
    const int f = blockIdx.y;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int words = (a.tiles + 1) >> 1;
    for (int t = threadIdx.x; t < words; t += 256) hist[t] = 0u;
    __syncthreads();
    const CamD cam = load_camera(a.poses + 7 * f);
    const double tt = a.times ? static_cast<double>(a.times[f]) : static_cast<double>(a.t0);
    const int64_t g0 = static_cast<int64_t>(blockIdx.x) * BIN_GROUP;
    WaveCells& W = wc[w];
#pragma unroll 1
    for (int k = 0; k < BIN_GROUP / 256; ++k) {
        const int64_t g = g0 + k * 256 + threadIdx.x;
        BinShape S;
        const bool has = g < a.n && project_one<EXT>(a, f, g, cam, tt, S);
        const uint32_t ncell = has ? static_cast<uint32_t>(S.rw * S.rh) : 0u;
        uint32_t total;
        const uint32_t start = wave_exclusive_scan(ncell, lane, total);
        W.shape[lane] = S;
        W.start[lane] = start;
        W.mask[lane] = 0ull;
        W.cnt[lane] = 0u;
        __builtin_amdgcn_wave_barrier();
        for (uint32_t b0 = 0; b0 < total; b0 += 64) {
            const uint32_t item = b0 + static_cast<uint32_t>(lane);
            const int o = chunk_owner(W.own, start, ncell, b0, lane);
            if (item < total) {
                const uint32_t cell = item - W.start[o];
                const BinShape& So = W.shape[o];
                const int ry = static_cast<int>(cell) / So.rw;
                const int tx = So.tx0 + (static_cast<int>(cell) - ry * So.rw), ty = So.ty0 + ry;
                if (shape_meets_tile(a, So, tx, ty)) {
                    const int tl = ty * a.tiles_x + tx;
                    atomicAdd(&hist[tl >> 1], 1u << ((tl & 1) << 4));
                    atomicAdd(&W.cnt[o], 1u);
                    if (So.rw * So.rh <= 64) atomicOr(&W.mask[o], 1ull << cell);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (g < a.n) {
            const int64_t i = static_cast<int64_t>(f) * a.n + g;
            a.gcnt[i] = W.cnt[lane];
            if (has) a.tmask[i] = W.mask[lane];
        }
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    uint32_t* bh = a.bhist + (static_cast<int64_t>(f) * a.bin_blocks + blockIdx.x) * a.tiles;
    uint32_t* tc = a.tcnt + static_cast<int64_t>(f) * a.tiles;
    for (int t = threadIdx.x; t < a.tiles; t += 256) {
        const uint32_t v = (hist[t >> 1] >> ((t & 1) << 4)) & 0xFFFFu;
        bh[t] = v;
        if (v) atomicAdd(&tc[t], v);
    }
}

// Write intersection (f, g) -> tile (tx, ty) with pre-sort slot goff + k at
// position next(tile) of the tile's bucket, below end(tile) (the bucket's end
// in the global-atomic scatter; the workspace's capacity in the LDS scatter,
// whose reservations check the counts).  The counts bound every write; a
// mismatch is an internal error, reported instead of written out of bounds.
template <typename Next, typename End>
__device__ __forceinline__ void emit_key(const Args& a, uint64_t key, uint32_t slot, int tx, int ty, Next next,
                                         End end) {
    const int tl = ty * a.tiles_x + tx;
    const uint32_t pos = next(tl);
    if (pos >= end(tl)) {
        a.status[ST_OVERFLOW] = 2u;
        return;
    }
    KeySlot ks;
    ks.key = key;
    ks.slot = slot;
    ks.pad = 0u;
    a.kv[pos] = ks;
}

// Key (fp32 depth bits << 32 | Gaussian index) of (f, g).
__device__ __forceinline__ uint64_t sort_key(float depth, int64_t g) {
    return (static_cast<uint64_t>(__float_as_uint(depth)) << 32) | static_cast<uint64_t>(g);
}

// Intersections of a Gaussian whose rectangle exceeds 64 tiles (no mask):
// the tests are repeated in the count pass's row-major order.
template <typename Next, typename End>
__device__ __forceinline__ void scatter_big(const Args& a, int64_t g, const Record& r, const BinShape& S,
                                            uint32_t cnt, uint32_t goff, Next next, End end) {
    const uint64_t key = sort_key(r.depth, g);
    uint32_t k = 0;
    for (int ty = S.ty0; ty < S.ty0 + S.rh; ++ty)
        for (int tx = S.tx0; tx < S.tx0 + S.rw; ++tx)
            if (shape_meets_tile(a, S, tx, ty)) {
                if (k >= cnt) {
                    a.status[ST_OVERFLOW] = 2u;
                    return;
                }
                emit_key(a, key, goff + k, tx, ty, next, end);
                ++k;
            }
}

struct WaveKeys {
    unsigned long long mask[64];
    unsigned long long key[64];
    uint32_t start[64];
    uint32_t own[64];
    uint32_t goff[64];
    int tx0[64], ty0[64], rw[64];
};

// Scatter counterpart: one global atomic per non-empty (workgroup, tile)
// reserves the workgroup's range in the tile's bucket; positions inside it are
// handed out by LDS atomics.  A wave deals out its Gaussians' intersections
// (the set bits of their masks) one per lane and step; the k-th set bit of a
// mask gets pre-sort slot goff + k, as the count pass ordered them.
__global__ __launch_bounds__(256) void k_scatter_lds(Args a) {
    if (overflowed(a.status)) return;
    // base[t]: next position of this workgroup's range in tile t's bucket
    extern __shared__ uint32_t base[];
    __shared__ WaveKeys wk[4];
    const int f = blockIdx.y;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t* bh = a.bhist + (static_cast<int64_t>(f) * a.bin_blocks + blockIdx.x) * a.tiles;
    const int64_t tile0 = static_cast<int64_t>(f) * a.tiles;
    // eight tiles per thread at a time: all counts are requested, then all
    // reservations, so each batch costs two memory round trips, not sixteen
    constexpr int RT = 8;
    for (int t0 = 0; t0 < a.tiles; t0 += 256 * RT) {
        uint32_t v[RT], o[RT], lo[RT], hi[RT];
#pragma unroll
        for (int k = 0; k < RT; ++k) {
            const int t = t0 + k * 256 + threadIdx.x;
            v[k] = t < a.tiles ? bh[t] : 0u;
        }
#pragma unroll
        for (int k = 0; k < RT; ++k) {
            const int t = t0 + k * 256 + threadIdx.x;
            o[k] = lo[k] = hi[k] = 0u;
            if (v[k]) {
                o[k] = atomicAdd(&a.tcur[tile0 + t], v[k]);
                lo[k] = a.toff[tile0 + t];
                hi[k] = a.toff[tile0 + t + 1];
            }
        }
#pragma unroll
        for (int k = 0; k < RT; ++k) {
            const int t = t0 + k * 256 + threadIdx.x;
            if (t < a.tiles) {
                const uint32_t b = v[k] ? lo[k] + o[k] : 0u;
                base[t] = b;
                if (v[k] && b + v[k] > hi[k]) a.status[ST_OVERFLOW] = 2u;  // counts disagree: internal error
            }
        }
    }
    __syncthreads();
    // a workgroup emits exactly its histogram's count per tile; the end
    // checked per key is only the workspace's (no write out of bounds even
    // if the counts disagreed, which the reservation above reports)
    auto next = [&](int tl) { return atomicAdd(&base[tl], 1u); };
    auto end = [&](int) { return static_cast<uint32_t>(a.k_cap); };
    const int64_t g0 = static_cast<int64_t>(blockIdx.x) * BIN_GROUP;
    WaveKeys& W = wk[w];
    // A Gaussian's count, depth, rectangle, mask and slot offset, requested
    // together (one memory round trip; a Gaussian without intersections
    // ignores them), and the next round's requested before this round's keys
    // are dealt out.  Only a Gaussian too large for a mask reads its record.
    struct In {
        uint32_t cnt;
        float depth;
        uint2 rc;
        uint64_t tm;
        uint32_t go;
    };
    auto load_in = [&](int k, In& x) {
        const int64_t g = g0 + k * 256 + threadIdx.x;
        const int64_t i = static_cast<int64_t>(f) * a.n + (g < a.n ? g : 0);
        x.cnt = g < a.n ? a.gcnt[i] : 0u;
        x.depth = a.dkey[i];
        x.rc = a.rect[i];
        x.tm = a.tmask[i];
        x.go = a.goff[i];
    };
    In nxt;
    load_in(0, nxt);
    static_assert(BIN_GROUP / 256 <= 32, "one bit per round");
    uint32_t big = 0u;  // rounds whose Gaussian has no mask, scattered after the loop
#pragma unroll 1
    for (int k = 0; k < BIN_GROUP / 256; ++k) {
        const int64_t g = g0 + k * 256 + threadIdx.x;
        const In cur = nxt;
        if (k + 1 < BIN_GROUP / 256) load_in(k + 1, nxt);
        const uint32_t cnt = cur.cnt;
        const uint2 rc = cur.rc;
        const uint64_t tm = cur.tm;
        const uint32_t go = cur.go;
        const bool small =
            cnt && ((rc.x >> 16) - (rc.x & 0xffff) + 1) * ((rc.y >> 16) - (rc.y & 0xffff) + 1) <= 64u;
        uint32_t total;
        const uint32_t start = wave_exclusive_scan(small ? cnt : 0u, lane, total);
        W.start[lane] = start;
        if (small) {
            W.mask[lane] = tm;
            W.key[lane] = sort_key(cur.depth, g);
            W.goff[lane] = go;
            W.tx0[lane] = rc.x & 0xffff;
            W.ty0[lane] = rc.y & 0xffff;
            W.rw[lane] = static_cast<int>(rc.x >> 16) - static_cast<int>(rc.x & 0xffff) + 1;
        }
        __builtin_amdgcn_wave_barrier();
        for (uint32_t b0 = 0; b0 < total; b0 += 64) {
            const uint32_t item = b0 + static_cast<uint32_t>(lane);
            const int o = chunk_owner(W.own, start, small ? cnt : 0u, b0, lane);
            if (item < total) {
                const uint32_t kk = item - W.start[o];
                const uint64_t m = W.mask[o];
                if (kk >= static_cast<uint32_t>(__popcll(m))) {  // counts and mask disagree: internal error
                    a.status[ST_OVERFLOW] = 2u;
                    continue;
                }
                const int bit = kth_set_bit(m, kk);
                const int ry = bit / W.rw[o];
                emit_key(a, W.key[o], W.goff[o] + kk, W.tx0[o] + (bit - ry * W.rw[o]), W.ty0[o] + ry, next, end);
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (cnt && !small) big |= 1u << k;
    }
    // out of the pipelined loop, whose registers the rectangle walk would add to
    while (big) {
        const int k = __builtin_ctz(big);
        big &= big - 1u;
        const int64_t g = g0 + k * 256 + threadIdx.x;
        const int64_t i = static_cast<int64_t>(f) * a.n + g;
        const Record r = a.rec[i];
        scatter_big(a, g, r, shape_from_record(r, a.rect[i]), a.gcnt[i], a.goff[i], next, end);
    }
}

// Fallback for tile grids too large for an LDS histogram: global atomics per
// intersection, one lane per Gaussian.
template <bool EXT>
__global__ __launch_bounds__(256) void k_project(Args a) {
    const int f = blockIdx.y;
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= a.n) return;
    const CamD cam = load_camera(a.poses + 7 * f);
    const double t = a.times ? static_cast<double>(a.times[f]) : static_cast<double>(a.t0);
    uint32_t* tc = a.tcnt + static_cast<int64_t>(f) * a.tiles;
    const int64_t i = static_cast<int64_t>(f) * a.n + g;
    BinShape S;
    uint32_t cnt = 0;
    if (project_one<EXT>(a, f, g, cam, t, S)) {
        uint64_t mask = 0;
        const bool small = S.rw * S.rh <= 64;
        for (int ry = 0; ry < S.rh; ++ry)
            for (int rx = 0; rx < S.rw; ++rx)
                if (shape_meets_tile(a, S, S.tx0 + rx, S.ty0 + ry)) {
                    ++cnt;
                    atomicAdd(&tc[(S.ty0 + ry) * a.tiles_x + S.tx0 + rx], 1u);
                    if (small) mask |= 1ull << (ry * S.rw + rx);
                }
        a.tmask[i] = mask;
    }
    a.gcnt[i] = cnt;
}

__global__ __launch_bounds__(256) void k_scatter(Args a) {
    if (overflowed(a.status)) return;
    const int f = blockIdx.y;
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= a.n) return;
    const int64_t tile0 = static_cast<int64_t>(f) * a.tiles;
    const int64_t i = static_cast<int64_t>(f) * a.n + g;
    const uint32_t cnt = a.gcnt[i];
    if (cnt == 0) return;
    const Record r = a.rec[i];
    const BinShape S = shape_from_record(r, a.rect[i]);
    scatter_big(a, g, r, S, cnt, a.goff[i],
                [&](int tl) { return a.toff[tile0 + tl] + atomicAdd(&a.tcur[tile0 + tl], 1u); },
                [&](int tl) { return a.toff[tile0 + tl + 1]; });
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
    if (!ext)
        hipLaunchKernelGGL(k_static_shapes, dim3(static_cast<uint32_t>((a.n + 255) / 256)), block, 0, stream, a);
    if (a.bhist) {
        const dim3 grid(static_cast<uint32_t>(a.bin_blocks), a.frames);
        const size_t lds = sizeof(uint32_t) * ((a.tiles + 1) / 2);
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
