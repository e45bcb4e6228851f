// Per-tile depth sort.  The binning pass already grouped the intersections by
// (frame, tile) (a counting sort on the tile digit); each tile's bucket is
// then sorted by the 64-bit key (fp32 depth bits, Gaussian index) in LDS by
// one workgroup: ranks by comparison within chunks of 16 keys, then by merging
// pairs of sorted runs level by level (binary search in the other run, the
// searches of a thread's elements interleaved).  Keys are unique within a
// bucket, so the order is fully determined (depth, ties by lower index)
// whatever order the atomics of the scatter produced.  Buckets longer than the
// LDS capacity are sorted in LDS chunks and merged in global memory (each
// element finds its place in the partner run by binary search).
#include "gv_internal.h"

namespace gv {

// Keys that pad the LDS buffers: above every real key (whose high word is the
// bit pattern of a finite depth) and distinct from each other.
__device__ __forceinline__ uint64_t pad_key(int e) { return 0xFFFFFFFF00000000ull | static_cast<uint32_t>(e); }

// Adds to rank[j0 + j] (j < NJ) the number of keys below x[j0 + j] in the
// sorted run of R keys at S + st[j0 + j] (R a power of two; slots past the
// run's keys hold keys above every real key): binary lifting, unrolled, the
// NJ searches interleaved so that their LDS reads are in flight together.
template <int R, int NJ, int EPT>
__device__ __forceinline__ void count_below_n(const uint64_t* S, int j0, const int (&st)[EPT],
                                              const uint64_t (&x)[EPT], int (&rank)[EPT]) {
    const uint64_t* p[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) p[j] = S + st[j0 + j];
#pragma unroll
    for (int step = R / 2; step >= 1; step /= 2) {
        uint64_t y[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) y[j] = p[j][step - 1];
#pragma unroll
        for (int j = 0; j < NJ; ++j) p[j] = y[j] < x[j0 + j] ? p[j] + step : p[j];
    }
    uint64_t y[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) y[j] = p[j][0];
#pragma unroll
    for (int j = 0; j < NJ; ++j)
        rank[j0 + j] += static_cast<int>(p[j] - (S + st[j0 + j])) + (y[j] < x[j0 + j] ? 1 : 0);
}

// count_below_n over the elements j of this wave that hold a key, j < EPT:
// element j of thread t is e = t + WG j, so they are a prefix of j, the same
// for the whole wave ((t & ~63) + WG j < live).  Up to four searches are
// interleaved at a time.  Lanes whose e is past `live` search as well (every
// window lies inside the buffer) and their results are ignored.
template <int R, int EPT>
__device__ __forceinline__ void count_below_wave(const uint64_t* S, int live, const int (&st)[EPT],
                                                 const uint64_t (&x)[EPT], int (&rank)[EPT]) {
    const int w0 = static_cast<int>(threadIdx.x) & ~63;
#pragma unroll
    for (int j0 = 0; j0 < EPT; j0 += 4) {
        int nj = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) nj += (j0 + j < EPT && w0 + WG * (j0 + j) < live) ? 1 : 0;
        if (nj == 0) break;
        if (nj == 4 && j0 + 4 <= EPT) count_below_n<R, (EPT < 4 ? EPT : 4), EPT>(S, j0, st, x, rank);
        else if (nj >= 3 && EPT >= 3) count_below_n<R, (EPT < 3 ? EPT : 3), EPT>(S, j0, st, x, rank);
        else if (nj >= 2 && EPT >= 2) count_below_n<R, (EPT < 2 ? EPT : 2), EPT>(S, j0, st, x, rank);
        else count_below_n<R, 1, EPT>(S, j0, st, x, rank);
        if (nj < 4) break;
    }
}

// count_below_wave for a run length known only at run time (a power of two,
// R <= runlen <= CAP).
template <int R, int CAP>
__device__ __forceinline__ void count_below_wave_upto(const uint64_t* S, int runlen, int live,
                                                      const int (&st)[CAP / WG], const uint64_t (&x)[CAP / WG],
                                                      int (&rank)[CAP / WG]) {
    if constexpr (R < CAP) {
        if (runlen > R) {
            count_below_wave_upto<2 * R, CAP>(S, runlen, live, st, x, rank);
            return;
        }
    }
    count_below_wave<R, CAP / WG>(S, live, st, x, rank);
}

// Merge levels R, 2R, ... below npad: a key's rank in the merged pair of runs
// is its rank in its own run plus the number of the other run's keys below it.
// Each level reads `cur` and writes its merged runs to `nxt`; the buffers
// swap after every level.
template <int R, int CAP>
__device__ __forceinline__ void merge_levels(uint64_t*& cur, uint64_t*& nxt, int npad, const uint64_t (&x)[CAP / WG],
                                             int (&rank)[CAP / WG]) {
    constexpr int EPT = CAP / WG;
    if constexpr (R < CAP) {
        if (R >= npad) return;
        // the thread index passes through an empty asm statement, so that the
        // compiler cannot compute every level's windows up front (registers)
        int t = static_cast<int>(threadIdx.x);
        asm volatile("" : "+v"(t));
        int st[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int e = t + WG * j;
            const int gb = e & ~(2 * R - 1);  // first element of the pair of runs
            st[j] = (e & R) ? gb : gb + R;    // the other run
        }
        count_below_wave<R, EPT>(cur, npad, st, x, rank);
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int e = t + WG * j;
            if (e < npad) nxt[(e & ~(2 * R - 1)) + rank[j]] = x[j];
        }
        __syncthreads();
        uint64_t* tmp = cur;
        cur = nxt;
        nxt = tmp;
        merge_levels<2 * R, CAP>(cur, nxt, npad, x, rank);
    }
}

// Ranks of the keys of one bucket segment of len <= CAP keys, in LDS.
// Thread t owns elements e = t + WG j (their keys and values stay in
// registers; only keys are exchanged through LDS).  Level 0 ranks every key
// within its chunk of 16 by comparison with the chunk's keys; each following
// level merges pairs of sorted runs (16 -> 32 -> 64 -> ...).  Each level
// writes its sorted runs (key at its rank) for the next level's searches.
// Padding keys lie above every real key (real depths are finite) and are
// distinct, so the ranks of a level are a permutation and every slot is
// written.  Returns the buffer (SA or SB) holding the keys in sorted order.
template <int CAP>
__device__ __forceinline__ uint64_t* lds_sort_ranks(const KeySlot* src, int len, uint64_t* SA, uint64_t* SB,
                                               uint64_t (&x)[CAP / WG], uint32_t (&v)[CAP / WG],
                                               int (&rank)[CAP / WG]) {
    constexpr int EPT = CAP / WG;
    int t = static_cast<int>(threadIdx.x);  // see merge_levels
    asm volatile("" : "+v"(t));
    const int npad = (len + 15) & ~15;
    // the last level merges groups of `top` keys; slots [npad, top) of both
    // buffers keep padding keys, so every run searched has its full length
    int top = 16;
    while (top < npad) top <<= 1;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int e = t + WG * j;
        if (e < len) {
            const KeySlot ks = src[e];
            x[j] = ks.key;
            v[j] = ks.slot;
        } else {
            x[j] = pad_key(e);
            v[j] = 0u;
        }
        if (e < npad) SA[e] = x[j];
        else if (e < top) SA[e] = SB[e] = pad_key(e);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int e = t + WG * j;
        rank[j] = 0;
        if (e < npad) {
            const uint64_t* C = SA + (e & ~15);
            int r = 0;
#pragma unroll
            for (int k = 0; k < 16; ++k) r += C[k] < x[j] ? 1 : 0;
            rank[j] = r;
            SB[(e & ~15) + r] = x[j];
        }
    }
    __syncthreads();
    uint64_t* cur = SB;
    uint64_t* nxt = SA;
    merge_levels<16, CAP>(cur, nxt, npad, x, rank);
    return cur;
}

// Number of elements of the sorted run R[0, len) whose key is strictly smaller.
__device__ __forceinline__ int64_t lower_rank(const KeySlot* R, int64_t len, uint64_t key) {
    int64_t lo = 0, hi = len;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (R[mid].key < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <int CAP>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(CAP <= 1024 ? 7 : 1))) void k_tile_sort(Args a) {
    if (overflowed(a.status)) return;
    const int64_t seg = blockIdx.x;
    uint32_t s, e;
    bucket_range(a, seg, s, e);
    const int64_t n = static_cast<int64_t>(e) - s;
    if (n <= 0) return;
    constexpr int EPT = CAP / WG;
    __shared__ uint64_t SA[CAP], SB[CAP];
    uint64_t x[EPT];
    uint32_t v[EPT];
    int rank[EPT];
    KeySlot* src = a.kv + s;
    if (n <= 2 * CAP) {
        // One run, or two: the first is sorted and written back in place, the
        // second sorted in LDS; the first's keys are then reloaded into the
        // other LDS buffer and every element adds the number of keys below it
        // in the other run (binary search in LDS).  One copy of the LDS sort
        // serves both runs.
        const int runs = n <= CAP ? 1 : 2;
        const uint64_t* K1 = nullptr;
#pragma unroll 1
        for (int run = 0; run < runs; ++run) {
            const int len = run == 0 ? (n < CAP ? static_cast<int>(n) : CAP) : static_cast<int>(n) - CAP;
            K1 = lds_sort_ranks<CAP>(src + run * CAP, len, SA, SB, x, v, rank);
            if (run + 1 < runs) {
#pragma unroll
                for (int j = 0; j < EPT; ++j) src[rank[j]] = KeySlot{x[j], v[j], 0u};
                __syncthreads();
            }
        }
        if (runs == 1) {
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                const int i = threadIdx.x + WG * j;
                if (i < n) {
                    a.sgid[s + rank[j]] = static_cast<uint32_t>(x[j]);
                    a.sslot[s + rank[j]] = v[j];
                }
            }
            return;
        }
        const int len1 = static_cast<int>(n) - CAP;
        uint64_t* K0 = K1 == SA ? SB : SA;
        // run 1's keys and padding fill K1[0, top1) (the group size of its last level)
        int top1 = 16;
        while (top1 < ((len1 + 15) & ~15)) top1 <<= 1;
        for (int i = threadIdx.x; i < CAP; i += WG) K0[i] = src[i].key;
        __syncthreads();
        int st[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) st[j] = 0;
        // run 1's elements: their rank in run 1 plus run 0's keys below them
        count_below_wave<CAP, EPT>(K0, len1, st, x, rank);
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int i = threadIdx.x + WG * j;
            if (i < len1) {
                a.sgid[s + rank[j]] = static_cast<uint32_t>(x[j]);
                a.sslot[s + rank[j]] = v[j];
            }
        }
        // run 0's elements: their position in run 0 plus run 1's keys below them
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int i = threadIdx.x + WG * j;
            const KeySlot e0 = src[i];
            x[j] = e0.key;
            v[j] = e0.slot;
            rank[j] = i;
        }
        count_below_wave_upto<16, CAP>(K1, top1, CAP, st, x, rank);
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            a.sgid[s + rank[j]] = static_cast<uint32_t>(x[j]);
            a.sslot[s + rank[j]] = v[j];
        }
        return;
    }
    // Long bucket: sorted runs of CAP in place, then pairwise merges.
    KeySlot* dst = a.tkv + s;
    for (int64_t c0 = 0; c0 < n; c0 += CAP) {
        const int len = static_cast<int>(n - c0 < CAP ? n - c0 : CAP);
        // every thread reads its elements of the chunk before the first
        // barrier inside lds_sort_ranks, so the chunk may then be overwritten
        lds_sort_ranks<CAP>(src + c0, len, SA, SB, x, v, rank);
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int i = threadIdx.x + WG * j;
            if (i < len) src[c0 + rank[j]] = KeySlot{x[j], v[j], 0u};
        }
        __syncthreads();
    }
    for (int64_t w = CAP; w < n; w <<= 1) {
        for (int64_t lo = 0; lo < n; lo += 2 * w) {
            const int64_t mid = lo + w < n ? lo + w : n;
            const int64_t hi = lo + 2 * w < n ? lo + 2 * w : n;
            for (int64_t i = lo + threadIdx.x; i < hi; i += WG) {
                const KeySlot e = src[i];
                int64_t pos;
                if (i < mid) pos = lo + (i - lo) + lower_rank(src + mid, hi - mid, e.key);
                else pos = lo + (i - mid) + lower_rank(src + lo, mid - lo, e.key);
                dst[pos] = e;
            }
        }
        __syncthreads();
        KeySlot* t = src;
        src = dst;
        dst = t;
    }
    for (int64_t i = threadIdx.x; i < n; i += WG) {
        const KeySlot e = src[i];
        a.sgid[s + i] = static_cast<uint32_t>(e.key);
        a.sslot[s + i] = e.slot;
    }
}

hipError_t launch_tile_sort(const Args& a, int64_t segments, hipStream_t stream) {
    if (segments <= 0) return hipSuccess;
    const dim3 grid(static_cast<uint32_t>(segments)), block(WG);
    switch (a.tune.sort_cap) {
        case 512: hipLaunchKernelGGL(k_tile_sort<512>, grid, block, 0, stream, a); break;
        case 1024: hipLaunchKernelGGL(k_tile_sort<1024>, grid, block, 0, stream, a); break;
        case 2048: hipLaunchKernelGGL(k_tile_sort<2048>, grid, block, 0, stream, a); break;
        default: hipLaunchKernelGGL(k_tile_sort<4096>, grid, block, 0, stream, a); break;
    }
    return hipGetLastError();
}

}  // namespace gv
