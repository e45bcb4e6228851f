// Per-tile depth sort.  The binning pass already grouped the intersections by
// (frame, tile) (a counting sort on the tile digit); each tile's bucket is
// then sorted by the 64-bit key (fp32 depth bits, Gaussian index) in LDS by
// one workgroup: ranks by comparison within chunks of 16 keys, then by merging
// pairs of sorted runs level by level (binary search in the other run).  Keys are unique within a bucket, so the order is fully determined
// (depth, ties by lower index) whatever order the atomics of the scatter
// produced.  Buckets longer than the LDS capacity are sorted in LDS chunks and
// merged in global memory (each element finds its place in the partner run by
// binary search).
#include "gv_internal.h"

namespace gv {

// Number of keys below x in the sorted run S[0, R) (R a power of two; slots
// past the run's keys hold keys above every real key): binary lifting.
__device__ __forceinline__ int count_below(const uint64_t* S, int R, uint64_t x) {
    int lo = 0;
    for (int step = R >> 1; step >= 1; step >>= 1)
        if (S[lo + step - 1] < x) lo += step;
    if (S[lo] < x) ++lo;
    return lo;
}

// Keys that pad the LDS buffers: above every real key (whose high word is the
// bit pattern of a finite depth) and distinct from each other.
__device__ __forceinline__ uint64_t pad_key(int e) { return 0xFFFFFFFF00000000ull | static_cast<uint32_t>(e); }

// Ranks of the keys of one bucket segment of len <= CAP keys, in LDS.
// Thread t owns elements e = t + WG j (their keys and values stay in
// registers; only keys are exchanged through LDS).  Level 0 ranks every key
// within its chunk of 16 by comparison with the chunk's keys; each following
// level merges pairs of sorted runs (16 -> 32 -> 64 -> ...): a key's rank in
// the merged run is its rank in its own run plus the number of the other
// run's keys below it.  Each level writes its sorted
// runs (key at its rank) for the next level's searches.  Padding keys lie
// above every real key (real depths are finite) and are distinct, so the
// ranks of a level are a permutation and every slot is written.  Returns the
// buffer (SA or SB) holding the keys in sorted order.
template <int CAP>
__device__ __forceinline__ uint64_t* lds_sort_ranks(const KeySlot* src, int len, uint64_t* SA, uint64_t* SB,
                                               uint64_t (&x)[CAP / WG], uint32_t (&v)[CAP / WG],
                                               int (&rank)[CAP / WG]) {
    constexpr int EPT = CAP / WG;
    const int npad = (len + 15) & ~15;
    // the last level merges groups of `top` keys; slots [npad, top) of both
    // buffers keep padding keys, so every run searched has its full length
    int top = 16;
    while (top < npad) top <<= 1;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int e = threadIdx.x + WG * j;
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
        const int e = threadIdx.x + WG * j;
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
    for (int R = 16; R < npad; R <<= 1) {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int e = threadIdx.x + WG * j;
            if (e >= npad) continue;
            const int gb = e & ~(2 * R - 1);  // first element of the pair of runs
            const int st = (e & R) ? gb : gb + R;  // the other run
            int r = rank[j];
            if (st < npad) r += count_below(cur + st, R, x[j]);
            rank[j] = r;
            nxt[gb + r] = x[j];
        }
        __syncthreads();
        uint64_t* tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
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
__global__ __launch_bounds__(WG) void k_tile_sort(Args a) {
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
    if (n <= CAP) {
        lds_sort_ranks<CAP>(a.kv + s, static_cast<int>(n), SA, SB, x, v, rank);
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
    KeySlot* src = a.kv + s;
    if (n <= 2 * CAP) {
        // Two runs: the first is sorted and written back in place, the
        // second sorted in LDS; the first's keys are then reloaded into the
        // other LDS buffer and every element adds the number of keys below it
        // in the other run (binary search in LDS).
        lds_sort_ranks<CAP>(src, CAP, SA, SB, x, v, rank);
#pragma unroll
        for (int j = 0; j < EPT; ++j) src[rank[j]] = KeySlot{x[j], v[j], 0u};
        __syncthreads();
        const int len1 = static_cast<int>(n) - CAP;
        const uint64_t* K1 = lds_sort_ranks<CAP>(src + CAP, len1, SA, SB, x, v, rank);
        uint64_t* K0 = K1 == SA ? SB : SA;
        // run 1's keys and padding fill K1[0, top1) (the group size of its last level)
        int top1 = 16;
        while (top1 < ((len1 + 15) & ~15)) top1 <<= 1;
        for (int i = threadIdx.x; i < CAP; i += WG) K0[i] = src[i].key;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int i = threadIdx.x + WG * j;
            if (i < len1) {
                const int r = rank[j] + count_below(K0, CAP, x[j]);
                a.sgid[s + r] = static_cast<uint32_t>(x[j]);
                a.sslot[s + r] = v[j];
            }
            const KeySlot e0 = src[i];
            const int r0 = i + count_below(K1, top1, e0.key);
            a.sgid[s + r0] = static_cast<uint32_t>(e0.key);
            a.sslot[s + r0] = e0.slot;
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
