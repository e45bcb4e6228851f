// Per-tile depth sort.  The binning pass already grouped the intersections by
// (frame, tile) (a counting sort on the tile digit); each tile's bucket is
// then sorted by the 64-bit key (fp32 depth bits, Gaussian index) in LDS by
// one workgroup: rank counting for short buckets, a bitonic network up to the
// LDS capacity.  Keys are unique within a bucket, so the order is fully
// determined (depth, ties by lower index) whatever order the atomics of the
// scatter produced.  Buckets longer than the LDS capacity are sorted in LDS
// chunks and merged in global memory (each element finds its place in the
// partner run by binary search).
#include "gv_internal.h"

namespace gv {

// Buckets up to this length are sorted by rank counting (O(n^2 / threads)
// comparisons, no barriers); longer ones by the bitonic network.
constexpr int RANK_SORT_MAX = 512;

template <int CAP>
__device__ __forceinline__ void bitonic_lds(uint64_t* K, uint32_t* V, int m) {
    for (int k = 2; k <= m; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int lj = __builtin_ctz(j);  // j is a power of two
            for (int p = threadIdx.x; p < (m >> 1); p += WG) {
                const int i = ((p >> lj) << (lj + 1)) | (p & (j - 1));
                const int l = i + j;
                const bool asc = (i & k) == 0;
                const uint64_t ki = K[i], kl = K[l];
                if ((ki > kl) == asc) {
                    K[i] = kl;
                    K[l] = ki;
                    const uint32_t t = V[i];
                    V[i] = V[l];
                    V[l] = t;
                }
            }
            __syncthreads();
        }
    }
}

__device__ __forceinline__ int next_pow2(int x) {
    int m = 2;
    while (m < x) m <<= 1;
    return m;
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
    __shared__ uint64_t K[CAP];
    __shared__ uint32_t V[CAP];
    if (n <= RANK_SORT_MAX) {
        // short bucket: every element's final position is the number of
        // smaller keys (keys are unique); no barriers after the load
        for (int i = threadIdx.x; i < n; i += WG) {
            const KeySlot ks = a.kv[s + i];
            K[i] = ks.key;
            V[i] = ks.slot;
        }
        __syncthreads();
        // each thread ranks element tid and, for buckets longer than WG,
        // element tid + WG, in one pass over the keys
        const int nn = static_cast<int>(n);
        const int i0 = threadIdx.x, i1 = threadIdx.x + WG;
        const uint64_t k0 = i0 < nn ? K[i0] : ~0ull, k1 = i1 < nn ? K[i1] : ~0ull;
        int r0 = 0, r1 = 0;
        if (nn > WG) {
            for (int k = 0; k < nn; ++k) {
                const uint64_t x = K[k];
                r0 += x < k0 ? 1 : 0;
                r1 += x < k1 ? 1 : 0;
            }
        } else if (i0 < nn) {
            int q0 = 0, q1 = 0;
            int k = 0;
            for (; k + 1 < nn; k += 2) {
                q0 += K[k] < k0 ? 1 : 0;
                q1 += K[k + 1] < k0 ? 1 : 0;
            }
            if (k < nn) q0 += K[k] < k0 ? 1 : 0;
            r0 = q0 + q1;
        }
        if (i0 < nn) {
            a.sgid[s + r0] = static_cast<uint32_t>(k0);
            a.sslot[s + r0] = V[i0];
        }
        if (i1 < nn) {
            a.sgid[s + r1] = static_cast<uint32_t>(k1);
            a.sslot[s + r1] = V[i1];
        }
        return;
    }
    if (n <= CAP) {
        const int m = next_pow2(static_cast<int>(n));
        for (int i = threadIdx.x; i < m; i += WG) {
            const KeySlot ks = i < n ? a.kv[s + i] : KeySlot{~0ull, 0u, 0u};
            K[i] = ks.key;
            V[i] = ks.slot;
        }
        __syncthreads();
        bitonic_lds<CAP>(K, V, m);
        for (int i = threadIdx.x; i < n; i += WG) {
            a.sgid[s + i] = static_cast<uint32_t>(K[i]);
            a.sslot[s + i] = V[i];
        }
        return;
    }
    // Long bucket: sorted runs of CAP in place, then pairwise merges.
    KeySlot* src = a.kv + s;
    KeySlot* dst = a.tkv + s;
    for (int64_t c0 = 0; c0 < n; c0 += CAP) {
        const int len = static_cast<int>(n - c0 < CAP ? n - c0 : CAP);
        const int m = next_pow2(len);
        for (int i = threadIdx.x; i < m; i += WG) {
            const KeySlot ks = i < len ? src[c0 + i] : KeySlot{~0ull, 0u, 0u};
            K[i] = ks.key;
            V[i] = ks.slot;
        }
        __syncthreads();
        bitonic_lds<CAP>(K, V, m);
        for (int i = threadIdx.x; i < len; i += WG) src[c0 + i] = KeySlot{K[i], V[i], 0u};
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
        case 1024: hipLaunchKernelGGL(k_tile_sort<1024>, grid, block, 0, stream, a); break;
        case 2048: hipLaunchKernelGGL(k_tile_sort<2048>, grid, block, 0, stream, a); break;
        default: hipLaunchKernelGGL(k_tile_sort<4096>, grid, block, 0, stream, a); break;
    }
    return hipGetLastError();
}

}  // namespace gv
