// Device-wide exclusive prefix sums of u32 counts (three passes: per-block
// scan with 64-bit block totals, scan of the block totals in one workgroup,
// add-back).  The grand total is kept in 64 bits so that an intersection count
// beyond 2^32 is detected as an overflow instead of wrapping.
#include "gv_internal.h"

namespace gv {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;  // 2048 counts per workgroup

// Exclusive scan of x across the 256 threads of the workgroup; returns the
// prefix and writes the workgroup total to *total.
template <typename U>
__device__ __forceinline__ U block_exclusive_scan(U x, U* total) {
    __shared__ U wsum[SCAN_THREADS / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    U inc = x;
    for (int d = 1; d < 64; d <<= 1) {
        const U y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    U before = 0, all = 0;
    for (int k = 0; k < SCAN_THREADS / 64; ++k) {
        if (k < w) before += wsum[k];
        all += wsum[k];
    }
    *total = all;
    __syncthreads();
    return before + inc - x;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_local(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                             int64_t count, unsigned long long* __restrict__ block_sums) {
    const int64_t base = static_cast<int64_t>(blockIdx.x) * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    if (base + SCAN_ITEMS <= count) {
        const uint4 lo = *reinterpret_cast<const uint4*>(in + base);
        const uint4 hi = *reinterpret_cast<const uint4*>(in + base + 4);
        v[0] = lo.x; v[1] = lo.y; v[2] = lo.z; v[3] = lo.w;
        v[4] = hi.x; v[5] = hi.y; v[6] = hi.z; v[7] = hi.w;
    } else {
        for (int k = 0; k < SCAN_ITEMS; ++k) v[k] = (base + k < count) ? in[base + k] : 0u;
    }
    uint32_t sum = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) sum += v[k];
    uint32_t total;
    uint32_t run = block_exclusive_scan<uint32_t>(sum, &total);
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < count) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// One workgroup: exclusive scan of the block totals in place; writes the
// grand total to out[count] (u32) and, if status_total_slot >= 0, to the
// status word, raising the overflow flag when it exceeds k_cap.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_block_sums(unsigned long long* __restrict__ block_sums, int64_t n_blocks,
                                                                  uint32_t* __restrict__ out, int64_t count,
                                                                  uint32_t* __restrict__ status, int check,
                                                                  int64_t k_cap) {
    const int64_t per = (n_blocks + SCAN_THREADS - 1) / SCAN_THREADS;
    const int64_t b0 = threadIdx.x * per;
    unsigned long long s = 0;
    for (int64_t b = b0; b < b0 + per && b < n_blocks; ++b) s += block_sums[b];
    unsigned long long total;
    unsigned long long run = block_exclusive_scan<unsigned long long>(s, &total);
    for (int64_t b = b0; b < b0 + per && b < n_blocks; ++b) {
        const unsigned long long v = block_sums[b];
        block_sums[b] = run;
        run += v;
    }
    if (threadIdx.x == 0) {
        out[count] = static_cast<uint32_t>(total);
        if (check) {
            status[ST_K_LO] = static_cast<uint32_t>(total);
            status[ST_K_HI] = static_cast<uint32_t>(total >> 32);
            if (total > static_cast<uint64_t>(k_cap)) status[ST_OVERFLOW] = 1u;
        }
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_add(uint32_t* __restrict__ out, int64_t count,
                                                           const unsigned long long* __restrict__ block_sums) {
    const uint32_t add = static_cast<uint32_t>(block_sums[blockIdx.x]);
    const int64_t base = static_cast<int64_t>(blockIdx.x) * SCAN_TILE;
    for (int k = threadIdx.x; k < SCAN_TILE; k += SCAN_THREADS) {
        const int64_t i = base + k;
        if (i < count) out[i] += add;
    }
}

int64_t scan_blocks(int64_t count) { return (count + SCAN_TILE - 1) / SCAN_TILE; }

// Exclusive scan in[count] -> out[count + 1] on `stream`; tmp holds
// scan_blocks(count) 64-bit values.
hipError_t exclusive_scan(const uint32_t* in, uint32_t* out, int64_t count, unsigned long long* tmp, uint32_t* status,
                          int check, int64_t k_cap, hipStream_t stream) {
    const int64_t nb = scan_blocks(count);
    if (nb > 0) {
        hipLaunchKernelGGL(k_scan_local, dim3(static_cast<uint32_t>(nb)), dim3(SCAN_THREADS), 0, stream, in, out, count,
                           tmp);
    }
    hipLaunchKernelGGL(k_scan_block_sums, dim3(1), dim3(SCAN_THREADS), 0, stream, tmp, nb, out, count, status, check,
                       k_cap);
    if (nb > 0) {
        hipLaunchKernelGGL(k_scan_add, dim3(static_cast<uint32_t>(nb)), dim3(SCAN_THREADS), 0, stream, out, count, tmp);
    }
    return hipGetLastError();
}

}  // namespace gv
