// Gaussian pyramid of target frames for the spatial hierarchy (Sec. 3.3):
// each level is the previous one blurred by the separable 5-tap binomial
// filter [1 4 6 4 1] / 16 and decimated by 2 (even rows and columns kept),
// borders mirrored without repeating the edge sample.  One thread per output
// pixel; HBM-bound (the 5 x 5 window is re-read from cache).
#include "gv_internal.h"

namespace gv {

__device__ __forceinline__ int mirror_index(int i, int n) {
    if (n == 1) return 0;
    while (i < 0 || i >= n) i = i < 0 ? -i : 2 * (n - 1) - i;
    return i;
}

__global__ __launch_bounds__(256) void k_pyr_reduce(const float* __restrict__ in, float* __restrict__ out,
                                                    int64_t planes, int H, int W, int Ho, int Wo) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int64_t per = static_cast<int64_t>(Ho) * Wo;
    if (i >= planes * per) return;
    const int64_t p = i / per;
    const int r = static_cast<int>(i - p * per);
    const int y = r / Wo, x = r - y * Wo;
    const float k[5] = {0.0625f, 0.25f, 0.375f, 0.25f, 0.0625f};
    const float* src = in + p * static_cast<int64_t>(H) * W;
    int xs[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) xs[d] = mirror_index(2 * x + d - 2, W);
    float acc = 0.0f;
#pragma unroll
    for (int dy = 0; dy < 5; ++dy) {
        const float* row = src + static_cast<int64_t>(mirror_index(2 * y + dy - 2, H)) * W;
        float h = 0.0f;
#pragma unroll
        for (int dx = 0; dx < 5; ++dx) h += k[dx] * row[xs[dx]];
        acc += k[dy] * h;
    }
    out[i] = acc;
}

}  // namespace gv

using namespace gv;

static bool pyramid_args_ok(int64_t planes, int32_t height, int32_t width, int32_t levels) {
    return planes >= 1 && height >= 1 && width >= 1 && height <= 65536 && width <= 65536 && levels >= 1 &&
           levels <= 16 && planes * static_cast<int64_t>(height) * width <= (int64_t(1) << 40);
}

extern "C" gv_status gv_pyramid_floats(int64_t planes, int32_t height, int32_t width, int32_t levels,
                                       int64_t* out_count) {
    if (!out_count || !pyramid_args_ok(planes, height, width, levels)) return GV_ERR_INVALID_ARG;
    int64_t total = 0;
    int h = height, w = width;
    for (int l = 1; l < levels; ++l) {
        h = (h + 1) / 2;
        w = (w + 1) / 2;
        total += planes * static_cast<int64_t>(h) * w;
    }
    *out_count = total;
    return GV_OK;
}

extern "C" gv_status gv_gaussian_pyramid(const float* images, int64_t planes, int32_t height, int32_t width,
                                         int32_t levels, float* out, void* stream) {
    if (!images || !pyramid_args_ok(planes, height, width, levels) || (levels > 1 && !out))
        return GV_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const float* src = images;
    float* dst = out;
    int h = height, w = width;
    for (int l = 1; l < levels; ++l) {
        const int ho = (h + 1) / 2, wo = (w + 1) / 2;
        const int64_t n = planes * static_cast<int64_t>(ho) * wo;
        hipLaunchKernelGGL(k_pyr_reduce, dim3(static_cast<uint32_t>((n + 255) / 256)), dim3(256), 0, st, src, dst,
                           planes, h, w, ho, wo);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return GV_ERR_HIP;
        src = dst;
        dst += n;
        h = ho;
        w = wo;
    }
    return GV_OK;
}
