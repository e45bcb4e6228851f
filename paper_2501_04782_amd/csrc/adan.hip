// Fused Adan step (the optimizer of Sec. 4.1) over several FP32 tensors in
// one launch: one element per thread, reading the parameter, its gradient and
// the four state words (m, v, n, previous gradient) and writing all but the
// gradient back.  HBM-bound: per element 24 B read (parameter, gradient,
// m, v, n, g_prev) and 20 B written (parameter, m, v, n, g_prev).
#include <cstring>

#include "gv_internal.h"

namespace gv {

struct AdanTensors {
    float* params[GV_ADAN_MAX_TENSORS];
    const float* grads[GV_ADAN_MAX_TENSORS];
    float* states[GV_ADAN_MAX_TENSORS];      // [4][count]: m, v, n, g_prev
    int64_t counts[GV_ADAN_MAX_TENSORS];
    int64_t offsets[GV_ADAN_MAX_TENSORS + 1];  // prefix sums of counts
    int n;
};

__global__ __launch_bounds__(256) void k_adan(AdanTensors T, gv_adan_params hp) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= T.offsets[T.n]) return;
    int t = 0;
    while (t + 1 < T.n && i >= T.offsets[t + 1]) ++t;
    const int64_t j = i - T.offsets[t];
    const int64_t c = T.counts[t];
    float* st = T.states[t];
    const float g = T.grads[t][j];
    float m, v, nn;
    if (hp.step == 0) {  // m0 = g0, v0 = 0, n0 = g0^2
        m = g;
        v = 0.0f;
        nn = g * g;
    } else {
        const float gp = st[3 * c + j];
        const float diff = g - gp;
        m = (1.0f - hp.beta1) * st[j] + hp.beta1 * g;
        v = hp.step == 1 ? diff : (1.0f - hp.beta2) * st[c + j] + hp.beta2 * diff;  // v1 = g1 - g0
        const float w = g + (1.0f - hp.beta2) * diff;
        nn = (1.0f - hp.beta3) * st[2 * c + j] + hp.beta3 * w * w;
    }
    st[j] = m;
    st[c + j] = v;
    st[2 * c + j] = nn;
    st[3 * c + j] = g;
    const float eta = hp.lr / sqrtf(nn + hp.eps);
    float* p = T.params[t] + j;
    *p = (*p - eta * (m + (1.0f - hp.beta2) * v)) / (1.0f + hp.weight_decay * hp.lr);
}

}  // namespace gv

using namespace gv;

extern "C" gv_status gv_adan_step(int32_t n_tensors, float* const* params, const float* const* grads,
                                  float* const* states, const int64_t* counts, const gv_adan_params* hp,
                                  void* stream) {
    if (n_tensors < 1 || n_tensors > GV_ADAN_MAX_TENSORS || !params || !grads || !states || !counts || !hp)
        return GV_ERR_INVALID_ARG;
    if (hp->step < 0 || !(hp->lr >= 0.0f) || !(hp->eps > 0.0f) || !(hp->weight_decay >= 0.0f)) return GV_ERR_INVALID_ARG;
    const float b[3] = {hp->beta1, hp->beta2, hp->beta3};
    for (float x : b)
        if (!(x >= 0.0f && x <= 1.0f)) return GV_ERR_INVALID_ARG;
    AdanTensors T;
    memset(&T, 0, sizeof(T));
    T.n = n_tensors;
    T.offsets[0] = 0;
    for (int t = 0; t < n_tensors; ++t) {
        if (counts[t] < 0 || (counts[t] > 0 && (!params[t] || !grads[t] || !states[t]))) return GV_ERR_INVALID_ARG;
        T.params[t] = params[t];
        T.grads[t] = grads[t];
        T.states[t] = states[t];
        T.counts[t] = counts[t];
        T.offsets[t + 1] = T.offsets[t] + counts[t];
    }
    const int64_t total = T.offsets[n_tensors];
    if (total == 0) return GV_OK;
    if (total > (int64_t(1) << 40)) return GV_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_adan, dim3(static_cast<uint32_t>((total + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), T, *hp);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? GV_OK : GV_ERR_HIP;
}
