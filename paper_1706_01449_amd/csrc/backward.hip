// Backward of a loss on the top-K scores with the top-K indices held fixed
// (not part of the paper).  S[u,k] = U[u] . I[idx[u,k]], G = dL/dS:
//   dU[u] = sum_k G[u,k] I[idx[u,k]]        gather, summed in k order (deterministic)
//   dI[i] += G[u,k] U[u]  for idx[u,k] = i  float32 atomic scatter-add
// One wave per user; lane j handles factor j (and j + 64, ...), so each row
// read of I and each row of atomics into dI is one coalesced 256-byte access.
#include "device_common.h"
#include "internal.h"

namespace mips {

__global__ void __launch_bounds__(256) topk_backward_kernel(const float* __restrict__ U,
                                                            const float* __restrict__ I,
                                                            int64_t n_u, int64_t n_i, int f, int K,
                                                            const int32_t* __restrict__ idx,
                                                            const float* __restrict__ G,
                                                            float* __restrict__ dU, float* dI) {
    const int lane = threadIdx.x & 63;
    const int64_t u = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    if (u >= n_u) return;
    const int32_t* ix = idx + u * K;
    const float* g = G + u * K;
    for (int j0 = 0; j0 < f; j0 += kWave) {
        const int j = j0 + lane;
        const bool on = j < f;
        const float uj = on ? U[u * f + j] : 0.0f;
        float acc = 0.0f;
        for (int k = 0; k < K; ++k) {
            const int64_t i = ix[k];
            const float gk = g[k];
            if (i < 0 || i >= n_i) continue;        // out-of-range entries are skipped
            if (on) {
                acc = fmaf(gk, I[i * f + j], acc);
                atomicAdd(&dI[i * f + j], gk * uj);
            }
        }
        if (on) dU[u * f + j] = acc;
    }
}

hipError_t launch_backward(const float* U, const float* I, int64_t n_u, int64_t n_i, int f, int K,
                           const int32_t* idx, const float* G, float* dU, float* dI, hipStream_t s) {
    hipError_t e = launch_zero(dI, (size_t)n_i * f * sizeof(float), s);
    if (e != hipSuccess) return e;
    const unsigned blocks = (unsigned)((n_u + 3) / 4);
    topk_backward_kernel<<<dim3(blocks), dim3(256), 0, s>>>(U, I, n_u, n_i, f, K, idx, G, dU, dI);
    return hipGetLastError();
}

}  // namespace mips
