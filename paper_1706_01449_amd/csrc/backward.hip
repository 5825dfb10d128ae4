// Backward of a loss on the top-K scores with the top-K indices held fixed
// (not part of the paper).  S[u,k] = U[u] . I[idx[u,k]], G = dL/dS:
//   dU[u] = sum_k G[u,k] I[idx[u,k]]        gather, summed in k order (deterministic)
//   dI[i] = sum of G[u,k] U[u] over the pairs with idx[u,k] = i
// dU: one wave per user; lane j handles factor j (and j + 64, ...), so each
// row read of I is one coalesced 256-byte access.
// dI: the (u, k) pairs are grouped by item (counts, offsets, scatter), then
// one wave sums 64 consecutive grouped pairs, adding one partial row to dI
// per item it meets; far fewer float32 atomics than one row per pair, which
// bound a direct scatter-add.  Pair counts of 2^31 or more use the direct
// scatter-add.
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

// dU only (the gather of topk_backward_kernel without the scatter).
__global__ void __launch_bounds__(256) topk_dU_kernel(const float* __restrict__ I, int64_t n_u,
                                                      int64_t n_i, int f, int K,
                                                      const int32_t* __restrict__ idx,
                                                      const float* __restrict__ G,
                                                      float* __restrict__ dU) {
    const int lane = threadIdx.x & 63;
    const int64_t u = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    if (u >= n_u) return;
    const int32_t* ix = idx + u * K;
    const float* g = G + u * K;
    for (int j0 = 0; j0 < f; j0 += kWave) {
        const int j = j0 + lane;
        const bool on = j < f;
        float acc = 0.0f;
        for (int k = 0; k < K; ++k) {
            const int64_t i = ix[k];
            if (i < 0 || i >= n_i) continue;        // out-of-range entries are skipped
            if (on) acc = fmaf(g[k], I[i * f + j], acc);
        }
        if (on) dU[u * f + j] = acc;
    }
}

// Pairs are grouped by item in workgroups of 1024 threads over 4096
// consecutive pairs: each workgroup first counts its pairs per item in an LDS
// hash table (linear probing), so a popular item costs one global atomic per
// workgroup instead of one per pair.  A pair whose probe sequence runs past
// kProbe slots falls back to a global atomic of its own.
constexpr int kGrpPairs = 4096, kGrpSlots = 8192, kProbe = 64;

struct GrpTable {
    int key[kGrpSlots];
    unsigned int cnt[kGrpSlots];
    unsigned int base[kGrpSlots];
};

__device__ __forceinline__ void grp_init(GrpTable& T) {
    for (int s = threadIdx.x; s < kGrpSlots; s += 1024) { T.key[s] = -1; T.cnt[s] = 0u; }
    __syncthreads();
}

// Slot of `item` in T (-1: table too crowded) and the pair's rank among the
// workgroup's pairs of that item.
__device__ __forceinline__ int grp_insert(GrpTable& T, int item, unsigned int* rank) {
    int h = (int)(((unsigned int)item * 2654435761u) >> 19);   // 13 bits
    for (int t = 0; t < kProbe; ++t) {
        const int k = atomicCAS(&T.key[h], -1, item);
        if (k == -1 || k == item) {
            *rank = atomicAdd(&T.cnt[h], 1u);
            return h;
        }
        h = (h + 1) & (kGrpSlots - 1);
    }
    return -1;
}

__global__ void __launch_bounds__(1024) bwd_count_kernel(const int32_t* __restrict__ idx, int64_t npairs,
                                                         int64_t n_i, unsigned int* cnt) {
    __shared__ GrpTable T;
    grp_init(T);
    const int64_t base = blockIdx.x * (int64_t)kGrpPairs;
    for (int q = 0; q < kGrpPairs / 1024; ++q) {
        const int64_t p = base + q * 1024 + threadIdx.x;
        if (p >= npairs) continue;
        const int64_t i = idx[p];
        if (i < 0 || i >= n_i) continue;
        unsigned int r;
        if (grp_insert(T, (int)i, &r) < 0) atomicAdd(&cnt[i], 1u);
    }
    __syncthreads();
    for (int s = threadIdx.x; s < kGrpSlots; s += 1024)
        if (T.key[s] >= 0) atomicAdd(&cnt[T.key[s]], T.cnt[s]);
}

// Exclusive prefix sum of cnt[0 .. n) into off and cur in three steps over
// blocks of 1024 counts: block sums, a scan of the block sums (one
// workgroup), then each block's scan plus its offset; total[0] = sum.
__device__ __forceinline__ unsigned int block_incl_scan(unsigned int v, unsigned int* sh,
                                                        unsigned int* tot) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const unsigned int x = t >= d ? sh[t - d] : 0u;
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    const unsigned int r = sh[t];
    *tot = sh[1023];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(1024) bwd_block_sum_kernel(const unsigned int* cnt, int64_t n,
                                                             unsigned int* bsum) {
    __shared__ unsigned int sh[1024];
    const int64_t i = blockIdx.x * (int64_t)1024 + threadIdx.x;
    unsigned int tot;
    block_incl_scan(i < n ? cnt[i] : 0u, sh, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) bwd_bsum_scan_kernel(unsigned int* bsum, int64_t nb,
                                                             unsigned int* total) {
    __shared__ unsigned int sh[1024];
    unsigned int carry = 0u;
    for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
        const int64_t b = b0 + threadIdx.x;
        const unsigned int v = b < nb ? bsum[b] : 0u;
        unsigned int tot;
        const unsigned int s = block_incl_scan(v, sh, &tot);
        if (b < nb) bsum[b] = carry + s - v;   // exclusive
        carry += tot;
    }
    if (threadIdx.x == 0) total[0] = carry;
}

__global__ void __launch_bounds__(1024) bwd_offsets_kernel(const unsigned int* cnt, int64_t n,
                                                           const unsigned int* bsum,
                                                           unsigned int* off, unsigned int* cur) {
    __shared__ unsigned int sh[1024];
    const int64_t i = blockIdx.x * (int64_t)1024 + threadIdx.x;
    const unsigned int v = i < n ? cnt[i] : 0u;
    unsigned int tot;
    const unsigned int s = block_incl_scan(v, sh, &tot);
    if (i < n) {
        off[i] = bsum[blockIdx.x] + s - v;
        cur[i] = off[i];
    }
}

// Pair indices grouped by item: each workgroup reserves one range per item
// it holds (one global atomic per item), then places its pairs by their
// LDS ranks.
__global__ void __launch_bounds__(1024) bwd_scatter_kernel(const int32_t* __restrict__ idx,
                                                           int64_t npairs, int64_t n_i,
                                                           unsigned int* cur, int* grouped) {
    __shared__ GrpTable T;
    grp_init(T);
    const int64_t base = blockIdx.x * (int64_t)kGrpPairs;
    int slot[kGrpPairs / 1024];
    unsigned int rank[kGrpPairs / 1024];
    for (int q = 0; q < kGrpPairs / 1024; ++q) {
        const int64_t p = base + q * 1024 + threadIdx.x;
        slot[q] = -2;                           // -2: no pair; -1: placed directly
        if (p >= npairs) continue;
        const int64_t i = idx[p];
        if (i < 0 || i >= n_i) continue;
        slot[q] = grp_insert(T, (int)i, &rank[q]);
        if (slot[q] < 0) grouped[atomicAdd(&cur[i], 1u)] = (int)p;
    }
    __syncthreads();
    for (int s = threadIdx.x; s < kGrpSlots; s += 1024)
        if (T.key[s] >= 0) T.base[s] = atomicAdd(&cur[T.key[s]], T.cnt[s]);
    __syncthreads();
    for (int q = 0; q < kGrpPairs / 1024; ++q) {
        const int64_t p = base + q * 1024 + threadIdx.x;
        if (slot[q] >= 0) grouped[T.base[slot[q]] + rank[q]] = (int)p;
    }
}

// Wave w sums grouped pairs [64 w, 64 w + 64): lane j accumulates factor j
// of G[p] U[p / K] while the item stays the same, and adds the partial row
// to dI when the item changes or the block ends.
__global__ void __launch_bounds__(256) bwd_dI_kernel(const float* __restrict__ U, int f, int K,
                                                     const int32_t* __restrict__ idx,
                                                     const float* __restrict__ G,
                                                     const int* __restrict__ grouped,
                                                     const unsigned int* total, float* dI) {
    const int lane = threadIdx.x & 63;
    const int64_t w = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t nt = total[0];
    const int64_t base = w * 64;
    if (base >= nt) return;
    const int m = (int)(nt - base < 64 ? nt - base : 64);
    // lane e holds entry e of the block: pair, item, gradient, user
    const int p = lane < m ? grouped[base + lane] : 0;
    const int item = lane < m ? idx[p] : -1;
    const float gp = lane < m ? G[p] : 0.0f;
    const int64_t up = (int64_t)(p / K);
    for (int j0 = 0; j0 < f; j0 += kWave) {
        const int j = j0 + lane;
        const bool on = j < f;
        float acc = 0.0f;
        int cur = __builtin_amdgcn_readlane(item, 0);
        for (int e = 0; e < m; e += 8) {
            float v[8], g[8];
            int it[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int ee = e + q < m ? e + q : m - 1;
                it[q] = __builtin_amdgcn_readlane(item, ee);
                g[q] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(gp), ee));
                const int64_t uu = __builtin_amdgcn_readlane((int)up, ee);
                v[q] = on ? U[uu * f + j] : 0.0f;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (e + q >= m) break;
                if (it[q] != cur) {
                    if (on) atomicAdd(&dI[(int64_t)cur * f + j], acc);
                    acc = 0.0f;
                    cur = it[q];
                }
                acc = fmaf(g[q], v[q], acc);
            }
        }
        if (on) atomicAdd(&dI[(int64_t)cur * f + j], acc);
    }
}

// Scratch of the grouped dI path: counts, offsets, cursors, total, block
// sums, grouped pairs (0 when the direct scatter-add is taken).
static size_t al256b(size_t x) { return (x + 255) & ~(size_t)255; }

size_t backward_scratch_bytes(int64_t n_i, int64_t npairs) {
    if (npairs >= ((int64_t)1 << 31)) return 0;
    const int64_t nblk = (n_i + 1023) / 1024;
    return 3 * al256b((size_t)n_i * 4) + 256 + al256b((size_t)nblk * 4) + (size_t)npairs * 4;
}

hipError_t launch_backward(const float* U, const float* I, int64_t n_u, int64_t n_i, int f, int K,
                           const int32_t* idx, const float* G, float* dU, float* dI,
                           void* scratch_in, hipStream_t s) {
    hipError_t e = launch_zero(dI, (size_t)n_i * f * sizeof(float), s);
    if (e != hipSuccess) return e;
    const unsigned blocks = (unsigned)((n_u + 3) / 4);
    const int64_t npairs = n_u * (int64_t)K;
    if (npairs >= ((int64_t)1 << 31)) {
        topk_backward_kernel<<<dim3(blocks), dim3(256), 0, s>>>(U, I, n_u, n_i, f, K, idx, G, dU, dI);
        return hipGetLastError();
    }
    // caller's scratch, else stream-ordered scratch
    unsigned char* scratch = (unsigned char*)scratch_in;
    const size_t nb = (size_t)n_i * 4, ab = al256b(nb);
    const int64_t nblk = (n_i + 1023) / 1024;
    const size_t bb = al256b((size_t)nblk * 4);
    if (!scratch &&
        (e = hipMallocAsync((void**)&scratch, backward_scratch_bytes(n_i, npairs), s)) != hipSuccess)
        return e;
    unsigned int* cnt = (unsigned int*)scratch;
    unsigned int* off = (unsigned int*)(scratch + ab);
    unsigned int* cur = (unsigned int*)(scratch + 2 * ab);
    unsigned int* total = (unsigned int*)(scratch + 3 * ab);
    unsigned int* bsum = (unsigned int*)(scratch + 3 * ab + 256);
    int* grouped = (int*)(scratch + 3 * ab + 256 + bb);
    const unsigned pb = (unsigned)((npairs + kGrpPairs - 1) / kGrpPairs);
    if ((e = launch_zero(cnt, nb, s)) == hipSuccess) {
        bwd_count_kernel<<<pb, 1024, 0, s>>>(idx, npairs, n_i, cnt);
        bwd_block_sum_kernel<<<(unsigned)nblk, 1024, 0, s>>>(cnt, n_i, bsum);
        bwd_bsum_scan_kernel<<<1, 1024, 0, s>>>(bsum, nblk, total);
        bwd_offsets_kernel<<<(unsigned)nblk, 1024, 0, s>>>(cnt, n_i, bsum, off, cur);
        bwd_scatter_kernel<<<pb, 1024, 0, s>>>(idx, npairs, n_i, cur, grouped);
        topk_dU_kernel<<<dim3(blocks), dim3(256), 0, s>>>(I, n_u, n_i, f, K, idx, G, dU);
        const int64_t waves = (npairs + 63) / 64;
        bwd_dI_kernel<<<(unsigned)((waves + 3) / 4), 256, 0, s>>>(U, f, K, idx, G, grouped, total, dI);
        e = hipGetLastError();
    }
    if (scratch_in) return e;
    const hipError_t e2 = hipFreeAsync(scratch, s);
    return e != hipSuccess ? e : e2;
}

}  // namespace mips
