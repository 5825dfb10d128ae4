// Maximus (paper Section III, Algorithm 1) on the GPU: index construction
// (k-means over users, per-cluster angle bound theta_b, every item ordered by
// the bound of Eq. (appx_bound), users grouped by cluster) and the query: the
// screen kernel's blocked walk down each cluster's list with per-user early
// termination, followed by the shared certification and fallback.
//
// Determinism: k-means sums are accumulated in 64-bit fixed point (integer
// adds are order independent), theta_b uses an atomic max, and the lists are
// ordered by a stable radix sort on (bound desc, item asc), so the index is
// identical from run to run.  Exactness never depends on the clustering.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/mips.h"
#include "device_common.h"
#include "internal.h"

namespace mips {

// ---------------------------------------------------------------------------
// Small helpers.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) absmax_kernel(const float* X, int64_t n, unsigned int* out) {
    __shared__ float wm[4];
    float m = 0.0f;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(X[i]));
    for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)   // one atomic per workgroup
        atomicMax(out, __float_as_uint(fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]))));
}

// 2^e with n * max|x| * 2^e < 2^61, so fixed-point sums of n values fit in int64.
__device__ __forceinline__ double fixed_scale(int64_t n, unsigned int absmax_bits) {
    const double m = (double)__uint_as_float(absmax_bits);
    if (!(m > 0.0)) return 1.0;
    const int e = 60 - (int)ceil(log2((double)n)) - (int)ceil(log2(m));
    return ldexp(1.0, e);
}

__global__ void gather_rows_kernel(const float* U, int f, const int* idx, int C, double* cent) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)C * f) return;
    const int c = (int)(t / f), j = (int)(t - (int64_t)c * f);
    cent[t] = (double)U[(int64_t)idx[c] * f + j];
}

__global__ void cent_prep_kernel(const double* cent, int C, int f, float* cent32, float* cnorm2) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    float s = 0.0f;
    for (int j = 0; j < f; ++j) {
        const float x = (float)cent[(int64_t)c * f + j];
        cent32[(int64_t)c * f + j] = x;
        s = fmaf(x, x, s);
    }
    cnorm2[c] = s;
}

// Nearest centroid by Euclidean distance ||u||^2 - 2 u.c + ||c||^2 (the
// ||u||^2 term is common); ties go to the lower centroid index.  One thread
// per user; centroids staged through LDS 64 at a time, factors 32 at a time.
__global__ void __launch_bounds__(256) assign_kernel(const float* __restrict__ U, int64_t n_u,
                                                     int f, const float* __restrict__ cent32,
                                                     const float* __restrict__ cnorm2, int C,
                                                     int* __restrict__ assign) {
    extern __shared__ float sc[];                 // [64][f]
    const int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool on = u < n_u;
    const float* urow = U + (on ? u : 0) * f;
    float best = __builtin_inff();
    int bi = 0;
    for (int c0 = 0; c0 < C; c0 += 64) {
        const int nc = min(64, C - c0);
        __syncthreads();
        for (int t = threadIdx.x; t < nc * f; t += blockDim.x) sc[t] = cent32[(int64_t)c0 * f + t];
        __syncthreads();
        float part[64];
#pragma unroll
        for (int q = 0; q < 64; ++q) part[q] = 0.0f;
        for (int j0 = 0; j0 < f; j0 += 32) {
            float x[32];
#pragma unroll
            for (int q = 0; q < 32; ++q) x[q] = (j0 + q < f) ? urow[j0 + q] : 0.0f;
#pragma unroll
            for (int c = 0; c < 64; ++c) {
                if (c < nc) {
                    float acc = part[c];
#pragma unroll
                    for (int q = 0; q < 32; ++q)
                        if (j0 + q < f) acc = fmaf(x[q], sc[c * f + j0 + q], acc);
                    part[c] = acc;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < 64; ++c) {
            if (c < nc) {
                const float d = fmaf(-2.0f, part[c], cnorm2[c0 + c]);
                if (d < best) { best = d; bi = c0 + c; }
            }
        }
    }
    if (on) assign[u] = bi;
}

// Fixed-point per-cluster sums and counts (order independent).  When the
// C x f sums fit in LDS a workgroup first aggregates its 256 users there, so
// each (cluster, factor) receives one global atomic per workgroup.
__global__ void __launch_bounds__(256) kmeans_sum_kernel(const float* __restrict__ U, int64_t n_u,
                                                         int f, const int* __restrict__ assign,
                                                         const unsigned int* absmax_bits,
                                                         unsigned long long* sums,
                                                         unsigned int* counts, int C) {
    __shared__ unsigned long long ls[4096];
    __shared__ unsigned int lc[512];
    const double scale = fixed_scale(n_u, *absmax_bits);
    const int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool local = (int64_t)C * f <= 4096 && C <= 512;
    if (local) {
        for (int t = threadIdx.x; t < C * f; t += blockDim.x) ls[t] = 0ull;
        for (int t = threadIdx.x; t < C; t += blockDim.x) lc[t] = 0u;
        __syncthreads();
    }
    if (u < n_u) {
        const int c = assign[u];
        const float* row = U + u * f;
        if (local) {
            atomicAdd(&lc[c], 1u);
            for (int j = 0; j < f; ++j)
                atomicAdd(&ls[c * f + j], (unsigned long long)llrint((double)row[j] * scale));
        } else {
            atomicAdd(&counts[c], 1u);
            for (int j = 0; j < f; ++j)
                atomicAdd(&sums[(int64_t)c * f + j], (unsigned long long)llrint((double)row[j] * scale));
        }
    }
    if (local) {
        __syncthreads();
        for (int t = threadIdx.x; t < C * f; t += blockDim.x)
            if (ls[t]) atomicAdd(&sums[t], ls[t]);
        for (int t = threadIdx.x; t < C; t += blockDim.x)
            if (lc[t]) atomicAdd(&counts[t], lc[t]);
    }
}

__global__ void kmeans_update_kernel(double* cent, int C, int f, const unsigned long long* sums,
                                     const unsigned int* counts, const unsigned int* absmax_bits,
                                     int64_t n_u) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)C * f) return;
    const int c = (int)(t / f);
    const unsigned int n = counts[c];
    if (n == 0) return;   // an empty cluster keeps its centroid
    const double scale = fixed_scale(n_u, *absmax_bits);
    cent[t] = (double)(long long)sums[t] / scale / (double)n;
}

// Kahan's stable angle between a and b (float64): 2 atan2(|a^ - b^|, |a^ + b^|).
__device__ __forceinline__ double stable_angle(const float* a, const double* b, int f, double na,
                                               double nb) {
    double d = 0.0, s = 0.0;
    for (int j = 0; j < f; ++j) {
        const double x = (double)a[j] / na, y = b[j] / nb;
        d += (x - y) * (x - y);
        s += (x + y) * (x + y);
    }
    return 2.0 * atan2(sqrt(d), sqrt(s));
}

// theta_b[c] = max over users of cluster c of the user-centroid angle (zero
// users left out).  Non-negative doubles order like their bit patterns.
// Workgroups stride over many users and keep the per-cluster maxima in LDS,
// then merge them with one atomic per cluster and workgroup.
__global__ void __launch_bounds__(256) theta_kernel(const float* __restrict__ U, int64_t n_u, int f,
                                                    const int* __restrict__ assign,
                                                    const double* __restrict__ cent,
                                                    const double* __restrict__ cnorm, int C,
                                                    unsigned long long* theta_bits) {
    __shared__ unsigned long long lt[4096];
    for (int c = threadIdx.x; c < C; c += blockDim.x) lt[c] = 0ull;
    __syncthreads();
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n_u;
         u += (int64_t)gridDim.x * blockDim.x) {
        const float* row = U + u * f;
        double n2 = 0.0;
        for (int j = 0; j < f; ++j) n2 += (double)row[j] * (double)row[j];
        const int c = assign[u];
        const double nc = cnorm[c];
        if (!(n2 > 0.0) || !(nc > 0.0)) continue;
        const double th = stable_angle(row, cent + (int64_t)c * f, f, sqrt(n2), nc);
        atomicMax(&lt[c], (unsigned long long)__double_as_longlong(th));
    }
    __syncthreads();
    for (int c = threadIdx.x; c < C; c += blockDim.x)
        if (lt[c]) atomicMax(&theta_bits[c], lt[c]);
}

__global__ void cnorm_kernel(const double* cent, int C, int f, double* cnorm) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    double s = 0.0;
    for (int j = 0; j < f; ++j) s += cent[(int64_t)c * f + j] * cent[(int64_t)c * f + j];
    cnorm[c] = sqrt(s);
}

// A zero centroid bounds nothing by angle: theta_b = pi (bound = ||i||).
__global__ void theta_fix_kernel(const double* cnorm, int C, double* theta) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    if (!(cnorm[c] > 0.0)) theta[c] = 3.14159265358979323846;
}

// Float bits -> unsigned key ordered like the floats, then complemented so
// that an ascending sort gives descending bounds.
__device__ __forceinline__ uint32_t desc_key(float x) {
    const uint32_t b = __float_as_uint(x);
    const uint32_t asc = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    return ~asc;
}
__device__ __forceinline__ float key_to_float(uint32_t k) {
    const uint32_t asc = ~k;
    const uint32_t b = (asc & 0x80000000u) ? (asc & 0x7fffffffu) : ~asc;
    return __uint_as_float(b);
}

// Bound of Eq. (appx_bound) for every (cluster, item) in float64:
// ||i|| cos(max(theta_ic - theta_b, 0)), widened by 2^-40 ||i|| for the
// float64 evaluation of the angles and rounded up to float32.
__global__ void bound_kernel(const float* __restrict__ I, int64_t n_i, int f,
                             const double* __restrict__ cent, const double* __restrict__ cnorm,
                             const double* __restrict__ theta, int C, uint32_t* keys, int* vals) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)C * n_i) return;
    const int c = (int)(t / n_i);
    const int64_t i = t - (int64_t)c * n_i;
    const float* row = I + i * f;
    double n2 = 0.0;
    for (int j = 0; j < f; ++j) n2 += (double)row[j] * (double)row[j];
    const double ni = sqrt(n2);
    double b;
    if (!(ni > 0.0)) {
        b = 0.0;
    } else if (!(cnorm[c] > 0.0)) {
        b = ni;
    } else {
        const double th = stable_angle(row, cent + (int64_t)c * f, f, ni, cnorm[c]);
        b = ni * cos(fmax(th - theta[c], 0.0));
    }
    const float b32 = round_up_f32(b + 0x1p-40 * ni * (1.0 + 0x1p-20));
    keys[t] = desc_key(b32);
    vals[t] = (int)i;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort pass (8-bit digit at `shift`) over independent
// segments of `len` (key, value) pairs; one 1024-thread workgroup per segment.
// Elements are ranked chunk by chunk in their current order, so equal digits
// keep their relative order.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) radix_pass_kernel(const uint32_t* __restrict__ kin,
                                                          const int* __restrict__ vin,
                                                          uint32_t* __restrict__ kout,
                                                          int* __restrict__ vout, int64_t len,
                                                          int shift) {
    __shared__ unsigned int run[256];          // next output slot of each digit
    __shared__ unsigned int wcnt[16][256];     // per-wave digit counts of the current chunk
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t base = (int64_t)blockIdx.x * len;
    // histogram -> exclusive scan
    for (int d = t; d < 16 * 256; d += 1024) (&wcnt[0][0])[d] = 0u;
    if (t < 256) run[t] = 0u;
    __syncthreads();
    for (int64_t i = t; i < len; i += 1024) atomicAdd(&run[(kin[base + i] >> shift) & 255u], 1u);
    __syncthreads();
    if (t == 0) {
        unsigned int acc = 0u;
        for (int d = 0; d < 256; ++d) { const unsigned int c = run[d]; run[d] = acc; acc += c; }
    }
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int64_t c0 = 0; c0 < len; c0 += 1024) {
        const int64_t i = c0 + t;
        const bool on = i < len;
        const uint32_t k = on ? kin[base + i] : 0u;
        const int v = on ? vin[base + i] : 0;
        const uint32_t d = (k >> shift) & 255u;
        // lanes of this wave holding the same digit
        uint64_t match = __builtin_amdgcn_ballot_w64(on);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t bb = __builtin_amdgcn_ballot_w64(((d >> bit) & 1u) != 0u);
            match &= ((d >> bit) & 1u) ? bb : ~bb;
        }
        const unsigned int rank_w = __builtin_popcountll(match & lt);
        if (on && rank_w == 0) wcnt[wv][d] = __builtin_popcountll(match);
        __syncthreads();
        if (on) {
            unsigned int pos = run[d] + rank_w;
            for (int q = 0; q < wv; ++q) pos += wcnt[q][d];
            kout[base + pos] = k;
            vout[base + pos] = v;
        }
        __syncthreads();
        if (t < 256) {
            unsigned int add = 0u;
            for (int q = 0; q < 16; ++q) { add += wcnt[q][t]; wcnt[q][t] = 0u; }
            run[t] += add;
        }
        __syncthreads();
    }
}

// Sorted (key, item) pairs -> padded walk lists and rounded-up bounds.
__global__ void lists_kernel(const uint32_t* keys, const int* vals, int64_t n_i, int64_t n_i_pad,
                             int C, int* lists, float* lbound) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)C * n_i_pad) return;
    const int c = (int)(t / n_i_pad);
    const int64_t p = t - (int64_t)c * n_i_pad;
    if (p < n_i) {
        lists[t] = vals[(int64_t)c * n_i + p];
        lbound[t] = key_to_float(keys[(int64_t)c * n_i + p]);
    } else {
        lists[t] = -1;
        lbound[t] = -__builtin_inff();
    }
}

// Per (cluster, tile of 32 list entries): max C and max G of its items.
__global__ void cblockmax_kernel(const int* lists, int64_t n_i_pad, int64_t n_blk, int C,
                                 const float* Corig, const float* Gorig, float2* out) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)C * n_blk) return;
    const int c = (int)(t / n_blk);
    const int64_t b = t - (int64_t)c * n_blk;
    float cm = 0.0f, gm = 0.0f;
    for (int q = 0; q < kTile; ++q) {
        const int item = lists[(int64_t)c * n_i_pad + b * kTile + q];
        if (item >= 0) {
            cm = fmaxf(cm, Corig[item]);
            gm = fmaxf(gm, Gorig[item]);
        }
    }
    out[t] = make_float2(cm, gm);
}

// ---------------------------------------------------------------------------
// Users grouped by cluster, in ascending user order inside each cluster (a
// stable counting sort on the cluster id, C <= 4096): per-chunk counts,
// per-cluster running offsets over the chunks, then a scatter that walks each
// chunk in order, 64 users at a time, ranking equal clusters within the wave.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) group_count_kernel(const int* assign, int64_t n, int64_t chunk,
                                                          int C, unsigned int* ccounts) {
    __shared__ unsigned int lc[4096];
    for (int c = threadIdx.x; c < C; c += blockDim.x) lc[c] = 0u;
    __syncthreads();
    const int64_t lo = blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    for (int64_t u = lo + threadIdx.x; u < hi; u += blockDim.x) atomicAdd(&lc[assign[u]], 1u);
    __syncthreads();
    for (int c = threadIdx.x; c < C; c += blockDim.x) ccounts[(int64_t)blockIdx.x * C + c] = lc[c];
}

// offs[k][c] = sum of ccounts[k'][c] over chunks k' < k; hist[c] = total of c
__global__ void group_offsets_kernel(unsigned int* ccounts, int nchunks, int C, unsigned int* hist) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    unsigned int run = 0u;
    for (int k = 0; k < nchunks; ++k) {
        const unsigned int v = ccounts[(int64_t)k * C + c];
        ccounts[(int64_t)k * C + c] = run;
        run += v;
    }
    hist[c] = run;
}

__global__ void __launch_bounds__(64) group_scatter_kernel(const int* assign, int64_t n, int64_t chunk,
                                                           int C, const unsigned int* offs,
                                                           const unsigned int* cstart, int* sorted) {
    __shared__ unsigned int next[4096];
    const int lane = threadIdx.x;
    for (int c = lane; c < C; c += 64) next[c] = cstart[c] + offs[(int64_t)blockIdx.x * C + c];
    __syncthreads();
    const int64_t lo = blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int64_t base = lo; base < hi; base += 64) {
        const int64_t u = base + lane;
        const bool on = u < hi;
        const int key = on ? assign[u] : -1;
        uint64_t left = ballot(on);
        while (left) {
            const int leader = __builtin_ctzll(left);
            const int k = __builtin_amdgcn_readlane(key, leader);
            const uint64_t m = ballot(key == k);
            if (key == k) sorted[next[k] + __builtin_popcountll(m & below)] = (int)u;
            __syncthreads();
            if (lane == leader) next[k] += (unsigned int)__builtin_popcountll(m);
            __syncthreads();
            left &= ~m;
        }
    }
}

// Fixed-point per-cluster sums over users already grouped by cluster:
// workgroup w takes sorted positions [w * 2048, (w + 1) * 2048), thread t
// factor t % f of rows t / f, t / f + 256 / f, ...; a thread adds its partial
// sum to the cluster's global sum only when the cluster changes along its
// rows, so a workgroup issues about f atomics per cluster it touches.
constexpr int kSortedSumRows = 2048;

__global__ void __launch_bounds__(256) kmeans_sum_sorted_kernel(const float* __restrict__ U,
                                                                int64_t n_u, int f,
                                                                const int* __restrict__ sorted,
                                                                const int* __restrict__ assign,
                                                                const unsigned int* absmax_bits,
                                                                unsigned long long* sums) {
    const int per = 256 / f;                 // rows per pass (f <= 256)
    const int r0 = threadIdx.x / f, j = threadIdx.x - r0 * f;
    if (r0 >= per) return;
    const double scale = fixed_scale(n_u, *absmax_bits);
    const int64_t lo = (int64_t)blockIdx.x * kSortedSumRows;
    const int64_t hi = lo + kSortedSumRows < n_u ? lo + kSortedSumRows : n_u;
    long long acc = 0;
    int cur = -1;
    for (int64_t p = lo + r0; p < hi; p += per) {
        const int u = sorted[p];
        const int c = assign[u];
        if (c != cur) {
            if (cur >= 0 && acc) atomicAdd(&sums[(int64_t)cur * f + j], (unsigned long long)acc);
            acc = 0;
            cur = c;
        }
        acc += llrint((double)U[(int64_t)u * f + j] * scale);
    }
    if (cur >= 0 && acc) atomicAdd(&sums[(int64_t)cur * f + j], (unsigned long long)acc);
}

__global__ void copy_counts_kernel(const unsigned int* hist, int C, unsigned int* counts) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < C) counts[c] = hist[c];
}

__global__ void iota_kernel(int* v, int64_t n) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < n) v[t] = (int)t;
}

// Users per cluster.  Each workgroup strides over many users and counts in
// LDS, then adds its non-zero counts (same-address device atomics are slow,
// so one per cluster and workgroup instead of one per user).
__global__ void __launch_bounds__(256) count_kernel(const int* assign, int64_t n, int C,
                                                    unsigned int* counts) {
    __shared__ unsigned int lc[4096];
    for (int c = threadIdx.x; c < C; c += blockDim.x) lc[c] = 0u;
    __syncthreads();
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&lc[assign[t]], 1u);
    __syncthreads();
    for (int c = threadIdx.x; c < C; c += blockDim.x)
        if (lc[c]) atomicAdd(&counts[c], lc[c]);
}

__global__ void set_ctrl_kernel(Ctrl* ctrl, unsigned int c, unsigned int e, unsigned int g) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctrl->cmax_bits = c;
        ctrl->emax_bits = e;
        ctrl->gmax_bits = g;
    }
}

static unsigned int grid_of(int64_t n, int b = 256) { return (unsigned int)((n + b - 1) / b); }

// Users grouped by cluster (ascending user order inside each cluster) into
// `sorted`; ghist[0..C) receives the cluster sizes and ghist[4096 + c] the
// first position of cluster c.  ccounts holds group_chunks(n_u) * C entries.
static int64_t group_chunk(int64_t n_u) { return std::max<int64_t>(4096, (n_u + 1023) / 1024); }
static int group_chunks(int64_t n_u) { return (int)((n_u + group_chunk(n_u) - 1) / group_chunk(n_u)); }

static hipError_t group_users(const int* assign, int64_t n_u, int C, unsigned int* ccounts,
                              unsigned int* ghist, int* sorted, hipStream_t s) {
    const int64_t chunk = group_chunk(n_u);
    const int nchunks = group_chunks(n_u);
    hipError_t e = launch_zero(ghist, (size_t)2 * kBuckets * sizeof(unsigned int), s);
    if (e != hipSuccess) return e;
    group_count_kernel<<<nchunks, 256, 0, s>>>(assign, n_u, chunk, C, ccounts);
    group_offsets_kernel<<<grid_of(C), 256, 0, s>>>(ccounts, nchunks, C, ghist);
    if ((e = launch_scan4096(ghist, s)) != hipSuccess) return e;
    group_scatter_kernel<<<nchunks, 64, 0, s>>>(assign, n_u, chunk, C, ccounts, ghist + kBuckets, sorted);
    return hipGetLastError();
}

}  // namespace mips

// ---------------------------------------------------------------------------
// The index (host side).
// ---------------------------------------------------------------------------
using namespace mips;

struct mips_maximus_index {
    int device = 0;
    int64_t n_u = 0, n_i = 0, n_blk = 0, n_i_pad = 0;
    int f = 0, C = 0, shared_blocks = 1;
    float* U = nullptr;
    float* I = nullptr;
    double* cent = nullptr;
    double* theta = nullptr;
    float* cent32 = nullptr;      // float32 centroids and their squared norms (assignment)
    float* cnorm2 = nullptr;
    double* cnorm = nullptr;      // float64 centroid norms (angles)
    int* assign = nullptr;
    int* sorted_users = nullptr;
    int* lists = nullptr;
    float* lbound = nullptr;
    // per screen precision (fp32, bf16, fp8)
    void* qrow[3] = {nullptr, nullptr, nullptr};
    float* Corig[3] = {nullptr, nullptr, nullptr};
    float* Gorig[3] = {nullptr, nullptr, nullptr};
    int* kexp = nullptr;
    float2* cblockmax[3] = {nullptr, nullptr, nullptr};
    unsigned int maxbits[3][3] = {};
    Ctrl* prep_ctrl = nullptr;            // device copies of maxbits, one Ctrl per precision
    // walk tiles for 1, 2 and 4 user blocks per wave
    int4* tiles[3] = {nullptr, nullptr, nullptr};
    int64_t ntiles[3] = {0, 0, 0};
    std::vector<void*> allocs;
    char* arena = nullptr;                // free space of the current chunk
    size_t arena_left = 0;
};

namespace {

int ub_slot(int UB) { return UB == 1 ? 0 : (UB == 2 ? 1 : 2); }

// Device memory of the index comes from a few chunks of kIndexChunk bytes
// (one hipMalloc and one hipFree each), carved into 256-byte aligned pieces;
// a piece of at least a chunk gets an allocation of its own.
constexpr size_t kIndexChunk = (size_t)32 << 20;

template <typename T>
hipError_t dalloc(mips_maximus_index* ix, T** p, size_t count) {
    const size_t bytes = ((count * sizeof(T) > 0 ? count * sizeof(T) : 1) + 255) & ~(size_t)255;
    if (bytes >= kIndexChunk) {
        void* q = nullptr;
        const hipError_t e = hipMalloc(&q, bytes);
        if (e != hipSuccess) return e;
        ix->allocs.push_back(q);
        *p = (T*)q;
        return hipSuccess;
    }
    if (bytes > ix->arena_left) {
        void* q = nullptr;
        const hipError_t e = hipMalloc(&q, kIndexChunk);
        if (e != hipSuccess) return e;
        ix->allocs.push_back(q);
        ix->arena = (char*)q;
        ix->arena_left = kIndexChunk;
    }
    *p = (T*)ix->arena;
    ix->arena += bytes;
    ix->arena_left -= bytes;
    return hipSuccess;
}

void free_index(mips_maximus_index* ix) {
    if (!ix) return;
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    if (have) (void)hipSetDevice(ix->device);
    for (void* p : ix->allocs) (void)hipFree(p);
    if (have) (void)hipSetDevice(cur);
    delete ix;
}

// Forgy initialisation: C distinct users drawn with a splitmix64 stream.
std::vector<int> forgy(int64_t n_u, int C, uint64_t seed) {
    uint64_t s = seed ^ 0x9E3779B97F4A7C15ull;
    auto next = [&]() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    std::vector<int> out;
    out.reserve(C);
    std::vector<int> sorted;
    while ((int)out.size() < C) {
        const int cand = (int)(next() % (uint64_t)n_u);
        auto it = std::lower_bound(sorted.begin(), sorted.end(), cand);
        if (it != sorted.end() && *it == cand) continue;
        sorted.insert(it, cand);
        out.push_back(cand);
    }
    std::sort(out.begin(), out.end());
    return out;
}

}  // namespace

// ---------------------------------------------------------------------------
// Queries for arbitrary user vectors (new users, or any subset).  A vector
// may use cluster c's list when its angle to the centroid is at most
// theta_b[c]: the bound of Eq. (appx_bound) only needs theta_uc <= theta_b
// (Section III-C), so such a vector is covered exactly like a member.  Each
// vector tries its nearest centroid; the others take the exact path.
// ---------------------------------------------------------------------------
__global__ void qcover_kernel(const float* __restrict__ Uq, int64_t n_q, int f,
                              const int* __restrict__ qassign, const double* __restrict__ cent,
                              const double* __restrict__ cnorm, const double* __restrict__ theta,
                              unsigned int* ccount, int* uflag, int* flist, Ctrl* ctrl) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n_q) return;
    const float* row = Uq + q * f;
    double n2 = 0.0;
    bool finite = true;
    for (int j = 0; j < f; ++j) {
        finite = finite && __builtin_isfinite(row[j]);
        n2 += (double)row[j] * (double)row[j];
    }
    const int c = qassign[q];
    bool covered = false;
    if (finite && n2 > 0.0) {
        if (!(cnorm[c] > 0.0)) {
            covered = true;                       // theta_b = pi: the bound is ||i||
        } else {
            const double th = stable_angle(row, cent + (int64_t)c * f, f, sqrt(n2), cnorm[c]);
            covered = th <= theta[c];
        }
    }
    if (!finite) atomicOr(&ctrl->nonfinite, 1u);
    if (covered) {
        atomicAdd(&ccount[c], 1u);
    } else {
        uflag[q] = 1;
        const unsigned int k = atomicAdd(&ctrl->fb_count, 1u);
        flist[k] = (int)q;
    }
}

__global__ void qscatter_kernel(int64_t n_q, const int* __restrict__ qassign,
                                const int* __restrict__ uflag, unsigned int* offs, int* sorted) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n_q || uflag[q]) return;
    const unsigned int pos = atomicAdd(&offs[qassign[q]], 1u);
    sorted[pos] = (int)q;
}

// tiles per cluster for runs of `span` users
__global__ void qtile_count_kernel(const unsigned int* ccount, int C, int span, unsigned int* tcount) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    tcount[c] = (ccount[c] + span - 1) / span;
}

__global__ void qtiles_kernel(const unsigned int* ccount, const unsigned int* cstart,
                              const unsigned int* toff, int C, int span, int4* tiles) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const unsigned int n = ccount[c];
    for (unsigned int o = 0, t = 0; o < n; o += span, ++t)
        tiles[toff[c] + t] = make_int4(c, (int)(cstart[c] + o), (int)min((unsigned int)span, n - o), 0);
}

extern "C" {

int mips_maximus_build(const float* U, int64_t n_u, const float* I, int64_t n_i, int32_t f,
                       int32_t n_clusters, int32_t kmeans_iters, uint64_t seed, int32_t block_items,
                       void* stream, mips_maximus_index** out_index) {
    if (!out_index) return fail(MIPS_ERR_ARG, "out_index is NULL");
    *out_index = nullptr;
    if (!U || !I) return fail(MIPS_ERR_ARG, "null array pointer");
    if (n_u < 1 || n_u >= ((int64_t)1 << 31)) return fail(MIPS_ERR_ARG, "n_u must be in [1, 2^31)");
    if (n_i < 1 || n_i >= ((int64_t)1 << 31)) return fail(MIPS_ERR_ARG, "n_i must be in [1, 2^31)");
    if (f < 1 || f > 256) return fail(MIPS_ERR_ARG, "f must be in [1, 256] (got %d)", f);
    if (n_clusters < 1 || n_clusters > 4096 || (int64_t)n_clusters > n_u)
        return fail(MIPS_ERR_ARG, "n_clusters must be in [1, min(n_u, 4096)] (got %d)", n_clusters);
    if (kmeans_iters < 0 || kmeans_iters > 100)
        return fail(MIPS_ERR_ARG, "kmeans_iters must be in [0, 100] (got %d)", kmeans_iters);
    if (block_items < 0) return fail(MIPS_ERR_ARG, "block_items must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    PhaseTimer timer(MIPS_PHASE_BUILD, s);

    mips_maximus_index* ix = new (std::nothrow) mips_maximus_index();
    if (!ix) return fail(MIPS_ERR_NOMEM, "host allocation failed");
    (void)hipGetDevice(&ix->device);
    const int C = n_clusters;
    ix->n_u = n_u;
    ix->n_i = n_i;
    ix->f = f;
    ix->C = C;
    ix->n_blk = (n_i + kTile - 1) / kTile;
    ix->n_i_pad = ix->n_blk * kTile;
    ix->shared_blocks = block_items > 0 ? (block_items + kTile - 1) / kTile : 1;

    hipError_t e = hipSuccess;
    auto fail_hip = [&](const char* what) {
        free_index(ix);
        return (e == hipErrorOutOfMemory) ? fail(MIPS_ERR_NOMEM, "%s: out of device memory", what)
                                          : hip_fail(e, what);
    };
#define TRY(x, what) do { if ((e = (x)) != hipSuccess) return fail_hip(what); } while (0)

    // copies of the inputs
    TRY(dalloc(ix, &ix->U, (size_t)n_u * f), "alloc U");
    TRY(dalloc(ix, &ix->I, (size_t)n_i * f), "alloc I");
    TRY(hipMemcpyAsync(ix->U, U, (size_t)n_u * f * sizeof(float), hipMemcpyDeviceToDevice, s), "copy U");
    TRY(hipMemcpyAsync(ix->I, I, (size_t)n_i * f * sizeof(float), hipMemcpyDeviceToDevice, s), "copy I");

    // ---- k-means (Section III-A) -----------------------------------------
    unsigned int* absmax = nullptr;
    unsigned long long* sums = nullptr;
    unsigned int* counts = nullptr;
    float* cent32 = nullptr;
    float* cnorm2 = nullptr;
    double* cnorm = nullptr;
    int* init_idx = nullptr;
    TRY(dalloc(ix, &ix->cent, (size_t)C * f), "alloc centroids");
    TRY(dalloc(ix, &ix->theta, (size_t)C), "alloc theta");
    TRY(dalloc(ix, &ix->assign, (size_t)n_u), "alloc assign");
    TRY(dalloc(ix, &absmax, 1), "alloc");
    TRY(dalloc(ix, &sums, (size_t)C * f), "alloc");
    TRY(dalloc(ix, &counts, (size_t)C), "alloc");
    unsigned int *ccounts = nullptr, *ghist = nullptr;
    TRY(dalloc(ix, &ix->sorted_users, (size_t)n_u), "alloc");
    TRY(dalloc(ix, &ccounts, (size_t)group_chunks(n_u) * C), "alloc");
    TRY(dalloc(ix, &ghist, (size_t)2 * kBuckets), "alloc");
    // sums in LDS per workgroup when C x f fits, else over users grouped by cluster
    const bool lds_sums = (int64_t)C * f <= 4096;
    TRY(dalloc(ix, &cent32, (size_t)C * f), "alloc");
    TRY(dalloc(ix, &cnorm2, (size_t)C), "alloc");
    TRY(dalloc(ix, &cnorm, (size_t)C), "alloc");
    TRY(dalloc(ix, &init_idx, (size_t)C), "alloc");
    {
        const std::vector<int> pick = forgy(n_u, C, seed);
        TRY(hipMemcpyAsync(init_idx, pick.data(), C * sizeof(int), hipMemcpyHostToDevice, s), "copy init");
        TRY(hipStreamSynchronize(s), "sync");   // `pick` leaves scope
    }
    TRY(launch_zero(absmax, sizeof(unsigned int), s), "zero");
    absmax_kernel<<<256, 256, 0, s>>>(ix->U, n_u * f, absmax);
    gather_rows_kernel<<<grid_of((int64_t)C * f), 256, 0, s>>>(ix->U, f, init_idx, C, ix->cent);
    const size_t lds_assign = (size_t)64 * f * sizeof(float);
    for (int it = 0; it <= kmeans_iters; ++it) {
        cent_prep_kernel<<<grid_of(C), 256, 0, s>>>(ix->cent, C, f, cent32, cnorm2);
        assign_kernel<<<grid_of(n_u), 256, lds_assign, s>>>(ix->U, n_u, f, cent32, cnorm2, C, ix->assign);
        if (it == kmeans_iters) break;   // final assignment after the last update
        TRY(launch_zero(sums, (size_t)C * f * sizeof(unsigned long long), s), "zero");
        TRY(launch_zero(counts, (size_t)C * sizeof(unsigned int), s), "zero");
        if (lds_sums) {
            kmeans_sum_kernel<<<grid_of(n_u), 256, 0, s>>>(ix->U, n_u, f, ix->assign, absmax, sums, counts, C);
        } else {
            TRY(group_users(ix->assign, n_u, C, ccounts, ghist, ix->sorted_users, s), "grouping");
            kmeans_sum_sorted_kernel<<<grid_of(n_u, kSortedSumRows), 256, 0, s>>>(
                ix->U, n_u, f, ix->sorted_users, ix->assign, absmax, sums);
            copy_counts_kernel<<<grid_of(C), 256, 0, s>>>(ghist, C, counts);
        }
        kmeans_update_kernel<<<grid_of((int64_t)C * f), 256, 0, s>>>(ix->cent, C, f, sums, counts, absmax, n_u);
    }
    TRY(hipGetLastError(), "k-means");

    // ---- theta_b (Algorithm 1, ConstructIndex) ----------------------------
    cnorm_kernel<<<grid_of(C), 256, 0, s>>>(ix->cent, C, f, cnorm);
    TRY(launch_zero(ix->theta, (size_t)C * sizeof(double), s), "zero");
    theta_kernel<<<std::min(grid_of(n_u), 1024u), 256, 0, s>>>(ix->U, n_u, f, ix->assign, ix->cent,
                                                               cnorm, C, (unsigned long long*)ix->theta);
    theta_fix_kernel<<<grid_of(C), 256, 0, s>>>(cnorm, C, ix->theta);
    TRY(hipGetLastError(), "theta_b");
    ix->cent32 = cent32;
    ix->cnorm2 = cnorm2;
    ix->cnorm = cnorm;

    // ---- bounds and per-cluster lists --------------------------------------
    {
        uint32_t *k0 = nullptr, *k1 = nullptr;
        int *v0 = nullptr, *v1 = nullptr;
        const size_t tot = (size_t)C * n_i;
        TRY(dalloc(ix, &k0, tot), "alloc keys");
        TRY(dalloc(ix, &k1, tot), "alloc keys");
        TRY(dalloc(ix, &v0, tot), "alloc vals");
        TRY(dalloc(ix, &v1, tot), "alloc vals");
        bound_kernel<<<grid_of((int64_t)tot), 256, 0, s>>>(ix->I, n_i, f, ix->cent, cnorm, ix->theta,
                                                           C, k0, v0);
        for (int pass = 0; pass < 4; ++pass) {
            const bool even = (pass & 1) == 0;
            radix_pass_kernel<<<C, 1024, 0, s>>>(even ? k0 : k1, even ? v0 : v1, even ? k1 : k0,
                                                  even ? v1 : v0, n_i, 8 * pass);
        }
        TRY(dalloc(ix, &ix->lists, (size_t)C * ix->n_i_pad), "alloc lists");
        TRY(dalloc(ix, &ix->lbound, (size_t)C * ix->n_i_pad), "alloc bounds");
        lists_kernel<<<grid_of((int64_t)C * ix->n_i_pad), 256, 0, s>>>(k0, v0, n_i, ix->n_i_pad, C,
                                                                       ix->lists, ix->lbound);
        TRY(hipGetLastError(), "lists");
        // users grouped by the final assignment
        TRY(group_users(ix->assign, n_u, C, ccounts, ghist, ix->sorted_users, s), "user grouping");
    }

    // ---- screen copies of the items for every precision --------------------
    {
        Ctrl* tctrl = nullptr;
        float* Etmp = nullptr;
        TRY(dalloc(ix, &tctrl, 3), "alloc");
        ix->prep_ctrl = tctrl;
        TRY(dalloc(ix, &Etmp, (size_t)n_i), "alloc");
        TRY(dalloc(ix, &ix->kexp, (size_t)n_i), "alloc");
        TRY(launch_zero(tctrl, 3 * sizeof(Ctrl), s), "zero");
        for (int prec = 0; prec < 3; ++prec) {
            ScreenPlan p;
            make_screen_plan(n_u, n_i, f, 1, prec, true, &p);
            const size_t esz = prec == PREC_FP32 ? 4 : (prec == PREC_BF16 ? 2 : 1);
            unsigned char* q = nullptr;
            TRY(dalloc(ix, &q, (size_t)n_i * p.f_pad * esz), "alloc screen rows");
            ix->qrow[prec] = q;
            TRY(dalloc(ix, &ix->Corig[prec], (size_t)n_i), "alloc");
            TRY(dalloc(ix, &ix->Gorig[prec], (size_t)n_i), "alloc");
            TRY(dalloc(ix, &ix->cblockmax[prec], (size_t)C * ix->n_blk), "alloc");
            ItemPrepArgs ia{};
            ia.I = ix->I;
            ia.n_i = n_i;
            ia.n_blk = ix->n_blk;
            ia.f = f;
            ia.f_pad = p.f_pad;
            ia.nch = p.nch;
            ia.gamma = p.gamma;
            ia.Corig = ix->Corig[prec];
            ia.Gorig = ix->Gorig[prec];
            ia.Eorig = Etmp;
            ia.kexp = ix->kexp;
            ia.qrow = q;
            ia.ctrl = tctrl + prec;
            if (p.fast) {
                TRY(launch_item_prep(prec, ia, false, s), "item screen copies");
                cblockmax_kernel<<<grid_of((int64_t)C * ix->n_blk), 256, 0, s>>>(
                    ix->lists, ix->n_i_pad, ix->n_blk, C, ix->Corig[prec], ix->Gorig[prec],
                    ix->cblockmax[prec]);
                TRY(hipGetLastError(), "tile maxima");
            } else if (prec == 0) {
                // no screen for these sizes (every query takes the exact path):
                // only the finiteness check of I is needed
                TRY(launch_nonfinite_scan(ix->I, 0, ix->I, n_i * f, tctrl, s), "finite check");
            }
        }
        Ctrl h[3];
        TRY(hipMemcpyAsync(h, tctrl, sizeof(h), hipMemcpyDeviceToHost, s), "read maxima");
        TRY(hipStreamSynchronize(s), "sync");
        for (int prec = 0; prec < 3; ++prec) {
            ix->maxbits[prec][0] = h[prec].cmax_bits;
            ix->maxbits[prec][1] = h[prec].emax_bits;
            ix->maxbits[prec][2] = h[prec].gmax_bits;
            if (h[prec].nonfinite) {
                free_index(ix);
                return fail(MIPS_ERR_NONFINITE, "I holds NaN or Inf");
            }
        }
    }

    // ---- walk tiles: runs of up to 32*UB users of one cluster --------------
    {
        TRY(launch_zero(counts, (size_t)C * sizeof(unsigned int), s), "zero");
        count_kernel<<<std::min(grid_of(n_u), 256u), 256, 0, s>>>(ix->assign, n_u, C, counts);
        std::vector<unsigned int> hc(C);
        TRY(hipMemcpyAsync(hc.data(), counts, C * sizeof(unsigned int), hipMemcpyDeviceToHost, s), "read counts");
        TRY(hipStreamSynchronize(s), "sync");
        const int ubs[3] = {1, 2, 4};
        for (int q = 0; q < 3; ++q) {
            const int span = kTile * ubs[q];
            std::vector<int4> tl;
            int64_t start = 0;
            for (int c = 0; c < C; ++c) {
                for (int64_t o = 0; o < (int64_t)hc[c]; o += span)
                    tl.push_back(make_int4(c, (int)(start + o), (int)std::min<int64_t>(span, hc[c] - o), 0));
                start += hc[c];
            }
            if (tl.empty()) tl.push_back(make_int4(0, 0, 0, 0));
            ix->ntiles[q] = (int64_t)tl.size();
            TRY(dalloc(ix, &ix->tiles[q], tl.size()), "alloc tiles");
            TRY(hipMemcpyAsync(ix->tiles[q], tl.data(), tl.size() * sizeof(int4), hipMemcpyHostToDevice, s), "copy tiles");
        }
        TRY(hipStreamSynchronize(s), "sync");
    }
#undef TRY
    *out_index = ix;
    return MIPS_OK;
}

void mips_maximus_free(mips_maximus_index* index) { free_index(index); }

}  // extern "C"

namespace {

// Workspace of a query of the index's own users: one layout for the size
// function and the query.
struct IndexQueryLayout {
    size_t ctrl, uflag, zero_end, flist, uscal, cnt, cand, fbkeys, total;
};

IndexQueryLayout index_query_layout(const mips_maximus_index* ix, const ScreenPlan& p) {
    IndexQueryLayout L{};
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o += (b + 255) & ~(size_t)255; return r; };
    L.ctrl = take(sizeof(Ctrl));
    L.uflag = take((size_t)ix->n_u * 4);
    L.zero_end = o;
    L.flist = take((size_t)ix->n_u * 4);
    L.uscal = take((size_t)ix->n_u * 16);
    L.cnt = take((size_t)p.n_ublk * 64 * 4);
    L.cand = take(cand_bytes(p.n_ublk, p.cap));
    L.fbkeys = take((size_t)p.fb_grid * ix->n_i * 8);
    L.total = o;
    return L;
}

// The plan of a query of the index's own users (walk tiles of the plan's
// block count).
ScreenPlan index_query_plan(const mips_maximus_index* ix, int32_t K, int32_t precision) {
    ScreenPlan p;
    make_screen_plan(ix->n_u, ix->n_i, ix->f, K, screen_prec(precision), true, &p);
    p.n_waves = p.fast ? ix->ntiles[ub_slot(p.UB)] : 0;
    p.n_ublk = p.n_waves * p.UB;
    return p;
}

}  // namespace

extern "C" {

size_t mips_maximus_query_workspace_size(const mips_maximus_index* ix, int32_t K, int32_t precision) {
    if (!ix || K < 1 || (int64_t)K > ix->n_i || K > kFallbackMaxK || !valid_prec(precision))
        return 0;
    return index_query_layout(ix, index_query_plan(ix, K, precision)).total;
}

}  // extern "C"

namespace {

// Walk (screen over the cluster lists), certification and the exact
// fallback for the users named by `tiles` / `sorted_users` (rows of U).
int walk_certify_fallback(const mips_maximus_index* ix, const ScreenPlan& p, int precision,
                          bool casc, const float* U, int64_t n_u, const int4* tiles, const int* sorted_users,
                          Ctrl* ctrl, int* uflag, int* flist, float4* uscal, int* cnt, int2* cand,
                          double* fbkeys, int32_t* out_idx, double* out_score, bool want_stats,
                          hipStream_t s) {
    hipError_t e;
    set_ctrl_kernel<<<1, 64, 0, s>>>(ctrl, ix->maxbits[precision][0], ix->maxbits[precision][1],
                                     ix->maxbits[precision][2]);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "set maxima");
    ScreenArgs a{};
    a.U = U;
    a.I = ix->I;
    a.n_u = n_u;
    a.n_i = ix->n_i;
    a.n_blk = ix->n_blk;
    a.n_i_pad = ix->n_i_pad;
    a.f = ix->f;
    a.f_pad = p.f_pad;
    a.nch = p.nch;
    a.K = p.K;
    a.cap = p.cap;
    a.kc = p.kc;
    a.gamma = p.gamma;
    a.walk = 1;
    a.warm_rounds = 1;
    a.shared_blocks = ix->shared_blocks;
    a.tiles = tiles;
    a.sorted_users = sorted_users;
    a.lists = ix->lists;
    a.lbound = ix->lbound;
    a.cblockmax = ix->cblockmax[precision];
    a.qrow = ix->qrow[precision];
    a.kexp = ix->kexp;
    a.Corig = ix->Corig[precision];
    a.Gorig = ix->Gorig[precision];
    if (casc && ix->qrow[PREC_BF16]) {
        // bfloat16 rows of the index for the certification cascade
        ScreenPlan pb;
        make_screen_plan(1, ix->n_i, ix->f, 1, PREC_BF16, true, &pb);
        a.qrow_b = ix->qrow[PREC_BF16];
        a.Gorig_b = ix->Gorig[PREC_BF16];
        a.maxb = &ix->prep_ctrl[PREC_BF16].cmax_bits;
        a.fpb = pb.f_pad;
    }
    a.want_stats = want_stats;
    a.ctrl = ctrl;
    a.uflag = uflag;
    a.flist = flist;
    a.uscal = uscal;
    a.n_ublk = p.n_ublk;
    a.cnt = cnt;
    a.cand = cand;
    a.out_idx = out_idx;
    a.out_score = out_score;
    if (p.fast) {
        if (p.n_waves > 0) {
            {
                PhaseTimer t(MIPS_PHASE_WALK, s);
                if ((e = launch_screen(p, a, s)) != hipSuccess) return hip_fail(e, "walk");
            }
            PhaseTimer t(MIPS_PHASE_CERTIFY, s);
            if ((e = launch_certify(p, a, s)) != hipSuccess) return hip_fail(e, "certify");
        }
    } else {
        if ((e = launch_flag_all(n_u, uflag, flist, ctrl, s)) != hipSuccess) return hip_fail(e, "flag all");
    }
    PhaseTimer t(MIPS_PHASE_FALLBACK, s);
    FallbackArgs fa{};
    fa.U = U;
    fa.I = ix->I;
    fa.n_u = n_u;
    fa.n_i = ix->n_i;
    fa.f = ix->f;
    fa.K = p.K;
    fa.flist = flist;
    fa.ctrl = ctrl;
    fa.keys = fbkeys;
    fa.out_idx = out_idx;
    fa.out_score = out_score;
    if ((e = launch_fallback(p, fa, s)) != hipSuccess) return hip_fail(e, "fallback");
    return MIPS_OK;
}

int check_query_args(const mips_maximus_index* ix, int32_t K, int32_t precision, int32_t* out_idx,
                     double* out_score) {
    if (!ix) return fail(MIPS_ERR_ARG, "index is NULL");
    if (!out_idx || !out_score) return fail(MIPS_ERR_ARG, "null output pointer");
    if (K < 1 || (int64_t)K > ix->n_i) return fail(MIPS_ERR_ARG, "K must be in [1, n_i] (got %d)", K);
    if (K > kFallbackMaxK) return fail(MIPS_ERR_UNSUPPORTED, "K > %d is not supported", kFallbackMaxK);
    if (!valid_prec(precision)) return fail(MIPS_ERR_ARG, "unknown precision %d", precision);
    return MIPS_OK;
}

// Workspace of a vector query: sizes in one place for the size function and
// the query.
struct QueryLayout {
    size_t ctrl, uflag, ccount, tcount, tiles, zero_end;
    size_t flist, uscal, qassign, sorted, cnt, cand, fbkeys, total;
    int64_t max_tiles;
};

QueryLayout query_layout(const mips_maximus_index* ix, const ScreenPlan& p, int64_t n_q) {
    QueryLayout L{};
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o += (b + 255) & ~(size_t)255; return r; };
    const int span = kTile * p.UB;
    L.max_tiles = p.fast ? (n_q + span - 1) / span + ix->C : 0;
    const int64_t n_ublk = L.max_tiles * p.UB;
    L.ctrl = take(sizeof(Ctrl));
    L.uflag = take((size_t)n_q * 4);
    L.ccount = take(2 * kBuckets * sizeof(unsigned int));
    L.tcount = take(2 * kBuckets * sizeof(unsigned int));
    L.tiles = take((size_t)std::max<int64_t>(L.max_tiles, 1) * sizeof(int4));
    L.zero_end = o;
    L.flist = take((size_t)n_q * 4);
    L.uscal = take((size_t)n_q * 16);
    L.qassign = take((size_t)n_q * 4);
    L.sorted = take((size_t)n_q * 4);
    L.cnt = take((size_t)n_ublk * 64 * 4);
    L.cand = take(cand_bytes(n_ublk, p.cap));
    L.fbkeys = take((size_t)p.fb_grid * ix->n_i * 8);
    L.total = o;
    return L;
}

}  // namespace

extern "C" {

int mips_maximus_query(const mips_maximus_index* ix, int32_t K, int32_t precision, int32_t* out_idx,
                       double* out_score, void* workspace, size_t workspace_bytes, void* stream,
                       mips_stats* stats) {
    int rc = check_query_args(ix, K, precision, out_idx, out_score);
    if (rc != MIPS_OK) return rc;
    const size_t need = mips_maximus_query_workspace_size(ix, K, precision);
    if (!workspace || workspace_bytes < need)
        return fail(MIPS_ERR_WORKSPACE, "workspace needs %zu bytes (got %zu)", need, workspace_bytes);
    if (((uintptr_t)workspace & 255) != 0) return fail(MIPS_ERR_ARG, "workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    const ScreenPlan p = index_query_plan(ix, K, precision);
    const int slot = ub_slot(p.UB);
    const IndexQueryLayout L = index_query_layout(ix, p);
    if (L.total > workspace_bytes)
        return fail(MIPS_ERR_WORKSPACE, "workspace layout needs %zu bytes (got %zu)", L.total, workspace_bytes);
    char* ws = (char*)workspace;
    Ctrl* ctrl = (Ctrl*)(ws + L.ctrl);
    int* uflag = (int*)(ws + L.uflag);
    const size_t zero_bytes = L.zero_end;
    int* flist = (int*)(ws + L.flist);
    float4* uscal = (float4*)(ws + L.uscal);
    int* cnt = (int*)(ws + L.cnt);
    int2* cand = (int2*)(ws + L.cand);
    double* fbkeys = (double*)(ws + L.fbkeys);
    hipError_t e;
    if ((e = launch_zero(ws, zero_bytes, s)) != hipSuccess) return hip_fail(e, "zero");
    rc = walk_certify_fallback(ix, p, screen_prec(precision), cascade_of(precision), ix->U, ix->n_u, ix->tiles[slot], ix->sorted_users,
                               ctrl, uflag, flist, uscal, cnt, cand, fbkeys, out_idx, out_score,
                               stats != nullptr, s);
    if (rc != MIPS_OK) return rc;
    if (stats) {
        rc = finish_stats(ctrl, s, ix->n_u, ix->n_i, stats);
        if (rc == MIPS_OK && !p.fast) {
            stats->items_scored = ix->n_u * ix->n_i;
            stats->mean_items_visited = (double)ix->n_i;
        }
        return rc;
    }
    return MIPS_OK;
}

size_t mips_maximus_query_users_workspace_size(const mips_maximus_index* ix, int64_t n_q,
                                               int32_t K, int32_t precision) {
    if (!ix || n_q < 1 || n_q >= ((int64_t)1 << 31) || K < 1 || (int64_t)K > ix->n_i ||
        K > kFallbackMaxK || !valid_prec(precision))
        return 0;
    ScreenPlan p;
    make_screen_plan(n_q, ix->n_i, ix->f, K, screen_prec(precision), true, &p);
    return query_layout(ix, p, n_q).total;
}

int mips_maximus_query_users(const mips_maximus_index* ix, const float* Uq, int64_t n_q, int32_t K,
                             int32_t precision, int32_t* out_idx, double* out_score,
                             void* workspace, size_t workspace_bytes, void* stream,
                             mips_stats* stats) {
    int rc = check_query_args(ix, K, precision, out_idx, out_score);
    if (rc != MIPS_OK) return rc;
    if (!Uq) return fail(MIPS_ERR_ARG, "Uq is NULL");
    if (n_q < 1 || n_q >= ((int64_t)1 << 31)) return fail(MIPS_ERR_ARG, "n_q must be in [1, 2^31)");
    const size_t need = mips_maximus_query_users_workspace_size(ix, n_q, K, precision);
    if (!workspace || workspace_bytes < need)
        return fail(MIPS_ERR_WORKSPACE, "workspace needs %zu bytes (got %zu)", need, workspace_bytes);
    if (((uintptr_t)workspace & 255) != 0) return fail(MIPS_ERR_ARG, "workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    ScreenPlan p;
    make_screen_plan(n_q, ix->n_i, ix->f, K, screen_prec(precision), true, &p);
    const QueryLayout L = query_layout(ix, p, n_q);
    p.n_waves = L.max_tiles;
    p.n_ublk = p.n_waves * p.UB;
    char* ws = (char*)workspace;
    Ctrl* ctrl = (Ctrl*)(ws + L.ctrl);
    int* uflag = (int*)(ws + L.uflag);
    unsigned int* ccount = (unsigned int*)(ws + L.ccount);   // counts, then starts
    unsigned int* tcount = (unsigned int*)(ws + L.tcount);   // tile counts, then offsets
    int4* tiles = (int4*)(ws + L.tiles);
    int* flist = (int*)(ws + L.flist);
    float4* uscal = (float4*)(ws + L.uscal);
    int* qassign = (int*)(ws + L.qassign);
    int* sorted = (int*)(ws + L.sorted);
    hipError_t e;
    if ((e = launch_zero(ws, L.zero_end, s)) != hipSuccess) return hip_fail(e, "zero");
    if (p.fast) {
        PhaseTimer t(MIPS_PHASE_WALK, s);
        const int C = ix->C, f = ix->f, span = kTile * p.UB;
        const size_t lds_assign = (size_t)64 * f * sizeof(float);
        assign_kernel<<<grid_of(n_q), 256, lds_assign, s>>>(Uq, n_q, f, ix->cent32, ix->cnorm2, C, qassign);
        qcover_kernel<<<grid_of(n_q), 256, 0, s>>>(Uq, n_q, f, qassign, ix->cent, ix->cnorm, ix->theta,
                                                   ccount, uflag, flist, ctrl);
        if ((e = launch_scan4096(ccount, s)) != hipSuccess) return hip_fail(e, "scan");
        qtile_count_kernel<<<grid_of(C), 256, 0, s>>>(ccount, C, span, tcount);
        if ((e = launch_scan4096(tcount, s)) != hipSuccess) return hip_fail(e, "scan");
        qtiles_kernel<<<grid_of(C), 256, 0, s>>>(ccount, ccount + kBuckets, tcount + kBuckets, C, span, tiles);
        qscatter_kernel<<<grid_of(n_q), 256, 0, s>>>(n_q, qassign, uflag, ccount + kBuckets, sorted);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "user grouping");
    }
    rc = walk_certify_fallback(ix, p, screen_prec(precision), cascade_of(precision), Uq, n_q, tiles, sorted, ctrl, uflag, flist, uscal,
                               (int*)(ws + L.cnt), (int2*)(ws + L.cand), (double*)(ws + L.fbkeys),
                               out_idx, out_score, stats != nullptr, s);
    if (rc != MIPS_OK) return rc;
    if (stats) {
        rc = finish_stats(ctrl, s, n_q, ix->n_i, stats);
        if (rc == MIPS_OK && !p.fast) {
            stats->items_scored = n_q * ix->n_i;
            stats->mean_items_visited = (double)ix->n_i;
        }
        return rc;
    }
    return MIPS_OK;
}

int mips_maximus_export(const mips_maximus_index* ix, int32_t* n_clusters, int32_t* f, int64_t* n_u,
                        int64_t* n_i, double* centroids, double* theta_b, int32_t* assign,
                        int32_t* lists, float* bounds, void* stream) {
    if (!ix) return fail(MIPS_ERR_ARG, "index is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (n_clusters) *n_clusters = ix->C;
    if (f) *f = ix->f;
    if (n_u) *n_u = ix->n_u;
    if (n_i) *n_i = ix->n_i;
    hipError_t e = hipSuccess;
    if (centroids && e == hipSuccess)
        e = hipMemcpyAsync(centroids, ix->cent, (size_t)ix->C * ix->f * sizeof(double), hipMemcpyDeviceToHost, s);
    if (theta_b && e == hipSuccess)
        e = hipMemcpyAsync(theta_b, ix->theta, (size_t)ix->C * sizeof(double), hipMemcpyDeviceToHost, s);
    if (assign && e == hipSuccess)
        e = hipMemcpyAsync(assign, ix->assign, (size_t)ix->n_u * sizeof(int), hipMemcpyDeviceToHost, s);
    for (int c = 0; c < ix->C && e == hipSuccess; ++c) {
        if (lists)
            e = hipMemcpyAsync(lists + (int64_t)c * ix->n_i, ix->lists + (int64_t)c * ix->n_i_pad,
                               (size_t)ix->n_i * sizeof(int), hipMemcpyDeviceToHost, s);
        if (bounds && e == hipSuccess)
            e = hipMemcpyAsync(bounds + (int64_t)c * ix->n_i, ix->lbound + (int64_t)c * ix->n_i_pad,
                               (size_t)ix->n_i * sizeof(float), hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "export");
    return MIPS_OK;
}

}  // extern "C"
