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
// dst = src (n floats) and max |x| over them (atomic max of the float bits);
// dst is 16-byte aligned, src float4 loads when it is too.  Four loads in
// flight per thread.
__global__ void __launch_bounds__(256) copy_absmax_kernel(const float* __restrict__ src,
                                                          float* __restrict__ dst, int64_t n,
                                                          unsigned int* out) {
    __shared__ float wm[4];
    float m = 0.0f;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if ((((uintptr_t)src) & 15) == 0) {
        const int64_t n4 = n >> 2;
        const float4* s4 = (const float4*)src;
        float4* d4 = (float4*)dst;
        for (int64_t i = t0; i < n4; i += 4 * stride) {
            float4 v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (i + r * stride < n4) v[r] = s4[i + r * stride];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (i + r * stride < n4) {
                    d4[i + r * stride] = v[r];
                    m = fmaxf(m, fmaxf(fmaxf(fabsf(v[r].x), fabsf(v[r].y)),
                                       fmaxf(fabsf(v[r].z), fabsf(v[r].w))));
                }
            }
        }
        for (int64_t k = (n4 << 2) + t0; k < n; k += stride) {
            dst[k] = src[k];
            m = fmaxf(m, fabsf(src[k]));
        }
    } else {
        for (int64_t k = t0; k < n; k += stride) {
            const float x = src[k];
            dst[k] = x;
            m = fmaxf(m, fabsf(x));
        }
    }
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

// splitmix64 (Steele, Lea and Flood 2014): output k of the stream seeded by s.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t s, uint64_t k) {
    uint64_t z = s + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Initial centroids: the user order cut into C strata [c n_u / C, (c+1) n_u / C)
// (each non-empty as C <= n_u), one user drawn uniformly from each, so the
// C users are distinct.
__global__ void forgy_kernel(const float* __restrict__ U, int64_t n_u, int f, int C, uint64_t seed,
                             double* cent) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)C * f) return;
    const int c = (int)(t / f), j = (int)(t - (int64_t)c * f);
    const int64_t lo = (int64_t)c * n_u / C, hi = (int64_t)(c + 1) * n_u / C;
    const uint64_t r = splitmix64_at(seed ^ 0x6A09E667F3BCC909ull, (uint64_t)c);
    const int64_t pick = lo + (int64_t)(r % (uint64_t)(hi - lo));
    cent[t] = (double)U[pick * f + j];
}

// ---------------------------------------------------------------------------
// Nearest centroid on the matrix cores.  Centroid c is extended to
// [c, ||c||^2, 0, ...] and user u to [u, -1/2, 0, ...] (length 2 ks), so the
// float32 product is u.c - ||c||^2 / 2, whose largest value over c marks the
// nearest centroid in Euclidean distance (||u||^2 is common to all c).  Ties
// go to the lower centroid index.
//
// 32x32x2 float32 MFMA tiles: centroids are rows (operand A), users columns
// (operand B); lane l holds user l%32 and the 16 centroids
// {8g + 4(l/32) + q} of the tile; lane half h = l/32 owns the extended
// coordinates [h ks, (h+1) ks).  The centroid operand is kept in a
// lane-ordered image (per tile: ks/2 pairs x 64 lanes x 2 floats, written
// by cent_prep_kernel) that a workgroup copies into LDS as it is.
// ---------------------------------------------------------------------------
struct AssignArgs {
    const float* U;
    int64_t n_u;
    int f, ks, C, ntile, chunk_tiles;
    int stage;                 // users staged through LDS (f <= 64)
    int lds_theta;             // final pass: per-workgroup theta maxima in LDS
    const float* img;          // ntile * ks * 64 floats
    int* assign;
    // angle passes: the index build's final pass takes theta_b of every
    // cluster from its members; a vector query tests each vector's cover
    const double* chat;        // unit centroids, C x f (zero rows for zero centroids)
    const double* cnorm;       // ||c|| in float64
    unsigned long long* theta_bits;
    const double* theta;       // cover test: theta_b
    int* uflag;                // cover test: 1 for a vector sent to the exact path
    int* flist;
    Ctrl* ctrl;
};

// Passes of the assignment kernel.
constexpr int kAssignPlain = 0, kAssignTheta = 1, kAssignCover = 2;

constexpr int kAssignWaves = 4;
constexpr int kAssignLds = 65536;      // dynamic LDS budget of the assignment kernel

__host__ __device__ inline int assign_ks(int f) { return 2 * ((f + 4) / 4); }   // even, 2 ks >= f + 1
inline size_t assign_theta_bytes(int C, bool final_pass) {
    return (final_pass && C <= 1024) ? (((size_t)C * 8 + 15) & ~(size_t)15) : 0;
}
inline size_t assign_stage_bytes(int f) { return f <= 64 ? (size_t)kAssignWaves * 32 * f * 4 : 0; }
inline int assign_chunk_tiles(int f, int C, bool final_pass) {
    const int ks = assign_ks(f), ntile = (C + 31) / 32;
    const size_t room = kAssignLds - assign_theta_bytes(C, final_pass) - assign_stage_bytes(f);
    const int fit = (int)(room / ((size_t)ks * 256));
    return std::max(1, std::min(ntile, fit));
}

template <int KS, int MODE>
__global__ void __launch_bounds__(256) assign_mfma_kernel(AssignArgs a) {
    constexpr bool FINAL = MODE == kAssignTheta;
    extern __shared__ __align__(16) unsigned char lds[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n = lane & 31, h = lane >> 5;
    const int f = a.f, ks = a.ks, ksp = ks >> 1;
    const size_t lt_bytes = FINAL && a.lds_theta ? (((size_t)a.C * 8 + 15) & ~(size_t)15) : 0;
    unsigned long long* lt = (unsigned long long*)lds;
    float* simg = (float*)(lds + lt_bytes);
    float* sus = simg + (size_t)a.chunk_tiles * ks * 64 + (size_t)wave * 32 * f;   // this wave's users
    const int nchunk = (a.ntile + a.chunk_tiles - 1) / a.chunk_tiles;
    const int64_t n_ublk = (a.n_u + 31) >> 5;

    auto stage_img = [&](int ch) {
        const int t0 = ch * a.chunk_tiles, nt = min(a.chunk_tiles, a.ntile - t0);
        const float4* src = (const float4*)(a.img + (size_t)t0 * ks * 64);
        float4* dst = (float4*)simg;
        const int n4 = nt * ks * 16;
        for (int e = threadIdx.x; e < n4; e += blockDim.x) dst[e] = src[e];
    };
    if (FINAL && a.lds_theta)
        for (int c = threadIdx.x; c < a.C; c += blockDim.x) lt[c] = 0ull;
    if (nchunk == 1) stage_img(0);
    __syncthreads();

    for (int64_t base = (int64_t)blockIdx.x * kAssignWaves; base < n_ublk;
         base += (int64_t)gridDim.x * kAssignWaves) {
        const int64_t blk = base + wave;
        const int64_t u0 = blk * 32;
        const int nrows = blk < n_ublk ? (int)min((int64_t)32, a.n_u - u0) : 0;
        const bool valid = n < nrows;
        const float* urow = a.U + (valid ? u0 + n : 0) * f;
        if (a.stage) {
            // coalesced copy of the block's rows (contiguous) into this
            // wave's LDS rows; LDS accesses of one wave complete in order
            const float* src = a.U + (nrows ? u0 : 0) * f;
            const int tot = nrows * f;
#pragma unroll 4
            for (int e = lane; e < tot; e += 64) sus[e] = src[e];
        }
        auto uval = [&](int j) -> float { return a.stage ? sus[n * f + j] : urow[j]; };
        float ub[KS];
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int j = h * ks + k;
            float v = 0.0f;
            if (k < ks) v = (j < f) ? (valid ? uval(j) : 0.0f) : (j == f ? -0.5f : 0.0f);
            ub[k] = v;
        }
        float bestv = -__builtin_inff();
        int besti = 0;
        for (int ch = 0; ch < nchunk; ++ch) {
            if (nchunk > 1) {
                __syncthreads();
                stage_img(ch);
                __syncthreads();
            }
            const int t0 = ch * a.chunk_tiles, nt = min(a.chunk_tiles, a.ntile - t0);
            for (int tl = 0; tl < nt; ++tl) {
                floatx16_t acc;
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
                const float2* ip = (const float2*)simg + (size_t)tl * ksp * 64 + lane;
#pragma unroll
                for (int kp = 0; kp < KS / 2; ++kp) {
                    if (kp < ksp) {
                        const float2 av = ip[kp * 64];
                        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, ub[2 * kp], acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.y, ub[2 * kp + 1], acc, 0, 0, 0);
                    }
                }
                const int cb = (t0 + tl) * 32 + 4 * h;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int c = cb + 8 * (r >> 2) + (r & 3);
                    if (c < a.C && acc[r] > bestv) { bestv = acc[r]; besti = c; }
                }
            }
        }
        {   // the user's two lanes hold disjoint centroid sets
            const float ov = xor32_f(bestv);
            const int oi = xor32_i(besti);
            if (ov > bestv || (ov == bestv && oi < besti)) { bestv = ov; besti = oi; }
        }
        if (MODE != kAssignCover && h == 0 && valid) a.assign[u0 + n] = besti;
        if constexpr (MODE != kAssignPlain) {
            // angle between the user and its centroid in float64 (Kahan:
            // 2 atan2(|u^ - c^|, |u^ + c^|)); lane half h sums the
            // coordinates j with (j / 2) % 2 == h, so the two halves read
            // neighbouring pairs of the unit centroid
            double n2 = 0.0;
            bool fin = true;
            for (int j = 2 * h; j < f; j += 4) {
                const float v0 = valid ? uval(j) : 0.0f;
                fin = fin && __builtin_isfinite(v0);
                const double x0 = (double)v0;
                n2 = fma(x0, x0, n2);
                if (j + 1 < f) {
                    const float v1 = valid ? uval(j + 1) : 0.0f;
                    fin = fin && __builtin_isfinite(v1);
                    const double x1 = (double)v1;
                    n2 = fma(x1, x1, n2);
                }
            }
            n2 += xor32_d(n2);
            fin = fin && xor32_i((int)fin) != 0;
            const double nc = a.cnorm[besti];
            const bool use = valid && n2 > 0.0 && nc > 0.0;
            double d = 0.0, s = 0.0;
            if (use) {
                const double rinv = 1.0 / sqrt(n2);
                const double* y = a.chat + (int64_t)besti * f;
                for (int j = 2 * h; j < f; j += 4) {
                    double y0, y1 = 0.0;
                    if ((f & 1) == 0) {          // 16-byte aligned pair
                        const double2 yy = *(const double2*)(y + j);
                        y0 = yy.x;
                        y1 = yy.y;
                    } else {
                        y0 = y[j];
                        if (j + 1 < f) y1 = y[j + 1];
                    }
                    const double x0 = (double)uval(j) * rinv;
                    const double p0 = x0 - y0, q0 = x0 + y0;
                    d = fma(p0, p0, d);
                    s = fma(q0, q0, s);
                    if (j + 1 < f) {
                        const double x1 = (double)uval(j + 1) * rinv;
                        const double p1 = x1 - y1, q1 = x1 + y1;
                        d = fma(p1, p1, d);
                        s = fma(q1, q1, s);
                    }
                }
            }
            d += xor32_d(d);
            s += xor32_d(s);
            if constexpr (MODE == kAssignTheta) {
                if (use && h == 0) {
                    const double th = 2.0 * atan2(sqrt(d), sqrt(s));
                    const unsigned long long bits = (unsigned long long)__double_as_longlong(th);
                    if (a.lds_theta) atomicMax(&lt[besti], bits);
                    else atomicMax(&a.theta_bits[besti], bits);
                }
            } else {
                // a vector may walk its nearest cluster's list when its angle to
                // the centroid is at most theta_b (a zero centroid has theta_b =
                // pi); the others, zero and non-finite rows take the exact path
                if (h == 0 && valid) {
                    bool cov = fin && n2 > 0.0;
                    if (cov && nc > 0.0) cov = 2.0 * atan2(sqrt(d), sqrt(s)) <= a.theta[besti];
                    const int64_t q = u0 + n;
                    if (!fin) atomicOr(&a.ctrl->nonfinite, 1u);
                    if (cov) {
                        a.assign[q] = besti;
                    } else {
                        a.assign[q] = -1;                 // left out of the grouping
                        a.uflag[q] = 1;
                        const unsigned int k = atomicAdd(&a.ctrl->fb_count, 1u);
                        a.flist[k] = (int)q;
                    }
                }
            }
        }
    }
    if (FINAL && a.lds_theta) {
        __syncthreads();
        for (int c = threadIdx.x; c < a.C; c += blockDim.x)
            if (lt[c]) atomicMax(&a.theta_bits[c], lt[c]);
    }
}

// Per 32-centroid tile (rows staged through LDS): float32 squared norms,
// float64 norms, unit centroids and the lane-ordered image of the extended
// centroids; also clears the cluster counts for the next update and, before
// the final assignment, theta_b.
__global__ void __launch_bounds__(256) cent_prep_kernel(const double* __restrict__ cent, int C, int f,
                                                        int ks, float* img, double* cnorm,
                                                        double* chat, unsigned int* counts,
                                                        double* theta_zero) {
    extern __shared__ double srows[];          // 32 x f
    __shared__ float n2s[32];
    __shared__ double nrm[32];
    const int t = blockIdx.x, tid = threadIdx.x;
    const int nr = min(32, C - t * 32);
    const double* src = cent + (int64_t)t * 32 * f;
    // rows through LDS unless they would not fit beside the static arrays
    const bool stage = f <= 254;
    if (stage)
        for (int e = tid; e < nr * f; e += blockDim.x) srows[e] = src[e];
    const double* rows = stage ? (const double*)srows : src;
    __syncthreads();
    if (tid < 32) {
        const int c = t * 32 + tid;
        float s = 0.0f;
        double s64 = 0.0;
        if (tid < nr) {
            for (int j = 0; j < f; ++j) {
                const double x = rows[tid * f + j];
                const float xf = (float)x;
                s = fmaf(xf, xf, s);
                s64 += x * x;
            }
            cnorm[c] = sqrt(s64);
            if (counts) counts[c] = 0u;
            if (theta_zero) theta_zero[c] = 0.0;
        }
        n2s[tid] = s;
        nrm[tid] = sqrt(s64);
    }
    __syncthreads();
    for (int e = tid; e < nr * f; e += blockDim.x) {
        const int r = e / f;
        const double nc = nrm[r];
        chat[(int64_t)t * 32 * f + e] = nc > 0.0 ? rows[e] * (1.0 / nc) : 0.0;
    }
    float* im = img + (size_t)t * ks * 64;
    for (int e = tid; e < ks * 64; e += blockDim.x) {
        const int kp = e >> 7, ln = (e >> 1) & 63, ee = e & 1;
        const int r = ln & 31, j = (ln >> 5) * ks + 2 * kp + ee;
        float v = 0.0f;
        if (r < nr) v = j < f ? (float)rows[r * f + j] : (j == f ? n2s[r] : 0.0f);
        im[e] = v;
    }
}

// ---------------------------------------------------------------------------
// k-means update.  Fixed-point per-cluster sums (int64 adds are order
// independent): workgroup (x, y) takes users [x R, (x+1) R) and clusters
// [y cs, (y+1) cs).  The rows' floats are read four at a time, four such
// loads in flight per thread, against the workgroup's assignments copied to
// LDS; the sums gather in LDS and each non-zero (cluster, factor) sum is
// added to the global one.
// ---------------------------------------------------------------------------
constexpr int kSumMaxRows = 2048;      // R <= kSumMaxRows (assignments in LDS)

__global__ void __launch_bounds__(256) kmeans_sum_kernel(const float* __restrict__ U, int64_t n_u, int f,
                                                         const int* __restrict__ assign,
                                                         const unsigned int* absmax_bits,
                                                         int64_t rows_per_wg, int cs,
                                                         unsigned long long* sums,
                                                         unsigned int* counts, int C) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int c0 = blockIdx.y * cs, ncs = min(cs, C - c0);
    if (ncs <= 0) return;                                         // whole workgroup
    unsigned long long* ls = (unsigned long long*)lds;            // [cs][f]
    unsigned int* lc = (unsigned int*)(ls + (size_t)cs * f);      // [cs]
    int* la = (int*)(lc + cs);                                    // [R] cluster - c0
    const int64_t lo = (int64_t)blockIdx.x * rows_per_wg;
    const int64_t hi = min(n_u, lo + rows_per_wg);
    const int nrow = (int)max((int64_t)0, hi - lo);
    for (int t = threadIdx.x; t < ncs * f; t += blockDim.x) ls[t] = 0ull;
    for (int t = threadIdx.x; t < ncs; t += blockDim.x) lc[t] = 0u;
    for (int t = threadIdx.x; t < nrow; t += blockDim.x) la[t] = assign[lo + t] - c0;
    __syncthreads();
    const double scale = fixed_scale(n_u, *absmax_bits);
    // rows_per_wg is a multiple of 4 and U 16-byte aligned: float4 groups
    const int nel = nrow * f, ng = (nel + 3) >> 2;
    const float4* U4 = (const float4*)(U + lo * f);
    for (int g0 = threadIdx.x; g0 < ng; g0 += 4 * 256) {
        float4 v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int g = g0 + 256 * r;
            if (4 * g + 4 <= nel) {
                v[r] = U4[g];
            } else if (g < ng) {
                const float* p = U + lo * f + 4 * g;
                v[r].x = p[0];
                v[r].y = 4 * g + 1 < nel ? p[1] : 0.0f;
                v[r].z = 4 * g + 2 < nel ? p[2] : 0.0f;
                v[r].w = 4 * g + 3 < nel ? p[3] : 0.0f;
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int g = g0 + 256 * r;
            if (g >= ng) continue;
            const float x[4] = {v[r].x, v[r].y, v[r].z, v[r].w};
            int row = (4 * g) / f;
            int j = 4 * g - row * f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (4 * g + q < nel) {
                    const int c = la[row];
                    if ((unsigned)c < (unsigned)ncs) {
                        atomicAdd(&ls[c * f + j], (unsigned long long)llrint((double)x[q] * scale));
                        if (j == 0) atomicAdd(&lc[c], 1u);
                    }
                }
                if (++j == f) { j = 0; ++row; }
            }
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < ncs * f; t += blockDim.x)
        if (ls[t]) atomicAdd(&sums[(int64_t)c0 * f + t], ls[t]);
    for (int t = threadIdx.x; t < ncs; t += blockDim.x)
        if (lc[t]) atomicAdd(&counts[c0 + t], lc[t]);
}

// New centroids from the sums (an empty cluster keeps its centroid); clears
// the sums for the next update.
__global__ void kmeans_update_kernel(double* cent, int C, int f, unsigned long long* sums,
                                     const unsigned int* counts, const unsigned int* absmax_bits,
                                     int64_t n_u) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)C * f) return;
    const int c = (int)(t / f);
    const unsigned int n = counts[c];
    const unsigned long long v = sums[t];
    sums[t] = 0ull;
    if (n == 0) return;
    const double scale = fixed_scale(n_u, *absmax_bits);
    cent[t] = (double)(long long)v / scale / (double)n;
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

// ---------------------------------------------------------------------------
// Bound of Eq. (appx_bound) for every (cluster, item) in float64:
// ||i|| cos(max(theta_ic - theta_b, 0)), theta_ic by Kahan's formula on the
// unit vectors, widened by 2^-40 ||i|| for the float64 evaluation and rounded
// up to float32.  Workgroup (x, y): items [256 x, 256 x + 256) against
// clusters [y cs, (y+1) cs).  With F > 0 (f <= F) the rows are staged through
// LDS and each thread keeps its unit item in registers; the unit centroid is
// the same for the whole wave.
// ---------------------------------------------------------------------------
template <int F>
__global__ void __launch_bounds__(256) bound_kernel(const float* __restrict__ I, int64_t n_i, int f,
                                                    const double* __restrict__ chat,
                                                    const double* __restrict__ cnorm,
                                                    const double* __restrict__ theta, int C, int cs,
                                                    uint32_t* __restrict__ keys) {
    extern __shared__ float srow[];       // F > 0: 256 x f floats, then unit centroids
    const int64_t i0 = (int64_t)blockIdx.x * 256, i = i0 + threadIdx.x;
    const bool on = i < n_i;
    const int c0 = blockIdx.y * cs, c1 = min(C, c0 + cs);
    double xh[F > 0 ? F : 1];
    double n2 = 0.0;
    if constexpr (F > 0) {
        const int nrow = (int)min((int64_t)256, n_i - i0);
        const float* src = I + i0 * f;
        for (int e = threadIdx.x; e < nrow * f; e += 256) srow[e] = src[e];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < F; ++j) {
            const double x = (on && j < f) ? (double)srow[threadIdx.x * f + j] : 0.0;
            xh[j] = x;
            n2 += x * x;
        }
    } else {
        const float* row = I + (on ? i : 0) * f;
        for (int j = 0; j < f; ++j) n2 += (double)row[j] * (double)row[j];
    }
    const double ni = sqrt(n2);
    const double rinv = ni > 0.0 ? 1.0 / ni : 0.0;
    if constexpr (F > 0) {
#pragma unroll
        for (int j = 0; j < F; ++j) xh[j] *= rinv;
    }
    const double slack = 0x1p-40 * ni * (1.0 + 0x1p-20);
    // F > 0: the rows' LDS then holds up to 128 unit centroids at a time
    // (256 f floats = 128 f doubles), read by the whole workgroup
    double* sc = (double*)srow;
    for (int cc = c0; cc < c1; cc += 128) {
        const int nb = min(128, c1 - cc);
        if constexpr (F > 0) {
            __syncthreads();
            for (int e = threadIdx.x; e < nb * f; e += 256) sc[e] = chat[(int64_t)cc * f + e];
            __syncthreads();
        }
        for (int c = cc; c < cc + nb; ++c) {
            const double nc = cnorm[c];
            double b;
            if (!(ni > 0.0)) {
                b = 0.0;
            } else if (!(nc > 0.0)) {
                b = ni;
            } else {
                double d = 0.0, s = 0.0;
                if constexpr (F > 0) {
                    const double* y = sc + (c - cc) * f;
#pragma unroll
                    for (int j = 0; j < F; ++j) {
                        if (j < f) {
                            const double yj = y[j];
                            const double p = xh[j] - yj, q = xh[j] + yj;
                            d = fma(p, p, d);
                            s = fma(q, q, s);
                        }
                    }
                } else {
                    const double* y = chat + (int64_t)c * f;
                    const float* row = I + (on ? i : 0) * f;
                    for (int j = 0; j < f; ++j) {
                        const double x = (double)row[j] * rinv;
                        const double p = x - y[j], q = x + y[j];
                        d = fma(p, p, d);
                        s = fma(q, q, s);
                    }
                }
                const double th = 2.0 * atan2(sqrt(d), sqrt(s));
                b = ni * cos(fmax(th - theta[c], 0.0));
            }
            if (on) keys[(int64_t)c * n_i + i] = desc_key(round_up_f32(b + slack));
        }
    }
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort (8-bit digit at `shift`) of C independent segments
// of `len` (key, value) pairs, each segment split into P parts of `part`
// pairs (grid P x C).  radix_hist_kernel counts the digits of every part;
// radix_scatter_kernel starts each digit of part p after all smaller digits
// of the segment and the same digit of parts before p, then ranks its pairs
// 1024 at a time in their current order (so equal digits keep their order).
// The first pass takes the item index as the value; the last writes the
// padded walk lists and their float bounds.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) radix_hist_kernel(const uint32_t* __restrict__ keys, int64_t len,
                                                         int64_t part, int shift, unsigned int* hist) {
    __shared__ unsigned int hc[256];
    const int P = gridDim.x, p = blockIdx.x, lane = threadIdx.x & 63;
    const int64_t seg = blockIdx.y;
    hc[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t lo = p * part, hi = min(len, lo + part);
    const uint32_t* k = keys + seg * len;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int64_t i0 = lo; i0 < hi; i0 += 256) {
        const int64_t i = i0 + threadIdx.x;
        const bool on = i < hi;
        const uint32_t d = on ? (k[i] >> shift) & 255u : 0u;
        // lanes with the same digit: one LDS add per digit and wave
        uint64_t match = __builtin_amdgcn_ballot_w64(on);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t bb = __builtin_amdgcn_ballot_w64(((d >> bit) & 1u) != 0u);
            match &= ((d >> bit) & 1u) ? bb : ~bb;
        }
        if (on && (match & lt) == 0ull) atomicAdd(&hc[d], (unsigned int)__builtin_popcountll(match));
    }
    __syncthreads();
    hist[(seg * 256 + threadIdx.x) * P + p] = hc[threadIdx.x];
}

template <bool FIRST, bool LAST>
__global__ void __launch_bounds__(1024) radix_scatter_kernel(const uint32_t* __restrict__ kin,
                                                             const int* __restrict__ vin,
                                                             uint32_t* __restrict__ kout,
                                                             int* __restrict__ vout, int64_t len,
                                                             int64_t part, int shift,
                                                             const unsigned int* __restrict__ hist,
                                                             int* lists, float* lbound, int64_t len_pad) {
    __shared__ unsigned int run[256];         // next output slot of each digit
    __shared__ unsigned int wsum[4];
    __shared__ unsigned int wcnt[16][256];    // per-wave digit counts of the current chunk
    __shared__ unsigned int woff[16][256];    // per-wave digit offsets of the current chunk
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int P = gridDim.x, p = blockIdx.x;
    const int64_t seg = blockIdx.y;
    unsigned int tot = 0u;
    if (t < 256) {
        const unsigned int* hs = hist + (seg * 256 + t) * P;
        unsigned int before = 0u;
        for (int q = 0; q < P; ++q) {
            const unsigned int v = hs[q];
            tot += v;
            if (q < p) before += v;
        }
        run[t] = before;
    }
    for (int d = t; d < 16 * 256; d += 1024) (&wcnt[0][0])[d] = 0u;
    // exclusive scan of the segment's digit totals (waves 0-3, 64 digits each)
    unsigned int x = tot;
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (t < 256 && lane == 63) wsum[wv] = x;
    __syncthreads();
    if (t < 256) {
        unsigned int pre = x - tot;
        for (int q = 0; q < wv; ++q) pre += wsum[q];
        run[t] += pre;
    }
    __syncthreads();
    const int64_t lo = p * part, hi = min(len, lo + part);
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    // the next chunk's pairs are loaded while this one is ranked
    bool on_n = lo + t < hi;
    uint32_t k_n = on_n ? kin[seg * len + lo + t] : 0u;
    int v_n = FIRST ? (int)(lo + t) : (on_n ? vin[seg * len + lo + t] : 0);
    for (int64_t c0 = lo; c0 < hi; c0 += 1024) {
        const bool on = on_n;
        const uint32_t k = k_n;
        const int v = v_n;
        {
            const int64_t in = c0 + 1024 + t;
            on_n = in < hi;
            k_n = on_n ? kin[seg * len + in] : 0u;
            v_n = FIRST ? (int)in : (on_n ? vin[seg * len + in] : 0);
        }
        const uint32_t d = (k >> shift) & 255u;
        uint64_t match = __builtin_amdgcn_ballot_w64(on);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t bb = __builtin_amdgcn_ballot_w64(((d >> bit) & 1u) != 0u);
            match &= ((d >> bit) & 1u) ? bb : ~bb;
        }
        const unsigned int rank_w = __builtin_popcountll(match & lt);
        if (on && rank_w == 0) wcnt[wv][d] = __builtin_popcountll(match);
        __syncthreads();
        if (t < 256) {
            unsigned int cq[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) cq[q] = wcnt[q][t];
            unsigned int acc = run[t];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                woff[q][t] = acc;
                wcnt[q][t] = 0u;
                acc += cq[q];
            }
            run[t] = acc;
        }
        __syncthreads();
        if (on) {
            const unsigned int pos = woff[wv][d] + rank_w;
            if (LAST) {
                lists[seg * len_pad + pos] = v;
                lbound[seg * len_pad + pos] = key_to_float(k);
            } else {
                kout[seg * len + pos] = k;
                vout[seg * len + pos] = v;
            }
        }
    }
    if (LAST && p == 0) {
        for (int64_t q = len + t; q < len_pad; q += 1024) {
            lists[seg * len_pad + q] = -1;
            lbound[seg * len_pad + q] = -__builtin_inff();
        }
    }
}

// Per item: (C_i, G_i of the three screen precisions) in one float4, so the
// tile maxima below gather one 16-byte value per list entry.
struct BlockMaxArgs {
    const int* lists;
    int64_t n_i, n_i_pad, n_blk;
    int C;
    const float* Corig;        // C_i (the same for every precision)
    const float* Gorig[3];     // null for a precision without a screen
    float4* cg4;               // n_i entries
    float2* out[3];            // null for a precision without a screen
};

__global__ void __launch_bounds__(256) item_cg4_kernel(BlockMaxArgs a) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= a.n_i) return;
    a.cg4[i] = make_float4(a.Corig[i], a.Gorig[0] ? a.Gorig[0][i] : 0.0f,
                           a.Gorig[1] ? a.Gorig[1][i] : 0.0f, a.Gorig[2] ? a.Gorig[2][i] : 0.0f);
}

// Per (cluster, tile of 32 list entries) and screen precision: max C and
// max G of its items.
__global__ void __launch_bounds__(256) cblockmax_kernel(BlockMaxArgs a) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)a.C * a.n_blk) return;
    const int c = (int)(t / a.n_blk);
    const int64_t b = t - (int64_t)c * a.n_blk;
    const int4* li = (const int4*)(a.lists + (int64_t)c * a.n_i_pad + b * kTile);
    float4 m = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll 2
    for (int q = 0; q < kTile / 4; ++q) {
        const int4 v = li[q];
        const int it[4] = {v.x, v.y, v.z, v.w};
        float4 g[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) g[r] = it[r] >= 0 ? a.cg4[it[r]] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            m.x = fmaxf(m.x, g[r].x);
            m.y = fmaxf(m.y, g[r].y);
            m.z = fmaxf(m.z, g[r].z);
            m.w = fmaxf(m.w, g[r].w);
        }
    }
    if (a.out[0]) a.out[0][t] = make_float2(m.x, m.y);
    if (a.out[1]) a.out[1][t] = make_float2(m.x, m.z);
    if (a.out[2]) a.out[2][t] = make_float2(m.x, m.w);
}

// ---------------------------------------------------------------------------
// Users grouped by cluster, in ascending user order inside each cluster (a
// stable counting sort on the cluster id, C <= 4096; a negative id leaves
// the user out): per-chunk counts
// (cluster-major), one wave per cluster scans them over the chunks, a scan
// over the clusters gives their starts, and one wave per chunk places its
// users 64 at a time, ranking equal clusters within the wave by ballots on
// the bits of the cluster id.
// ---------------------------------------------------------------------------
constexpr int kGroupChunk = 1024;

__global__ void __launch_bounds__(256) group_count_kernel(const int* __restrict__ assign, int64_t n, int C,
                                                          int nch, unsigned int* ccounts) {
    __shared__ unsigned int lc[4096];
    for (int c = threadIdx.x; c < C; c += blockDim.x) lc[c] = 0u;
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * kGroupChunk, hi = min(n, lo + kGroupChunk);
    for (int64_t u = lo + threadIdx.x; u < hi; u += blockDim.x) {
        const int c = assign[u];
        if (c >= 0) atomicAdd(&lc[c], 1u);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < C; c += blockDim.x) ccounts[(int64_t)c * nch + blockIdx.x] = lc[c];
}

// ccounts[c][k] -> users of cluster c in chunks before k; hist[c] = size of c
__global__ void __launch_bounds__(64) group_scan_kernel(unsigned int* ccounts, int nch, unsigned int* hist) {
    const int c = blockIdx.x, lane = threadIdx.x;
    unsigned int* row = ccounts + (int64_t)c * nch;
    unsigned int carry = 0u;
    for (int k0 = 0; k0 < nch; k0 += 64) {
        const int k = k0 + lane;
        const unsigned int v = k < nch ? row[k] : 0u;
        unsigned int x = v;
        for (int off = 1; off < 64; off <<= 1) {
            const unsigned int y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (k < nch) row[k] = carry + x - v;
        carry += __shfl(x, 63);
    }
    if (lane == 0) hist[c] = carry;
}

__global__ void __launch_bounds__(64) group_scatter_kernel(const int* __restrict__ assign, int64_t n, int C,
                                                           int nch, const unsigned int* __restrict__ offs,
                                                           const unsigned int* __restrict__ cstart,
                                                           int* sorted) {
    __shared__ unsigned int next[4096];
    const int lane = threadIdx.x, k = blockIdx.x;
    for (int c = lane; c < C; c += 64) next[c] = cstart[c] + offs[(int64_t)c * nch + k];
    __syncthreads();
    const int64_t lo = (int64_t)k * kGroupChunk, hi = min(n, lo + kGroupChunk);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int nbits = C > 1 ? 32 - __builtin_clz((unsigned)(C - 1)) : 0;
    int key[kGroupChunk / 64];
#pragma unroll
    for (int q = 0; q < kGroupChunk / 64; ++q) {
        const int64_t u = lo + q * 64 + lane;
        key[q] = u < hi ? assign[u] : 0;
    }
#pragma unroll
    for (int q = 0; q < kGroupChunk / 64; ++q) {
        const int64_t u = lo + q * 64 + lane;
        const bool on = u < hi && key[q] >= 0;
        uint64_t m = ballot(on);
        for (int b = 0; b < nbits; ++b) {
            const bool bit = ((key[q] >> b) & 1) != 0;
            const uint64_t bb = ballot(bit);
            m &= bit ? bb : ~bb;
        }
        // one wave: every lane reads its cursor before the group's last lane
        // advances it (LDS accesses of a wave complete in order)
        if (on) {
            sorted[next[key[q]] + __builtin_popcountll(m & below)] = (int)u;
            if ((m >> lane) == 1ull) next[key[q]] += (unsigned int)__builtin_popcountll(m);
        }
    }
}

// ---------------------------------------------------------------------------
// Walk tiles: runs of up to span = 32, 64 and 128 users of one cluster.
// Tile counts per cluster and their exclusive offsets (one workgroup, three
// spans), then one thread per tile slot; slots past the last tile get an
// empty tile.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) tile_offsets_kernel(const unsigned int* __restrict__ ccount, int C,
                                                            unsigned int* toff) {
    __shared__ unsigned int part[1024];
    const int t = threadIdx.x;
    for (int q = 0; q < 3; ++q) {
        const unsigned int span = (unsigned int)kTile << q;
        unsigned int v[4], sum = 0u;
        for (int r = 0; r < 4; ++r) {
            const int c = t * 4 + r;
            v[r] = c < C ? (ccount[c] + span - 1) / span : 0u;
            sum += v[r];
        }
        part[t] = sum;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const unsigned int add = (t >= off) ? part[t - off] : 0u;
            __syncthreads();
            part[t] += add;
            __syncthreads();
        }
        unsigned int run = part[t] - sum;
        for (int r = 0; r < 4; ++r) {
            toff[q * (kBuckets + 1) + t * 4 + r] = run;
            run += v[r];
        }
        if (t == 1023) toff[q * (kBuckets + 1) + kBuckets] = part[t];   // total
        __syncthreads();
    }
}

struct TileEmitArgs {
    const unsigned int* ccount;
    const unsigned int* cstart;
    const unsigned int* toff;      // 3 x (kBuckets + 1)
    int C;
    int64_t max_tiles[3];
    int4* tiles[3];
};

__global__ void __launch_bounds__(256) tiles_emit_kernel(TileEmitArgs a) {
    const int q = blockIdx.y;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= a.max_tiles[q]) return;
    const unsigned int* to = a.toff + q * (kBuckets + 1);
    if (t >= (int64_t)to[kBuckets]) {
        a.tiles[q][t] = make_int4(0, 0, 0, 0);
        return;
    }
    // the last cluster whose first tile is at or before t
    int lo = 0, hi = a.C - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int64_t)to[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    const unsigned int span = (unsigned int)kTile << q;
    const unsigned int o = (unsigned int)(t - to[lo]) * span;
    a.tiles[q][t] = make_int4(lo, (int)(a.cstart[lo] + o), (int)min(span, a.ccount[lo] - o), 0);
}

__global__ void copy_maxima_kernel(Ctrl* ctrl, const Ctrl* src) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctrl->cmax_bits = src->cmax_bits;
        ctrl->emax_bits = src->emax_bits;
        ctrl->gmax_bits = src->gmax_bits;
    }
}

static unsigned int grid_of(int64_t n, int b = 256) { return (unsigned int)((n + b - 1) / b); }

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
    double* cnorm = nullptr;      // float64 centroid norms
    double* chat = nullptr;       // unit centroids (angles)
    float* img = nullptr;         // lane-ordered extended centroids (assignment)
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
    Ctrl* prep_ctrl = nullptr;            // item maxima (and NaN flag), one Ctrl per precision
    // walk tiles for 1, 2 and 4 user blocks per wave: ntiles slots, an upper
    // bound on the tile count; slots past the last tile hold empty tiles
    int4* tiles[3] = {nullptr, nullptr, nullptr};
    int64_t ntiles[3] = {0, 0, 0};
    // per screen precision: the first wpre tiles of every list in operand order
    int wpre[3] = {0, 0, 0};
    void* wpacked[3] = {nullptr, nullptr, nullptr};
    float2* wcg[3] = {nullptr, nullptr, nullptr};
    int* wscale = nullptr;
    // device memory of the index and the build's temporaries (released when
    // the build ends): blocks of the library's cache, with their sizes
    std::vector<std::pair<void*, size_t>> allocs, tmp;
};

namespace {

int ub_slot(int UB) { return UB == 1 ? 0 : (UB == 2 ? 1 : 2); }

// Device memory for the walk prefix tiles of one screen precision.
constexpr size_t kWalkPrefixBytes = (size_t)16 << 20;

// Device memory of the index and of its build temporaries comes from the
// library's block cache (a released index leaves its blocks for the next).
template <typename T>
hipError_t dalloc(mips_maximus_index* ix, T** p, size_t count, bool temp = false) {
    void* q = nullptr;
    size_t got = 0;
    const hipError_t e = cache_alloc(&q, &got, count * sizeof(T));
    if (e != hipSuccess) return e;
    (temp ? ix->tmp : ix->allocs).push_back({q, got});
    *p = (T*)q;
    return hipSuccess;
}

// Waits for all work on the index's device (a query on any stream may still
// read it), then returns its blocks to the cache.
void free_index(mips_maximus_index* ix) {
    if (!ix) return;
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    if (have) (void)hipSetDevice(ix->device);
    (void)hipDeviceSynchronize();
    for (auto& q : ix->allocs) cache_release(q.first, q.second);
    for (auto& q : ix->tmp) cache_release(q.first, q.second);
    if (have) (void)hipSetDevice(cur);
    delete ix;
}

// Nearest centroid of n_u user rows (float32 MFMA); the final pass of the
// build also takes theta_b into theta_bits.
hipError_t launch_assign(const mips_maximus_index* ix, const float* U, int64_t n_u, int* assign,
                         int mode, unsigned long long* theta_bits, int* uflag, int* flist, Ctrl* ctrl,
                         hipStream_t s) {
    const bool final_pass = mode == kAssignTheta;
    AssignArgs a{};
    a.U = U;
    a.n_u = n_u;
    a.f = ix->f;
    a.ks = assign_ks(ix->f);
    a.C = ix->C;
    a.ntile = (ix->C + 31) / 32;
    a.chunk_tiles = assign_chunk_tiles(ix->f, ix->C, final_pass);
    a.stage = ix->f <= 64;
    a.lds_theta = final_pass && ix->C <= 1024;
    a.img = ix->img;
    a.assign = assign;
    a.chat = ix->chat;
    a.cnorm = ix->cnorm;
    a.theta_bits = theta_bits;
    a.theta = ix->theta;
    a.uflag = uflag;
    a.flist = flist;
    a.ctrl = ctrl;
    const size_t lds = assign_theta_bytes(ix->C, final_pass) + (size_t)a.chunk_tiles * a.ks * 256 +
                       assign_stage_bytes(ix->f);
    const int64_t n_ublk = (n_u + 31) / 32;
    const unsigned grid = (unsigned)std::min<int64_t>((n_ublk + kAssignWaves - 1) / kAssignWaves, 1024);
#define ASSIGN_LAUNCH(KS)                                                                   \
    do {                                                                                    \
        if (mode == kAssignTheta) assign_mfma_kernel<KS, kAssignTheta><<<grid, 256, lds, s>>>(a); \
        else if (mode == kAssignCover) assign_mfma_kernel<KS, kAssignCover><<<grid, 256, lds, s>>>(a); \
        else assign_mfma_kernel<KS, kAssignPlain><<<grid, 256, lds, s>>>(a);                \
    } while (0)
    if (a.ks <= 16) ASSIGN_LAUNCH(16);
    else if (a.ks <= 32) ASSIGN_LAUNCH(32);
    else if (a.ks <= 64) ASSIGN_LAUNCH(64);
    else ASSIGN_LAUNCH(132);
#undef ASSIGN_LAUNCH
    return hipGetLastError();
}

}  // namespace

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
    const int ks = assign_ks(f), ntile = (C + 31) / 32;

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
    TRY(hipMemcpyAsync(ix->I, I, (size_t)n_i * f * sizeof(float), hipMemcpyDeviceToDevice, s), "copy I");

    // ---- k-means (Section III-A) -----------------------------------------
    TRY(dalloc(ix, &ix->cent, (size_t)C * f), "alloc centroids");
    TRY(dalloc(ix, &ix->chat, (size_t)C * f), "alloc centroids");
    TRY(dalloc(ix, &ix->cnorm, (size_t)C), "alloc");
    TRY(dalloc(ix, &ix->img, (size_t)ntile * ks * 64), "alloc");
    TRY(dalloc(ix, &ix->assign, (size_t)n_u), "alloc assign");
    TRY(dalloc(ix, &ix->sorted_users, (size_t)n_u), "alloc");
    // state that starts at zero, cleared by one launch
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t z_absmax = 0, z_sums = al(4), z_counts = z_sums + al((size_t)C * f * 8),
                 z_ghist = z_counts + al((size_t)C * 4), z_end = z_ghist + al((size_t)2 * kBuckets * 4);
    TRY(dalloc(ix, &ix->theta, (size_t)C), "alloc theta");
    unsigned char* zb = nullptr;
    TRY(dalloc(ix, &zb, z_end, true), "alloc");
    unsigned int* absmax = (unsigned int*)(zb + z_absmax);
    unsigned long long* sums = (unsigned long long*)(zb + z_sums);
    unsigned int* counts = (unsigned int*)(zb + z_counts);
    unsigned int* ghist = (unsigned int*)(zb + z_ghist);
    TRY(launch_zero(zb, z_end, s), "zero");
    // the index's copy of U and max |u| (the fixed-point scale of the sums)
    copy_absmax_kernel<<<std::min(grid_of((n_u * f) / 16 + 1), 2048u), 256, 0, s>>>(U, ix->U, n_u * f, absmax);
    forgy_kernel<<<grid_of((int64_t)C * f), 256, 0, s>>>(ix->U, n_u, f, C, seed, ix->cent);
    // sums: clusters in slices whose (cluster, factor) sums fit in LDS beside
    // the assignments of up to kSumMaxRows rows (64 KB in all)
    const size_t per_c = (size_t)f * 8 + 4;
    int cs = (int)std::min<int64_t>(C, (65536 - 4 * kSumMaxRows) / per_c);
    cs = (C + (C + cs - 1) / cs - 1) / ((C + cs - 1) / cs);    // even slices
    const int nsl = (C + cs - 1) / cs;
    int64_t rows = std::min<int64_t>(kSumMaxRows, std::max<int64_t>(256, (n_u * nsl + 511) / 512));
    rows &= ~(int64_t)3;
    const unsigned sum_gx = (unsigned)((n_u + rows - 1) / rows);
    const size_t sum_lds = (size_t)cs * f * 8 + (size_t)cs * 4 + (size_t)rows * 4;
    for (int it = 0; it <= kmeans_iters; ++it) {
        const bool last = it == kmeans_iters;
        cent_prep_kernel<<<ntile, 256, f <= 254 ? (size_t)32 * f * 8 : 0, s>>>(
            ix->cent, C, f, ks, ix->img, ix->cnorm, ix->chat, counts, last ? ix->theta : nullptr);
        // the final assignment also gives theta_b (Algorithm 1, ConstructIndex)
        TRY(launch_assign(ix, ix->U, n_u, ix->assign, last ? kAssignTheta : kAssignPlain,
                          (unsigned long long*)ix->theta, nullptr, nullptr, nullptr, s), "assignment");
        if (last) break;
        kmeans_sum_kernel<<<dim3(sum_gx, nsl), 256, sum_lds, s>>>(ix->U, n_u, f, ix->assign, absmax, rows,
                                                                 cs, sums, counts, C);
        kmeans_update_kernel<<<grid_of((int64_t)C * f), 256, 0, s>>>(ix->cent, C, f, sums, counts, absmax, n_u);
    }
    theta_fix_kernel<<<grid_of(C), 256, 0, s>>>(ix->cnorm, C, ix->theta);
    TRY(hipGetLastError(), "k-means");

    // ---- bounds and per-cluster lists --------------------------------------
    {
        uint32_t *k0 = nullptr, *k1 = nullptr;
        int *v0 = nullptr, *v1 = nullptr;
        const size_t tot = (size_t)C * n_i;
        TRY(dalloc(ix, &k0, tot, true), "alloc keys");
        TRY(dalloc(ix, &k1, tot, true), "alloc keys");
        TRY(dalloc(ix, &v0, tot, true), "alloc vals");
        TRY(dalloc(ix, &v1, tot, true), "alloc vals");
        const unsigned nbx = grid_of(n_i);
        const int want = std::max(1, std::min(C, 1024 / (int)nbx));
        const int bcs = (C + want - 1) / want;
        const unsigned bsl = (unsigned)((C + bcs - 1) / bcs);
        const int F = f <= 16 ? 16 : (f <= 32 ? 32 : (f <= 64 ? 64 : 0));
        const size_t blds = F ? (size_t)256 * f * 4 : 0;
        const dim3 bg(nbx, bsl);
        switch (F) {
            case 16: bound_kernel<16><<<bg, 256, blds, s>>>(ix->I, n_i, f, ix->chat, ix->cnorm, ix->theta, C, bcs, k0); break;
            case 32: bound_kernel<32><<<bg, 256, blds, s>>>(ix->I, n_i, f, ix->chat, ix->cnorm, ix->theta, C, bcs, k0); break;
            case 64: bound_kernel<64><<<bg, 256, blds, s>>>(ix->I, n_i, f, ix->chat, ix->cnorm, ix->theta, C, bcs, k0); break;
            default: bound_kernel<0><<<bg, 256, 0, s>>>(ix->I, n_i, f, ix->chat, ix->cnorm, ix->theta, C, bcs, k0); break;
        }
        TRY(hipGetLastError(), "bounds");
        TRY(dalloc(ix, &ix->lists, (size_t)C * ix->n_i_pad), "alloc lists");
        TRY(dalloc(ix, &ix->lbound, (size_t)C * ix->n_i_pad), "alloc bounds");
        const int P = (int)std::max<int64_t>(1, std::min<int64_t>(512 / C, (n_i + 1023) / 1024));
        const int64_t part = (n_i + P - 1) / P;
        unsigned int* rh = nullptr;
        TRY(dalloc(ix, &rh, (size_t)C * 256 * P, true), "alloc");
        const dim3 rg(P, C);
        radix_hist_kernel<<<rg, 256, 0, s>>>(k0, n_i, part, 0, rh);
        radix_scatter_kernel<true, false><<<rg, 1024, 0, s>>>(k0, nullptr, k1, v1, n_i, part, 0, rh, nullptr, nullptr, 0);
        radix_hist_kernel<<<rg, 256, 0, s>>>(k1, n_i, part, 8, rh);
        radix_scatter_kernel<false, false><<<rg, 1024, 0, s>>>(k1, v1, k0, v0, n_i, part, 8, rh, nullptr, nullptr, 0);
        radix_hist_kernel<<<rg, 256, 0, s>>>(k0, n_i, part, 16, rh);
        radix_scatter_kernel<false, false><<<rg, 1024, 0, s>>>(k0, v0, k1, v1, n_i, part, 16, rh, nullptr, nullptr, 0);
        radix_hist_kernel<<<rg, 256, 0, s>>>(k1, n_i, part, 24, rh);
        radix_scatter_kernel<false, true><<<rg, 1024, 0, s>>>(k1, v1, nullptr, nullptr, n_i, part, 24, rh,
                                                              ix->lists, ix->lbound, ix->n_i_pad);
        TRY(hipGetLastError(), "lists");
    }

    // ---- users grouped by the final assignment ------------------------------
    {
        const int nch = (int)((n_u + kGroupChunk - 1) / kGroupChunk);
        unsigned int* ccounts = nullptr;
        TRY(dalloc(ix, &ccounts, (size_t)C * nch, true), "alloc");
        group_count_kernel<<<nch, 256, 0, s>>>(ix->assign, n_u, C, nch, ccounts);
        group_scan_kernel<<<C, 64, 0, s>>>(ccounts, nch, ghist);
        TRY(launch_scan4096(ghist, s), "scan");
        group_scatter_kernel<<<nch, 64, 0, s>>>(ix->assign, n_u, C, nch, ccounts, ghist + kBuckets,
                                                ix->sorted_users);
        TRY(hipGetLastError(), "user grouping");
    }

    // ---- screen copies of the items for every precision --------------------
    {
        Ctrl* tctrl = nullptr;
        float* Etmp = nullptr;
        TRY(dalloc(ix, &tctrl, 3), "alloc");
        ix->prep_ctrl = tctrl;
        TRY(dalloc(ix, &Etmp, (size_t)n_i, true), "alloc");
        TRY(dalloc(ix, &ix->kexp, (size_t)n_i), "alloc");
        TRY(launch_zero(tctrl, 3 * sizeof(Ctrl), s), "zero");
        BlockMaxArgs bm{};
        bm.lists = ix->lists;
        bm.n_i = n_i;
        bm.n_i_pad = ix->n_i_pad;
        bm.n_blk = ix->n_blk;
        bm.C = C;
        float4* cg4 = nullptr;
        TRY(dalloc(ix, &cg4, (size_t)n_i, true), "alloc");
        bm.cg4 = cg4;
        bool any = false;
        ItemPrepArgs ias[3] = {};
        const ItemPrepArgs* iap[3] = {nullptr, nullptr, nullptr};
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
            ItemPrepArgs& ia = ias[prec];
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
                iap[prec] = &ia;
                bm.Corig = ix->Corig[prec];
                bm.Gorig[prec] = ix->Gorig[prec];
                bm.out[prec] = ix->cblockmax[prec];
                any = true;
            } else if (prec == 0) {
                // no screen for these sizes (every query takes the exact path):
                // only the finiteness check of I is needed
                TRY(launch_nonfinite_scan(ix->I, 0, ix->I, n_i * f, tctrl, s), "finite check");
            }
        }
        if (any) {
            TRY(launch_item_stats3(iap, s), "item screen copies");
            item_cg4_kernel<<<grid_of(n_i), 256, 0, s>>>(bm);
            cblockmax_kernel<<<grid_of((int64_t)C * ix->n_blk), 256, 0, s>>>(bm);
            TRY(hipGetLastError(), "tile maxima");
            // walk prefix tiles: at most kWalkPrefixBytes per precision
            for (int prec = 0; prec < 3; ++prec) {
                if (!iap[prec]) continue;
                const size_t op = prec == PREC_FP32 ? 4 : (prec == PREC_BF16 ? 16 : 32);
                const size_t tile_bytes = (size_t)iap[prec]->nch * kWave * op;
                const int64_t fit = (int64_t)(kWalkPrefixBytes / (tile_bytes * (size_t)C));
                const int wpre = (int)std::min<int64_t>(ix->n_blk, std::max<int64_t>(1, fit));
                unsigned char* pk = nullptr;
                TRY(dalloc(ix, &pk, (size_t)C * wpre * tile_bytes), "alloc prefix tiles");
                TRY(dalloc(ix, &ix->wcg[prec], (size_t)C * wpre * kTile), "alloc");
                if (prec == PREC_FP8) TRY(dalloc(ix, &ix->wscale, (size_t)C * wpre * kTile), "alloc");
                ix->wpre[prec] = wpre;
                ix->wpacked[prec] = pk;
                WalkPackArgs wa{};
                wa.lists = ix->lists;
                wa.n_i_pad = ix->n_i_pad;
                wa.wpre = wpre;
                wa.f_pad = iap[prec]->f_pad;
                wa.nch = iap[prec]->nch;
                wa.qrow = ix->qrow[prec];
                wa.kexp = ix->kexp;
                wa.Corig = ix->Corig[prec];
                wa.Gorig = ix->Gorig[prec];
                wa.packed = pk;
                wa.cg = ix->wcg[prec];
                wa.scale = prec == PREC_FP8 ? ix->wscale : nullptr;
                TRY(launch_walk_pack(prec, wa, C, s), "walk prefix tiles");
            }
        }
    }

    // ---- walk tiles: runs of up to 32*UB users of one cluster --------------
    {
        unsigned int* toff = nullptr;
        TRY(dalloc(ix, &toff, (size_t)3 * (kBuckets + 1), true), "alloc");
        tile_offsets_kernel<<<1, 1024, 0, s>>>(ghist, C, toff);
        TileEmitArgs ta{};
        ta.ccount = ghist;
        ta.cstart = ghist + kBuckets;
        ta.toff = toff;
        ta.C = C;
        int64_t most = 0;
        for (int q = 0; q < 3; ++q) {
            const int64_t span = (int64_t)kTile << q;
            ix->ntiles[q] = (n_u + span - 1) / span + C;
            TRY(dalloc(ix, &ix->tiles[q], (size_t)ix->ntiles[q]), "alloc tiles");
            ta.max_tiles[q] = ix->ntiles[q];
            ta.tiles[q] = ix->tiles[q];
            most = std::max(most, ix->ntiles[q]);
        }
        tiles_emit_kernel<<<dim3(grid_of(most), 3), 256, 0, s>>>(ta);
        TRY(hipGetLastError(), "walk tiles");
    }

    // ---- the one host check: NaN or Inf in I --------------------------------
    {
        Ctrl h[3];
        TRY(hipMemcpyAsync(h, ix->prep_ctrl, sizeof(h), hipMemcpyDeviceToHost, s), "read flags");
        TRY(hipStreamSynchronize(s), "sync");
        for (int prec = 0; prec < 3; ++prec) {
            if (h[prec].nonfinite) {
                free_index(ix);
                return fail(MIPS_ERR_NONFINITE, "I holds NaN or Inf");
            }
        }
    }
    // the stream has finished with the temporaries
    for (auto& q : ix->tmp) cache_release(q.first, q.second);
    ix->tmp.clear();
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
    copy_maxima_kernel<<<1, 64, 0, s>>>(ctrl, ix->prep_ctrl + precision);
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
    a.wpre = ix->wpre[precision];
    a.wpacked = ix->wpacked[precision];
    a.wcg = ix->wcg[precision];
    a.wscale = ix->wscale;
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
    a.cand_lm = !fused_certify(p.prec, p.KM, p.UB);          // the layout the screen kernel writes
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
    size_t ctrl, uflag, ccount, zero_end;
    size_t toff, tiles, flist, uscal, qassign, sorted, ccounts, cnt, cand, fbkeys, total;
    int64_t max_tiles;
    int nch;
};

QueryLayout query_layout(const mips_maximus_index* ix, const ScreenPlan& p, int64_t n_q) {
    QueryLayout L{};
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o += (b + 255) & ~(size_t)255; return r; };
    const int span = kTile * p.UB;
    L.max_tiles = p.fast ? (n_q + span - 1) / span + ix->C : 0;
    const int64_t n_ublk = L.max_tiles * p.UB;
    L.nch = (int)((n_q + kGroupChunk - 1) / kGroupChunk);
    L.ctrl = take(sizeof(Ctrl));
    L.uflag = take((size_t)n_q * 4);
    L.ccount = take(2 * kBuckets * sizeof(unsigned int));      // cluster sizes, then starts
    L.zero_end = o;
    L.toff = take(3 * (kBuckets + 1) * sizeof(unsigned int));
    L.tiles = take((size_t)std::max<int64_t>(L.max_tiles, 1) * sizeof(int4));
    L.flist = take((size_t)n_q * 4);
    L.uscal = take((size_t)n_q * 16);
    L.qassign = take((size_t)n_q * 4);
    L.sorted = take((size_t)n_q * 4);
    L.ccounts = take((size_t)ix->C * L.nch * sizeof(unsigned int));
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

// ---------------------------------------------------------------------------
// Queries for arbitrary user vectors (new users, or any subset).  A vector
// may use cluster c's list when its angle to the centroid is at most
// theta_b[c]: the bound of Eq. (appx_bound) only needs theta_uc <= theta_b
// (Section III-C), so such a vector is covered exactly like a member.  Each
// vector tries its nearest centroid; the others take the exact path.
// ---------------------------------------------------------------------------
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
    unsigned int* toff = (unsigned int*)(ws + L.toff);       // tile offsets per span
    unsigned int* ccounts = (unsigned int*)(ws + L.ccounts);
    int4* tiles = (int4*)(ws + L.tiles);
    int* flist = (int*)(ws + L.flist);
    float4* uscal = (float4*)(ws + L.uscal);
    int* qassign = (int*)(ws + L.qassign);
    int* sorted = (int*)(ws + L.sorted);
    hipError_t e;
    if ((e = launch_zero(ws, L.zero_end, s)) != hipSuccess) return hip_fail(e, "zero");
    if (p.fast) {
        PhaseTimer t(MIPS_PHASE_WALK, s);
        const int C = ix->C;
        // nearest cluster and its cover test in one pass
        if ((e = launch_assign(ix, Uq, n_q, qassign, kAssignCover, nullptr, uflag, flist, ctrl, s)) != hipSuccess)
            return hip_fail(e, "assignment");
        // covered vectors grouped by cluster (stable), then their walk tiles
        group_count_kernel<<<L.nch, 256, 0, s>>>(qassign, n_q, C, L.nch, ccounts);
        group_scan_kernel<<<C, 64, 0, s>>>(ccounts, L.nch, ccount);
        if ((e = launch_scan4096(ccount, s)) != hipSuccess) return hip_fail(e, "scan");
        group_scatter_kernel<<<L.nch, 64, 0, s>>>(qassign, n_q, C, L.nch, ccounts, ccount + kBuckets, sorted);
        tile_offsets_kernel<<<1, 1024, 0, s>>>(ccount, C, toff);
        TileEmitArgs ta{};
        ta.ccount = ccount;
        ta.cstart = ccount + kBuckets;
        ta.toff = toff;
        ta.C = C;
        const int slot = ub_slot(p.UB);
        ta.max_tiles[slot] = L.max_tiles;
        ta.tiles[slot] = tiles;
        tiles_emit_kernel<<<dim3(grid_of(L.max_tiles), 3), 256, 0, s>>>(ta);
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
