// Item preparation for the screen: per-item norms and screen copies, a
// descending-norm item order, and the item tiles packed in matrix-core
// operand order with per-tile bound maxima.
//
// Why a norm order: the paper's brute force scores items in storage order
// (Section II-C).  Here the items are streamed in roughly descending ||i||
// so that each user's K-th best score is found early; after that almost no
// score of a 32 x 32 tile can reach it and the fused top-K stays on its fast
// path.  The order changes speed only: the final order is decided by the
// float64 keys and the original item index.
#include "device_common.h"
#include "internal.h"

namespace mips {

__global__ void zero_kernel(uint4* p, size_t n16) {
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

__global__ void zero_tail_kernel(unsigned char* p, size_t n) {
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Zero `bytes` bytes at p (p 16-byte aligned): whole 16-byte words first,
// then the tail byte by byte, so nothing past p + bytes is touched.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    const size_t n16 = bytes / 16;
    if (n16) {
        size_t blocks = (n16 + 255) / 256;
        if (blocks > 4096) blocks = 4096;
        zero_kernel<<<dim3((unsigned)blocks), dim3(256), 0, s>>>((uint4*)p, n16);
    }
    const size_t tail = bytes - n16 * 16;
    if (tail) zero_tail_kernel<<<dim3(1), dim3(16), 0, s>>>((unsigned char*)p + n16 * 16, tail);
    return hipGetLastError();
}

// Sixteen lanes per item (lane q takes factors q, q+16, ...; f_pad <= 128):
// float64 norms of the row, of its screen copy and of the residual, the
// descending-norm bucket, and the global maxima (reduced over the wave, one
// atomic per wave).  The order of the float64 partial sums only moves the
// last bits; every norm is rounded up and the per-user slack covers the rest.
constexpr int kPrepLanes = 16;
constexpr int kPrepPer = 128 / kPrepLanes;      // factors per lane at f_pad = 128

// Screen copy, norms and bucket of item i for precision PREC from its
// factors x (lane q of the item's 16 holds factors q, q + 16, ...), whose
// float64 sum of squares s2, largest magnitude and finiteness are already
// reduced over the 16 lanes; (C, E, G) raise the running maxima.
template <int PREC>
__device__ __forceinline__ void item_stats_one(const ItemPrepArgs& a, int64_t i, bool on, int q,
                                               const float (&x)[kPrepPer], double s2, float amax,
                                               bool finite, unsigned int& cb, unsigned int& eb,
                                               unsigned int& gb) {
    int k = 0;
    if (PREC == PREC_FP8) k = e4m3_row_scale_exp(amax);
    double r2 = 0.0, q2 = 0.0;
#pragma unroll
    for (int e = 0; e < kPrepPer; ++e) {
        const int j = q + e * kPrepLanes;
        if (!on || j >= a.f_pad) continue;
        if (PREC == PREC_FP32) {
            ((float*)a.qrow)[i * a.f_pad + j] = x[e];
        } else if (PREC == PREC_BF16) {
            const uint16_t hb = f32_to_bf16_bits(x[e]);
            const double d = (double)bf16_bits_to_f32(hb);
            r2 += ((double)x[e] - d) * ((double)x[e] - d);
            q2 += d * d;
            ((uint16_t*)a.qrow)[i * a.f_pad + j] = hb;
        } else {
            const uint32_t b = e4m3_encode(__builtin_ldexpf(x[e], -k));
            const double d = __builtin_ldexp((double)e4m3_decode(b), k);
            r2 += ((double)x[e] - d) * ((double)x[e] - d);
            q2 += d * d;
            ((uint8_t*)a.qrow)[i * a.f_pad + j] = (uint8_t)b;
        }
    }
    if (PREC == PREC_FP32) {
        q2 = s2;
    } else {
        for (int off = kPrepLanes / 2; off >= 1; off >>= 1) {
            r2 += __shfl_xor(r2, off, kPrepLanes);
            q2 += __shfl_xor(q2, off, kPrepLanes);
        }
    }
    float C = norm_up_f32(sqrt(s2));
    float E = norm_up_f32(sqrt(q2));
    float G = (PREC == PREC_FP32) ? 0.0f : norm_up_f32(sqrt(r2) + (double)a.gamma * sqrt(q2));
    if (!finite || !on) { C = 0.0f; E = 0.0f; G = 0.0f; }
    if (on && q == 0) {
        if (PREC == PREC_FP8) a.kexp[i] = k;
        a.Corig[i] = C;
        a.Gorig[i] = G;
        a.Eorig[i] = E;
        if (!finite) atomicOr(&a.ctrl->nonfinite, 1u);
        if (a.bucket) {
            // descending ||i||: 16 buckets per octave from the float bits
            int bk = (kBuckets - 1) - (int)(__float_as_uint(C) >> 19);
            bk = bk < 0 ? 0 : (bk >= kBuckets ? kBuckets - 1 : bk);
            a.bucket[i] = bk;
        }
    }
    // all values are >= 0, so their bit patterns order as integers
    cb = max(cb, __float_as_uint(C));
    eb = max(eb, __float_as_uint(E));
    gb = max(gb, __float_as_uint(G));
}

// Item i's factors for its 16 lanes and their float64 sum of squares,
// largest magnitude and finiteness, reduced over the 16 lanes.
__device__ __forceinline__ void item_load(const ItemPrepArgs& a, int64_t i, bool on, int q,
                                          float (&x)[kPrepPer], double& s2, float& amax,
                                          bool& finite) {
    const float* row = a.I + (on ? i : 0) * a.f;
    s2 = 0.0;
    amax = 0.0f;
    finite = true;
#pragma unroll
    for (int e = 0; e < kPrepPer; ++e) {
        const int j = q + e * kPrepLanes;
        x[e] = (on && j < a.f) ? row[j] : 0.0f;
        finite = finite && __builtin_isfinite(x[e]);
        s2 += (double)x[e] * (double)x[e];
        amax = fmaxf(amax, fabsf(x[e]));
    }
    for (int off = kPrepLanes / 2; off >= 1; off >>= 1) {
        s2 += __shfl_xor(s2, off, kPrepLanes);
        amax = fmaxf(amax, __shfl_xor(amax, off, kPrepLanes));
        // every lane must take part in the exchange (no short-circuit)
        const int fp = __shfl_xor((int)finite, off, kPrepLanes);
        finite = finite && (fp != 0);
    }
}

// The global maxima are reduced over the whole workgroup (one atomic per
// workgroup and value: same-address atomics serialise).
__device__ __forceinline__ void item_maxima_flush(Ctrl* ctrl, unsigned int cb, unsigned int eb,
                                                  unsigned int gb, unsigned int (&smax)[3][4]) {
    for (int off = 32; off >= 1; off >>= 1) {
        cb = max(cb, (unsigned int)__shfl_xor((int)cb, off));
        eb = max(eb, (unsigned int)__shfl_xor((int)eb, off));
        gb = max(gb, (unsigned int)__shfl_xor((int)gb, off));
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        smax[0][wv] = cb;
        smax[1][wv] = eb;
        smax[2][wv] = gb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int m[3];
        for (int v = 0; v < 3; ++v)
            m[v] = max(max(smax[v][0], smax[v][1]), max(smax[v][2], smax[v][3]));
        atomicMax(&ctrl->cmax_bits, m[0]);
        atomicMax(&ctrl->emax_bits, m[1]);
        atomicMax(&ctrl->gmax_bits, m[2]);
    }
    __syncthreads();
}

template <int PREC>
__global__ void __launch_bounds__(256) item_stats_kernel(ItemPrepArgs a) {
    __shared__ unsigned int smax[3][4];
    const int q = threadIdx.x & (kPrepLanes - 1);
    unsigned int cb = 0u, eb = 0u, gb = 0u;
    for (int64_t base = (int64_t)blockIdx.x * (256 / kPrepLanes); base < a.n_i;
         base += (int64_t)gridDim.x * (256 / kPrepLanes)) {
        const int64_t i = base + threadIdx.x / kPrepLanes;
        const bool on = i < a.n_i;
        float x[kPrepPer];
        double s2;
        float amax;
        bool finite;
        item_load(a, i, on, q, x, s2, amax, finite);
        item_stats_one<PREC>(a, i, on, q, x, s2, amax, finite, cb, eb, gb);
    }
    item_maxima_flush(a.ctrl, cb, eb, gb, smax);
}

// The three screen precisions of the same items in one pass over I (a
// Maximus index keeps all three); `mask` bit p enables precision p.
__global__ void __launch_bounds__(256) item_stats3_kernel(ItemPrepArgs a0, ItemPrepArgs a1,
                                                          ItemPrepArgs a2, int mask) {
    __shared__ unsigned int smax[3][4];
    const int q = threadIdx.x & (kPrepLanes - 1);
    unsigned int cb[3] = {0u, 0u, 0u}, eb[3] = {0u, 0u, 0u}, gb[3] = {0u, 0u, 0u};
    for (int64_t base = (int64_t)blockIdx.x * (256 / kPrepLanes); base < a0.n_i;
         base += (int64_t)gridDim.x * (256 / kPrepLanes)) {
        const int64_t i = base + threadIdx.x / kPrepLanes;
        const bool on = i < a0.n_i;
        float x[kPrepPer];
        double s2;
        float amax;
        bool finite;
        item_load(a0, i, on, q, x, s2, amax, finite);
        if (mask & 1) item_stats_one<PREC_FP32>(a0, i, on, q, x, s2, amax, finite, cb[0], eb[0], gb[0]);
        if (mask & 2) item_stats_one<PREC_BF16>(a1, i, on, q, x, s2, amax, finite, cb[1], eb[1], gb[1]);
        if (mask & 4) item_stats_one<PREC_FP8>(a2, i, on, q, x, s2, amax, finite, cb[2], eb[2], gb[2]);
    }
    if (mask & 1) item_maxima_flush(a0.ctrl, cb[0], eb[0], gb[0], smax);
    if (mask & 2) item_maxima_flush(a1.ctrl, cb[1], eb[1], gb[1], smax);
    if (mask & 4) item_maxima_flush(a2.ctrl, cb[2], eb[2], gb[2], smax);
}

// Exclusive scan of the bucket counts (one workgroup of 1024 threads).
__global__ void __launch_bounds__(1024) bucket_scan_kernel(unsigned int* hist) {
    __shared__ unsigned int part[1024];
    int t = threadIdx.x;
    unsigned int v[4];
    unsigned int sum = 0;
    for (int q = 0; q < 4; ++q) { v[q] = hist[t * 4 + q]; sum += v[q]; }
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        unsigned int add = (t >= off) ? part[t - off] : 0u;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    unsigned int run = part[t] - sum;   // exclusive prefix of this thread's group
    for (int q = 0; q < 4; ++q) { hist[kBuckets + t * 4 + q] = run; run += v[q]; }
}

// Bucket counts: each workgroup counts its 256 items in LDS and adds the
// non-zero counts to the global histogram (one atomic per bucket and
// workgroup instead of one per item on a few hot buckets).
__global__ void __launch_bounds__(256) bucket_count_kernel(ItemPrepArgs a) {
    __shared__ unsigned int lh[kBuckets];
    for (int t = threadIdx.x; t < kBuckets; t += blockDim.x) lh[t] = 0u;
    __syncthreads();
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < a.n_i) atomicAdd(&lh[a.bucket[i]], 1u);
    __syncthreads();
    for (int t = threadIdx.x; t < kBuckets; t += blockDim.x)
        if (lh[t]) atomicAdd(&a.hist[t], lh[t]);
}

// Scatter into bucket order: ranks within the workgroup from LDS atomics,
// one global atomic per bucket and workgroup reserves the range.  The order
// inside a bucket is arbitrary (it changes speed only).
__global__ void __launch_bounds__(256) bucket_scatter_kernel(ItemPrepArgs a) {
    __shared__ unsigned int lh[kBuckets];
    for (int t = threadIdx.x; t < kBuckets; t += blockDim.x) lh[t] = 0u;
    __syncthreads();
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int bk = i < a.n_i ? a.bucket[i] : 0;
    unsigned int local = 0;
    if (i < a.n_i) local = atomicAdd(&lh[bk], 1u);
    __syncthreads();
    for (int t = threadIdx.x; t < kBuckets; t += blockDim.x)
        if (lh[t]) lh[t] = atomicAdd(&a.hist[kBuckets + t], lh[t]);
    __syncthreads();
    if (i < a.n_i) a.perm[lh[bk] + local] = (int)i;
}

// One 64-thread workgroup per item tile: copy the 32 items' screen rows into
// operand order (lane l = row l%32, half l/32 of the factors, chunk c) and
// reduce the tile maxima of C and G.
template <int PREC>
__global__ void __launch_bounds__(64) item_pack_kernel(ItemPrepArgs a) {
    const int64_t b = blockIdx.x;
    const int lane = threadIdx.x, m = lane & 31, h = lane >> 5;
    const int64_t p = b * kTile + m;
    const int item = (p < a.n_i) ? a.perm[p] : -1;
    if (p >= a.n_i && h == 0) a.perm[p] = -1;   // padded positions: no item
    const int half = a.f_pad / 2;
    if (PREC == PREC_BF16) {
        const uint4* src = (const uint4*)a.qrow;
        uint4* dst = (uint4*)a.packed;
        for (int c = 0; c < a.nch; ++c) {
            uint4 v = make_uint4(0, 0, 0, 0);
            if (item >= 0) v = src[((int64_t)item * a.f_pad + h * half + c * 8) / 8];
            dst[(b * a.nch + c) * kWave + lane] = v;
        }
    } else if (PREC == PREC_FP8) {
        const uint4* src = (const uint4*)a.qrow;
        uint4* dst = (uint4*)a.packed;
        for (int c = 0; c < a.nch; ++c) {
            uint4 v0 = make_uint4(0, 0, 0, 0), v1 = v0;
            if (item >= 0) {
                int64_t o = ((int64_t)item * a.f_pad + h * half + c * 32) / 16;
                v0 = src[o];
                v1 = src[o + 1];
            }
            int64_t d = ((b * a.nch + c) * kWave + lane) * 2;
            dst[d] = v0;
            dst[d + 1] = v1;
        }
        if (h == 0) a.pscale[p] = (item >= 0 ? a.kexp[item] : 0) + 127;
    } else {
        const float* src = (const float*)a.qrow;
        float* dst = (float*)a.packed;
        for (int c = 0; c < a.nch; ++c) {
            float v = 0.0f;
            if (item >= 0) v = src[(int64_t)item * a.f_pad + h * half + c];
            dst[(b * a.nch + c) * kWave + lane] = v;
        }
    }
    float cm = (item >= 0) ? a.Corig[item] : 0.0f;
    float gm = (item >= 0) ? a.Gorig[item] : 0.0f;
    if (a.cgpos && h == 0) a.cgpos[p] = make_float4(cm, gm, __int_as_float(item), 0.0f);
    for (int off = 16; off >= 1; off >>= 1) {
        cm = fmaxf(cm, __shfl_xor(cm, off));
        gm = fmaxf(gm, __shfl_xor(gm, off));
    }
    if (lane == 0) a.blockmax[b] = make_float2(cm, gm);
}

// Walk prefix tiles: tile t of cluster c holds list entries t 32 .. t 32 + 31
// in the layout of item_pack_kernel (one workgroup of 64 lanes per tile).
template <int PREC>
__global__ void __launch_bounds__(64) walk_pack_kernel(WalkPackArgs a) {
    const int t = blockIdx.x, c = blockIdx.y;
    const int lane = threadIdx.x, m = lane & 31, h = lane >> 5;
    const int64_t p = (int64_t)t * kTile + m;
    const int item = a.lists[(int64_t)c * a.n_i_pad + p];
    const int64_t tile = (int64_t)c * a.wpre + t;
    const int half = a.f_pad / 2;
    if (PREC == PREC_BF16) {
        const uint4* src = (const uint4*)a.qrow;
        uint4* dst = (uint4*)a.packed;
        for (int cc = 0; cc < a.nch; ++cc) {
            uint4 v = make_uint4(0, 0, 0, 0);
            if (item >= 0) v = src[((int64_t)item * a.f_pad + h * half + cc * 8) / 8];
            dst[(tile * a.nch + cc) * kWave + lane] = v;
        }
    } else if (PREC == PREC_FP8) {
        const uint4* src = (const uint4*)a.qrow;
        uint4* dst = (uint4*)a.packed;
        for (int cc = 0; cc < a.nch; ++cc) {
            uint4 v0 = make_uint4(0, 0, 0, 0), v1 = v0;
            if (item >= 0) {
                const int64_t o = ((int64_t)item * a.f_pad + h * half + cc * 32) / 16;
                v0 = src[o];
                v1 = src[o + 1];
            }
            const int64_t d = ((tile * a.nch + cc) * kWave + lane) * 2;
            dst[d] = v0;
            dst[d + 1] = v1;
        }
        if (h == 0) a.scale[tile * kTile + m] = (item >= 0 ? a.kexp[item] : 0) + 127;
    } else {
        const float* src = (const float*)a.qrow;
        float* dst = (float*)a.packed;
        for (int cc = 0; cc < a.nch; ++cc) {
            float v = 0.0f;
            if (item >= 0) v = src[(int64_t)item * a.f_pad + h * half + cc];
            dst[(tile * a.nch + cc) * kWave + lane] = v;
        }
    }
    if (h == 0)
        a.cg[tile * kTile + m] = item >= 0 ? make_float2(a.Corig[item], a.Gorig[item]) : make_float2(0.0f, 0.0f);
}

hipError_t launch_walk_pack(int prec, const WalkPackArgs& a, int C, hipStream_t s) {
    if (a.wpre <= 0) return hipSuccess;
    const dim3 g((unsigned)a.wpre, (unsigned)C);
    switch (prec) {
        case PREC_FP32: walk_pack_kernel<PREC_FP32><<<g, 64, 0, s>>>(a); break;
        case PREC_BF16: walk_pack_kernel<PREC_BF16><<<g, 64, 0, s>>>(a); break;
        default: walk_pack_kernel<PREC_FP8><<<g, 64, 0, s>>>(a); break;
    }
    return hipGetLastError();
}

__global__ void nonfinite_scan_kernel(const float* U, int64_t nu, const float* I, int64_t ni,
                                      Ctrl* ctrl) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (int64_t j = i; j < nu; j += stride) bad = bad || !__builtin_isfinite(U[j]);
    for (int64_t j = i; j < ni; j += stride) bad = bad || !__builtin_isfinite(I[j]);
    if (bad) atomicOr(&ctrl->nonfinite, 1u);
}

// Suffix maxima of the per-tile norm maxima (one 1024-thread workgroup:
// each thread owns a contiguous run of tiles).
__global__ void __launch_bounds__(1024) tailmax_kernel(const float2* blockmax, int64_t n_blk,
                                                       float* tailmax) {
    __shared__ float part[1024];
    const int t = threadIdx.x;
    const int64_t per = (n_blk + 1023) / 1024;
    const int64_t lo = t * per, hi = lo + per < n_blk ? lo + per : n_blk;
    float m = 0.0f;
    for (int64_t b = lo; b < hi; ++b) m = fmaxf(m, blockmax[b].x);
    part[t] = m;
    __syncthreads();
    // inclusive suffix max over the threads' runs (Hillis-Steele), then
    // exclusive by reading the next thread's entry
    for (int off = 1; off < 1024; off <<= 1) {
        const float o = (t + off < 1024) ? part[t + off] : 0.0f;
        __syncthreads();
        part[t] = fmaxf(part[t], o);
        __syncthreads();
    }
    float after = (t + 1 < 1024) ? part[t + 1] : 0.0f;
    for (int64_t b = hi - 1; b >= lo; --b) {
        after = fmaxf(after, blockmax[b].x);
        tailmax[b] = after;
    }
}

hipError_t launch_tailmax(const float2* blockmax, int64_t n_blk, float* tailmax, hipStream_t s) {
    tailmax_kernel<<<1, 1024, 0, s>>>(blockmax, n_blk, tailmax);
    return hipGetLastError();
}

// Exclusive scan of 4096 counts at hist[0..4096) into hist[4096..8192).
hipError_t launch_scan4096(unsigned int* hist, hipStream_t s) {
    bucket_scan_kernel<<<1, 1024, 0, s>>>(hist);
    return hipGetLastError();
}

hipError_t launch_nonfinite_scan(const float* U, int64_t nu_elems, const float* I,
                                 int64_t ni_elems, Ctrl* ctrl, hipStream_t s) {
    nonfinite_scan_kernel<<<dim3(1024), dim3(256), 0, s>>>(U, nu_elems, I, ni_elems, ctrl);
    return hipGetLastError();
}

hipError_t launch_item_stats3(const ItemPrepArgs* const (&a)[3], hipStream_t s) {
    int mask = 0;
    const ItemPrepArgs* any = nullptr;
    for (int p = 0; p < 3; ++p) {
        if (!a[p]) continue;
        if (a[p]->f_pad > 128 || a[p]->f > a[p]->f_pad) return hipErrorInvalidValue;
        mask |= 1 << p;
        any = a[p];
    }
    if (!any) return hipSuccess;
    const int64_t groups = (any->n_i + 256 / kPrepLanes - 1) / (256 / kPrepLanes);
    const unsigned ns = (unsigned)(groups < 256 ? groups : 256);
    item_stats3_kernel<<<ns, 256, 0, s>>>(a[0] ? *a[0] : *any, a[1] ? *a[1] : *any, a[2] ? *a[2] : *any,
                                          mask);
    return hipGetLastError();
}

hipError_t launch_item_prep(int prec, const ItemPrepArgs& a, bool pack, hipStream_t s) {
    const unsigned nb = (unsigned)((a.n_i + 255) / 256);
    if (a.f_pad > 128 || a.f > a.f_pad) return hipErrorInvalidValue;
    // at most 256 workgroups, each striding over the items 16 at a time
    const int64_t groups = (a.n_i + 256 / kPrepLanes - 1) / (256 / kPrepLanes);
    const unsigned ns = (unsigned)(groups < 256 ? groups : 256);
    switch (prec) {
        case PREC_FP32: item_stats_kernel<PREC_FP32><<<ns, 256, 0, s>>>(a); break;
        case PREC_BF16: item_stats_kernel<PREC_BF16><<<ns, 256, 0, s>>>(a); break;
        default: item_stats_kernel<PREC_FP8><<<ns, 256, 0, s>>>(a); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !pack) return e;
    bucket_count_kernel<<<nb, 256, 0, s>>>(a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    bucket_scan_kernel<<<1, 1024, 0, s>>>(a.hist);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    bucket_scatter_kernel<<<nb, 256, 0, s>>>(a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const unsigned tiles = (unsigned)a.n_blk;
    switch (prec) {
        case PREC_FP32: item_pack_kernel<PREC_FP32><<<tiles, 64, 0, s>>>(a); break;
        case PREC_BF16: item_pack_kernel<PREC_BF16><<<tiles, 64, 0, s>>>(a); break;
        default: item_pack_kernel<PREC_FP8><<<tiles, 64, 0, s>>>(a); break;
    }
    return hipGetLastError();
}

}  // namespace mips
