// Score tiles on the matrix cores fused with a per-user streaming top-K
// (the brute force of paper Section II-C and the blocked walk of Maximus,
// Section III-C/III-D), then certification with a float64 rescore, and the
// exact float64 fallback.
//
// Tile layout.  One wave owns UB blocks of 32 users for the whole item sweep.
// A 32x32 output tile has items as rows (operand A) and users as columns
// (operand B), so lane l of the wave holds user l%32 and the 16 items
// {8g + 4*(l/32) + q : g, q = 0..3} of the tile.  Both operands are indexed
// the same way over the factors: lane half h = l/32 owns the contiguous
// factor range [h*f_pad/2, (h+1)*f_pad/2), chunk c the next E of them.
//
// Streaming top-K.  Each lane keeps a register list of the KM largest lower
// bounds it has seen (K real slots below KM-K +inf pads, so the last entry is
// its K-th largest), and tau_u = max over the user's two lanes of that entry
// is a valid lower bound on the user's K-th largest key.  Per tile a lane
// takes the max of its 16 screened scores and compares it once with
// tau_u - e_tile(u); only when some lane passes does the wave walk the 16
// scores, insert their lower bounds and append (score, position) to the
// user's candidate buffer.  The score matrix is never written out.
//
// Error bound of a screened score s (float32 accumulation of the screen
// copies u', i'):
//   |key(u,i) - s| <= A_u C_i + B_u G_i,
//   A_u = ||u - u'|| + f 2^-52 ||u||,  B_u = ||u'||,
//   C_i = ||i||,  G_i = ||i - i'|| + gamma ||i'||,
// with gamma = n 2^-22 / (1 - n 2^-22) for the n products of a dot product
// (4x the float32 unit roundoff, covering any summation order of the
// accumulation); for the float32 screen A_u = (f 2^-52 + gamma) ||u||, B = 0.
// A per-user slack (2^-20 of the largest magnitude involved) absorbs the
// float32 rounding of every threshold and bound computed here.
#pragma once

#include <type_traits>

#include "device_common.h"
#include "internal.h"

namespace mips {

// ---------------------------------------------------------------------------
// Screen precisions: operand type and matrix-core instruction per chunk.
// ---------------------------------------------------------------------------
template <int PREC> struct Prec;

template <> struct Prec<PREC_FP32> {
    typedef float Op;
    static constexpr int E = 1;                  // factors per lane per chunk
    static constexpr int ESZ = 4;                // bytes per factor
    __device__ static Op zero() { return 0.0f; }
    __device__ static Op load_packed(const void* base, int64_t b, int c, int nch, int lane) {
        return ((const float*)base)[(b * nch + c) * kWave + lane];
    }
    __device__ static Op load_row(const void* q, int64_t item, int f_pad, int off) {
        return ((const float*)q)[item * f_pad + off];
    }
    __device__ static floatx16_t mma(Op a, Op b, floatx16_t acc, int, int) {
        return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
};

template <> struct Prec<PREC_BF16> {
    typedef bf16x8_t Op;
    static constexpr int E = 8;
    static constexpr int ESZ = 2;
    __device__ static Op zero() { return __builtin_bit_cast(Op, intx4_t{0, 0, 0, 0}); }
    __device__ static Op load_packed(const void* base, int64_t b, int c, int nch, int lane) {
        return __builtin_bit_cast(Op, ((const intx4_t*)base)[(b * nch + c) * kWave + lane]);
    }
    __device__ static Op load_row(const void* q, int64_t item, int f_pad, int off) {
        return __builtin_bit_cast(Op, ((const intx4_t*)q)[(item * f_pad + off) >> 3]);
    }
    __device__ static floatx16_t mma(Op a, Op b, floatx16_t acc, int, int) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
};

template <> struct Prec<PREC_FP8> {
    typedef intx8_t Op;
    static constexpr int E = 32;
    static constexpr int ESZ = 1;
    __device__ static Op zero() { return intx8_t{0, 0, 0, 0, 0, 0, 0, 0}; }
    __device__ static Op load_packed(const void* base, int64_t b, int c, int nch, int lane) {
        return ((const intx8_t*)base)[(b * nch + c) * kWave + lane];
    }
    __device__ static Op load_row(const void* q, int64_t item, int f_pad, int off) {
        return ((const intx8_t*)q)[(item * f_pad + off) >> 5];
    }
    // E8M0 scales: lane's row of A (item) and column of B (user).
    __device__ static floatx16_t mma(Op a, Op b, floatx16_t acc, int sa, int sb) {
        return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, acc, 0, 0, 0, sa, 0, sb);
    }
};

__device__ __forceinline__ double dot64(const float* __restrict__ u, const float* __restrict__ v,
                                        int f) {
    double acc = 0.0;
    for (int j = 0; j < f; ++j) acc = __fma_rn((double)u[j], (double)v[j], acc);
    return acc;
}

// Order of the result: a before b iff a has the larger key, or equal keys
// and the lower item index.
__device__ __forceinline__ bool before(double ka, int ia, double kb, int ib) {
    return ka > kb || (ka == kb && ia < ib);
}

// float64 key of (u, i) summed left to right; the row loads are issued in
// batches of 16 factors so that one memory latency covers 16 FMAs.
__device__ __forceinline__ double key64(const float* __restrict__ u, const float* __restrict__ v,
                                        int f) {
    double acc = 0.0;
    int j = 0;
    if ((f & 1) == 0) {
        const float2* u2 = (const float2*)u;
        const float2* v2 = (const float2*)v;
        for (; j + 16 <= f; j += 16) {
            float2 x[8], y[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) { x[q] = u2[(j >> 1) + q]; y[q] = v2[(j >> 1) + q]; }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                acc = __fma_rn((double)x[q].x, (double)y[q].x, acc);
                acc = __fma_rn((double)x[q].y, (double)y[q].y, acc);
            }
        }
    }
    for (; j < f; ++j) acc = __fma_rn((double)u[j], (double)v[j], acc);
    return acc;
}

// float64 keys of u against up to four item rows (it[q] < 0: skipped), each
// summed left to right; the loads of all rows of an 8-factor batch are
// issued together, so one memory latency covers up to 32 FMAs.
__device__ __forceinline__ void keys4(const float* __restrict__ u, const float* __restrict__ I,
                                      int f, const int (&it)[4], double (&acc)[4]) {
    const float* v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        v[q] = I + (int64_t)(it[q] >= 0 ? it[q] : 0) * f;
        acc[q] = 0.0;
    }
    int j = 0;
    if ((f & 1) == 0) {
        const float2* u2 = (const float2*)u;
        for (; j + 8 <= f; j += 8) {
            float2 x[4], y[4][4];
#pragma unroll
            for (int e = 0; e < 4; ++e) x[e] = u2[(j >> 1) + e];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (it[q] < 0) continue;
                const float2* v2 = (const float2*)v[q];
#pragma unroll
                for (int e = 0; e < 4; ++e) y[q][e] = v2[(j >> 1) + e];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (it[q] < 0) continue;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    acc[q] = __fma_rn((double)x[e].x, (double)y[q][e].x, acc[q]);
                    acc[q] = __fma_rn((double)x[e].y, (double)y[q][e].y, acc[q]);
                }
            }
        }
    }
    for (; j < f; ++j) {
        const double x = (double)u[j];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (it[q] >= 0) acc[q] = __fma_rn(x, (double)v[q][j], acc[q]);
    }
}

__device__ __forceinline__ void flag_user(const ScreenArgs& a, int64_t u) {
    if (atomicCAS(&a.uflag[u], 0, 1) == 0) {
        unsigned int k = atomicAdd(&a.ctrl->fb_count, 1u);
        a.flist[k] = (int)u;
    }
}

// Users of user block `ub` of wave `w`: brute force takes them in order, the
// walk takes them from its tile (all users of a tile share one cluster).
__device__ __forceinline__ int64_t user_of(const ScreenArgs& a, int UB, int64_t w, int ub, int n,
                                           const int4& tile, bool* valid) {
    if (a.walk) {
        int r = ub * kTile + n;
        *valid = r < tile.z;
        return *valid ? (int64_t)a.sorted_users[tile.y + r] : 0;
    }
    int64_t u = (w * UB + ub) * kTile + n;
    *valid = u < a.n_u;
    return *valid ? u : 0;
}

// Maximum / minimum that propagate NaN (IEEE 754-2019 maximum): they map to
// the three-input v_maximum3 / v_minimum3 without the operand quieting that
// fmaxf needs.  Scores are finite or -inf here (a NaN only arises from
// non-finite input, whose users are sent to the exact path).
__device__ __forceinline__ float vmax(float a, float b) { return __builtin_elementwise_maximum(a, b); }
__device__ __forceinline__ float vmin(float a, float b) { return __builtin_elementwise_minimum(a, b); }

// Entry `idx` (wave-uniform, known only at run time) of a register list
// sorted in descending order: the max over the entries from idx on.  Written
// as a masked reduction so that the list stays in registers (a select chain
// would be turned into an indexed load from scratch memory).
template <int KM>
__device__ __forceinline__ float pick_sorted(const float (&l)[KM], int idx) {
    float v = -__builtin_inff();
#pragma unroll
    for (int q = 0; q < KM; ++q) v = vmax(v, (q >= idx) ? l[q] : -__builtin_inff());
    return v;
}

// Insert x into a register list sorted in descending order, keeping its KM
// largest entries: the new entry q is the median of old entries q-1, q and x
// (one exact v_med3_f32 per slot, all independent).
template <int KM>
__device__ __forceinline__ void list_insert(float (&l)[KM], float x) {
#pragma unroll
    for (int q = KM - 1; q >= 1; --q) l[q] = __builtin_amdgcn_fmed3f(l[q - 1], l[q], x);
    l[0] = vmax(l[0], x);
}

template <int KM>
__device__ __forceinline__ void list_reset(float (&l)[KM], int K) {
#pragma unroll
    for (int q = 0; q < KM; ++q) l[q] = (q < KM - K) ? __builtin_inff() : -__builtin_inff();
}

// Valid lower bound on a user's K-th largest key from the two lanes' lists:
// each lane's K-th largest entry, and the min over the two lanes of their
// ceil(K/2)-th largest (together at least K values reach it).
template <int KM>
__device__ __forceinline__ float list_tau(const float (&l)[KM], int hidx, bool k_is_km) {
    const float t = l[KM - 1];
    // with K == KM (the usual case) the entry's slot is a compile-time index
    const float th = k_is_km ? l[KM - KM / 2 - 1] : pick_sorted(l, hidx);
    const float tp = xor32_f(t), thp = xor32_f(th);
    return vmax(vmax(t, tp), vmin(th, thp));
}

// The walk tests each hit against the pair's own bound (the item norms of
// its tile, gathered with the operands) where the extra registers keep two
// waves per SIMD: lists of up to 16 entries, at most 64 bfloat16 or 32
// float32 factors.
__host__ __device__ constexpr bool pair_bound_walk(bool walk, int prec, int km, int nch) {
    return walk && km <= 16 && (prec != PREC_BF16 || nch <= 4) && (prec != PREC_FP32 || nch <= 16);
}

// Warm-up sets of per-slot maxima (16 slots per set) used to seed tau.
__host__ __device__ constexpr int warm_sets(int km) {
    return km <= 16 ? 2 : (km <= 32 ? 3 : 4);
}



// ---------------------------------------------------------------------------
// The screen kernel.
// ---------------------------------------------------------------------------
// Sweep modes: the brute force, the norm-pruned brute force (stop test over
// the suffix maxima of the norm-ordered tiles) and the Maximus walk.
constexpr int kSweepBrute = 0, kSweepPruned = 1, kSweepWalk = 2;

template <int PREC, int KM, int NCH, int UB, int MODE>
// bmax_base: a.blockmax (brute force, norm-pruned) or a.cblockmax (walk), as
// a separate restrict-qualified argument: the compiler can then prove that no
// store of the kernel reaches it and reads the per-tile maxima with scalar
// loads (through the struct it issues vector loads, whose waits would also
// drain the operand loads in flight).
__global__ void __launch_bounds__(64) screen_kernel(const ScreenArgs a,
                                                    const float2* __restrict__ bmax_base) {
    constexpr bool WALK = MODE == kSweepWalk;
    typedef Prec<PREC> P;
    typedef typename P::Op Op;
    constexpr int E = P::E;
    constexpr int S = warm_sets(KM);
    const int lane = threadIdx.x, n = lane & 31, h = lane >> 5;
    const int64_t w = blockIdx.x;
    const int half = a.f_pad / 2;
    const float ninf = -__builtin_inff(), pinf = __builtin_inff();

    int4 tile = make_int4(0, 0, 0, 0);
    if (WALK) tile = a.tiles[w];
    const int cluster = tile.x;

    const float Cmax = __uint_as_float(a.ctrl->cmax_bits);
    const float Emax = __uint_as_float(a.ctrl->emax_bits);
    const float Gmax = __uint_as_float(a.ctrl->gmax_bits);

    Op bu[UB][NCH];
    float Au[UB], Bu[UB], slk[UB], tau[UB], tauf[UB], Nup[UB];
    int ustop[UB];                // walk: tiles visited before the user stopped
    // K-lists: registers, or LDS (lane-major, conflict-free) where they or
    // the operands would take most of the registers (four user blocks, 32
    // operand registers per block, lists of 32 or more entries); the lists
    // are touched only when a tile has hits.
    constexpr int OPR = NCH * (PREC == PREC_FP32 ? 1 : (PREC == PREC_BF16 ? 4 : 8));
    constexpr bool LDSL = UB >= 4 || OPR >= 32 || KM >= 32;
    float lst[UB][LDSL ? 1 : KM];
    __shared__ float s_lst[LDSL ? UB * KM * kWave : 1];
    auto list_load = [&](int ub, float (&L)[KM]) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < KM; ++q) {
            if constexpr (LDSL) L[q] = s_lst[(ub * KM + q) * kWave + lane];
            else L[q] = lst[ub][q];
        }
    };
    auto list_store = [&](int ub, const float (&L)[KM]) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < KM; ++q) {
            if constexpr (LDSL) s_lst[(ub * KM + q) * kWave + lane] = L[q];
            else lst[ub][q] = L[q];
        }
    };
    int cnt[UB], uscale[UB];
    bool dgn[UB];                 // degenerate user: already on the exact path
    bool act[UB];

    // ---- prologue: load, quantise and measure this wave's users ----------
    // The 32 user rows of a block are first copied to LDS with all their
    // loads issued together (one memory latency per block; one row per lane
    // would take one per factor batch), and each lane reads its user's
    // factors from there.  Brute force and norm-pruned sweep: the rows are
    // consecutive in U (one coalesced copy) and the copy goes to the K-list
    // array where that is in LDS and large enough (the lists are first
    // written after the prologue); walk: gathered, lane j loading factor j
    // of each row, into an LDS buffer of its own (f_pad <= 64).  A buffer
    // of its own for the float32 brute force was measured slower (8.45 vs
    // 8.52 ms on 480,000 x 17,770), so there each lane reads its own row.
    constexpr int kStageMax = 2 * kTile * NCH * E;    // floats of 32 rows at f = f_pad
    constexpr bool kStageL = !WALK && LDSL && UB * KM * kWave >= kStageMax;
    constexpr bool kStageS = WALK && PREC != PREC_FP8 && kStageMax <= kTile * kWave;
    constexpr bool kStage = kStageL || kStageS;
    constexpr int kStageIt = (kStageMax + kWave - 1) / kWave;
    __shared__ float s_stage[kStageS ? kStageMax : 1];
    float* const stage = kStageL ? s_lst : s_stage;
#pragma unroll
    for (int ub = 0; ub < UB; ++ub) {
        bool valid;
        const int64_t u = user_of(a, UB, w, ub, n, tile, &valid);
        const float* urow = a.U + u * a.f;
        if constexpr (kStage && !WALK) {
            const int64_t u0 = (w * UB + ub) * kTile;
            const int64_t left = a.n_u - u0;
            const int nf = (int)(left <= 0 ? 0 : (left < kTile ? left : kTile)) * a.f;
            const float* src = a.U + u0 * a.f;
            float v[kStageIt];
#pragma unroll
            for (int t = 0; t < kStageIt; ++t) {
                const int i = lane + t * kWave;
                v[t] = (i < nf) ? src[i] : 0.0f;
            }
            __syncthreads();                          // the previous block's reads are done
#pragma unroll
            for (int t = 0; t < kStageIt; ++t) {
                const int i = lane + t * kWave;
                if (i < nf) stage[i] = v[t];
            }
            __syncthreads();
        } else if constexpr (kStage) {
            // f <= f_pad <= 64: lane j holds factor j of row t
            const int rows = tile.z - ub * kTile;     // users of this block (may be <= 0)
            const int mine = (lane < rows && lane < kTile) ? a.sorted_users[tile.y + ub * kTile + lane] : 0;
            float v[kTile];
#pragma unroll
            for (int t = 0; t < kTile; ++t) {
                const int ut = __builtin_amdgcn_readlane(mine, t);
                v[t] = (t < rows && lane < a.f) ? a.U[(int64_t)ut * a.f + lane] : 0.0f;
            }
            __syncthreads();                          // the previous block's reads are done
#pragma unroll
            for (int t = 0; t < kTile; ++t)
                if (lane < a.f) stage[t * a.f + lane] = v[t];
            __syncthreads();
        }
        auto ux = [&](int j) __attribute__((always_inline)) -> float {
            if constexpr (kStage) return stage[n * a.f + j];   // the staged copy
            else return urow[j];
        };
        double s2 = 0.0, r2 = 0.0, q2 = 0.0;
        float amax = 0.0f;
        bool finite = true;
        if (valid) {
            for (int j = h * half; j < h * half + half && j < a.f; ++j) {
                const float x = ux(j);
                finite = finite && ((__float_as_uint(x) & 0x7f800000u) != 0x7f800000u);
                s2 += (double)x * (double)x;
                amax = fmaxf(amax, fabsf(x));
            }
        }
        int k = 0;
        if (PREC == PREC_FP8) {
            amax = fmaxf(amax, xor32_f(amax));
            k = e4m3_row_scale_exp(amax);
        }
        uscale[ub] = k + 127;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            Op op = P::zero();
            if (valid) {
                const int j0 = h * half + c * E;
                if constexpr (PREC == PREC_FP32) {
                    const float x = (j0 < a.f) ? ux(j0) : 0.0f;
                    op = __builtin_bit_cast(Op, x);
                } else if constexpr (PREC == PREC_BF16) {
                    uint32_t wd[4];
#pragma unroll
                    for (int e = 0; e < 8; e += 2) {
                        const float x0 = (j0 + e < a.f) ? ux(j0 + e) : 0.0f;
                        const float x1 = (j0 + e + 1 < a.f) ? ux(j0 + e + 1) : 0.0f;
                        const uint16_t b0 = f32_to_bf16_bits(x0), b1 = f32_to_bf16_bits(x1);
                        const double d0 = bf16_bits_to_f32(b0), d1 = bf16_bits_to_f32(b1);
                        r2 += ((double)x0 - d0) * ((double)x0 - d0) + ((double)x1 - d1) * ((double)x1 - d1);
                        q2 += d0 * d0 + d1 * d1;
                        wd[e / 2] = (uint32_t)b0 | ((uint32_t)b1 << 16);
                    }
                    op = __builtin_bit_cast(Op, intx4_t{(int)wd[0], (int)wd[1], (int)wd[2], (int)wd[3]});
                } else {
                    uint32_t wd[8];
#pragma unroll
                    for (int e = 0; e < 32; e += 4) {
                        uint32_t word = 0;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const float x = (j0 + e + q < a.f) ? ux(j0 + e + q) : 0.0f;
                            const uint32_t byte = e4m3_encode(__builtin_ldexpf(x, -k));
                            const double d = __builtin_ldexp((double)e4m3_decode(byte), k);
                            r2 += ((double)x - d) * ((double)x - d);
                            q2 += d * d;
                            word |= byte << (8 * q);
                        }
                        wd[e / 4] = word;
                    }
                    op = __builtin_bit_cast(Op, intx8_t{(int)wd[0], (int)wd[1], (int)wd[2], (int)wd[3],
                                                        (int)wd[4], (int)wd[5], (int)wd[6], (int)wd[7]});
                }
            }
            bu[ub][c] = op;
        }
        s2 += xor32_d(s2);
        r2 += xor32_d(r2);
        q2 += xor32_d(q2);
        // every lane must take part in the exchange (no short-circuit)
        const int finite_p = xor32_i((int)finite);
        finite = finite && (finite_p != 0);
        const double N64 = sqrt(s2);
        float A, B;
        if constexpr (PREC == PREC_FP32) {
            A = norm_up_f32(((double)a.f * 0x1p-52 + (double)a.gamma) * N64);
            B = 0.0f;
        } else {
            A = norm_up_f32(sqrt(r2) + (double)a.f * 0x1p-52 * N64);
            B = norm_up_f32(sqrt(q2));
        }
        const double M = N64 * Cmax * 1.01 + (double)B * Emax * 1.01 + (double)A * Cmax +
                         (double)B * Gmax;
        Au[ub] = A;
        Bu[ub] = B;
        slk[ub] = round_up_f32(M * 0x1p-20 + 0x1p-100);
        Nup[ub] = norm_up_f32(N64);
        const bool degenerate = !finite || !(N64 > 0.0) || !(N64 * (double)Cmax < 0x1p100);
        if (valid && degenerate && h == 0) {
            if (!finite) atomicOr(&a.ctrl->nonfinite, 1u);
            flag_user(a, u);
        }
        act[ub] = valid && !degenerate;
        dgn[ub] = degenerate;
        tau[ub] = ninf;
        cnt[ub] = 0;
        ustop[ub] = -1;
    }

    // list slot of the ceil(K/2)-th largest real entry (KM-K +inf pads first)
    const int hidx = KM - (a.K / 2) - 1;
    const bool k_is_km = a.K == KM;
    const int n_blk = (int)a.n_blk;   // < 2^26 (n_i < 2^31): 32-bit scalar tile arithmetic
    const int* clist = WALK ? a.lists + (int64_t)cluster * a.n_i_pad : nullptr;
    // per-tile bound maxima (max C_i, max G_i over the tile's items)
    const float2* bmax = WALK ? bmax_base + (int64_t)cluster * n_blk : bmax_base;

    // This lane's A-operand chunks of tile b (row n), the row's item index
    // (-1 past the end) and, for E4M3, the row's E8M0 scale byte.
    auto load_tile = [&](int b, Op (&ai)[NCH], int& item, int& iscale, float2& cg)
        __attribute__((always_inline)) {
        const int64_t p = (int64_t)b * kTile + n;
        if constexpr (!WALK) {
#pragma unroll
            for (int c = 0; c < NCH; ++c)
                ai[c] = P::load_packed(a.packed, b, c, NCH, lane);
            item = 0;                               // hits name positions (no item needed)
            if (PREC == PREC_FP8) iscale = a.pscale[p];
        } else {
            item = clist[p];                        // -1 past the last item
            if (b < a.wpre) {
                // a prefix tile: operands already in matrix-core order
                const int64_t tl = (int64_t)cluster * a.wpre + b;
#pragma unroll
                for (int c = 0; c < NCH; ++c) ai[c] = P::load_packed(a.wpacked, tl, c, NCH, lane);
                if constexpr (pair_bound_walk(WALK, PREC, KM, NCH)) cg = a.wcg[tl * kTile + n];
                if (PREC == PREC_FP8) iscale = a.wscale[tl * kTile + n];
            } else {
                const int64_t row = item >= 0 ? item : 0;
                if constexpr (pair_bound_walk(WALK, PREC, KM, NCH))
                    cg = make_float2(a.Corig[row], a.Gorig[row]);   // for the per-pair bound
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    ai[c] = P::load_row(a.qrow, row, a.f_pad, h * half + c * E);
                    if (item < 0) ai[c] = P::zero();
                }
                if (PREC == PREC_FP8) iscale = (item >= 0) ? a.kexp[item] + 127 : 127;
            }
        }
    };

    // Scores of user block ub on tile b: items (rows) x users (columns).  Rows
    // past the last item hold zero operands (score 0); the warm-up sets them
    // to -inf here, the sweep drops them where it looks at rows (their item
    // index is -1), so its common path carries no test for them.
    const int n_full = (int)(a.n_i / kTile);   // tiles without rows past the last item
    auto score_one = [&](int b, const Op (&ai)[NCH], int iscale, int ub) __attribute__((always_inline))
        -> floatx16_t {
        floatx16_t acc = {};
#pragma unroll
        for (int c = 0; c < NCH; ++c) acc = P::mma(ai[c], bu[ub][c], acc, iscale, uscale[ub]);
        return acc;
    };
    auto mask_rows = [&](int b, floatx16_t& acc) __attribute__((always_inline)) {
        if (b >= n_full) {
            const int rem = (int)(a.n_i - (int64_t)b * kTile);   // rows of tile b holding items
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (8 * (r >> 2) + 4 * h + (r & 3) >= rem) acc[r] = ninf;
        }
    };

    // ---- warm-up -------------------------------------------------------------
    // Brute force: the lower bounds of every item of the W leading tiles (the
    // largest norms) go into the K-lists, tile by tile for all blocks, so tau
    // starts at the K-th largest lower bound over those items; the main sweep
    // covers tiles W and later, and the leading tiles are scored once more at
    // the end, with the final tau, to record their candidates (with no list
    // update).  Hits, which cost far more than a tile test, are thereby mostly
    // the user's final candidates.
    constexpr bool DENSE_WARM = MODE == kSweepBrute;
    const int W = DENSE_WARM ? (a.warm_rounds * S < n_blk ? a.warm_rounds * S : n_blk) : 0;
    if constexpr (DENSE_WARM) {
        float L[UB][KM];
#pragma unroll
        for (int ub = 0; ub < UB; ++ub) list_reset(L[ub], a.K);
        for (int b = 0; b < W; ++b) {
            Op ai[NCH];
            int it = -1, sc = 127;
            float2 cgw;
            load_tile(b, ai, it, sc, cgw);
            const float2 bmw = bmax[b];
#pragma unroll
            for (int ub = 0; ub < UB; ++ub) {
                floatx16_t acc = score_one(b, ai, sc, ub);
                mask_rows(b, acc);
                const float ee = fmaf(Au[ub], bmw.x, fmaf(Bu[ub], bmw.y, slk[ub]));
#pragma unroll
                for (int r = 0; r < 16; ++r) list_insert(L[ub], acc[r] - ee);
            }
        }
#pragma unroll
        for (int ub = 0; ub < UB; ++ub) {
            tau[ub] = list_tau(L[ub], hidx, k_is_km);
            list_store(ub, L[ub]);
            tauf[ub] = act[ub] ? tau[ub] : pinf;
        }
    } else {
    // Walk and norm-pruned sweep: tau from per-slot maxima of the leading
    // tiles.  Slot (s, r) keeps the max over tiles b = s (mod S) of this
    // lane's row r: each slot max is the screened score of one distinct item,
    // so the K-th largest of their lower bounds (over the user's two lanes)
    // is a valid lower bound on the user's K-th largest key.  The leading
    // tiles hold the largest-norm items (norm-pruned) or the best-bound items
    // (walk).
    // One user block at a time, so that only one block's slot maxima are live.
#pragma unroll
    for (int ub = 0; ub < UB; ++ub) {
        float gm[S * 16];
#pragma unroll
        for (int q = 0; q < S * 16; ++q) gm[q] = ninf;
        for (int rd = 0; rd < a.warm_rounds; ++rd) {
#pragma unroll
            for (int sidx = 0; sidx < S; ++sidx) {
                const int b = rd * S + sidx;
                if (b < n_blk) {
                    Op ai[NCH];
                    int it = -1, sc = 127;
                    float2 cgw;
                    load_tile(b, ai, it, sc, cgw);
                    floatx16_t acc = score_one(b, ai, sc, ub);
                    mask_rows(b, acc);
#pragma unroll
                    for (int r = 0; r < 16; ++r) gm[sidx * 16 + r] = vmax(gm[sidx * 16 + r], acc[r]);
                }
            }
        }
        // every warm-up item has e <= A Cmax + B Gmax + slack
        const float ew = fmaf(Au[ub], Cmax, fmaf(Bu[ub], Gmax, slk[ub]));
        float L[KM];
        list_reset(L, a.K);
#pragma unroll
        for (int q = 0; q < S * 16; ++q) list_insert(L, gm[q] - ew);
        tau[ub] = list_tau(L, hidx, k_is_km);
        list_reset(L, a.K);
        list_store(ub, L);
        tauf[ub] = act[ub] ? tau[ub] : pinf;
    }
    }

    // Streaming top-K over one user block of one tile: a wave-wide test of
    // the lanes' tile maxima against tau_u - e_tile(u); only when some lane
    // passes are the row groups and rows walked.
    // A hit is appended as (score, reference): the walk names the item (its
    // tile rows come from a list, gathered by item), the brute force names
    // the sorted position b 32 + row, which needs no exchange between lanes;
    // certification maps positions to items.  The store goes to slot
    // min(count, cap - 1): a list that overflows sends its user to the exact
    // path, whatever its last slot holds.
    const int lane_slot0 = lane;
    // candidate list layout: element-major for the fused certification (one
    // lane per user), lane-major for the certification kernels
    constexpr bool kCandLM = !fused_certify(PREC, KM, UB);
    auto test_block = [&](int b, int ub, const floatx16_t& sc, int item, float2 cg)
        __attribute__((always_inline)) {
        // the tile's bound maxima, read (scalar load) where they are used: a
        // vector load issued with the tile's operands was carried to the
        // next iteration by a copy at the loop's back edge, and the wait for
        // that copy also drained the operand loads issued after it
        const float2 bm = bmax[b];
        const float ee = fmaf(Au[ub], bm.x, fmaf(Bu[ub], bm.y, slk[ub]));
        const float thr = tauf[ub] - ee;
        // maxima of the four row groups {4g .. 4g+3}, then of the tile
        float gm4[4];
#pragma unroll
        for (int g = 0; g < 4; ++g)
            gm4[g] = vmax(vmax(sc[4 * g], sc[4 * g + 1]), vmax(sc[4 * g + 2], sc[4 * g + 3]));
        const float m = vmax(vmax(gm4[0], gm4[1]), vmax(gm4[2], gm4[3]));
        if (!ballot(m >= thr)) return;
        float L[KM];
        list_load(ub, L);
        // a group is walked only when some lane's group maximum passes
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            if (!ballot(gm4[g] >= thr)) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float v = sc[4 * g + q];
                bool hit = v >= thr;
                if (ballot(hit)) {
                    const int row = 8 * g + 4 * h + q;
                    int ref;
                    if constexpr (WALK) {
                        // item index of output row 8g + 4h + q, held by lane
                        // (row); -1 for rows past the end of the list
                        ref = __builtin_amdgcn_ds_bpermute(row << 2, item);
                        hit = hit && ref >= 0;
                    } else {
                        // rows past the last item hold zero operands (score 0)
                        ref = b * kTile + row;
                        hit = hit && (int64_t)ref < a.n_i;
                    }
                    float lb = v - ee;
                    if constexpr (pair_bound_walk(WALK, PREC, KM, NCH)) {
                        // walk tiles mix item norms, so the tile's bound is
                        // loose: test the pair's own bound
                        const float ci = __int_as_float(
                            __builtin_amdgcn_ds_bpermute(row << 2, __float_as_int(cg.x)));
                        const float gi = __int_as_float(
                            __builtin_amdgcn_ds_bpermute(row << 2, __float_as_int(cg.y)));
                        const float ei = fmaf(Au[ub], ci, fmaf(Bu[ub], gi, slk[ub]));
                        hit = hit && (v + ei >= tauf[ub]);
                        lb = v - ei;
                    }
                    if (hit) {
                        list_insert(L, lb);
                        int2* const cb = a.cand + cand_base(w * UB + ub, lane_slot0, a.cap, kCandLM);
                        cb[(cnt[ub] < a.cap ? cnt[ub] : a.cap - 1) * cand_stride(kCandLM)] =
                            make_int2(__float_as_int(v), ref);
                        cnt[ub] += 1;
                    }
                }
            }
        }
        tau[ub] = vmax(tau[ub], list_tau(L, hidx, k_is_km));
        tauf[ub] = act[ub] ? tau[ub] : pinf;
        list_store(ub, L);
    };

    // Stop test after tile b (Section III-C); returns false once every user
    // of the wave has stopped.  Every unvisited item i has key <=
    // ||u|| bound_j(i) + f 2^-53 ||u|| ||i||, and the list is sorted, so the
    // next entry's bound covers all of them.  The norm-pruned brute force is
    // the same test with theta_b = pi (bound = ||i||), over the suffix maxima
    // of its norm-ordered tiles.
    auto stop_after = [&](int b) __attribute__((always_inline)) -> bool {
        if constexpr (MODE == kSweepBrute) return true;
        const int64_t pnext = (int64_t)(b + 1) * kTile;
        bool any = false;
        if (b + 1 >= (WALK ? a.shared_blocks : 1)) {
            float bnext;
            if constexpr (WALK)
                bnext = (pnext < a.n_i) ? a.lbound[(int64_t)cluster * a.n_i_pad + pnext] : ninf;
            else
                bnext = (b + 1 < n_blk) ? a.tailmax[b + 1] : ninf;
#pragma unroll
            for (int ub = 0; ub < UB; ++ub) {
                if (act[ub] && fmaf(Nup[ub], bnext, slk[ub]) < tau[ub]) {
                    act[ub] = false;
                    tauf[ub] = pinf;
                    ustop[ub] = b + 1;
                }
                any = any || act[ub];
            }
        } else {
#pragma unroll
            for (int ub = 0; ub < UB; ++ub) any = any || act[ub];
        }
        return ballot(any) != 0;
    };

    // ---- item sweep --------------------------------------------------------
    // With four user blocks, products and tests are interleaved over the
    // blocks: the products of block j of tile b go into one of two
    // accumulator tiles while the test of the block before it (block j - 1,
    // or the last block of tile b - 1) reads the other, so the matrix cores
    // work while the vector unit tests.  Block j of tile b uses accumulator
    // (b UB + j) mod 2.  With one or two blocks, whose product chains are long
    // (float32: 25 dependent products per block at f = 50) or few, all
    // products of a tile come first (independent chains interleave), then the
    // tests, and another wave of the SIMD keeps the matrix cores busy.  Operands
    // are loaded two tiles ahead into alternating register sets, issued as
    // soon as the tile's last products have read them; the loads are
    // unconditional (tile index clamped to the last tile), so the loop body is
    // straight-line code apart from the tests' branches.
    int b_done = n_blk;           // tiles visited (the walk may stop early)
    const int b0 = W;             // first tile of the main sweep
    if (n_blk > b0) {
        const int last = n_blk - 1;
        Op ops[2][NCH];
        int itm[2] = {-1, -1}, scl[2] = {127, 127};
        float2 cgx[2] = {make_float2(0.0f, 0.0f), make_float2(0.0f, 0.0f)};
        floatx16_t acc[2];
        int itP = -1;                 // the previous tile's item and norms
        float2 cgP = make_float2(0.0f, 0.0f);
        load_tile(b0, ops[0], itm[0], scl[0], cgx[0]);
        load_tile(b0 + 1 < n_blk ? b0 + 1 : b0, ops[1], itm[1], scl[1], cgx[1]);
        // tile b from operand set T (= b mod 2); false: every user stopped
        // after tile b - 1 (tile b's products are then unused)
        auto sweep = [&](int b, auto tconst) __attribute__((always_inline)) -> bool {
            constexpr int T = decltype(tconst)::value;
            const int itC = itm[T], scC = scl[T];
            const float2 cgC = cgx[T];
            if constexpr (UB <= 2) {
                // all products of the tile (independent chains, interleaved
                // by the compiler), then the tests and the stop test
#pragma unroll
                for (int j = 0; j < UB; ++j) acc[j] = score_one(b, ops[T], scC, j);
                // float32 (25 products per block at f = 50): keep the products,
                // the next loads and the tests in this order; hoisting the
                // tests' threshold arithmetic above the products made them
                // wait for every operand of the tile (measured 8.3 vs 9.1 ms
                // on 480,000 x 17,770; for the bfloat16 screen at f = 100 the
                // free schedule was faster)
                if constexpr (PREC == PREC_FP32) __builtin_amdgcn_sched_barrier(0);
                load_tile(b + 2 < last ? b + 2 : last, ops[T], itm[T], scl[T], cgx[T]);
#pragma unroll
                for (int j = 0; j < UB; ++j) test_block(b, j, acc[j], itC, cgC);
                return stop_after(b);
            } else {
#pragma unroll
                for (int j = 0; j < UB; ++j) {
                    acc[(T * UB + j) & 1] = score_one(b, ops[T], scC, j);
                    if (j == UB - 1)
                        load_tile(b + 2 < last ? b + 2 : last, ops[T], itm[T], scl[T], cgx[T]);
                    if (j == 0) {
                        if (b > b0) {
                            test_block(b - 1, UB - 1, acc[(T * UB + 1) & 1], itP, cgP);
                            if (!stop_after(b - 1)) return false;
                        }
                    } else {
                        test_block(b, j - 1, acc[(T * UB + j - 1) & 1], itC, cgC);
                    }
                }
                itP = itC;
                cgP = cgC;
                return true;
            }
        };
        // a false sweep: every user stopped after tile b (two blocks or
        // fewer) or after tile b - 1 (rotated blocks)
        constexpr int kStopLag = UB <= 2 ? 1 : 0;
        if constexpr (MODE != kSweepWalk && UB >= 2) {
            // The loop runs while both tiles of a pair exist, every path
            // through its body passes both halves, and an odd last tile is
            // swept after it.  An exit between the halves gives the
            // wait-count analysis a path on which the first half's operand
            // loads are the newest at the loop head, which then waits for
            // every load in flight (the two-tile prefetch lost on every
            // other tile).  A stop after the first half (norm-pruned sweep)
            // takes effect after the second, whose tile then finds no active
            // user: no hit and no state change, one tile of products spent
            // out of hundreds.  The walk, a few tiles long, keeps the exit,
            // and so does the one-block sweep (float32 at f = 100: 50 chained
            // products per tile; measured 266 -> 317 ms with this loop).
            int b = b0;
            if constexpr (MODE == kSweepBrute) {
                for (; b + 1 < n_blk; b += 2) {
                    sweep(b, std::integral_constant<int, 0>{});
                    sweep(b + 1, std::integral_constant<int, 1>{});
                }
                if (b < n_blk) sweep(b, std::integral_constant<int, 0>{});
            } else {
                for (; b + 1 < n_blk; b += 2) {
                    const bool live0 = sweep(b, std::integral_constant<int, 0>{});
                    const bool live1 = sweep(b + 1, std::integral_constant<int, 1>{});
                    if (!live0) { b_done = b + kStopLag; break; }
                    if (!live1) { b_done = b + 1 + kStopLag; break; }
                }
                if (b_done == n_blk && b < n_blk && !sweep(b, std::integral_constant<int, 0>{}))
                    b_done = b + kStopLag;
            }
        } else {
            for (int b = b0; b < n_blk; b += 2) {
                if (!sweep(b, std::integral_constant<int, 0>{})) { b_done = b + kStopLag; break; }
                if (b + 1 >= n_blk) break;
                if (!sweep(b + 1, std::integral_constant<int, 1>{})) { b_done = b + 1 + kStopLag; break; }
            }
        }
        if (UB > 2 && b_done == n_blk) {
            // the last block of the last tile (accumulator ((last - b0) UB + UB - 1) mod 2)
            if (((last - b0) & 1) == 0) test_block(last, UB - 1, acc[(UB - 1) & 1], itP, cgP);
            else test_block(last, UB - 1, acc[(2 * UB - 1) & 1], itP, cgP);
        }
    }

    // ---- brute force: candidates of the leading tiles, final tau ------------
    if constexpr (DENSE_WARM) {
        for (int b = 0; b < W; ++b) {
            Op ai[NCH];
            int it = -1, sc = 127;
            float2 cgw;
            load_tile(b, ai, it, sc, cgw);
            const float2 bm = bmax[b];
            const int rem = (int)(a.n_i - (int64_t)b * kTile);   // rows holding items
#pragma unroll
            for (int ub = 0; ub < UB; ++ub) {
                const floatx16_t v = score_one(b, ai, sc, ub);
                const float thr = tauf[ub] - fmaf(Au[ub], bm.x, fmaf(Bu[ub], bm.y, slk[ub]));
                float m = vmax(v[0], v[1]);
#pragma unroll
                for (int r = 2; r < 16; r += 2) m = vmax(m, vmax(v[r], v[r + 1]));
                if (!ballot(m >= thr)) continue;
                int2* const cb = a.cand + cand_base(w * UB + ub, lane_slot0, a.cap, kCandLM);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = 8 * (r >> 2) + 4 * h + (r & 3);
                    if (v[r] >= thr && row < rem) {
                        cb[(cnt[ub] < a.cap ? cnt[ub] : a.cap - 1) * cand_stride(kCandLM)] =
                            make_int2(__float_as_int(v[r]), b * kTile + row);
                        cnt[ub] += 1;
                    }
                }
            }
        }
    }

    // ---- certification in the same wave (short K-lists) ----------------------
    // Lane 32h + n certifies user n of user block h: it walks the user's two
    // candidate lists (its own half and the one of lane n + 32 or n), keeps
    // the pairs whose upper bound reaches tau_u, rescores them in float64,
    // and keeps the K best by (key desc, index asc) in a sorted register list
    // (only pairs whose key reaches tau_u can be among them).  The user goes
    // to the exact path when a list overflowed or fewer than K keys reach
    // tau_u.  Same rules as certify_kernel, without the round trip through
    // memory for the per-user state.
    if constexpr (fused_certify(PREC, KM, UB)) {
#pragma unroll
      for (int ps = 0; ps < UB / 2; ++ps) {
        // pass ps: lanes of half h certify the users of block 2 ps + h
        const int b0 = 2 * ps, b1 = 2 * ps + 1;
        const int ubl = b0 + h;
        const int x0 = xor32_i(cnt[b0]);
        const int x1 = xor32_i(cnt[b1]);
        const int cA = (h == 1) ? x1 : cnt[b0];          // the list of lane n
        const int cB = (h == 1) ? cnt[b1] : x0;          // the list of lane n + 32
        const float ut = (h == 1) ? tau[b1] : tau[b0];
        const bool ud = (h == 1) ? dgn[b1] : dgn[b0];
        const float uA = (h == 1) ? Au[b1] : Au[b0];
        const float uB = (h == 1) ? Bu[b1] : Bu[b0];
        const float us = (h == 1) ? slk[b1] : slk[b0];
        bool valid = false;
        const int64_t u = user_of(a, UB, w, ubl, n, tile, &valid);
        unsigned long long st_cand = 0, st_resc = 0, st_max = 0;
        double st_abs = 0.0, st_rel = 0.0;
        if (valid && !ud) {
            const int cap = a.cap;
            const int m0 = cA < cap ? cA : cap, m1 = cB < cap ? cB : cap;
            bool bad = (cA > cap) || (cB > cap);
            const int tot = m0 + m1;
            // the user's two lists (its lane n and lane n + 32 halves)
            const int64_t base0 = cand_base(w * UB + ubl, n, cap, kCandLM);
            const int64_t base1 = cand_base(w * UB + ubl, n + 32, cap, kCandLM);
            constexpr int cst = kCandLM ? 1 : kCandStride;
            const float* urow = a.U + u * a.f;
            double tau64 = (double)ut;   // kept pairs: key >= tau64
            float thr = ut;              // rescored pairs: upper bound >= thr (<= tau64)
            double unorm = 0.0;
            if (a.want_stats) {
                for (int j = 0; j < a.f; ++j) unorm += (double)urow[j] * (double)urow[j];
                unorm = sqrt(unorm);
            }
            double tk[KM];
            int ti[KM];
#pragma unroll
            for (int q = 0; q < KM; ++q) { tk[q] = -__builtin_inf(); ti[q] = 0x7fffffff; }
            int nkeep = 0;
            for (int j0 = 0; j0 < tot; j0 += 8) {
                int2 e[8];
                float Ci[8], Gi[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int j = j0 + q;
                    e[q] = make_int2(0, -1);
                    if (j < tot) e[q] = a.cand[(j < m0) ? base0 + j * cst : base1 + (j - m0) * cst];
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int ref = e[q].y;
                    if constexpr (WALK) {
                        Ci[q] = (ref >= 0) ? a.Corig[ref] : 0.0f;
                        Gi[q] = (ref >= 0) ? a.Gorig[ref] : 0.0f;
                    } else {
                        // sorted position: its norms and its item in one 16-byte read
                        const float4 cg = (ref >= 0) ? a.cgpos[ref] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                        Ci[q] = cg.x;
                        Gi[q] = cg.y;
                        e[q].y = (ref >= 0) ? __float_as_int(cg.z) : -1;
                    }
                }
                int it[8];
                bool anyk = false;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const float sv = __int_as_float(e[q].x);
                    const float eb = fmaf(uA, Ci[q], fmaf(uB, Gi[q], us));
                    it[q] = (e[q].y >= 0 && sv + eb >= thr) ? e[q].y : -1;
                    anyk = anyk || it[q] >= 0;
                }
                if (!anyk) continue;
                double k8[8];
                {
                    // two groups of four rows (one memory latency per 32 FMAs)
                    const int ia[4] = {it[0], it[1], it[2], it[3]}, ib[4] = {it[4], it[5], it[6], it[7]};
                    double ka[4], kb[4];
                    keys4(urow, a.I, a.f, ia, ka);
                    keys4(urow, a.I, a.f, ib, kb);
#pragma unroll
                    for (int q = 0; q < 4; ++q) { k8[q] = ka[q]; k8[q + 4] = kb[q]; }
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    if (it[q] < 0) continue;
                    const double key = k8[q];
                    ++st_resc;
                    if (a.want_stats) {
                        const double err = fabs((double)__int_as_float(e[q].x) - key);
                        st_abs = fmax(st_abs, err);
                        const double scale = unorm * (double)Ci[q];
                        if (scale > 0.0) st_rel = fmax(st_rel, err / scale);
                    }
                    if (key < tau64) continue;   // beaten by K items
                    ++nkeep;
                    // insert into the sorted list: every slot from the old list
                    const int ix = it[q];
#pragma unroll
                    for (int q2 = KM - 1; q2 >= 1; --q2) {
                        const bool above = before(key, ix, tk[q2 - 1], ti[q2 - 1]);
                        const bool here = before(key, ix, tk[q2], ti[q2]);
                        const double nk = above ? tk[q2 - 1] : (here ? key : tk[q2]);
                        const int ni = above ? ti[q2 - 1] : (here ? ix : ti[q2]);
                        tk[q2] = nk;
                        ti[q2] = ni;
                    }
                    if (before(key, ix, tk[0], ti[0])) { tk[0] = key; ti[0] = ix; }
                }
                // once K keys are kept, the K-th largest of them is at most
                // the user's K-th largest key: later pairs below it need no
                // rescore
                if (nkeep >= a.K) {
                    double kth = tk[KM - 1];
                    if (!k_is_km) {
#pragma unroll
                        for (int q = 0; q < KM; ++q)
                            if (q == a.K - 1) kth = tk[q];
                    }
                    if (kth > tau64) {
                        tau64 = kth;
                        thr = fmaxf(thr, __double2float_rd(kth));
                    }
                }
            }
            st_cand = (unsigned long long)(cA + cB);
            st_max = st_cand;
            if (bad || nkeep < a.K) {
                flag_user(a, u);
            } else {
#pragma unroll
                for (int q = 0; q < KM; ++q) {
                    if (q < a.K) {
                        a.out_idx[u * a.K + q] = ti[q];
                        a.out_score[u * a.K + q] = tk[q];
                    }
                }
            }
        } else if (valid) {
            st_max = (unsigned long long)(cA + cB);
        }
        if (a.want_stats) {
            for (int off = 32; off >= 1; off >>= 1) {
                st_cand += __shfl_xor(st_cand, off);
                st_resc += __shfl_xor(st_resc, off);
                st_max = max(st_max, (unsigned long long)__shfl_xor(st_max, off));
                st_abs = fmax(st_abs, __shfl_xor(st_abs, off));
                st_rel = fmax(st_rel, __shfl_xor(st_rel, off));
            }
            if (lane == 0) {
                if (st_cand) atomicAdd(&a.ctrl->cand_total, st_cand);
                if (st_resc) atomicAdd(&a.ctrl->rescored, st_resc);
                if (st_max) atomicMax(&a.ctrl->cand_max, st_max);
                atomic_max_nonneg((double*)&a.ctrl->max_abs_err, st_abs);
                atomic_max_nonneg((double*)&a.ctrl->max_rel_err, st_rel);
            }
        }
      }
    }

    // ---- hand the per-user state to certification -------------------------
    unsigned long long visited = 0;
#pragma unroll
    for (int ub = 0; ub < UB; ++ub) {
        const int64_t ublk = w * UB + ub;
        if (ublk < a.n_ublk) a.cnt[(ublk << 6) + lane] = cnt[ub];
        bool valid;
        const int64_t u = user_of(a, UB, w, ub, n, tile, &valid);
        if (valid && h == 0) {
            a.uscal[u] = make_float4(Au[ub], Bu[ub], slk[ub], tau[ub]);
            const int64_t tiles_seen = (ustop[ub] >= 0) ? ustop[ub] : b_done;
            visited += (unsigned long long)(tiles_seen * kTile < a.n_i ? tiles_seen * kTile : a.n_i);
        }
    }
    if (a.want_stats) {
        for (int off = 32; off >= 1; off >>= 1) visited += __shfl_xor(visited, off);
        if (lane == 0 && visited) atomicAdd(&a.ctrl->visited, visited);
    }
}

template <int PREC, int KM, int NCH>
static hipError_t go_screen(const ScreenPlan& p, const ScreenArgs& a, hipStream_t s) {
    // blocks per wave: fewer where a stop test keeps waves until their
    // slowest user stops
    constexpr int UBS = ub_for(PREC, KM, NCH, true), UBB = ub_for(PREC, KM, NCH, false);
    const dim3 grid((unsigned)p.n_waves), blk(64);
    if (a.walk) {
        if (p.UB != UBS) return hipErrorInvalidValue;   // plan and kernel disagree
        screen_kernel<PREC, KM, NCH, UBS, kSweepWalk><<<grid, blk, 0, s>>>(a, a.cblockmax);
    } else if (a.prune) {
        if (p.UB != UBB) return hipErrorInvalidValue;
        screen_kernel<PREC, KM, NCH, UBB, kSweepPruned><<<grid, blk, 0, s>>>(a, a.blockmax);
    } else {
        if (p.UB != UBB) return hipErrorInvalidValue;
        screen_kernel<PREC, KM, NCH, UBB, kSweepBrute><<<grid, blk, 0, s>>>(a, a.blockmax);
    }
    return hipGetLastError();
}

template <int PREC, int NCH>
static hipError_t screen_km(const ScreenPlan& p, const ScreenArgs& a, hipStream_t s) {
    switch (p.KM) {
        case 1:  return go_screen<PREC, 1, NCH>(p, a, s);
        case 8:  return go_screen<PREC, 8, NCH>(p, a, s);
        case 10: return go_screen<PREC, 10, NCH>(p, a, s);
        case 16: return go_screen<PREC, 16, NCH>(p, a, s);
        case 32: return go_screen<PREC, 32, NCH>(p, a, s);
        default: return go_screen<PREC, 64, NCH>(p, a, s);
    }
}

}  // namespace mips
