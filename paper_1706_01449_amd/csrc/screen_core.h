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

// Certification runs at the end of the screen kernel when the K-list fits a
// small sorted register list, two user blocks keep every lane busy (one user
// per lane), and the screen keeps few candidates per user (not E4M3, whose
// hundreds of candidates per user make one lane per user too slow; there the
// separate kernel spreads a user over 16 or 64 lanes).
__host__ __device__ constexpr bool fused_certify(int prec, int km, int ub) {
    return prec != PREC_FP8 && km <= 16 && ub == 2;
}

// ---------------------------------------------------------------------------
// The screen kernel.
// ---------------------------------------------------------------------------
template <int PREC, int KM, int NCH, int UB, bool WALK>
__global__ void __launch_bounds__(64) screen_kernel(const ScreenArgs a) {
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
    float lst[UB][KM];
    int cnt[UB], uscale[UB];
    bool dgn[UB];                 // degenerate user: already on the exact path
    bool act[UB];
    int2* cptr[UB];

    // ---- prologue: load, quantise and measure this wave's users ----------
#pragma unroll
    for (int ub = 0; ub < UB; ++ub) {
        bool valid;
        const int64_t u = user_of(a, UB, w, ub, n, tile, &valid);
        const float* urow = a.U + u * a.f;
        double s2 = 0.0, r2 = 0.0, q2 = 0.0;
        float amax = 0.0f;
        bool finite = true;
        if (valid) {
            for (int j = h * half; j < h * half + half && j < a.f; ++j) {
                const float x = urow[j];
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
                    const float x = (j0 < a.f) ? urow[j0] : 0.0f;
                    op = __builtin_bit_cast(Op, x);
                } else if constexpr (PREC == PREC_BF16) {
                    uint32_t wd[4];
#pragma unroll
                    for (int e = 0; e < 8; e += 2) {
                        const float x0 = (j0 + e < a.f) ? urow[j0 + e] : 0.0f;
                        const float x1 = (j0 + e + 1 < a.f) ? urow[j0 + e + 1] : 0.0f;
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
                            const float x = (j0 + e + q < a.f) ? urow[j0 + e + q] : 0.0f;
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
        cptr[ub] = a.cand + (((w * UB + ub) << 6) + lane) * (int64_t)a.cap;   // lane-major lists
        list_reset(lst[ub], a.K);
    }

    // list slot of the ceil(K/2)-th largest real entry (KM-K +inf pads first)
    const int hidx = KM - (a.K / 2) - 1;
    const bool k_is_km = a.K == KM;
    const int n_blk = (int)a.n_blk;   // < 2^26 (n_i < 2^31): 32-bit scalar tile arithmetic
    const int* clist = WALK ? a.lists + (int64_t)cluster * a.n_i_pad : nullptr;
    // per-tile bound maxima (prefetched with the tile operands)
    const float2* bmax = WALK ? a.cblockmax + (int64_t)cluster * n_blk : a.blockmax;

    // This lane's A-operand chunks of tile b (row n), the row's item index
    // (-1 past the end) and, for E4M3, the row's E8M0 scale byte.
    auto load_tile = [&](int b, Op (&ai)[NCH], int& item, int& iscale, float2& bm, float2& cg)
        __attribute__((always_inline)) {
        const int64_t p = (int64_t)b * kTile + n;
        bm = bmax[b];
        if constexpr (!WALK) {
#pragma unroll
            for (int c = 0; c < NCH; ++c)
                ai[c] = P::load_packed(a.packed, b, c, NCH, lane);
            item = a.perm[p];                       // -1 past the last item
            if (PREC == PREC_FP8) iscale = a.pscale[p];
        } else {
            item = clist[p];                        // -1 past the last item
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
    };

    // Score tile: acc[ub] = items (rows) x users (columns); rows past the
    // last item are set to -inf.
    auto score_tile = [&](int b, const Op (&ai)[NCH], int iscale, floatx16_t (&acc)[UB])
        __attribute__((always_inline)) {
#pragma unroll
        for (int ub = 0; ub < UB; ++ub) {
            floatx16_t z = {};
            acc[ub] = z;
#pragma unroll
            for (int c = 0; c < NCH; ++c)
                acc[ub] = P::mma(ai[c], bu[ub][c], acc[ub], iscale, uscale[ub]);
        }
        if ((int64_t)(b + 1) * kTile > a.n_i) {
#pragma unroll
            for (int ub = 0; ub < UB; ++ub)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    if ((int64_t)b * kTile + 8 * (r >> 2) + 4 * h + (r & 3) >= a.n_i) acc[ub][r] = ninf;
        }
    };

    // ---- warm-up: seed tau from per-slot maxima of the leading tiles -----
    // Slot (s, r) keeps the max over tiles b = s (mod S) of this lane's row r:
    // each slot max is the screened score of one distinct item, so the K-th
    // largest of their lower bounds (over the user's two lanes) is a valid
    // lower bound on the user's K-th largest key.  The leading tiles hold the
    // largest-norm items (brute force) or the best-bound items (walk).
    {
        float gm[UB][S * 16];
#pragma unroll
        for (int ub = 0; ub < UB; ++ub)
#pragma unroll
            for (int q = 0; q < S * 16; ++q) gm[ub][q] = ninf;
        for (int rd = 0; rd < a.warm_rounds; ++rd) {
#pragma unroll
            for (int sidx = 0; sidx < S; ++sidx) {
                const int b = rd * S + sidx;
                if (b < n_blk) {
                    Op ai[NCH];
                    int it = -1, sc = 127;
                    float2 bmw;
                    float2 cgw;
                    load_tile(b, ai, it, sc, bmw, cgw);
                    floatx16_t acc[UB];
                    score_tile(b, ai, sc, acc);
#pragma unroll
                    for (int ub = 0; ub < UB; ++ub)
#pragma unroll
                        for (int r = 0; r < 16; ++r)
                            gm[ub][sidx * 16 + r] = vmax(gm[ub][sidx * 16 + r], acc[ub][r]);
                }
            }
        }
#pragma unroll
        for (int ub = 0; ub < UB; ++ub) {
            // every warm-up item has e <= A Cmax + B Gmax + slack
            const float ew = fmaf(Au[ub], Cmax, fmaf(Bu[ub], Gmax, slk[ub]));
#pragma unroll
            for (int q = 0; q < S * 16; ++q) list_insert(lst[ub], gm[ub][q] - ew);
            tau[ub] = list_tau(lst[ub], hidx, k_is_km);
            list_reset(lst[ub], a.K);
            tauf[ub] = act[ub] ? tau[ub] : pinf;
        }
    }

    // Streaming top-K over tile b; returns false once every user of a walk
    // wave has stopped.
    auto epi_tile = [&](int b, floatx16_t (&acc)[UB], int item, float2 bm, float2 cg)
        __attribute__((always_inline)) -> bool {
#pragma unroll
        for (int ub = 0; ub < UB; ++ub) {
            const float ee = fmaf(Au[ub], bm.x, fmaf(Bu[ub], bm.y, slk[ub]));
            const float thr = tauf[ub] - ee;
            // maxima of the four row groups {4g .. 4g+3}, then of the tile
            float gm4[4];
#pragma unroll
            for (int g = 0; g < 4; ++g)
                gm4[g] = vmax(vmax(acc[ub][4 * g], acc[ub][4 * g + 1]),
                              vmax(acc[ub][4 * g + 2], acc[ub][4 * g + 3]));
            const float m = vmax(vmax(gm4[0], gm4[1]), vmax(gm4[2], gm4[3]));
            if (ballot(m >= thr)) {
                // a group is walked only when some lane's group maximum passes
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    if (!ballot(gm4[g] >= thr)) continue;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int r = 4 * g + q;
                        const float v = acc[ub][r];
                        bool hit = (v >= thr) && (v > ninf);
                        if (ballot(hit)) {
                            // item index of output row 8g + 4h + q, held by lane (row)
                            const int row = 8 * g + 4 * h + q;
                            const int orig = __builtin_amdgcn_ds_bpermute(row << 2, item);
                            float lb = v - ee;
                            if constexpr (pair_bound_walk(WALK, PREC, KM, NCH)) {
                                // walk tiles mix item norms, so the tile's
                                // bound is loose: test the pair's own bound
                                const float ci = __int_as_float(
                                    __builtin_amdgcn_ds_bpermute(row << 2, __float_as_int(cg.x)));
                                const float gi = __int_as_float(
                                    __builtin_amdgcn_ds_bpermute(row << 2, __float_as_int(cg.y)));
                                const float ei = fmaf(Au[ub], ci, fmaf(Bu[ub], gi, slk[ub]));
                                hit = hit && (v + ei >= tauf[ub]);
                                lb = v - ei;
                            }
                            if (hit) {
                                list_insert(lst[ub], lb);
                                if (cnt[ub] < a.cap)
                                    cptr[ub][cnt[ub]] = make_int2(__float_as_int(v), orig);
                                cnt[ub] += 1;
                            }
                        }
                    }
                }
                tau[ub] = vmax(tau[ub], list_tau(lst[ub], hidx, k_is_km));
                tauf[ub] = act[ub] ? tau[ub] : pinf;
            }
        }
        if constexpr (!WALK) {
            if (!a.prune) return true;
        }
        // Stop test after this tile (Section III-C): every unvisited item i has
        // key <= ||u|| bound_j(i) + f 2^-53 ||u|| ||i||, and the list is sorted,
        // so the next entry's bound covers all of them.  The norm-pruned brute
        // force is the same test with theta_b = pi (bound = ||i||), over the
        // suffix maxima of its norm-ordered tiles.
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
    // Operands are loaded two tiles ahead into alternating register sets; the
    // loads are unconditional (tile index clamped to the last tile) so the
    // loop body is straight-line code with exact wait counts.
    int b_done = n_blk;           // tiles visited (the walk may stop early)
    if (n_blk > 0) {
        const int last = n_blk - 1;
        Op oA[NCH], oB[NCH];
        int itA = -1, itB = -1, scA = 127, scB = 127;
        float2 bmA, bmB, cgA = make_float2(0.0f, 0.0f), cgB = make_float2(0.0f, 0.0f);
        floatx16_t acc[UB];
        load_tile(0, oA, itA, scA, bmA, cgA);
        load_tile(n_blk > 1 ? 1 : 0, oB, itB, scB, bmB, cgB);
        for (int b = 0; b < n_blk; b += 2) {
            score_tile(b, oA, scA, acc);
            const int eA = itA;
            const float2 mA = bmA, gA = cgA;
            load_tile(b + 2 < last ? b + 2 : last, oA, itA, scA, bmA, cgA);
            if (!epi_tile(b, acc, eA, mA, gA)) { b_done = b + 1; break; }
            if (b + 1 >= n_blk) break;
            score_tile(b + 1, oB, scB, acc);
            const int eB = itB;
            const float2 mB = bmB, gB = cgB;
            load_tile(b + 3 < last ? b + 3 : last, oB, itB, scB, bmB, cgB);
            if (!epi_tile(b + 1, acc, eB, mB, gB)) { b_done = b + 2; break; }
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
        const int ubl = h;
        const int x0 = xor32_i(cnt[0]);
        const int x1 = xor32_i(cnt[UB - 1]);
        const int cA = (ubl == 1) ? x1 : cnt[0];          // the list of lane n
        const int cB = (ubl == 1) ? cnt[UB - 1] : x0;     // the list of lane n + 32
        const float uA = (ubl == 1) ? Au[UB - 1] : Au[0];
        const float uB = (ubl == 1) ? Bu[UB - 1] : Bu[0];
        const float us = (ubl == 1) ? slk[UB - 1] : slk[0];
        const float ut = (ubl == 1) ? tau[UB - 1] : tau[0];
        const bool ud = (ubl == 1) ? dgn[UB - 1] : dgn[0];
        bool valid = false;
        const int64_t u = (h < UB) ? user_of(a, UB, w, ubl, n, tile, &valid) : 0;
        unsigned long long st_cand = 0, st_resc = 0, st_max = 0;
        double st_abs = 0.0, st_rel = 0.0;
        if (valid && !ud) {
            const int cap = a.cap;
            const int m0 = cA < cap ? cA : cap, m1 = cB < cap ? cB : cap;
            bool bad = (cA > cap) || (cB > cap);
            const int tot = m0 + m1;
            const int2* list0 = a.cand + (((w * UB + ubl) << 6) + n) * (int64_t)cap;
            const int2* list1 = a.cand + (((w * UB + ubl) << 6) + n + 32) * (int64_t)cap;
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
            for (int j0 = 0; j0 < tot; j0 += 4) {
                int2 e[4];
                float Ci[4], Gi[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int j = j0 + q;
                    e[q] = make_int2(0, -1);
                    if (j < tot) e[q] = (j < m0) ? list0[j] : list1[j - m0];
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int item = e[q].y;
                    Ci[q] = (item >= 0) ? a.Corig[item] : 0.0f;
                    Gi[q] = (item >= 0) ? a.Gorig[item] : 0.0f;
                }
                int it[4];
                bool anyk = false;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float sv = __int_as_float(e[q].x);
                    const float eb = fmaf(uA, Ci[q], fmaf(uB, Gi[q], us));
                    it[q] = (e[q].y >= 0 && sv + eb >= thr) ? e[q].y : -1;
                    anyk = anyk || it[q] >= 0;
                }
                if (!anyk) continue;
                double k4[4];
                keys4(urow, a.I, a.f, it, k4);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (it[q] < 0) continue;
                    const double key = k4[q];
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

template <int PREC, int KM, int NCH, int UB>
static hipError_t go_screen(const ScreenPlan& p, const ScreenArgs& a, hipStream_t s) {
    if (a.walk)
        screen_kernel<PREC, KM, NCH, UB, true><<<dim3((unsigned)p.n_waves), dim3(64), 0, s>>>(a);
    else
        screen_kernel<PREC, KM, NCH, UB, false><<<dim3((unsigned)p.n_waves), dim3(64), 0, s>>>(a);
    return hipGetLastError();
}

template <int PREC, int NCH>
static hipError_t screen_km(const ScreenPlan& p, const ScreenArgs& a, hipStream_t s) {
    switch (p.KM) {
        case 1:  return go_screen<PREC, 1, NCH, ub_for(PREC, 1, NCH)>(p, a, s);
        case 8:  return go_screen<PREC, 8, NCH, ub_for(PREC, 8, NCH)>(p, a, s);
        case 10: return go_screen<PREC, 10, NCH, ub_for(PREC, 10, NCH)>(p, a, s);
        case 16: return go_screen<PREC, 16, NCH, ub_for(PREC, 16, NCH)>(p, a, s);
        case 32: return go_screen<PREC, 32, NCH, ub_for(PREC, 32, NCH)>(p, a, s);
        default: return go_screen<PREC, 64, NCH, ub_for(PREC, 64, NCH)>(p, a, s);
    }
}

}  // namespace mips
