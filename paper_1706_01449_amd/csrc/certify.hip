// Certification of the screen's candidates with a float64 rescore, the exact
// float64 fallback, and the screen launch dispatcher.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "screen_core.h"

namespace mips {

// ---------------------------------------------------------------------------
// Certification: keep the candidates whose upper bound reaches tau_u,
// rescore them in float64 (left to right), and emit the first K by
// (key desc, item index asc).  Same wave/user mapping as the screen.
// ---------------------------------------------------------------------------
// G lanes per user (a group, contiguous in the wave), EM kept pairs per lane.
// The screen left each user two candidate lists (its two lanes' halves);
// lane g of the group takes entries g, g+G, ... of their concatenation,
// rescores in float64 those whose upper bound reaches tau_u, and writes the
// ones whose key reaches tau_u to its LDS slots.  The rank of a kept pair among the group's kept
// pairs by (key desc, index asc) is its output position.  A user goes to the
// exact fallback when a candidate list overflowed, a lane kept more than EM
// pairs, or fewer than K pairs were kept.
template <int G, int EM>
__global__ void __launch_bounds__(256) certify_kernel(const ScreenArgs a, int UB, int64_t n_ublk) {
    __shared__ double skey[256 * EM];
    __shared__ int sidx[256 * EM];
    __shared__ int scnt[256];
    const int t = threadIdx.x;
    const int g = t & (G - 1);
    const int gbase = t - g;                 // first thread of this group
    const int64_t slotu = (blockIdx.x * (int64_t)256 + t) / G;   // user slot in screen order
    const int64_t ublk = slotu >> 5;
    const int n = (int)(slotu & 31);
    const int K = a.K;

    bool valid = false;
    int64_t u = 0;
    int c0 = 0, c1 = 0;
    if (ublk < n_ublk) {
        const int64_t w = ublk / UB;
        const int ub = (int)(ublk - w * UB);
        int4 tile = make_int4(0, 0, 0, 0);
        if (a.walk) tile = a.tiles[w];
        u = user_of(a, UB, w, ub, n, tile, &valid);
        c0 = a.cnt[(ublk << 6) + n];
        c1 = a.cnt[(ublk << 6) + n + 32];
    }
    const bool flagged = valid ? (a.uflag[u] != 0) : true;
    bool bad = (c0 > a.cap) || (c1 > a.cap);
    const int m0 = min(c0, a.cap), m1 = min(c1, a.cap);
    const int tot = flagged ? 0 : m0 + m1;
    int kept = 0, rescored = 0;
    double st_abs = 0.0, st_rel = 0.0;
    if (!flagged) {
        const float4 us = a.uscal[u];
        const double tau64 = (double)us.w;
        const float* urow = a.U + u * a.f;
        double unorm = 0.0;   // ||u||, for the relative error statistic only
        if (a.want_stats) {
            for (int j = 0; j < a.f; ++j) unorm += (double)urow[j] * (double)urow[j];
            unorm = sqrt(unorm);
        }
        // the user's two lists (lanes n and n+32 of its screen wave)
        const int64_t base0 = cand_base(ublk, n, a.cap, a.cand_lm), base1 = cand_base(ublk, n + 32, a.cap, a.cand_lm);
        const int cst = cand_stride(a.cand_lm);
        for (int j0 = g; j0 < tot; j0 += 4 * G) {
            int2 e[4];
            float Ci[4], Gi[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = j0 + q * G;
                e[q] = make_int2(0, -1);
                if (j < tot) e[q] = a.cand[(j < m0) ? base0 + j * cst : base1 + (j - m0) * cst];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) e[q].y = cand_item(a, e[q].y);
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
                const int item = e[q].y;
                const float sv = __int_as_float(e[q].x);
                const float eb = fmaf(us.x, Ci[q], fmaf(us.y, Gi[q], us.z));
                it[q] = (item >= 0 && sv + eb >= us.w) ? item : -1;
                anyk = anyk || it[q] >= 0;
            }
            if (!anyk) continue;
            double k4[4];
            keys4(urow, a.I, a.f, it, k4);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int item = it[q];
                if (item < 0) continue;
                const float sv = __int_as_float(e[q].x);
                const double key = k4[q];
                ++rescored;
                if (a.want_stats) {
                    const double err = fabs((double)sv - key);
                    st_abs = fmax(st_abs, err);
                    const double scale = unorm * (double)Ci[q];
                    if (scale > 0.0) st_rel = fmax(st_rel, err / scale);
                }
                // tau_u is at most the K-th largest key, so a pair whose key
                // is below it is beaten by K items and needs no rank
                if (key < tau64) continue;
                if (kept < EM) {
                    skey[t * EM + kept] = key;
                    sidx[t * EM + kept] = item;
                }
                ++kept;
            }
        }
    }
    if (kept > EM) bad = true;
    scnt[t] = kept < EM ? kept : EM;
    // group totals and flags
    int gk = kept;
    int gb = bad ? 1 : 0;
    for (int off = G / 2; off >= 1; off >>= 1) {
        gk += __shfl_xor(gk, off, G);
        gb |= __shfl_xor(gb, off, G);
    }
    __syncthreads();
    if (valid && !flagged) {
        if (gb || gk < K) {
            if (g == 0) flag_user(a, u);
        } else {
            const int own = scnt[t];
            for (int x = 0; x < own; ++x) {
                const double kx = skey[t * EM + x];
                const int ix = sidx[t * EM + x];
                int rank = 0;
                for (int q = 0; q < G; ++q) {
                    const int o = gbase + q;
                    const int no = scnt[o];
                    for (int y = 0; y < no; ++y)
                        rank += before(skey[o * EM + y], sidx[o * EM + y], kx, ix) ? 1 : 0;
                }
                if (rank < K) {
                    a.out_idx[u * K + rank] = ix;
                    a.out_score[u * K + rank] = kx;
                }
            }
        }
    }
    if (!a.want_stats) return;
    // statistics: reduce over the wave, one atomic each
    unsigned long long st_cand = (g == 0 && !flagged) ? (unsigned long long)(c0 + c1) : 0ull;
    unsigned long long st_max = (g == 0 && valid) ? (unsigned long long)(c0 + c1) : 0ull;
    unsigned long long st_resc = (unsigned long long)rescored;
    for (int off = 32; off >= 1; off >>= 1) {
        st_cand += __shfl_xor(st_cand, off);
        st_resc += __shfl_xor(st_resc, off);
        st_max = max(st_max, (unsigned long long)__shfl_xor(st_max, off));
        st_abs = fmax(st_abs, __shfl_xor(st_abs, off));
        st_rel = fmax(st_rel, __shfl_xor(st_rel, off));
    }
    if ((t & 63) == 0) {
        if (st_cand) atomicAdd(&a.ctrl->cand_total, st_cand);
        if (st_resc) atomicAdd(&a.ctrl->rescored, st_resc);
        if (st_max) atomicMax(&a.ctrl->cand_max, st_max);
        atomic_max_nonneg((double*)&a.ctrl->max_abs_err, st_abs);
        atomic_max_nonneg((double*)&a.ctrl->max_rel_err, st_rel);
    }
}

// ---------------------------------------------------------------------------
// Certification with one wave per user, for long candidate lists (E4M3, or
// K > 16).  The candidates whose upper bound reaches the threshold are
// rescored 64 at a time: their item rows are staged through LDS in blocks of
// 16 factors with coalesced loads (64-byte row segments rather than one
// scattered 8-byte load per lane), and lane r continues the left-to-right
// float64 sum of row r.  After each block of 64 rescored pairs the K-th
// largest key seen so far replaces tau_u when larger (it is the K-th largest
// key of a subset, so still at most the user's K-th largest key), which
// removes most later candidates before their rows are read.  Kept pairs
// (key >= threshold) stay in LDS, pruned to the threshold after each block.
//
// Cascade (CASC, E4M3 screens): before the float64 rescore, each block of 64
// surviving candidates is re-screened with bfloat16 copies of the user and
// item rows (float32 sum, the screen's error bound with bfloat16 residual
// norms).  The K-th largest bfloat16 lower bound also raises the threshold,
// and only pairs whose bfloat16 upper bound reaches it are rescored, which
// reads 2-byte instead of 4-byte factors for most of the E4M3 candidates.
// ---------------------------------------------------------------------------
constexpr int kCwCols = 16;      // factors per staged block
constexpr int kCwKeys = 128;     // kept pairs per user (more: exact fallback)

template <int VEC, bool CASC>
__global__ void __launch_bounds__(64) certify_wave_kernel(const ScreenArgs a, int UB, int64_t n_ublk) {
    typedef float __attribute__((ext_vector_type(VEC))) vec_t;
    constexpr int NV = kCwCols / VEC;          // vectors per row and block
    constexpr int LOADS = 64 * NV / 64;        // vector loads per lane and block
    constexpr int CB = 2 * kCwCols;            // bfloat16 factors per staged block
    constexpr int LB = CB / 8;                 // 16-byte loads per lane and block (bfloat16)
    __shared__ double su[256];
    __shared__ float sub[CASC ? 256 : 1];      // bfloat16 copy of u (as floats)
    __shared__ int2 pend[128];                 // candidates passing the screen's bound
    __shared__ int2 pend2[CASC ? 128 : 1];     // ... and the bfloat16 bound
    __shared__ __attribute__((aligned(16))) float stage[64][kCwCols + 4];
    __shared__ double skey[kCwKeys];
    __shared__ int sidx[kCwKeys];
    __shared__ double slb[CASC ? kCwKeys : 1]; // bfloat16 lower bounds >= threshold
    const int lane = threadIdx.x;
    const uint64_t below = (1ull << lane) - 1ull;
    const int64_t ublk = (int64_t)blockIdx.x >> 5;
    const int n = (int)(blockIdx.x & 31);
    if (ublk >= n_ublk) return;
    const int64_t w = ublk / UB;
    const int ub = (int)(ublk - w * UB);
    int4 tile = make_int4(0, 0, 0, 0);
    if (a.walk) tile = a.tiles[w];
    bool valid;
    const int64_t u = user_of(a, UB, w, ub, n, tile, &valid);
    if (!valid) return;
    const int c0 = a.cnt[(ublk << 6) + n], c1 = a.cnt[(ublk << 6) + n + 32];
    const bool flagged = a.uflag[u] != 0;
    const bool over = c0 > a.cap || c1 > a.cap;
    if (flagged || over) {
        if (lane == 0) {
            if (!flagged) flag_user(a, u);
            if (a.want_stats) {
                if (!flagged) atomicAdd(&a.ctrl->cand_total, (unsigned long long)(c0 + c1));
                atomicMax(&a.ctrl->cand_max, (unsigned long long)(c0 + c1));
            }
        }
        return;
    }
    const int f = a.f, K = a.K;
    const float* urow = a.U + u * f;
    for (int j = lane; j < f; j += 64) su[j] = (double)urow[j];
    // bfloat16 re-screen bound of this user (as in the screen's prologue)
    float Ab = 0.0f, Bb = 0.0f, Sb = 0.0f;
    if (CASC) {
        double s2 = 0.0, r2 = 0.0, q2 = 0.0;
        for (int j = lane; j < a.fpb; j += 64) {
            const float x = j < f ? urow[j] : 0.0f;
            const float d = bf16_bits_to_f32(f32_to_bf16_bits(x));
            s2 += (double)x * (double)x;
            r2 += ((double)x - (double)d) * ((double)x - (double)d);
            q2 += (double)d * (double)d;
            sub[j] = d;
        }
        for (int off = 32; off >= 1; off >>= 1) {
            s2 += __shfl_xor(s2, off);
            r2 += __shfl_xor(r2, off);
            q2 += __shfl_xor(q2, off);
        }
        const double N64 = sqrt(s2);
        Ab = norm_up_f32(sqrt(r2) + (double)f * 0x1p-52 * N64);
        Bb = norm_up_f32(sqrt(q2));
        const double Cmax = (double)__uint_as_float(a.maxb[0]);
        const double Emax = (double)__uint_as_float(a.maxb[1]);
        const double Gmax = (double)__uint_as_float(a.maxb[2]);
        const double M = N64 * Cmax * 1.01 + (double)Bb * Emax * 1.01 + (double)Ab * Cmax +
                         (double)Bb * Gmax;
        Sb = round_up_f32(M * 0x1p-20 + 0x1p-100);
    }
    const float4 us = a.uscal[u];
    double tau64 = (double)us.w;       // kept pairs: key >= tau64
    float thr = us.w;                  // candidates: upper bound >= thr (thr <= tau64)
    const int tot = c0 + c1;
    const int64_t base0 = cand_base(ublk, n, a.cap, a.cand_lm), base1 = cand_base(ublk, n + 32, a.cap, a.cand_lm);
    const int cst = cand_stride(a.cand_lm);
    __syncthreads();
    double unorm = 0.0;   // ||u||, for the relative error statistic only
    if (a.want_stats) {
        for (int j = 0; j < f; ++j) unorm += su[j] * su[j];
        unorm = sqrt(unorm);
    }
    int npend = 0, npend2 = 0, nk = 0, nlb = 0, rescored = 0;
    bool lost = false;                 // more than kCwKeys kept pairs
    double st_abs = 0.0, st_rel = 0.0;

    // K-th largest of v[0 .. m) (-inf when m < K): the entry with fewer than
    // K values above it and at least K at or above it.
    auto kth_of = [&](const double* v, int m) __attribute__((always_inline)) {
        double kth = -__builtin_inf();
        if (m < K) return kth;
        for (int x = lane; x < m; x += 64) {
            const double vx = v[x];
            int gt = 0, ge = 0;
            for (int y = 0; y < m; ++y) {
                const double vy = v[y];
                gt += vy > vx ? 1 : 0;
                ge += vy >= vx ? 1 : 0;
            }
            if (gt < K && ge >= K) kth = vx;
        }
        for (int off = 32; off >= 1; off >>= 1) kth = fmax(kth, __shfl_xor(kth, off));
        return kth;
    };
    // drop the entries of v (and of ix, when given) below t; returns the count left
    auto prune = [&](double* v, int* ix, int m, double t) __attribute__((always_inline)) {
        double kv[kCwKeys / 64];
        int ki[kCwKeys / 64];
        bool kp[kCwKeys / 64];
#pragma unroll
        for (int q = 0; q < kCwKeys / 64; ++q) {
            const int x = q * 64 + lane;
            kp[q] = x < m && v[x] >= t;
            kv[q] = kp[q] ? v[x] : 0.0;
            ki[q] = (kp[q] && ix) ? ix[x] : 0;
        }
        __syncthreads();
        int r = 0;
#pragma unroll
        for (int q = 0; q < kCwKeys / 64; ++q) {
            const uint64_t bq = ballot(kp[q]);
            if (kp[q]) {
                const int p2 = r + __builtin_popcountll(bq & below);
                v[p2] = kv[q];
                if (ix) ix[p2] = ki[q];
            }
            r += __builtin_popcountll(bq);
        }
        __syncthreads();
        return r;
    };

    // Rescore src[0 .. nr) in float64: stage the rows, sum, keep keys >=
    // tau64, then raise tau64 / thr to the K-th largest kept key and prune.
    auto rescore = [&](const int2* src, int nr) __attribute__((always_inline)) {
        const float* rowp[LOADS];
        int col[LOADS];
#pragma unroll
        for (int s = 0; s < LOADS; ++s) {
            const int e = s * 64 + lane, r = e / NV;
            col[s] = (e - r * NV) * VEC;
            rowp[s] = (r < nr) ? a.I + (int64_t)src[r].y * f : nullptr;
        }
        vec_t v[LOADS];
        auto load = [&](int j0) __attribute__((always_inline)) {
#pragma unroll
            for (int s = 0; s < LOADS; ++s) {
                const int c = j0 + col[s];
                if (rowp[s] && c < f) v[s] = *(const vec_t*)(rowp[s] + c);
            }
        };
        load(0);
        double acc = 0.0;
        for (int j0 = 0; j0 < f; j0 += kCwCols) {
            __syncthreads();   // the previous block's sums have read the stage
#pragma unroll
            for (int s = 0; s < LOADS; ++s) {
                const int e = s * 64 + lane, r = e / NV;
                if (rowp[s] && j0 + col[s] < f) *(vec_t*)&stage[r][col[s]] = v[s];
            }
            __syncthreads();
            if (j0 + kCwCols < f) load(j0 + kCwCols);
            const int nc = min(kCwCols, f - j0);
            if (lane < nr) {
                if (nc == kCwCols) {
#pragma unroll
                    for (int c = 0; c < kCwCols; ++c)
                        acc = __fma_rn(su[j0 + c], (double)stage[lane][c], acc);
                } else {
                    for (int c = 0; c < nc; ++c)
                        acc = __fma_rn(su[j0 + c], (double)stage[lane][c], acc);
                }
            }
        }
        const bool has = lane < nr;
        const int2 ent = has ? src[lane] : make_int2(0, -1);
        if (has && a.want_stats) {
            const double err = fabs((double)__int_as_float(ent.x) - acc);
            st_abs = fmax(st_abs, err);
            const double scale = unorm * (double)a.Corig[ent.y];
            if (scale > 0.0) st_rel = fmax(st_rel, err / scale);
        }
        rescored += nr;
        const bool take = has && acc >= tau64;
        const uint64_t bt = ballot(take);
        const int pos = nk + __builtin_popcountll(bt & below);
        if (take && pos < kCwKeys) { skey[pos] = acc; sidx[pos] = ent.y; }
        nk += __builtin_popcountll(bt);
        if (nk > kCwKeys) { lost = true; nk = kCwKeys; }
        __syncthreads();
        if (nk < K || lost) return;
        const double kth = kth_of(skey, nk);
        if (kth > tau64) {
            tau64 = kth;
            thr = fmaxf(thr, __double2float_rd(kth));
        }
        nk = prune(skey, sidx, nk, tau64);
    };

    // bfloat16 re-screen of pend[0 .. nr) into pend2 (CASC only).
    auto cascade = [&](int nr) __attribute__((always_inline)) {
        const uint16_t* rowb[LB];
        int colb[LB];
#pragma unroll
        for (int s = 0; s < LB; ++s) {
            const int e = s * 64 + lane, r = e / (CB / 8);
            colb[s] = (e - r * (CB / 8)) * 8;
            rowb[s] = (r < nr) ? (const uint16_t*)a.qrow_b + (int64_t)pend[r].y * a.fpb : nullptr;
        }
        float acc = 0.0f;
        for (int j0 = 0; j0 < a.fpb; j0 += CB) {
            intx4_t v[LB];
#pragma unroll
            for (int s = 0; s < LB; ++s)
                if (rowb[s] && j0 + colb[s] < a.fpb) v[s] = *(const intx4_t*)(rowb[s] + j0 + colb[s]);
            __syncthreads();   // the previous block's sums have read the stage
#pragma unroll
            for (int s = 0; s < LB; ++s) {
                const int e = s * 64 + lane, r = e / (CB / 8);
                if (rowb[s] && j0 + colb[s] < a.fpb) *(intx4_t*)&stage[r][colb[s] / 2] = v[s];
            }
            __syncthreads();
            const int nc = min(CB, a.fpb - j0);
            if (lane < nr) {
                if (nc == CB) {
                    const intx4_t* rs4 = (const intx4_t*)&stage[lane][0];
#pragma unroll
                    for (int q = 0; q < CB / 8; ++q) {
                        const intx4_t wv = rs4[q];
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const uint32_t wd = (uint32_t)wv[t];
                            acc = fmaf(sub[j0 + 8 * q + 2 * t], __uint_as_float(wd << 16), acc);
                            acc = fmaf(sub[j0 + 8 * q + 2 * t + 1], __uint_as_float(wd & 0xffff0000u), acc);
                        }
                    }
                } else {
                    const uint16_t* rs = (const uint16_t*)&stage[lane][0];
                    for (int c = 0; c < nc; ++c) acc = fmaf(sub[j0 + c], bf16_bits_to_f32(rs[c]), acc);
                }
            }
        }
        const bool has = lane < nr;
        const int2 ent = has ? pend[lane] : make_int2(0, -1);
        float lb = -__builtin_inff(), ubd = -__builtin_inff();
        if (has) {
            const float e = fmaf(Ab, a.Corig[ent.y], fmaf(Bb, a.Gorig_b[ent.y], Sb));
            lb = acc - e;
            ubd = acc + e;
        }
        // lower bounds of distinct items: their K-th largest raises thr
        const bool tl = has && lb >= thr;
        const uint64_t bl = ballot(tl);
        const int pl = nlb + __builtin_popcountll(bl & below);
        if (tl && pl < kCwKeys) slb[pl] = (double)lb;
        nlb = min(kCwKeys, nlb + __builtin_popcountll(bl));   // a subset still bounds
        __syncthreads();
        const double kl = kth_of(slb, nlb);
        if (kl > (double)thr) {
            thr = (float)kl;   // a float32 lower bound: exact
            tau64 = fmax(tau64, kl);
        }
        if (nlb >= K) nlb = prune(slb, nullptr, nlb, (double)thr);
        // pairs whose bfloat16 upper bound reaches thr go to the rescore
        const bool pass = has && ubd >= thr;
        const uint64_t bp = ballot(pass);
        if (pass) pend2[npend2 + __builtin_popcountll(bp & below)] = ent;
        npend2 += __builtin_popcountll(bp);
        if (npend2 >= 64) {
            __syncthreads();
            rescore(pend2, 64);
            const int rest = npend2 - 64;
            const int2 t = (lane < rest) ? pend2[64 + lane] : make_int2(0, -1);
            __syncthreads();
            if (lane < rest) pend2[lane] = t;
            npend2 = rest;
        }
    };

    for (int base = 0; base < tot; base += 64) {
        const int j = base + lane;
        int2 e = make_int2(0, -1);
        if (j < tot) e = a.cand[(j < c0) ? base0 + j * cst : base1 + (j - c0) * cst];
        e.y = cand_item(a, e.y);
        bool keep = false;
        if (e.y >= 0) {
            const float eb = fmaf(us.x, a.Corig[e.y], fmaf(us.y, a.Gorig[e.y], us.z));
            keep = __int_as_float(e.x) + eb >= thr;
        }
        const uint64_t bk = ballot(keep);
        if (keep) pend[npend + __builtin_popcountll(bk & below)] = e;
        npend += __builtin_popcountll(bk);
        if (npend >= 64) {
            __syncthreads();
            if (CASC) cascade(64); else rescore(pend, 64);
            const int rest = npend - 64;
            const int2 t = (lane < rest) ? pend[64 + lane] : make_int2(0, -1);
            __syncthreads();
            if (lane < rest) pend[lane] = t;
            npend = rest;
        }
    }
    if (npend > 0) {
        __syncthreads();
        if (CASC) cascade(npend); else rescore(pend, npend);
    }
    if (CASC && npend2 > 0) {
        __syncthreads();
        rescore(pend2, npend2);
    }
    if (lost || nk < K) {
        if (lane == 0) flag_user(a, u);
    } else {
        for (int x = lane; x < nk; x += 64) {
            const double kx = skey[x];
            const int ix = sidx[x];
            int rank = 0;
            for (int y = 0; y < nk; ++y) rank += before(skey[y], sidx[y], kx, ix) ? 1 : 0;
            if (rank < K) {
                a.out_idx[u * K + rank] = ix;
                a.out_score[u * K + rank] = kx;
            }
        }
    }
    if (!a.want_stats) return;
    for (int off = 32; off >= 1; off >>= 1) {
        st_abs = fmax(st_abs, __shfl_xor(st_abs, off));
        st_rel = fmax(st_rel, __shfl_xor(st_rel, off));
    }
    if (lane == 0) {
        atomicAdd(&a.ctrl->cand_total, (unsigned long long)tot);
        atomicMax(&a.ctrl->cand_max, (unsigned long long)tot);
        if (rescored) atomicAdd(&a.ctrl->rescored, (unsigned long long)rescored);
        atomic_max_nonneg((double*)&a.ctrl->max_abs_err, st_abs);
        atomic_max_nonneg((double*)&a.ctrl->max_rel_err, st_rel);
    }
}

// ---------------------------------------------------------------------------
// Exact float64 fallback: all keys of a flagged user, radix selection of the
// K-th (key desc, index asc), then ranks.  Used for users whose candidate
// buffer overflowed, degenerate users (zero, non-finite, out of range) and
// requests outside the screen's compiled shapes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long ordered(double k) {
    unsigned long long b = (unsigned long long)__double_as_longlong(k);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// Keys of one user against all items, 256 items per step: the items' rows
// are staged through LDS 32 factors at a time with coalesced loads, then
// each thread continues its item's left-to-right float64 sum.
constexpr int kFbRows = 256, kFbCols = 32;

__device__ __forceinline__ void fallback_keys(const FallbackArgs& a, const float* su,
                                              float (*srow)[kFbCols + 1], double* keys) {
    const int tid = threadIdx.x;
    const int f = a.f;
    for (int64_t base = 0; base < a.n_i; base += kFbRows) {
        const int nr = (int)min((int64_t)kFbRows, a.n_i - base);
        const float* src = a.I + base * f;
        double acc = 0.0;
        for (int j0 = 0; j0 < f; j0 += kFbCols) {
            const int nc = min(kFbCols, f - j0);
            __syncthreads();
            for (int e = tid; e < kFbRows * kFbCols; e += kFbRows) {
                const int r = e / kFbCols, c = e - r * kFbCols;
                if (r < nr && c < nc) srow[r][c] = src[(int64_t)r * f + j0 + c];
            }
            __syncthreads();
            if (tid < nr)
                for (int c = 0; c < nc; ++c)
                    acc = __fma_rn((double)su[j0 + c], (double)srow[tid][c], acc);
        }
        if (tid < nr) keys[base + tid] = acc;
    }
    __syncthreads();
}

// Keys of the first a.pre_users fallback users, spread over the device:
// workgroup (x, y) takes users y, y + gridDim.y, ... and item blocks
// x, x + gridDim.x, ... of 256 items, one item per thread with its row read
// directly (a wave's rows are re-read from the cache line by line), the
// user's row from LDS.  User t's keys go to slot t.
__global__ void __launch_bounds__(256) fallback_keys_kernel(const FallbackArgs a) {
    __shared__ float su[256];
    const unsigned int count = min(a.ctrl->fb_count, (unsigned)a.pre_users);
    const int64_t nb = (a.n_i + 255) / 256;
    for (unsigned int t = blockIdx.y; t < count; t += gridDim.y) {
        const int64_t u = a.flist[t];
        __syncthreads();
        for (int j = threadIdx.x; j < a.f; j += 256) su[j] = a.U[u * a.f + j];
        __syncthreads();
        for (int64_t blk = blockIdx.x; blk < nb; blk += gridDim.x) {
            const int64_t i = blk * 256 + threadIdx.x;
            if (i >= a.n_i) continue;
            const float* row = a.I + i * a.f;
            double acc = 0.0;
            int j = 0;
            if ((a.f & 1) == 0) {
                const float2* r2 = (const float2*)row;
                for (; j + 16 <= a.f; j += 16) {
                    float2 y[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) y[e] = r2[(j >> 1) + e];
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        acc = __fma_rn((double)su[j + 2 * e], (double)y[e].x, acc);
                        acc = __fma_rn((double)su[j + 2 * e + 1], (double)y[e].y, acc);
                    }
                }
            }
            for (; j < a.f; ++j) acc = __fma_rn((double)su[j], (double)row[j], acc);
            a.keys[(int64_t)t * a.n_i + i] = acc;
        }
    }
}

// KMAX: the largest K the kernel serves (its LDS slots for the selected
// pairs); the small instance leaves room for several workgroups per CU.
template <int KMAX>
__global__ void __launch_bounds__(256) fallback_kernel(const FallbackArgs a) {
    __shared__ unsigned int hist[256];
    __shared__ double skey[KMAX];
    __shared__ int sidx[KMAX];
    __shared__ float su[256];
    __shared__ float srow[kFbRows][kFbCols + 1];
    __shared__ unsigned long long s_prefix;
    __shared__ unsigned int s_need, s_sel, s_wave[4];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const unsigned int count = a.ctrl->fb_count;
    double* keys = a.keys + (int64_t)blockIdx.x * a.n_i;
    const int K = a.K;
    for (unsigned int t = blockIdx.x; t < count; t += gridDim.x) {
        const int64_t u = a.flist[t];
        const float* urow = a.U + u * a.f;
        __syncthreads();
        if (t >= (unsigned)a.pre_users) {     // keys not precomputed by fallback_keys_kernel
            for (int j = tid; j < a.f; j += 256) su[j] = urow[j];
            fallback_keys(a, su, srow, keys);
        }
        if (tid == 0) { s_prefix = 0ull; s_need = (unsigned)K; s_sel = 0u; }
        __syncthreads();
        unsigned long long mask = 0ull;
        for (int pass = 7; pass >= 0; --pass) {
            hist[tid] = 0u;
            __syncthreads();
            const unsigned long long prefix = s_prefix;
            for (int64_t i = tid; i < a.n_i; i += 256) {
                const unsigned long long m = ordered(keys[i]);
                if ((m & mask) == prefix) atomicAdd(&hist[(m >> (8 * pass)) & 255u], 1u);
            }
            __syncthreads();
            if (tid == 0) {
                unsigned int need = s_need, cum = 0u;
                int d = 255;
                for (; d > 0; --d) {
                    if (cum + hist[d] >= need) break;
                    cum += hist[d];
                }
                s_need = need - cum;
                s_prefix = prefix | ((unsigned long long)d << (8 * pass));
            }
            mask |= 255ull << (8 * pass);
            __syncthreads();
        }
        const unsigned long long T = s_prefix;
        const unsigned int take_eq = s_need;   // items equal to T to take, lowest indices first
        unsigned int eq_before = 0u;
        for (int64_t base = 0; base < a.n_i; base += 256) {
            const int64_t i = base + tid;
            unsigned long long m = 0ull;
            double k = 0.0;
            if (i < a.n_i) { k = keys[i]; m = ordered(k); }
            const bool gt = i < a.n_i && m > T;
            const bool eq = i < a.n_i && m == T;
            const unsigned long long bal = __builtin_amdgcn_ballot_w64(eq);
            const unsigned int below = __builtin_popcountll(bal & ((1ull << lane) - 1ull));
            if (lane == 0) s_wave[wv] = __builtin_popcountll(bal);
            __syncthreads();
            unsigned int rank = eq_before + below;
            for (int q = 0; q < wv; ++q) rank += s_wave[q];
            const unsigned int chunk_eq = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
            if (gt || (eq && rank < take_eq)) {
                const unsigned int slot = atomicAdd(&s_sel, 1u);
                if (slot < (unsigned)KMAX) { skey[slot] = k; sidx[slot] = (int)i; }
            }
            eq_before += chunk_eq;
            __syncthreads();
        }
        const int sel = (int)min(s_sel, (unsigned)K);
        for (int s = tid; s < sel; s += 256) {
            const double kx = skey[s];
            const int ix = sidx[s];
            int rank = 0;
            for (int y = 0; y < sel; ++y) rank += before(skey[y], sidx[y], kx, ix) ? 1 : 0;
            if (rank < K) {
                a.out_idx[u * K + rank] = ix;
                a.out_score[u * K + rank] = kx;
            }
        }
        __syncthreads();
    }
}

__global__ void flag_all_kernel(int64_t n_u, int* uflag, int* flist, Ctrl* ctrl) {
    int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (u < n_u) { uflag[u] = 1; flist[u] = (int)u; }
    if (u == 0) ctrl->fb_count = (unsigned int)n_u;
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
hipError_t launch_screen(const ScreenPlan& p, const ScreenArgs& a, hipStream_t s) {
    if (p.prec == PREC_BF16) return launch_screen_bf16(p, a, s);
    if (p.prec == PREC_FP8) return launch_screen_fp8(p, a, s);
    return launch_screen_fp32(p, a, s);
}

// Per-user bin of kept candidates in certification (LDS).
hipError_t launch_certify(const ScreenPlan& p, const ScreenArgs& a, hipStream_t s) {
    if (fused_certify(p.prec, p.KM, p.UB)) return hipSuccess;   // done by the screen kernel
    // one wave per user for long candidate lists (E4M3, or K > 16), a group
    // of lanes per user for short ones (the certification test knob forces
    // either kernel)
    bool wave = p.prec == PREC_FP8 || p.K > 16;
    if (debug_certify_kernel() == 1) wave = true;
    if (debug_certify_kernel() == 2) wave = false;
    if (wave) {
        const uintptr_t base = (uintptr_t)a.I;
        const dim3 grid((unsigned)(p.n_ublk * 32)), blk(64);
        // bfloat16 cascade for E4M3 screens when the caller prepared its rows
        const bool casc = p.prec == PREC_FP8 && a.qrow_b != nullptr;
        if (casc) {
            if (p.f % 4 == 0 && base % 16 == 0)
                certify_wave_kernel<4, true><<<grid, blk, 0, s>>>(a, p.UB, p.n_ublk);
            else if (p.f % 2 == 0 && base % 8 == 0)
                certify_wave_kernel<2, true><<<grid, blk, 0, s>>>(a, p.UB, p.n_ublk);
            else
                certify_wave_kernel<1, true><<<grid, blk, 0, s>>>(a, p.UB, p.n_ublk);
        } else {
            if (p.f % 4 == 0 && base % 16 == 0)
                certify_wave_kernel<4, false><<<grid, blk, 0, s>>>(a, p.UB, p.n_ublk);
            else if (p.f % 2 == 0 && base % 8 == 0)
                certify_wave_kernel<2, false><<<grid, blk, 0, s>>>(a, p.UB, p.n_ublk);
            else
                certify_wave_kernel<1, false><<<grid, blk, 0, s>>>(a, p.UB, p.n_ublk);
        }
        return hipGetLastError();
    }
    // lanes per user G and LDS slots per lane EM (pairs whose key reaches
    // tau_u): 64 per user for the float32/bfloat16 screens at K <= 16, 256
    // for larger K or E4M3 at K <= 16, 1024 for E4M3 at larger K
    const bool fp8 = p.prec == PREC_FP8;
    const int G = (!fp8 && p.K <= 16) ? 8 : ((fp8 && p.K > 16) ? 64 : 16);
    const int64_t threads = p.n_ublk * 32 * G;
    const dim3 grid((unsigned)((threads + 255) / 256)), blk(256);
    if (G == 8)
        certify_kernel<8, 8><<<grid, blk, 0, s>>>(a, p.UB, p.n_ublk);
    else if (G == 16)
        certify_kernel<16, 16><<<grid, blk, 0, s>>>(a, p.UB, p.n_ublk);
    else
        certify_kernel<64, 16><<<grid, blk, 0, s>>>(a, p.UB, p.n_ublk);
    return hipGetLastError();
}

hipError_t launch_flag_all(int64_t n_u, int* uflag, int* flist, Ctrl* ctrl, hipStream_t s) {
    flag_all_kernel<<<dim3((unsigned)((n_u + 255) / 256)), dim3(256), 0, s>>>(n_u, uflag, flist, ctrl);
    return hipGetLastError();
}

hipError_t launch_fallback(const ScreenPlan& p, const FallbackArgs& a_in, hipStream_t s) {
    // keys of the first fb_grid fallback users across the whole device (each
    // user's keys land in the slot of the workgroup that selects them), the
    // rest inside the selection kernel
    FallbackArgs a = a_in;
    a.pre_users = p.fb_grid;
    const unsigned xb = (unsigned)std::min<int64_t>(32, (a.n_i + 255) / 256);
    fallback_keys_kernel<<<dim3(xb, 16), dim3(256), 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.K <= 64)
        fallback_kernel<64><<<dim3((unsigned)p.fb_grid), dim3(256), 0, s>>>(a);
    else
        fallback_kernel<kFallbackMaxK><<<dim3((unsigned)p.fb_grid), dim3(256), 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace mips
