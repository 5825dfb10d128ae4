// Certification of the screen's candidates with a float64 rescore, the exact
// float64 fallback, and the screen launch dispatcher.
#include "screen_core.h"

namespace mips {

// ---------------------------------------------------------------------------
// Certification: keep the candidates whose upper bound reaches tau_u,
// rescore them in float64 (left to right), and emit the first K by
// (key desc, item index asc).  Same wave/user mapping as the screen.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool before(double ka, int ia, double kb, int ib) {
    return ka > kb || (ka == kb && ia < ib);
}

// float64 key of (u, i): left-to-right sum over the factors, read two floats
// at a time when both rows are 8-byte aligned (f even).
__device__ __forceinline__ double dot64_rows(const float* __restrict__ u,
                                             const float* __restrict__ v, int f) {
    double acc = 0.0;
    if ((f & 1) == 0) {
        const float2* u2 = (const float2*)u;
        const float2* v2 = (const float2*)v;
        for (int j = 0; j < (f >> 1); ++j) {
            const float2 x = u2[j], y = v2[j];
            acc = __fma_rn((double)x.x, (double)y.x, acc);
            acc = __fma_rn((double)x.y, (double)y.y, acc);
        }
        return acc;
    }
    return dot64(u, v, f);
}

// One wave per block of 32 users (same lane mapping as the screen: lane l
// holds half l/32 of user l%32's candidates).
__global__ void __launch_bounds__(64) certify_kernel(const ScreenArgs a, int UB) {
    extern __shared__ unsigned char smem[];
    const int K = a.K;
    double* skey = (double*)smem;                       // [64][K]
    int* sidx = (int*)(smem + sizeof(double) * 64 * K); // [64][K]
    __shared__ int scnt[64];
    const int lane = threadIdx.x, n = lane & 31, h = lane >> 5;
    const int64_t ublk = blockIdx.x;
    const int64_t w = ublk / UB;
    const int ub = (int)(ublk - w * UB);
    int4 tile = make_int4(0, 0, 0, 0);
    if (a.walk) tile = a.tiles[w];
    double* mykey = skey + lane * K;
    int* myidx = sidx + lane * K;

    bool valid;
    const int64_t u = user_of(a, UB, w, ub, n, tile, &valid);
    const int c = valid ? a.cnt[(ublk << 6) + lane] : 0;
    const bool flagged = valid ? (a.uflag[u] != 0) : true;
    const float4 us = valid ? a.uscal[u] : make_float4(0.f, 0.f, 0.f, 0.f);
    const bool bad = c > a.cap;
    int kept = 0;
    unsigned long long st_resc = 0;
    double st_abs = 0.0, st_rel = 0.0;
    if (!flagged) {
        const float* urow = a.U + u * a.f;
        const int cm = min(c, a.cap);
        const int2* cbase = a.cand + ((ublk * a.cap) << 6) + lane;
        constexpr int CH = 4;     // candidates fetched together
        for (int s0 = 0; s0 < cm; s0 += CH) {
            int2 e[CH];
            float Ci[CH], Gi[CH];
#pragma unroll
            for (int q = 0; q < CH; ++q) e[q] = (s0 + q < cm) ? cbase[(int64_t)(s0 + q) << 6] : make_int2(0, -1);
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                Ci[q] = (e[q].y >= 0) ? a.Corig[e[q].y] : 0.0f;
                Gi[q] = (e[q].y >= 0) ? a.Gorig[e[q].y] : 0.0f;
            }
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                const int item = e[q].y;
                if (item < 0) continue;
                const float sv = __int_as_float(e[q].x);
                const float eb = fmaf(us.x, Ci[q], fmaf(us.y, Gi[q], us.z));
                if (!(sv + eb >= us.w)) continue;
                const double key = dot64_rows(urow, a.I + (int64_t)item * a.f, a.f);
                const double err = fabs((double)sv - key);
                st_abs = fmax(st_abs, err);
                const double scale = (us.y > 0.0f ? (double)us.y : (double)us.x) * (double)Ci[q];
                if (scale > 0.0) st_rel = fmax(st_rel, err / scale);
                ++st_resc;
                // insert into this lane's sorted top-K list
                const int len = kept < K ? kept : K;
                ++kept;
                if (len == K && !before(key, item, mykey[K - 1], myidx[K - 1])) continue;
                int pos = (len < K) ? len : K - 1;
                while (pos > 0 && before(key, item, mykey[pos - 1], myidx[pos - 1])) {
                    mykey[pos] = mykey[pos - 1];
                    myidx[pos] = myidx[pos - 1];
                    --pos;
                }
                mykey[pos] = key;
                myidx[pos] = item;
            }
        }
    }
    const int own = kept < K ? kept : K;
    scnt[lane] = own;
    __syncthreads();
    const int other = scnt[lane ^ 32];
    const int tot = kept + xor32_i(kept);
    const int bad_p = xor32_i((int)bad);   // all lanes exchange
    const bool anybad = bad || (bad_p != 0);
    const int ctot = c + xor32_i(c);
    if (valid && !flagged) {
        if (anybad || tot < K) {
            if (h == 0) flag_user(a, u);
        } else {
            const double* pk = skey + (lane ^ 32) * K;
            const int* pi = sidx + (lane ^ 32) * K;
            for (int x = 0; x < own; ++x) {
                const double kx = mykey[x];
                const int ix = myidx[x];
                int rank = x;   // own list is sorted
                for (int y = 0; y < other; ++y) rank += before(pk[y], pi[y], kx, ix) ? 1 : 0;
                if (rank < K) {
                    a.out_idx[u * K + rank] = ix;
                    a.out_score[u * K + rank] = kx;
                }
            }
        }
    }
    // wave reductions of the statistics, one atomic each
    unsigned long long st_cand = (!flagged) ? (unsigned long long)c : 0ull;
    unsigned long long st_max = (valid && h == 0) ? (unsigned long long)ctot : 0ull;
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

__global__ void __launch_bounds__(256) fallback_kernel(const FallbackArgs a) {
    __shared__ unsigned int hist[256];
    __shared__ double skey[kFallbackMaxK];
    __shared__ int sidx[kFallbackMaxK];
    __shared__ unsigned long long s_prefix;
    __shared__ unsigned int s_need, s_sel, s_wave[4];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const unsigned int count = a.ctrl->fb_count;
    double* keys = a.keys + (int64_t)blockIdx.x * a.n_i;
    const int K = a.K;
    for (unsigned int t = blockIdx.x; t < count; t += gridDim.x) {
        const int64_t u = a.flist[t];
        const float* urow = a.U + u * a.f;
        for (int64_t i = tid; i < a.n_i; i += 256) keys[i] = dot64(urow, a.I + i * a.f, a.f);
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
                if (slot < (unsigned)kFallbackMaxK) { skey[slot] = k; sidx[slot] = (int)i; }
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

hipError_t launch_certify(const ScreenPlan& p, const ScreenArgs& a, hipStream_t s) {
    const size_t shm = (sizeof(double) + sizeof(int)) * 64 * (size_t)p.K;
    certify_kernel<<<dim3((unsigned)p.n_ublk), dim3(64), shm, s>>>(a, p.UB);
    return hipGetLastError();
}

hipError_t launch_flag_all(int64_t n_u, int* uflag, int* flist, Ctrl* ctrl, hipStream_t s) {
    flag_all_kernel<<<dim3((unsigned)((n_u + 255) / 256)), dim3(256), 0, s>>>(n_u, uflag, flist, ctrl);
    return hipGetLastError();
}

hipError_t launch_fallback(const ScreenPlan& p, const FallbackArgs& a, hipStream_t s) {
    fallback_kernel<<<dim3((unsigned)p.fb_grid), dim3(256), 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace mips
