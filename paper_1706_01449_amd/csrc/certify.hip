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

// Largest index t in [0, n) with off[t] <= j (off non-decreasing, off[0] = 0).
__device__ __forceinline__ int seg_of(const int* off, int n, int j) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= j) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// One wave per block of 32 users.  The screen left each lane l (user l%32,
// half l/32) a list of candidates; here the whole wave works on them in
// lockstep: (1) every candidate whose upper bound reaches the user's tau is
// kept and binned per user in LDS, (2) the kept pairs are rescored in
// float64 (user rows staged in LDS), (3) each kept pair's rank among its
// user's kept pairs by (key desc, index asc) decides its output slot.
// Users whose candidate lists or bins overflowed, or who kept fewer than K,
// go to the exact fallback.
__global__ void __launch_bounds__(64) certify_kernel(const ScreenArgs a, int UB, int segcap) {
    extern __shared__ double smem_d[];
    const int f = a.f, K = a.K;
    const int lane = threadIdx.x, n = lane & 31, h = lane >> 5;
    const int64_t ublk = blockIdx.x;
    const int64_t w = ublk / UB;
    const int ub = (int)(ublk - w * UB);
    int4 tile = make_int4(0, 0, 0, 0);
    if (a.walk) tile = a.tiles[w];

    // LDS carve-up
    double* segk = smem_d;                                  // [32][segcap] keys
    int* segi = (int*)(segk + 32 * segcap);                 // [32][segcap] items
    float* urow = (float*)(segi + 32 * segcap);             // [32][f] user rows
    __shared__ float4 us[32];
    __shared__ int uval[32], ucnt[32], uoff[33], ubad[32];
    __shared__ int coff[65];
    __shared__ int64_t uid_s[32];

    // ---- users of this block ---------------------------------------------
    bool valid;
    const int64_t u = user_of(a, UB, w, ub, n, tile, &valid);
    const int c = valid ? a.cnt[(ublk << 6) + lane] : 0;
    if (h == 0) {
        const bool fl = valid ? (a.uflag[u] != 0) : true;
        uval[n] = (valid && !fl) ? 1 : 0;
        us[n] = valid ? a.uscal[u] : make_float4(0.f, 0.f, 0.f, 0.f);
        ucnt[n] = 0;
        ubad[n] = 0;
        uid_s[n] = u;
    }
    __syncthreads();
    if (c > a.cap && uval[n]) ubad[n] = 1;                   // either half overflowed
    // lanes' candidate counts -> prefix offsets (skipping users not certified here)
    const int cc = uval[n] ? min(c, a.cap) : 0;
    {
        int incl = cc;
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(incl, off);
            if (lane >= off) incl += v;
        }
        coff[lane + 1] = incl;
        if (lane == 0) coff[0] = 0;
    }
    // stage the user rows (row r of the block = user r)
    for (int t = lane; t < 32 * f; t += 64) {
        const int r = t / f, j = t - r * f;
        urow[t] = uval[r] ? a.U[uid_s[r] * f + j] : 0.0f;
    }
    __syncthreads();
    const int total = coff[64];

    // ---- (1) filter -------------------------------------------------------
    for (int j = lane; j < total; j += 64) {
        const int l = seg_of(coff, 64, j);
        const int slot = j - coff[l];
        const int2 e = a.cand[((ublk * a.cap + slot) << 6) + l];
        const int item = e.y;
        const int r = l & 31;
        const float4 s4 = us[r];
        const float sv = __int_as_float(e.x);
        const float eb = fmaf(s4.x, a.Corig[item], fmaf(s4.y, a.Gorig[item], s4.z));
        if (sv + eb >= s4.w) {
            const int k = atomicAdd(&ucnt[r], 1);
            if (k < segcap) {
                segi[r * segcap + k] = item;
                segk[r * segcap + k] = (double)sv;   // screened score, replaced by the key
            } else {
                ubad[r] = 1;
            }
        }
    }
    __syncthreads();
    if (lane < 32) {
        const int kept = min(ucnt[lane], segcap);
        if (uval[lane] && kept < K) ubad[lane] = 1;
        int incl = (uval[lane] && !ubad[lane]) ? kept : 0;
        for (int off = 1; off < 32; off <<= 1) {
            const int v = __shfl_up(incl, off, 32);
            if (lane >= off) incl += v;
        }
        uoff[lane + 1] = incl;
        if (lane == 0) uoff[0] = 0;
    }
    __syncthreads();
    const int ktot = uoff[32];

    // ---- (2) float64 rescore ----------------------------------------------
    double st_abs = 0.0, st_rel = 0.0;
    for (int j = lane; j < ktot; j += 64) {
        const int r = seg_of(uoff, 32, j);
        const int k = j - uoff[r];
        const int item = segi[r * segcap + k];
        const float* ur = urow + r * f;
        const float* ir = a.I + (int64_t)item * f;
        double acc = 0.0;
        if ((f & 1) == 0) {
            const float2* i2 = (const float2*)ir;
            for (int q = 0; q < (f >> 1); ++q) {
                const float2 y = i2[q];
                acc = __fma_rn((double)ur[2 * q], (double)y.x, acc);
                acc = __fma_rn((double)ur[2 * q + 1], (double)y.y, acc);
            }
        } else {
            for (int q = 0; q < f; ++q) acc = __fma_rn((double)ur[q], (double)ir[q], acc);
        }
        const double sv = segk[r * segcap + k];
        const double err = fabs(sv - acc);
        st_abs = fmax(st_abs, err);
        const float4 s4 = us[r];
        const double scale = (s4.y > 0.0f ? (double)s4.y : (double)s4.x) * (double)a.Corig[item];
        if (scale > 0.0) st_rel = fmax(st_rel, err / scale);
        segk[r * segcap + k] = acc;
    }
    __syncthreads();

    // ---- (3) ranks and output ---------------------------------------------
    for (int j = lane; j < ktot; j += 64) {
        const int r = seg_of(uoff, 32, j);
        const int k = j - uoff[r];
        const int nk = uoff[r + 1] - uoff[r];
        const double kx = segk[r * segcap + k];
        const int ix = segi[r * segcap + k];
        int rank = 0;
        for (int y = 0; y < nk; ++y)
            rank += before(segk[r * segcap + y], segi[r * segcap + y], kx, ix) ? 1 : 0;
        if (rank < K) {
            const int64_t uu = uid_s[r];
            a.out_idx[uu * K + rank] = ix;
            a.out_score[uu * K + rank] = kx;
        }
    }
    if (lane < 32 && uval[lane] && ubad[lane]) flag_user(a, uid_s[lane]);

    // statistics: one atomic each per wave
    unsigned long long st_cand = (unsigned long long)cc;
    const int ctot = c + xor32_i(c);
    unsigned long long st_max = (h == 0 && valid) ? (unsigned long long)ctot : 0ull;
    unsigned long long st_resc = (lane == 0) ? (unsigned long long)ktot : 0ull;
    for (int off = 32; off >= 1; off >>= 1) {
        st_cand += __shfl_xor(st_cand, off);
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

// Per-user bin of kept candidates in certification (LDS).
// Largest dynamic LDS one workgroup of the certification kernel may use on
// the current device (queried once; raised above the 64 KB default when the
// device allows it).
static size_t certify_lds_limit() {
    static size_t limit = 0;
    if (limit == 0) {
        int dev = 0, v = 0;
        size_t lim = 64 * 1024;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            v > 0)
            lim = (size_t)v;
        if (lim > 150 * 1024) lim = 150 * 1024;
        limit = lim;
    }
    return limit;
}

// Bins hold the kept candidates of one user: room for K plus the screen's
// usual surplus (the E4M3 screen keeps several times more), within the LDS
// a workgroup may use.  A user whose bin overflows goes to the fallback.
static int certify_segcap(const ScreenPlan& p) {
    const int want = (p.prec == PREC_FP8) ? 8 * p.K + 192 : 2 * p.K + 48;
    const size_t avail = certify_lds_limit() - 2048 - (size_t)32 * p.f * sizeof(float);
    const int room = (int)(avail / (32 * (sizeof(double) + sizeof(int))));
    return want < room ? want : room;
}

size_t certify_lds_bytes(const ScreenPlan& p) {
    return (size_t)32 * certify_segcap(p) * (sizeof(double) + sizeof(int)) + (size_t)32 * p.f * sizeof(float);
}

hipError_t launch_certify(const ScreenPlan& p, const ScreenArgs& a, hipStream_t s) {
    const size_t shm = certify_lds_bytes(p);
    if (shm > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)certify_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
    }
    certify_kernel<<<dim3((unsigned)p.n_ublk), dim3(64), shm, s>>>(a, p.UB, certify_segcap(p));
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
