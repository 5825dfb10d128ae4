// C ABI of libmips (declared in include/mips.h): argument checks, launch
// plans, workspace carving, kernel sequencing, statistics and kernel timing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/mips.h"
#include "internal.h"

namespace mips {

// ---------------------------------------------------------------------------
// Errors.
// ---------------------------------------------------------------------------
static thread_local char g_msg[512] = "";

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(MIPS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// Kernel timing: event pairs recorded on the caller's stream.
// ---------------------------------------------------------------------------
struct PhaseRecord {
    int phase;
    hipEvent_t start, stop;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<PhaseRecord> g_prof_pending;
static std::vector<hipEvent_t> g_prof_pool;

static hipEvent_t pool_event() {
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

PhaseTimer::PhaseTimer(int phase, hipStream_t s) : phase_(phase), stream_(s) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (!g_prof_on) return;
    start_ = pool_event();
    stop_ = pool_event();
    if (start_ && stop_ && hipEventRecord(start_, s) == hipSuccess) active_ = true;
}

PhaseTimer::~PhaseTimer() {
    if (!active_) return;
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (hipEventRecord(stop_, stream_) == hipSuccess)
        g_prof_pending.push_back({phase_, start_, stop_});
}

// ---------------------------------------------------------------------------
// Plans and workspace layout.
// ---------------------------------------------------------------------------
static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

static std::atomic<int> g_dbg_cand_cap{0}, g_dbg_certify{0};
int debug_cand_cap() { return g_dbg_cand_cap.load(std::memory_order_relaxed); }
int debug_certify_kernel() { return g_dbg_certify.load(std::memory_order_relaxed); }

bool make_screen_plan(int64_t n_u, int64_t n_i, int f, int K, int prec, bool stops, ScreenPlan* out) {
    ScreenPlan p;
    p.prec = prec;
    p.f = f;
    p.K = K;
    p.n_u = n_u;
    p.n_i = n_i;
    p.fast = (K <= 64 && f <= 128);
    // Factor chunks per matrix-core instruction sequence: the compiled chunk
    // count is the smallest one that covers f; factors past f are zero.
    if (prec == PREC_FP32) {
        const int need = (f + 1) / 2;                       // 2 factors per 32x32x2 step
        static const int opts[] = {8, 16, 25, 32, 50, 64};
        p.NCH = 64;
        for (int o : opts) if (o >= need) { p.NCH = o; break; }
        p.f_pad = 2 * p.NCH;
    } else if (prec == PREC_BF16) {
        const int need = (f + 15) / 16;                     // 16 factors per 32x32x16 step
        p.NCH = need <= 1 ? 1 : (need <= 2 ? 2 : (need <= 4 ? 4 : 8));
        p.f_pad = 16 * p.NCH;
    } else {
        const int need = (f + 63) / 64;                     // 64 factors per 32x32x64 step
        p.NCH = need <= 1 ? 1 : 2;
        p.f_pad = 64 * p.NCH;
    }
    p.nch = p.NCH;
    p.KM = K <= 1 ? 1 : (K <= 8 ? 8 : (K <= 10 ? 10 : (K <= 16 ? 16 : (K <= 32 ? 32 : 64))));
    p.UB = ub_for(prec, p.KM, p.NCH, stops);
    // Candidate slots per lane (half a user's items): room for the K-list
    // entries plus the items that pass before the threshold settles; the
    // coarser E4M3 screen keeps several times more.
    if (prec == PREC_FP8)
        p.cap = std::max(512, 8 * p.KM + 64);
    else
        p.cap = std::max(64, 2 * p.KM + 32);
    // Test knob: fewer candidate slots per lane (forces the overflow fallback).
    if (const int v = debug_cand_cap(); v >= 1) p.cap = v;
    p.kc = p.cap;
    p.n_blk = (n_i + 31) / 32;
    p.n_i_pad = p.n_blk * 32;
    p.n_waves = (n_u + 32 * p.UB - 1) / (32 * p.UB);
    p.n_ublk = p.n_waves * p.UB;
    p.fb_grid = (int)std::min<int64_t>(1024, std::max<int64_t>(1, n_u));
    const double n = (prec == PREC_FP32) ? (double)(p.f_pad + 1) : (double)p.f_pad;
    const double g = n * 0x1p-22 / (1.0 - n * 0x1p-22);
    p.gamma = (float)(g * (1.0 + 0x1p-20));
    *out = p;
    return true;
}

struct BmmLayout {
    size_t ctrl, ctrlb, hist, uflag, zero_end;
    size_t flist, uscal, bucket, perm, Corig, Gorig, Eorig, kexp, qrow, packed, pscale, blockmax,
        tailmax, cgpos;
    size_t qrowb, Gorigb, Eorigb;   // bfloat16 rows of the E4M3 certification cascade
    size_t cnt, cand, fbkeys, total;
};

// bfloat16 row stride of the cascade: f rounded up to 8 (16-byte rows)
static int cascade_stride(int f) { return (f + 7) & ~7; }

static BmmLayout bmm_layout(const ScreenPlan& p) {
    BmmLayout L{};
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o += al256(b); return r; };
    const size_t esz = p.prec == PREC_FP32 ? 4 : (p.prec == PREC_BF16 ? 2 : 1);
    const bool casc = p.fast && p.prec == PREC_FP8;
    L.ctrl = take(sizeof(Ctrl));
    L.ctrlb = take(sizeof(Ctrl));
    L.hist = take(2 * kBuckets * sizeof(unsigned int));
    L.uflag = take((size_t)p.n_u * 4);
    L.zero_end = o;
    L.flist = take((size_t)p.n_u * 4);
    L.uscal = take((size_t)p.n_u * 16);
    if (p.fast) {
        L.bucket = take((size_t)p.n_i * 4);
        L.perm = take((size_t)p.n_i_pad * 4);
        L.Corig = take((size_t)p.n_i * 4);
        L.Gorig = take((size_t)p.n_i * 4);
        L.Eorig = take((size_t)p.n_i * 4);
        L.kexp = take((size_t)p.n_i * 4);
        L.qrow = take((size_t)p.n_i * p.f_pad * esz);
        L.packed = take((size_t)p.n_i_pad * p.f_pad * esz);
        L.pscale = take((size_t)p.n_i_pad * 4);
        L.blockmax = take((size_t)p.n_blk * 8);
        L.cgpos = take((size_t)p.n_i_pad * 16);
        L.tailmax = take((size_t)p.n_blk * 4);
        if (casc) {
            L.qrowb = take((size_t)p.n_i * cascade_stride(p.f) * 2);
            L.Gorigb = take((size_t)p.n_i * 4);
            L.Eorigb = take((size_t)p.n_i * 4);
        }
        L.cnt = take((size_t)p.n_ublk * 64 * 4);
        L.cand = take(cand_bytes(p.n_ublk, p.cap));
    }
    L.fbkeys = take((size_t)p.fb_grid * p.n_i * 8);
    L.total = o;
    return L;
}

static int check_common(int64_t n_u, int64_t n_i, int f, int K, int prec) {
    if (n_u < 1) return fail(MIPS_ERR_ARG, "n_u must be >= 1 (got %lld)", (long long)n_u);
    if (n_i < 1 || n_i >= ((int64_t)1 << 31))
        return fail(MIPS_ERR_ARG, "n_i must be in [1, 2^31) (got %lld)", (long long)n_i);
    if (n_u >= ((int64_t)1 << 31)) return fail(MIPS_ERR_ARG, "n_u must be < 2^31");
    if (f < 1 || f > 256) return fail(MIPS_ERR_ARG, "f must be in [1, 256] (got %d)", f);
    if (K < 1 || (int64_t)K > n_i) return fail(MIPS_ERR_ARG, "K must be in [1, n_i] (got %d)", K);
    if (!valid_prec(prec)) return fail(MIPS_ERR_ARG, "unknown precision %d", prec);
    if (K > kFallbackMaxK)
        return fail(MIPS_ERR_UNSUPPORTED, "K > %d is not supported (got %d)", kFallbackMaxK, K);
    return MIPS_OK;
}

int finish_stats(Ctrl* dctrl, hipStream_t s, int64_t n_u, int64_t n_i, mips_stats* stats) {
    Ctrl h{};
    hipError_t e = hipMemcpyAsync(&h, dctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "reading statistics");
    std::memset(stats, 0, sizeof(*stats));
    stats->candidates_total = (int64_t)h.cand_total;
    stats->candidates_max_per_user = (int64_t)h.cand_max;
    stats->rescored_pairs = (int64_t)h.rescored;
    stats->overflow_users = (int64_t)h.fb_count;
    stats->items_scored = (int64_t)h.visited;
    stats->mean_items_visited = n_u > 0 ? (double)h.visited / (double)n_u : 0.0;
    double d;
    std::memcpy(&d, &h.max_abs_err, 8);
    stats->max_screen_abs_err = d;
    std::memcpy(&d, &h.max_rel_err, 8);
    stats->max_screen_rel_err = d;
    stats->nonfinite_input = h.nonfinite ? 1 : 0;
    (void)n_i;
    if (h.nonfinite) return fail(MIPS_ERR_NONFINITE, "U or I holds NaN or Inf");
    return MIPS_OK;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free backward: one static array per device,
// resolved once per device to its device address (the array's name in host
// code is only a stand-in for the symbol).  Held until the process ends.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[MIPS_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

int noalloc_scratch(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(MIPS_ERR_UNSUPPORTED, "device %d >= %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr || ((uintptr_t)ptr & 255) != 0) return fail(MIPS_ERR_HIP, "scratch symbol has no aligned address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MIPS_OK;
}

// ---------------------------------------------------------------------------
// Device memory of indexes and of Optimus' scratch: blocks from hipMalloc,
// kept in a per-process cache when released, so that repeated builds, frees
// and Optimus calls reuse them instead of mapping device pages again (a
// hipMalloc of tens of MB costs about 0.1 ms).  A release is only made once
// no work on the device can still use the block.  The cache keeps at most
// kCacheLimit bytes; beyond that the oldest blocks are freed.
// ---------------------------------------------------------------------------
struct CachedBlock {
    int dev;
    void* p;
    size_t bytes;
};
static std::mutex g_cache_mu;
static std::vector<CachedBlock> g_cache;
static size_t g_cache_bytes = 0;
constexpr size_t kCacheLimit = (size_t)4 << 30;

static size_t cache_round(size_t bytes) {
    const size_t g = bytes >= ((size_t)1 << 20) ? ((size_t)1 << 20) : 4096;
    return (std::max<size_t>(bytes, 1) + g - 1) / g * g;
}

hipError_t cache_alloc(void** p, size_t* bytes_out, size_t bytes) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    bytes = cache_round(bytes);
    {
        // smallest cached block of this device that holds the request
        // without wasting more than half of itself
        std::lock_guard<std::mutex> g(g_cache_mu);
        int best = -1;
        for (int k = 0; k < (int)g_cache.size(); ++k) {
            const CachedBlock& c = g_cache[k];
            if (c.dev == dev && c.bytes >= bytes && c.bytes <= 2 * bytes &&
                (best < 0 || c.bytes < g_cache[best].bytes))
                best = k;
        }
        if (best >= 0) {
            *p = g_cache[best].p;
            *bytes_out = g_cache[best].bytes;
            g_cache_bytes -= g_cache[best].bytes;
            g_cache.erase(g_cache.begin() + best);
            return hipSuccess;
        }
    }
    e = hipMalloc(p, bytes);
    if (e == hipErrorOutOfMemory) {
        // give the cached blocks of this device back and try once more
        (void)hipGetLastError();
        std::vector<void*> drop;
        {
            std::lock_guard<std::mutex> g(g_cache_mu);
            for (int k = (int)g_cache.size() - 1; k >= 0; --k) {
                if (g_cache[k].dev != dev) continue;
                drop.push_back(g_cache[k].p);
                g_cache_bytes -= g_cache[k].bytes;
                g_cache.erase(g_cache.begin() + k);
            }
        }
        for (void* q : drop) (void)hipFree(q);
        e = hipMalloc(p, bytes);
    }
    if (e == hipSuccess) *bytes_out = bytes;
    return e;
}

void cache_release(void* p, size_t bytes) {
    if (!p) return;
    int dev = -1;
    (void)hipGetDevice(&dev);
    std::vector<void*> drop;
    {
        std::lock_guard<std::mutex> g(g_cache_mu);
        g_cache.push_back({dev, p, bytes});
        g_cache_bytes += bytes;
        while (g_cache_bytes > kCacheLimit && !g_cache.empty()) {
            drop.push_back(g_cache.front().p);
            g_cache_bytes -= g_cache.front().bytes;
            g_cache.erase(g_cache.begin());
        }
    }
    for (void* q : drop) (void)hipFree(q);
}

}  // namespace mips

using namespace mips;

extern "C" {

const char* mips_status_string(int status) {
    switch (status) {
        case MIPS_OK: return "MIPS_OK";
        case MIPS_ERR_ARG: return "MIPS_ERR_ARG";
        case MIPS_ERR_NONFINITE: return "MIPS_ERR_NONFINITE";
        case MIPS_ERR_HIP: return "MIPS_ERR_HIP";
        case MIPS_ERR_WORKSPACE: return "MIPS_ERR_WORKSPACE";
        case MIPS_ERR_NOMEM: return "MIPS_ERR_NOMEM";
        case MIPS_ERR_UNSUPPORTED: return "MIPS_ERR_UNSUPPORTED";
        default: return "MIPS_ERR_UNKNOWN";
    }
}

const char* mips_last_error_message(void) { return g_msg; }

int mips_profile_enable(int enable) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_on = enable != 0;
    return MIPS_OK;
}

int mips_profile_read(double* ms, int64_t* launches) {
    std::vector<PhaseRecord> recs;
    {
        std::lock_guard<std::mutex> g(g_prof_mu);
        recs.swap(g_prof_pending);
    }
    int rc = MIPS_OK;
    for (auto& r : recs) {
        float t = 0.0f;
        hipError_t e = hipEventSynchronize(r.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, r.start, r.stop);
        if (e != hipSuccess) {
            rc = hip_fail(e, "profile event");
        } else if (r.phase >= 0 && r.phase < MIPS_PROFILE_PHASES) {
            if (ms) ms[r.phase] += (double)t;
            if (launches) launches[r.phase] += 1;
        }
    }
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (auto& r : recs) {
        g_prof_pool.push_back(r.start);
        g_prof_pool.push_back(r.stop);
    }
    return rc;
}

static int backward_args(const float* U, const float* I, int64_t n_u, int64_t n_i, int32_t f,
                         int32_t K, const int32_t* idx, const float* grad_scores, const float* dU,
                         const float* dI) {
    if (n_u < 1 || n_i < 1 || n_i >= ((int64_t)1 << 31) || n_u >= ((int64_t)1 << 31))
        return fail(MIPS_ERR_ARG, "n_u, n_i must be in [1, 2^31)");
    if (f < 1 || f > 4096) return fail(MIPS_ERR_ARG, "f must be in [1, 4096] (got %d)", f);
    if (K < 1) return fail(MIPS_ERR_ARG, "K must be >= 1 (got %d)", K);
    if (!U || !I || !idx || !grad_scores || !dU || !dI) return fail(MIPS_ERR_ARG, "null array pointer");
    return MIPS_OK;
}

int mips_topk_backward(const float* U, const float* I, int64_t n_u, int64_t n_i, int32_t f,
                       int32_t K, const int32_t* idx, const float* grad_scores, float* dU,
                       float* dI, void* stream) {
    const int rc = backward_args(U, I, n_u, n_i, f, K, idx, grad_scores, dU, dI);
    if (rc != MIPS_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    PhaseTimer t(MIPS_PHASE_BACKWARD, s);
    hipError_t e = launch_backward(U, I, n_u, n_i, f, K, idx, grad_scores, dU, dI, nullptr, s);
    if (e != hipSuccess) return hip_fail(e, "backward");
    return MIPS_OK;
}

int mips_topk_backward_noalloc(const float* U, const float* I, int64_t n_u, int64_t n_i, int32_t f,
                               int32_t K, const int32_t* idx, const float* grad_scores, float* dU,
                               float* dI, void* stream) {
    int rc = backward_args(U, I, n_u, n_i, f, K, idx, grad_scores, dU, dI);
    if (rc != MIPS_OK) return rc;
    const size_t need = backward_scratch_bytes(n_i, n_u * (int64_t)K);
    if (need > MIPS_NOALLOC_SCRATCH_BYTES)
        return fail(MIPS_ERR_UNSUPPORTED,
                    "mips_topk_backward_noalloc: n_i = %lld and n_u K = %lld need %zu bytes of "
                    "scratch; its static scratch holds %zu (12 n_i + 4 n_u K + 4 KiB at most)",
                    (long long)n_i, (long long)(n_u * (int64_t)K), need,
                    (size_t)MIPS_NOALLOC_SCRATCH_BYTES);
    void* ptr = nullptr;
    if ((rc = noalloc_scratch(&ptr)) != MIPS_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    PhaseTimer t(MIPS_PHASE_BACKWARD, s);
    // with n_u K >= 2^31 the direct scatter-add runs and needs no scratch
    hipError_t e = launch_backward(U, I, n_u, n_i, f, K, idx, grad_scores, dU, dI,
                                   need ? ptr : nullptr, s);
    if (e != hipSuccess) return hip_fail(e, "backward");
    return MIPS_OK;
}

size_t mips_bmm_topk_workspace_size(int64_t n_u, int64_t n_i, int32_t f, int32_t K,
                                    int32_t precision) {
    if (check_common(n_u, n_i, f, K, precision) != MIPS_OK) return 0;
    // one plan for both sweeps (the norm-pruned one takes the brute force's
    // user blocks per wave)
    ScreenPlan p;
    make_screen_plan(n_u, n_i, f, K, screen_prec(precision), false, &p);
    return bmm_layout(p).total;
}

int mips_debug_set(int32_t knob, int32_t value) {
    if (value < 0) return fail(MIPS_ERR_ARG, "debug knob values are >= 0 (got %d)", value);
    switch (knob) {
        case MIPS_DEBUG_CAND_CAP: g_dbg_cand_cap.store(value); return MIPS_OK;
        case MIPS_DEBUG_CERTIFY_KERNEL:
            if (value > 2) return fail(MIPS_ERR_ARG, "certification kernel must be 0, 1 or 2");
            g_dbg_certify.store(value);
            return MIPS_OK;
        default: return fail(MIPS_ERR_ARG, "unknown debug knob %d", knob);
    }
}

}  // extern "C"

// Brute force (prune = 0) or norm-pruned brute force (prune = 1).
static int bmm_impl(const float* U, int64_t n_u, const float* I, int64_t n_i, int32_t f, int32_t K,
                    int32_t precision, int32_t* out_idx, double* out_score, void* workspace,
                    size_t workspace_bytes, void* stream, mips_stats* stats, int prune) {
    int rc = check_common(n_u, n_i, f, K, precision);
    if (rc != MIPS_OK) return rc;
    if (!U || !I || !out_idx || !out_score) return fail(MIPS_ERR_ARG, "null array pointer");
    const bool casc = cascade_of(precision);
    precision = screen_prec(precision);
    ScreenPlan p;
    // the norm-pruned sweep takes the brute force's user blocks per wave
    make_screen_plan(n_u, n_i, f, K, precision, false, &p);
    const BmmLayout L = bmm_layout(p);
    if (!workspace || workspace_bytes < L.total)
        return fail(MIPS_ERR_WORKSPACE, "workspace needs %zu bytes (got %zu)", L.total, workspace_bytes);
    if (((uintptr_t)workspace & 255) != 0) return fail(MIPS_ERR_ARG, "workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)workspace;
    Ctrl* ctrl = (Ctrl*)(ws + L.ctrl);
    hipError_t e;

    {
        PhaseTimer t(MIPS_PHASE_ITEM_PREP, s);
        if ((e = launch_zero(ws, L.zero_end, s)) != hipSuccess) return hip_fail(e, "zero");
        if (p.fast) {
            ItemPrepArgs ia{};
            ia.I = I;
            ia.n_i = n_i;
            ia.n_blk = p.n_blk;
            ia.f = f;
            ia.f_pad = p.f_pad;
            ia.nch = p.nch;
            ia.gamma = p.gamma;
            ia.Corig = (float*)(ws + L.Corig);
            ia.Gorig = (float*)(ws + L.Gorig);
            ia.Eorig = (float*)(ws + L.Eorig);
            ia.kexp = (int*)(ws + L.kexp);
            ia.qrow = ws + L.qrow;
            ia.bucket = (int*)(ws + L.bucket);
            ia.hist = (unsigned int*)(ws + L.hist);
            ia.perm = (int*)(ws + L.perm);
            ia.packed = ws + L.packed;
            ia.pscale = (int*)(ws + L.pscale);
            ia.blockmax = (float2*)(ws + L.blockmax);
            ia.cgpos = (float4*)(ws + L.cgpos);
            ia.ctrl = ctrl;
            if ((e = launch_item_prep(precision, ia, true, s)) != hipSuccess)
                return hip_fail(e, "item preparation");
            if (casc) {
                // bfloat16 rows and residual norms for the certification cascade
                ItemPrepArgs ib{};
                ib.I = I;
                ib.n_i = n_i;
                ib.n_blk = p.n_blk;
                ib.f = f;
                ib.f_pad = cascade_stride(f);
                ib.nch = p.nch;
                const double n = (double)ib.f_pad;
                ib.gamma = (float)(n * 0x1p-22 / (1.0 - n * 0x1p-22) * (1.0 + 0x1p-20));
                ib.Corig = (float*)(ws + L.Corig);   // the same rounded-up norms
                ib.Gorig = (float*)(ws + L.Gorigb);
                ib.Eorig = (float*)(ws + L.Eorigb);
                ib.qrow = ws + L.qrowb;
                ib.ctrl = (Ctrl*)(ws + L.ctrlb);
                if ((e = launch_item_prep(PREC_BF16, ib, false, s)) != hipSuccess)
                    return hip_fail(e, "cascade rows");
            }
            if (prune &&
                (e = launch_tailmax(ia.blockmax, p.n_blk, (float*)(ws + L.tailmax), s)) != hipSuccess)
                return hip_fail(e, "tile norm maxima");
        } else {
            if ((e = launch_nonfinite_scan(U, n_u * f, I, n_i * f, ctrl, s)) != hipSuccess)
                return hip_fail(e, "finite check");
        }
    }
    ScreenArgs a{};
    a.U = U;
    a.I = I;
    a.n_u = n_u;
    a.n_i = n_i;
    a.n_blk = p.n_blk;
    a.n_i_pad = p.n_i_pad;
    a.f = f;
    a.f_pad = p.f_pad;
    a.nch = p.nch;
    a.K = K;
    a.cap = p.cap;
    a.kc = p.kc;
    a.gamma = p.gamma;
    a.ctrl = ctrl;
    a.want_stats = stats != nullptr;
    a.warm_rounds = 6;
    a.uflag = (int*)(ws + L.uflag);
    a.flist = (int*)(ws + L.flist);
    a.uscal = (float4*)(ws + L.uscal);
    a.out_idx = out_idx;
    a.out_score = out_score;
    if (p.fast) {
        a.packed = ws + L.packed;
        a.pscale = (const int*)(ws + L.pscale);
        a.blockmax = (const float2*)(ws + L.blockmax);
        a.cgpos = (const float4*)(ws + L.cgpos);
        a.tailmax = (const float*)(ws + L.tailmax);
        a.prune = prune;
        a.perm = (const int*)(ws + L.perm);
        a.qrow = ws + L.qrow;
        a.kexp = (const int*)(ws + L.kexp);
        a.Corig = (const float*)(ws + L.Corig);
        a.Gorig = (const float*)(ws + L.Gorig);
        if (casc) {
            a.qrow_b = ws + L.qrowb;
            a.Gorig_b = (const float*)(ws + L.Gorigb);
            a.maxb = &((const Ctrl*)(ws + L.ctrlb))->cmax_bits;
            a.fpb = cascade_stride(f);
        }
        a.n_ublk = p.n_ublk;
        a.cnt = (int*)(ws + L.cnt);
        a.cand = (int2*)(ws + L.cand);
        a.cand_lm = !fused_certify(p.prec, p.KM, p.UB);      // the layout the screen kernel writes
        {
            PhaseTimer t(MIPS_PHASE_SCREEN, s);
            if ((e = launch_screen(p, a, s)) != hipSuccess) return hip_fail(e, "screen");
        }
        {
            PhaseTimer t(MIPS_PHASE_CERTIFY, s);
            if ((e = launch_certify(p, a, s)) != hipSuccess) return hip_fail(e, "certify");
        }
    } else {
        if ((e = launch_flag_all(n_u, a.uflag, a.flist, ctrl, s)) != hipSuccess)
            return hip_fail(e, "flag all");
    }
    {
        PhaseTimer t(MIPS_PHASE_FALLBACK, s);
        FallbackArgs fa{};
        fa.U = U;
        fa.I = I;
        fa.n_u = n_u;
        fa.n_i = n_i;
        fa.f = f;
        fa.K = K;
        fa.flist = a.flist;
        fa.ctrl = ctrl;
        fa.keys = (double*)(ws + L.fbkeys);
        fa.out_idx = out_idx;
        fa.out_score = out_score;
        if ((e = launch_fallback(p, fa, s)) != hipSuccess) return hip_fail(e, "fallback");
    }
    if (stats) {
        rc = finish_stats(ctrl, s, n_u, n_i, stats);
        if (rc == MIPS_OK && !p.fast) stats->items_scored = n_u * n_i, stats->mean_items_visited = (double)n_i;
        return rc;
    }
    return MIPS_OK;
}

extern "C" {

int mips_bmm_topk(const float* U, int64_t n_u, const float* I, int64_t n_i, int32_t f, int32_t K,
                  int32_t precision, int32_t* out_idx, double* out_score, void* workspace,
                  size_t workspace_bytes, void* stream, mips_stats* stats) {
    return bmm_impl(U, n_u, I, n_i, f, K, precision, out_idx, out_score, workspace,
                    workspace_bytes, stream, stats, 0);
}

int mips_norm_pruned_topk(const float* U, int64_t n_u, const float* I, int64_t n_i, int32_t f,
                          int32_t K, int32_t precision, int32_t* out_idx, double* out_score,
                          void* workspace, size_t workspace_bytes, void* stream, mips_stats* stats) {
    return bmm_impl(U, n_u, I, n_i, f, K, precision, out_idx, out_score, workspace,
                    workspace_bytes, stream, stats, 1);
}

}  // extern "C"

