// Online, sample-based choice between the brute force and the Maximus index
// (paper Section IV, "Optimus"): build the index, time both methods on a
// random sample of users, extrapolate each to the whole batch (the index
// estimate includes its construction), then finish the remaining users with
// the faster one and reuse the sampled answers.
//
// On the GPU the sample must be large enough to fill the device, the analogue
// of the paper's rule that the sample occupy the CPU's L2 cache: a brute-force
// screen of fewer users than one full wave of workgroups under-reports its
// throughput.  Both methods are exact, so the choice changes speed only.
#include <algorithm>
#include <cstdint>
#include <utility>
#include <vector>

#include "../../include/mips.h"
#include "device_common.h"
#include "internal.h"

namespace mips {

namespace {

__global__ void gather_rows_f32(const float* __restrict__ U, int f, const int* __restrict__ ids,
                                int64_t n, float* __restrict__ out) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n * f) return;
    const int64_t r = t / f;
    out[t] = U[(int64_t)ids[r] * f + (t - r * f)];
}

__global__ void scatter_results(const int* __restrict__ ids, int64_t n, int K,
                                const int32_t* __restrict__ idx, const double* __restrict__ sc,
                                int32_t* __restrict__ out_idx, double* __restrict__ out_score) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n * K) return;
    const int64_t r = t / K;
    const int64_t k = t - r * K;
    out_idx[(int64_t)ids[r] * K + k] = idx[t];
    out_score[(int64_t)ids[r] * K + k] = sc[t];
}

unsigned grid1(int64_t n) { return (unsigned)((n + 255) / 256); }

// The systematic sample on the device: sample user k < ns is
// floor((k n_u + off) / ns) (strictly increasing as ns <= n_u).  ids[k]
// receives sample user k, ids[ns + r] the r-th other user in ascending order.
// User u has c = ceil((u ns - off) / n_u) sample users below it (clamped to
// [0, ns]) and is sample user c when floor((c n_u + off) / ns) == u.
__global__ void sample_ids_kernel(int64_t n_u, int64_t ns, int64_t off, int* ids) {
    const int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (u >= n_u) return;
    const int64_t num = u * ns - off;
    int64_t c = num <= 0 ? 0 : (num + n_u - 1) / n_u;
    if (c > ns) c = ns;
    const bool in = c < ns && (c * n_u + off) / ns == u;
    if (in) ids[c] = (int)u;
    else ids[ns + (u - c)] = (int)u;
}

// splitmix64 (Steele, Lea and Flood 2014): seeded stream for the sample.
uint64_t splitmix(uint64_t& x) {
    uint64_t z = (x += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Device buffers from the library's block cache, released when the scope
// ends, after the stream has finished with them.
struct Scratch {
    hipStream_t s;
    std::vector<std::pair<void*, size_t>> p;
    explicit Scratch(hipStream_t st) : s(st) {}
    ~Scratch() {
        (void)hipStreamSynchronize(s);
        for (auto& q : p) cache_release(q.first, q.second);
    }
    template <typename T>
    hipError_t alloc(T** out, size_t count) {
        void* q = nullptr;
        size_t got = 0;
        hipError_t e = cache_alloc(&q, &got, std::max<size_t>(count * sizeof(T), 256));
        if (e == hipSuccess) {
            p.push_back({q, got});
            *out = (T*)q;
        }
        return e;
    }
};

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    Timer() {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
    }
    ~Timer() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
    void start(hipStream_t s) { (void)hipEventRecord(a, s); }
    double stop(hipStream_t s) {
        (void)hipEventRecord(b, s);
        (void)hipEventSynchronize(b);
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, a, b);
        return (double)ms;
    }
};

}  // namespace
}  // namespace mips

using namespace mips;

extern "C" int mips_optimus_topk(const float* U, int64_t n_u, const float* I, int64_t n_i, int32_t f,
                                 int32_t K, int32_t precision, int32_t n_clusters,
                                 int32_t kmeans_iters, uint64_t seed, int64_t sample_users,
                                 int32_t* out_idx, double* out_score, void* stream,
                                 mips_optimus_report* report) {
    if (!U || !I || !out_idx || !out_score) return fail(MIPS_ERR_ARG, "null pointer argument");
    if (sample_users < 0) return fail(MIPS_ERR_ARG, "sample_users must be >= 0");
    if (n_u < 1 || n_u >= ((int64_t)1 << 31)) return fail(MIPS_ERR_ARG, "n_u must be in [1, 2^31)");
    if ((int64_t)n_clusters > n_u || n_clusters < 1 || n_clusters > 4096)
        return fail(MIPS_ERR_ARG, "n_clusters must be in [1, min(n_u, 4096)] (got %d)", n_clusters);
    if (kmeans_iters < 0 || kmeans_iters > 100)
        return fail(MIPS_ERR_ARG, "kmeans_iters must be in [0, 100] (got %d)", kmeans_iters);
    // argument checks of the two methods, before anything is enqueued
    if (K > kFallbackMaxK && (int64_t)K <= n_i)
        return fail(MIPS_ERR_UNSUPPORTED, "K > %d is not supported", kFallbackMaxK);
    if (mips_bmm_topk_workspace_size(n_u, n_i, f, K, precision) == 0)
        return fail(MIPS_ERR_ARG, "invalid sizes or precision for the brute force");
    hipStream_t s = (hipStream_t)stream;
    mips_optimus_report rep{};

    // ---- the sample: kDefaultSample users or 1%, whichever is larger --------
    const int64_t kDefaultSample = 131072;
    int64_t ns = sample_users > 0 ? sample_users : std::max<int64_t>(kDefaultSample, n_u / 100);
    ns = std::min(ns, n_u);
    // systematic sample with a seeded offset: users floor((k n_u + off) / ns),
    // k = 0 .. ns-1 (evenly spread), then the other users in order
    uint64_t st = seed ^ 0x6f7074696d7573ull;
    const int64_t off = (int64_t)(splitmix(st) % (uint64_t)n_u);
    const int64_t nr = n_u - ns;
    rep.sample_users = ns;

    Scratch sc(s);
    hipError_t e;
    int* ids = nullptr;
    float *Us = nullptr, *Ur = nullptr;
    int32_t *bi = nullptr, *mi = nullptr, *ri = nullptr;
    double *bs = nullptr, *ms = nullptr, *rs = nullptr;
#define TRY(x, what) do { if ((e = (x)) != hipSuccess) return (e == hipErrorOutOfMemory) ? fail(MIPS_ERR_NOMEM, "%s: out of device memory", what) : hip_fail(e, what); } while (0)
    TRY(sc.alloc(&ids, (size_t)n_u), "alloc");
    TRY(sc.alloc(&Us, (size_t)ns * f), "alloc");
    TRY(sc.alloc(&bi, (size_t)ns * K), "alloc");
    TRY(sc.alloc(&mi, (size_t)ns * K), "alloc");
    TRY(sc.alloc(&bs, (size_t)ns * K), "alloc");
    TRY(sc.alloc(&ms, (size_t)ns * K), "alloc");
    if (nr > 0) {
        TRY(sc.alloc(&Ur, (size_t)nr * f), "alloc");
        TRY(sc.alloc(&ri, (size_t)nr * K), "alloc");
        TRY(sc.alloc(&rs, (size_t)nr * K), "alloc");
    }
    sample_ids_kernel<<<grid1(n_u), 256, 0, s>>>(n_u, ns, off, ids);
    gather_rows_f32<<<grid1(ns * f), 256, 0, s>>>(U, f, ids, ns, Us);
    if (nr > 0) gather_rows_f32<<<grid1(nr * f), 256, 0, s>>>(U, f, ids + ns, nr, Ur);
    TRY(hipGetLastError(), "gather");

    // ---- brute force on the sample ------------------------------------------
    const size_t wb = std::max(mips_bmm_topk_workspace_size(ns, n_i, f, K, precision),
                               nr > 0 ? mips_bmm_topk_workspace_size(nr, n_i, f, K, precision) : 0);
    unsigned char* wsb = nullptr;
    TRY(sc.alloc(&wsb, wb), "alloc workspace");
    Timer tm;
    int rc;
    tm.start(s);
    rc = mips_bmm_topk(Us, ns, I, n_i, f, K, precision, bi, bs, wsb, wb, s, nullptr);
    if (rc != MIPS_OK) return rc;
    rep.bmm_sample_ms = tm.stop(s);

    // ---- index construction and queries on the sample -------------------------
    mips_maximus_index* ix = nullptr;
    tm.start(s);
    rc = mips_maximus_build(U, n_u, I, n_i, f, n_clusters, kmeans_iters, seed, 0, s, &ix);
    if (rc != MIPS_OK) return rc;
    rep.build_ms = tm.stop(s);
    struct IndexGuard {
        mips_maximus_index* ix;
        ~IndexGuard() { mips_maximus_free(ix); }
    } guard{ix};
    const size_t wq = std::max(mips_maximus_query_users_workspace_size(ix, ns, K, precision),
                               nr > 0 ? mips_maximus_query_users_workspace_size(ix, nr, K, precision) : 0);
    unsigned char* wsq = nullptr;
    TRY(sc.alloc(&wsq, wq), "alloc workspace");
    tm.start(s);
    rc = mips_maximus_query_users(ix, Us, ns, K, precision, mi, ms, wsq, wq, s, nullptr);
    if (rc != MIPS_OK) return rc;
    rep.maximus_sample_ms = tm.stop(s);

    // ---- extrapolate and choose ------------------------------------------------
    const double scale = (double)n_u / (double)ns;
    rep.est_bmm_ms = rep.bmm_sample_ms * scale;
    rep.est_maximus_ms = rep.build_ms + rep.maximus_sample_ms * scale;
    rep.choice = rep.est_maximus_ms < rep.est_bmm_ms ? MIPS_OPTIMUS_MAXIMUS : MIPS_OPTIMUS_BMM;
    const bool use_max = rep.choice == MIPS_OPTIMUS_MAXIMUS;

    // ---- finish the other users with the chosen method, reuse the sample ------
    tm.start(s);
    if (nr > 0) {
        rc = use_max ? mips_maximus_query_users(ix, Ur, nr, K, precision, ri, rs, wsq, wq, s, nullptr)
                     : mips_bmm_topk(Ur, nr, I, n_i, f, K, precision, ri, rs, wsb, wb, s, nullptr);
        if (rc != MIPS_OK) return rc;
        scatter_results<<<grid1(nr * K), 256, 0, s>>>(ids + ns, nr, K, ri, rs, out_idx, out_score);
    }
    scatter_results<<<grid1(ns * K), 256, 0, s>>>(ids, ns, K, use_max ? mi : bi, use_max ? ms : bs,
                                                  out_idx, out_score);
    TRY(hipGetLastError(), "scatter");
    rep.finish_ms = tm.stop(s);
#undef TRY
    if (report) *report = rep;
    return MIPS_OK;
}
