/*
 * mips.h -- C ABI of libmips: exact batch top-K maximum inner product search
 * on one AMD Instinct MI355X (gfx950).
 *
 * The problem (paper Section II-B, "Problem Statement: Batch Exact MIPS"):
 * given user vectors U (n_u x f) and item vectors I (n_i x f), return for
 * every user the K items with the largest inner product u.i.
 *
 * Result contract (identical for every entry point and every precision):
 *   key(u, i)  = the float64 value of  acc <- +0; for j = 0..f-1:
 *                acc <- RN64(acc + (double)U[u,j] * (double)I[i,j])
 *                (each float32 x float32 product is exact in float64, so the
 *                 left-to-right order of the additions is the only choice);
 *   top-K(u)   = the first K items when all items are ordered by
 *                (key descending, item index ascending).
 * out_idx[u*K + k] is the k-th item of top-K(u) and out_score[u*K + k] its
 * key.  The paper computes ratings in double precision and leaves the
 * summation order and the tie rule open; this library fixes both as above so
 * that exactly one answer is correct.
 *
 * Precision: the bulk of the scoring runs on the matrix cores in float32,
 * bfloat16 or OCP E4M3 (per-row power-of-two scaled), always with float32
 * accumulation.  Each screened score s carries a rigorous error bound e with
 * s - e <= key <= s + e; every item whose upper bound reaches the running
 * K-th best lower bound is kept and only those are rescored in float64.  The
 * precision therefore changes speed, never the answer.
 *
 * Conventions for every function below:
 *  - Array pointers are DEVICE pointers owned by the caller, row-major and
 *    contiguous (float32 unless stated).  The library never frees them and
 *    keeps none of them after the call returns (the Maximus index copies
 *    what it needs).
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  All work
 *    is enqueued on it and the call returns without synchronising, unless
 *    `stats` is non-NULL: then the call synchronises the stream and fills
 *    `stats` (host memory).
 *  - Argument errors are reported before anything is enqueued.  No C++
 *    exception crosses this interface.  Return values are mips_status codes
 *    (0 on success, negative on failure); mips_last_error_message() gives a
 *    thread-local description of the most recent failure.
 *  - Non-finite inputs are detected on the device.  They are reported as
 *    MIPS_ERR_NONFINITE only when `stats` forces a synchronisation (and in
 *    stats->nonfinite_input); the outputs are then unspecified.
 *  - Calls that share a workspace must not overlap in time (different
 *    streams need different workspaces).
 *  - Device memory: mips_maximus_build and mips_optimus_topk take their
 *    device memory from a block cache owned by the library (hipMalloc
 *    blocks).  Released blocks stay cached, up to 4 GiB per process, and
 *    are reused by later calls, so repeated builds do not map device pages
 *    again.  A block is released only when no work on the device can still
 *    use it.  mips_topk_backward takes stream-ordered scratch
 *    (hipMallocAsync / hipFreeAsync on `stream`).
 */
#ifndef MIPS_H
#define MIPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MIPS_OK = 0,
    MIPS_ERR_ARG = -1,          /* bad argument; nothing was enqueued                 */
    MIPS_ERR_NONFINITE = -2,    /* NaN or Inf in U or I (reported only with stats)    */
    MIPS_ERR_HIP = -3,          /* a HIP runtime call or kernel launch failed         */
    MIPS_ERR_WORKSPACE = -4,    /* workspace NULL or smaller than *_workspace_size()  */
    MIPS_ERR_NOMEM = -5,        /* the library could not allocate (Maximus index)     */
    MIPS_ERR_UNSUPPORTED = -6   /* valid request outside what this build supports     */
} mips_status;

typedef enum {
    MIPS_PREC_FP32 = 0,         /* float32 matrix-core screen                          */
    MIPS_PREC_BF16 = 1,         /* bfloat16 (round-to-nearest-even) screen             */
    MIPS_PREC_FP8_E4M3 = 2,     /* OCP E4M3 screen with per-row power-of-two scales    */
    MIPS_PREC_FP8_E4M3_BF16 = 3 /* the E4M3 screen, its candidates re-screened in       *
                                 * bfloat16 (with the bfloat16 bound) before the        *
                                 * float64 rescore: fewer pairs rescored, more passes   */
} mips_precision;

/* Host-side counters of one call; filled only when a non-NULL pointer is passed. */
typedef struct {
    int64_t candidates_total;        /* (user, item) pairs the screen kept for certification     */
    int64_t candidates_max_per_user; /* largest per-user candidate count                           */
    int64_t rescored_pairs;          /* pairs rescored in float64 after certification              */
    int64_t overflow_users;          /* users finished on the exact fallback path                  */
    int64_t items_scored;            /* (user, item) pairs scored by the screen (unpadded)          */
    double  mean_items_visited;      /* mean items scored per user (n_i for brute force)            */
    double  max_screen_abs_err;      /* max |screened score - key| over rescored pairs              */
    double  max_screen_rel_err;      /* same, divided by ||u|| ||i||                                 */
    int32_t nonfinite_input;         /* 1 if U or I held NaN or Inf                                 */
    int32_t reserved;
} mips_stats;

/* ------------------------------------------------------------------------- *
 * Brute force: blocked matrix multiply fused with a per-user streaming top-K
 * (paper Section II-C, "Blocked Matrix Multiply").  The score matrix U I^T is
 * produced tile by tile on the matrix cores and never written to memory.
 * ------------------------------------------------------------------------- */

/* Bytes of device workspace mips_bmm_topk needs for these sizes (0 if the
 * sizes are invalid).  Does not touch the GPU. */
size_t mips_bmm_topk_workspace_size(int64_t n_u, int64_t n_i, int32_t f, int32_t K,
                                    int32_t precision);

/* Top-K of every user.
 *   U          n_u x f float32 (device)        I      n_i x f float32 (device)
 *   K          1 <= K <= n_i; K <= 4096 (larger: MIPS_ERR_UNSUPPORTED)
 *   precision  a mips_precision value
 *   out_idx    n_u x K int32 (device, written)  out_score n_u x K float64 (device, written)
 *   workspace  device buffer of at least mips_bmm_topk_workspace_size() bytes,
 *              256-byte aligned, owned by the caller; contents on entry ignored
 * Limits: 1 <= n_u, 1 <= n_i < 2^31, 1 <= f <= 256.  Fast screening paths
 * cover K <= 64 and f <= 128; other valid requests run on the exact float64
 * fallback kernel (same result, slower). */
int mips_bmm_topk(const float* U, int64_t n_u, const float* I, int64_t n_i, int32_t f, int32_t K,
                  int32_t precision, int32_t* out_idx, double* out_score,
                  void* workspace, size_t workspace_bytes, void* stream, mips_stats* stats);

/* Norm-pruned brute force: mips_bmm_topk with early termination.  The items
 * are already scored in descending-norm tile order; after each tile a user
 * stops once ||u|| times the largest ||i|| of all later tiles (plus the
 * rounding slack) is below its K-th best lower bound tau_u, since every later
 * item then has key < tau_u <= the K-th largest key.  This is the stop test
 * of Algorithm 1 (Section III-C) with theta_b = pi, i.e. the bound ||i|| of
 * Eq. (appx_bound) for a cluster with no angular information, and the
 * length-based pruning the paper discusses for existing indexes
 * (Section II-D).  Same arguments, workspace size
 * (mips_bmm_topk_workspace_size) and result as mips_bmm_topk;
 * stats->mean_items_visited reports the items scored per user. */
int mips_norm_pruned_topk(const float* U, int64_t n_u, const float* I, int64_t n_i, int32_t f,
                          int32_t K, int32_t precision, int32_t* out_idx, double* out_score,
                          void* workspace, size_t workspace_bytes, void* stream, mips_stats* stats);

/* ------------------------------------------------------------------------- *
 * Maximus (paper Section III, Algorithm 1): k-means over users
 * (Section III-A), per cluster the largest user-centroid angle theta_b and
 * every item ordered by the bound of Eq. (appx_bound)
 * ||i|| cos(max(theta_ic - theta_b, 0)) (Section III-B, ConstructIndex), then
 * per user a walk down its cluster's list in item blocks shared by the
 * cluster's users (Section III-D), stopping once ||u|| times the bound of the
 * next item is below the K-th best score (Section III-C, QueryIndex).
 * ------------------------------------------------------------------------- */
typedef struct mips_maximus_index mips_maximus_index; /* opaque; owns device memory */

/* Build the index.
 *   n_clusters   1 <= C <= min(n_u, 4096)   kmeans_iters  0 <= iters <= 100 Lloyd updates
 *   seed         picks the C initial centroids (Forgy initialisation)
 *   block_items  0 = default; otherwise the number of leading list items scored for
 *                every user of a cluster before any may stop (the paper's B), rounded up
 *                to the item tile (32)
 *   out_index    receives the index; free it with mips_maximus_free()
 * The index copies U and I (and their screen copies); the caller may free them
 * afterwards.  Everything runs on the device; `stream` is synchronised once,
 * at the end, to report NaN or Inf in I (MIPS_ERR_NONFINITE).  Index memory
 * and build temporaries come from the library's block cache (see "Device
 * memory" above).  Returns MIPS_ERR_NOMEM if device memory runs out. */
int mips_maximus_build(const float* U, int64_t n_u, const float* I, int64_t n_i, int32_t f,
                       int32_t n_clusters, int32_t kmeans_iters, uint64_t seed,
                       int32_t block_items, void* stream, mips_maximus_index** out_index);

/* Workspace bytes for mips_maximus_query (0 on bad arguments). */
size_t mips_maximus_query_workspace_size(const mips_maximus_index* index, int32_t K,
                                         int32_t precision);

/* Top-K of every user of the index, same contract and output as mips_bmm_topk
 * (out_idx / out_score are n_u x K in the original user order).  Read-only on
 * the index: concurrent queries with separate workspaces are allowed.
 * stats->mean_items_visited reports the mean walk length w-bar of Eq. (runtime). */
int mips_maximus_query(const mips_maximus_index* index, int32_t K, int32_t precision,
                       int32_t* out_idx, double* out_score, void* workspace,
                       size_t workspace_bytes, void* stream, mips_stats* stats);

/* Top-K of arbitrary user vectors against the index's items: new users that
 * were not clustered, or any subset of the indexed users (the paper's
 * serving setting, Section III-E, and the user samples of the optimizer,
 * Section IV-A).  Each row of Uq is assigned to its nearest centroid
 * (Euclidean, as in the build); when its angle to that centroid is at most
 * the cluster's theta_b, the bound of Eq. (appx_bound) holds for it and it
 * walks that cluster's list; otherwise (or for a zero or non-finite row) it
 * takes the exact float64 path.  Same result contract as mips_bmm_topk.
 *   Uq         n_q x f float32 (device), f as in the index; 1 <= n_q < 2^31
 *   out_idx    n_q x K int32, out_score n_q x K float64 (device, written)
 *   workspace  at least mips_maximus_query_users_workspace_size() bytes,
 *              256-byte aligned, caller-owned
 * Read-only on the index. */
size_t mips_maximus_query_users_workspace_size(const mips_maximus_index* index, int64_t n_q,
                                               int32_t K, int32_t precision);
int mips_maximus_query_users(const mips_maximus_index* index, const float* Uq, int64_t n_q,
                             int32_t K, int32_t precision, int32_t* out_idx, double* out_score,
                             void* workspace, size_t workspace_bytes, void* stream,
                             mips_stats* stats);

/* Release the index (NULL is ignored): waits until the device is idle (a
 * query on any stream may still read the index), then returns its memory to
 * the library's block cache. */
void mips_maximus_free(mips_maximus_index* index);

/* Index description, for tests and reports (host memory, NULL fields skipped).
 * centroids C x f float64, theta_b C float64, assign n_u int32,
 * lists C x n_i int32 (item indices in walk order), bounds C x n_i float32
 * (the rounded-up bound of each list entry, in walk order).
 * Synchronises `stream`. */
int mips_maximus_export(const mips_maximus_index* index, int32_t* n_clusters, int32_t* f,
                        int64_t* n_u, int64_t* n_i, double* centroids, double* theta_b,
                        int32_t* assign, int32_t* lists, float* bounds, void* stream);

/* ------------------------------------------------------------------------- *
 * Optimus (paper Section IV): online, sample-based choice between the brute
 * force and the Maximus index.  Builds the index on all users, times both
 * methods on a seeded random sample of users, extrapolates each to the whole
 * batch (the index estimate includes its construction time), finishes the
 * remaining users with the faster method and reuses the sampled answers.
 * The sample is systematic: users floor((k n_u + off) / s), k < s, with a
 * seeded random offset 0 <= off < n_u (evenly spread over the user order),
 * chosen on the device.
 * Both methods are exact: the result is the mips_bmm_topk contract whatever
 * the choice.
 *   sample_users  0 = default: max(131072, n_u / 100), at most n_u (a sample
 *                 below one full wave of screen workgroups under-reports the
 *                 brute force's throughput); otherwise the sample size
 *   n_clusters, kmeans_iters, seed  as for mips_maximus_build (seed also draws
 *                 the sample)
 *   report        host memory, filled when non-NULL
 * Allocates its own device memory (stream-ordered, released before
 * returning) and synchronises `stream` (the timings need it).  Returns MIPS_ERR_NOMEM when device memory
 * runs out.
 * ------------------------------------------------------------------------- */
typedef enum { MIPS_OPTIMUS_BMM = 0, MIPS_OPTIMUS_MAXIMUS = 1 } mips_optimus_choice;

typedef struct {
    int32_t choice;              /* a mips_optimus_choice                                  */
    int32_t reserved;
    int64_t sample_users;        /* users in the sample                                    */
    double  build_ms;            /* Maximus index construction                             */
    double  bmm_sample_ms;       /* brute force on the sample                              */
    double  maximus_sample_ms;   /* Maximus queries on the sample                          */
    double  est_bmm_ms;          /* brute force extrapolated to all users                  */
    double  est_maximus_ms;      /* construction + queries extrapolated to all users       */
    double  finish_ms;           /* the chosen method on the other users, results in place */
} mips_optimus_report;

int mips_optimus_topk(const float* U, int64_t n_u, const float* I, int64_t n_i, int32_t f,
                      int32_t K, int32_t precision, int32_t n_clusters, int32_t kmeans_iters,
                      uint64_t seed, int64_t sample_users, int32_t* out_idx, double* out_score,
                      void* stream, mips_optimus_report* report);

/* ------------------------------------------------------------------------- *
 * Backward of a loss on the top-K scores (not in the paper).  With the top-K
 * indices fixed, S[u,k] = U[u] . I[idx[u,k]] and G = dL/dS:
 *   dU[u]  = sum_k G[u,k] I[idx[u,k]]                      (gather)
 *   dI[i]  = sum over (u,k) with idx[u,k] = i of G[u,k] U[u]  (scatter-add)
 * dU (n_u x f) and dI (n_i x f) are overwritten.  dU is summed in k order
 * and is deterministic.  For dI the pairs are grouped by item and summed in
 * runs, each run added with float32 atomics, so its last bits may vary run
 * to run.  idx entries outside [0, n_i) are skipped.  The grouping takes
 * stream-ordered scratch (hipMallocAsync / hipFreeAsync on `stream`) of
 * about 12 n_i + 4 n_u K bytes.
 * Limits: 1 <= n_u, n_i < 2^31; 1 <= f <= 4096; K >= 1.
 * ------------------------------------------------------------------------- */
int mips_topk_backward(const float* U, const float* I, int64_t n_u, int64_t n_i, int32_t f,
                       int32_t K, const int32_t* idx, const float* grad_scores, float* dU,
                       float* dI, void* stream);

/* ------------------------------------------------------------------------- *
 * mips_topk_backward_noalloc: the same operation and arguments as
 * mips_topk_backward, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight training or serving loops, harnesses that
 * forbid hipMalloc).  It calls no hipMalloc, hipFree or allocating library
 * routine: the item grouping's scratch is a static device array of
 * MIPS_NOALLOC_SCRATCH_BYTES bytes, one per device, that the library holds
 * from its first call on that device until the process ends.
 * The scratch needed is about 12 n_i + 4 n_u K bytes (+ 4 KiB); larger calls
 * return MIPS_ERR_UNSUPPORTED before anything is enqueued (use
 * mips_topk_backward for them).  With n_u K >= 2^31 no scratch is used.
 * Every call on a device shares that device's array: calls that overlap on
 * one device (two streams, or two host threads) race and must be ordered by
 * the caller.  The arrays it clears are cleared by kernels on `stream`.
 * Other arguments, limits, errors and results: as mips_topk_backward.
 * ------------------------------------------------------------------------- */
#define MIPS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int mips_topk_backward_noalloc(const float* U, const float* I, int64_t n_u, int64_t n_i,
                               int32_t f, int32_t K, const int32_t* idx,
                               const float* grad_scores, float* dU, float* dI, void* stream);

/* ------------------------------------------------------------------------- *
 * Diagnostics.
 * ------------------------------------------------------------------------- */
const char* mips_status_string(int status);
const char* mips_last_error_message(void);

/* Testing only.  Process-wide knobs that force rare paths so tests can reach
 * them on small inputs; 0 (the initial value) means normal operation.  They
 * change speed, never the result:
 *   MIPS_DEBUG_CAND_CAP        candidate slots per lane of the screen (>= 1);
 *                              a small cap overflows the lists and sends users
 *                              to the exact float64 fallback
 *   MIPS_DEBUG_CERTIFY_KERNEL  1 = certify with one wave per user, 2 = with a
 *                              group of lanes per user (where the screen does
 *                              not certify in its own tail)
 * Returns MIPS_ERR_ARG for an unknown knob or value.  Not for concurrent use
 * with calls that read the knobs. */
typedef enum { MIPS_DEBUG_CAND_CAP = 0, MIPS_DEBUG_CERTIFY_KERNEL = 1 } mips_debug_knob;
int mips_debug_set(int32_t knob, int32_t value);

/* Kernel timing.  While enabled, every kernel phase launched by this library
 * is bracketed by HIP events recorded on the caller's stream (no host
 * synchronisation).  mips_profile_read() waits for the recorded events, adds
 * their durations into `ms` and `launches` (arrays of MIPS_PROFILE_PHASES,
 * indexed by mips_profile_phase) and clears the record. */
typedef enum {
    MIPS_PHASE_ITEM_PREP = 0,   /* item norms, screen copies, norm order, packing   */
    MIPS_PHASE_SCREEN = 1,      /* matrix-core score tiles + streaming top-K          */
    MIPS_PHASE_CERTIFY = 2,     /* certification + float64 rescore + final order      */
    MIPS_PHASE_FALLBACK = 3,    /* exact float64 path for flagged users               */
    MIPS_PHASE_BUILD = 4,       /* Maximus index construction                         */
    MIPS_PHASE_WALK = 5,        /* Maximus blocked walk (screen over list blocks)     */
    MIPS_PHASE_BACKWARD = 6,    /* dU gather + dI scatter                             */
    MIPS_PROFILE_PHASES = 7
} mips_profile_phase;

int mips_profile_enable(int enable);
int mips_profile_read(double* ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* MIPS_H */
