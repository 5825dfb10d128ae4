/*
 * CPU oracle for exact batch top-K maximum inner product search.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.
 *
 * What it computes (Section II-B, problem statement; Section II-C, brute
 * force): for every user vector u and every item vector i the rating u.i,
 * then the K items with the largest ratings.  The paper evaluates in double
 * precision but does not fix a summation order or a tie rule, so this oracle
 * fixes both:
 *
 *   key(u, i)  = acc after  acc <- 0; for j = 0..f-1: acc <- RN64(acc + u_j * i_j)
 *                (each FP32 x FP32 product is exact in FP64, so only the
 *                 left-to-right order of the additions matters)
 *   top-K(u)   = the first K items when all items are ordered by
 *                (key descending, item index ascending).
 *
 * Two selection modes give the same first K entries:
 *   mode 0: full sort of all n_i (key, index) pairs with qsort;
 *   mode 1: a sorted list of K entries kept by insertion (the role the
 *           paper's min-heap plays), for large inputs.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double key;
    int32_t idx;
} oracle_entry;

/* Strict total order: a before b iff a.key > b.key, or equal keys and a.idx < b.idx. */
static int entry_before(const oracle_entry *a, const oracle_entry *b) {
    if (a->key > b->key) return 1;
    if (a->key < b->key) return 0;
    return a->idx < b->idx;
}

static int entry_cmp(const void *pa, const void *pb) {
    const oracle_entry *a = (const oracle_entry *)pa;
    const oracle_entry *b = (const oracle_entry *)pb;
    if (entry_before(a, b)) return -1;
    if (entry_before(b, a)) return 1;
    return 0;
}

/* The rating of one (user, item) pair in double precision, summed left to right. */
double oracle_key(const float *u, const float *i, int32_t f) {
    double acc = 0.0;
    for (int32_t j = 0; j < f; ++j) {
        double p = (double)u[j] * (double)i[j];
        acc = acc + p;
    }
    return acc;
}

/* All keys of one user: out[i] = key(u, item i). */
void oracle_user_keys(const float *u, const float *I, int64_t n_i, int32_t f, double *out) {
    for (int64_t i = 0; i < n_i; ++i) out[i] = oracle_key(u, I + i * (int64_t)f, f);
}

/*
 * Keys of given pairs: out[r*K + k] = key(U[r], I[idx[r*K + k]]) for rows
 * r < n_u.  Returns -1 if an index lies outside [0, n_i).
 */
int oracle_pair_keys(const float *U, int64_t n_u, const float *I, int64_t n_i, int32_t f,
                     int32_t K, const int32_t *idx, double *out) {
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t r = 0; r < n_u; ++r) {
        for (int32_t k = 0; k < K; ++k) {
            const int32_t i = idx[r * K + k];
            if (i < 0 || i >= n_i) {
                bad = 1;
                out[r * K + k] = 0.0;
                continue;
            }
            out[r * K + k] = oracle_key(U + r * (int64_t)f, I + (int64_t)i * f, f);
        }
    }
    return bad ? -1 : 0;
}

/*
 * Top-K for each user.  U is n_u x f, I is n_i x f, both row-major float32.
 * out_idx and out_key are n_u x K.  Returns 0 on success, -1 on bad
 * arguments, -2 on allocation failure.  nthreads <= 0 uses the OpenMP default.
 */
int oracle_topk(const float *U, int64_t n_u, const float *I, int64_t n_i, int32_t f, int32_t K,
                int32_t mode, int32_t *out_idx, double *out_key, int32_t nthreads) {
    if (!U || !I || !out_idx || !out_key) return -1;
    if (n_u < 0 || n_i < 1 || f < 1 || K < 1 || K > n_i) return -1;
    if (mode != 0 && mode != 1) return -1;
    int failed = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        oracle_entry *buf = NULL;
        if (mode == 0)
            buf = (oracle_entry *)malloc((size_t)n_i * sizeof(oracle_entry));
        else
            buf = (oracle_entry *)malloc((size_t)(K + 1) * sizeof(oracle_entry));
        if (!buf) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(static)
        for (int64_t u = 0; u < n_u; ++u) {
            if (!buf) continue;
            const float *urow = U + u * (int64_t)f;
            int32_t *oi = out_idx + u * (int64_t)K;
            double *ok = out_key + u * (int64_t)K;
            if (mode == 0) {
                for (int64_t i = 0; i < n_i; ++i) {
                    buf[i].key = oracle_key(urow, I + i * (int64_t)f, f);
                    buf[i].idx = (int32_t)i;
                }
                qsort(buf, (size_t)n_i, sizeof(oracle_entry), entry_cmp);
            } else {
                int32_t len = 0;
                for (int64_t i = 0; i < n_i; ++i) {
                    oracle_entry e;
                    e.key = oracle_key(urow, I + i * (int64_t)f, f);
                    e.idx = (int32_t)i;
                    if (len == K && !entry_before(&e, &buf[K - 1])) continue;
                    int32_t pos = (len < K) ? len : K - 1;
                    while (pos > 0 && entry_before(&e, &buf[pos - 1])) {
                        buf[pos] = buf[pos - 1];
                        --pos;
                    }
                    buf[pos] = e;
                    if (len < K) ++len;
                }
            }
            for (int32_t k = 0; k < K; ++k) {
                oi[k] = buf[k].idx;
                ok[k] = buf[k].key;
            }
        }
        free(buf);
    }
    return failed ? -2 : 0;
}

/* Number of OpenMP threads a parallel region uses (for reporting). */
int oracle_num_threads(int32_t nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
    return n;
#else
    (void)nthreads;
    return 1;
#endif
}
