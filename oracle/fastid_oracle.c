/*
 * FastID reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of the all-pairs SNP
 * comparison of Samsi et al., "A Linear Algebra Approach to Fast DNA Mixture
 * Analysis Using GPUs" (arXiv 1707.00516).  It works on UNPACKED profiles: one
 * byte per SNP locus, value 0 (minor allele absent) or 1 (minor allele
 * present).  It never sees bit-packed words, so it is independent of any bit
 * order or word width chosen by the GPU library.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this code.  The GPU library shares no code with it.
 *
 * Definitions followed:
 *   - Section II-A, Eq. 1: P_ij = POPCOUNT(AND(XOR(R_i, Q_j), R_i)).  Per locus
 *     the summand is (r XOR q) AND r, i.e. 1 exactly when the reference carries
 *     the minor allele and the query does not (mode ORACLE_MIXTURE).
 *   - Section II-A, identity comparison of two individuals: the population count
 *     of XOR(R, Q), the number of loci whose minor-allele state differs (mode
 *     ORACLE_IDENTITY).
 *   - Algorithm 2 (naive all-pairs): a triple loop over unknown samples, known
 *     samples and the profile length; here the innermost loop runs over loci
 *     rather than packed words, which gives the same count.
 *   - Section II-B: the result is the N_R x N_Q overloaded product C = AB; it is
 *     stored here query-major, counts[q * n_refs + r], the same values.
 *
 * Selection (not in the paper; the per-query reductions it suggests in
 * Section IV): top-k = the k smallest (count, reference index) pairs in
 * lexicographic order, found by sorting the whole row; threshold = every
 * reference with count <= T, in ascending index order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_MIXTURE 0
#define ORACLE_IDENTITY 1

/* Returns 0 on success, -1 if any byte is not 0/1 or an argument is invalid. */
int oracle_check_bytes(const uint8_t* b, int64_t n)
{
    if (!b && n > 0) return -1;
    for (int64_t i = 0; i < n; ++i)
        if (b[i] > 1) return -1;
    return 0;
}

/* Eq. 1 / XOR identity for one (reference, query) pair over L loci. */
int32_t oracle_count_pair(const uint8_t* ref, const uint8_t* qry, int32_t n_loci, int mode)
{
    int32_t p = 0;
    for (int32_t k = 0; k < n_loci; ++k) {
        uint8_t a = (uint8_t)(ref[k] ^ qry[k]);     /* XOR(R, Q)            */
        if (mode == ORACLE_MIXTURE) a = (uint8_t)(a & ref[k]); /* AND(., R) */
        p += a;                                     /* POPCOUNT accumulates */
    }
    return p;
}

/*
 * Algorithm 2: counts[q * n_refs + r] = P(ref r, query q).
 * refs: n_refs x n_loci bytes, queries: n_q x n_loci bytes (row-major).
 */
int oracle_counts(const uint8_t* refs, int64_t n_refs,
                  const uint8_t* qrys, int64_t n_q,
                  int32_t n_loci, int mode, int32_t* counts)
{
    if (n_refs < 0 || n_q < 0 || n_loci < 0) return -1;
    if (mode != ORACLE_MIXTURE && mode != ORACLE_IDENTITY) return -1;
    /* Rows of the result are independent; threads split the query loop only. */
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < n_q; ++q)
        for (int64_t r = 0; r < n_refs; ++r)
            counts[q * n_refs + r] =
                oracle_count_pair(refs + r * (int64_t)n_loci, qrys + q * (int64_t)n_loci,
                                  n_loci, mode);
    return 0;
}

/*
 * Counts for an explicit list of (query row, reference row) pairs; used to
 * check sampled outputs of very large problems one at a time.
 */
int oracle_count_pairs(const uint8_t* refs, const uint8_t* qrys, int32_t n_loci, int mode,
                       const int64_t* ref_rows, const int64_t* qry_rows, int64_t n_pairs,
                       int32_t* out)
{
    if (mode != ORACLE_MIXTURE && mode != ORACLE_IDENTITY) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_pairs; ++i)
        out[i] = oracle_count_pair(refs + ref_rows[i] * (int64_t)n_loci,
                                   qrys + qry_rows[i] * (int64_t)n_loci, n_loci, mode);
    return 0;
}

typedef struct { int32_t count; int64_t idx; } oracle_pair;

static int pair_cmp(const void* a, const void* b)
{
    const oracle_pair* x = (const oracle_pair*)a;
    const oracle_pair* y = (const oracle_pair*)b;
    if (x->count != y->count) return x->count < y->count ? -1 : 1;
    if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
    return 0;
}

/*
 * Top-k of each row of a count matrix counts[n_q][n_refs]: sort the whole row
 * by (count, index) and keep the first min(k, n_refs) pairs; missing entries
 * (k > n_refs) are (INT32_MAX, -1).
 */
int oracle_topk(const int32_t* counts, int64_t n_q, int64_t n_refs, int32_t k,
                int32_t* out_cnt, int64_t* out_idx)
{
    if (k < 1 || n_q < 0 || n_refs < 0) return -1;
    oracle_pair* row = (oracle_pair*)malloc(sizeof(oracle_pair) * (size_t)(n_refs > 0 ? n_refs : 1));
    if (!row) return -2;
    for (int64_t q = 0; q < n_q; ++q) {
        for (int64_t r = 0; r < n_refs; ++r) {
            row[r].count = counts[q * n_refs + r];
            row[r].idx = r;
        }
        qsort(row, (size_t)n_refs, sizeof(oracle_pair), pair_cmp);
        for (int32_t j = 0; j < k; ++j) {
            if (j < n_refs) {
                out_cnt[q * k + j] = row[j].count;
                out_idx[q * k + j] = row[j].idx;
            } else {
                out_cnt[q * k + j] = INT32_MAX;
                out_idx[q * k + j] = -1;
            }
        }
    }
    free(row);
    return 0;
}

/*
 * Threshold hits of each row, in CSR form: offs[n_q + 1]; for row q the hits
 * are idx[offs[q] .. offs[q+1]) ascending, with their counts.  A NULL idx/cnt
 * only counts the hits (offs is still filled).  cap bounds the arrays; returns
 * the total hit count, or -1 on bad arguments / -2 if cap is too small.
 */
int64_t oracle_threshold(const int32_t* counts, int64_t n_q, int64_t n_refs,
                         const int32_t* thr, int64_t cap,
                         int64_t* offs, int64_t* idx, int32_t* cnt)
{
    if (n_q < 0 || n_refs < 0) return -1;
    int64_t n = 0;
    for (int64_t q = 0; q < n_q; ++q) {
        offs[q] = n;
        for (int64_t r = 0; r < n_refs; ++r) {
            if (counts[q * n_refs + r] <= thr[q]) {
                if (idx && cnt) {
                    if (n >= cap) return -2;
                    idx[n] = r;
                    cnt[n] = counts[q * n_refs + r];
                }
                ++n;
            }
        }
    }
    offs[n_q] = n;
    return n;
}

/* Number of threads the parallel loops above use (1 without OpenMP). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
