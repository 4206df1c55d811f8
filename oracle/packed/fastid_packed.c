/*
 * FastID on x86: a packed CPU baseline -- TEST AND MEASUREMENT INFRASTRUCTURE.
 *
 * The paper's starting point is FastID running on x86 CPUs: profiles packed
 * one bit per SNP into machine words, compared word by word with a bitwise
 * operation and a population count (Section I, Section II-A, Algorithm 2).
 * This file is that program written for today's x86 cores: 64-bit words,
 * OpenMP threads over blocks of references, and, where the CPU has it, the
 * AVX-512 per-lane population count (eight words per instruction).
 *
 * Counts (Section II-A):
 *   mixture  (mode 0): C[q][r] = sum over words of popcount(R & ~Q)   (Eq. 1)
 *   identity (mode 1): C[q][r] = sum over words of popcount(R ^ Q)
 * Top-k: the k smallest (count, reference index) pairs of each query, ties
 * to the lowest index, padded with (INT32_MAX, -1).
 *
 * It is a second CPU implementation, independent of both the byte oracle
 * (fastid_oracle.c, which never sees a packed word) and the GPU library: it
 * packs its own words from 0/1 bytes and shares no code with either.  Its
 * own pins are the byte oracle's outputs (tests/test_cpu_packed.py).  Only
 * the test suite and the benchmark's CPU-baseline leg load it.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <immintrin.h>

#define CP_MIXTURE 0
#define CP_IDENTITY 1

/* 64-bit words per packed row (no padding words). */
int32_t cp_words(int32_t n_loci) { return (n_loci + 63) / 64; }

/* 0/1 bytes [n][ld] -> rows [n][cp_words(L)]: locus k = bit k % 64 of word
 * k / 64 (the word layout is this file's own; any fixed layout shared by
 * both operands gives the same counts).  Returns -1 on a byte above 1. */
int cp_pack(const uint8_t* bytes, int64_t n, int32_t n_loci, int64_t ld, uint64_t* out)
{
    const int32_t W = cp_words(n_loci);
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < n; ++i) {
        const uint8_t* src = bytes + i * ld;
        uint64_t* dst = out + i * W;
        for (int32_t w = 0; w < W; ++w) {
            uint64_t word = 0;
            for (int32_t b = 0; b < 64 && 64 * w + b < n_loci; ++b) {
                const uint8_t x = src[64 * w + b];
                bad |= x > 1;
                word |= (uint64_t)(x & 1u) << b;
            }
            dst[w] = word;
        }
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------ counts */
static inline int32_t pair_scalar(const uint64_t* r, const uint64_t* q, int32_t W, int mode)
{
    int32_t c = 0;
    for (int32_t w = 0; w < W; ++w)
        c += __builtin_popcountll(mode == CP_MIXTURE ? (r[w] & ~q[w]) : (r[w] ^ q[w]));
    return c;
}

/* Counts of one query q against nr consecutive references in row layout
 * (rows of W words).  Generic x86-64: one popcnt per word. */
__attribute__((target("popcnt"))) static void rows_popcnt(const uint64_t* q, const uint64_t* rs, int64_t nr,
                                                          int32_t W, int mode, int32_t* out)
{
    for (int64_t j = 0; j < nr; ++j) out[j] = pair_scalar(rs + j * W, q, W, mode);
}

static void rows_plain(const uint64_t* q, const uint64_t* rs, int64_t nr, int32_t W, int mode, int32_t* out)
{
    for (int64_t j = 0; j < nr; ++j) out[j] = pair_scalar(rs + j * W, q, W, mode);
}

/* AVX-512 works on a block of references transposed into groups of eight:
 * tb[(g * W + w) * 8 + l] = word w of reference 8 g + l (zero past the
 * block), so lane l of one vector is reference 8 g + l and a query word is
 * broadcast to all lanes: no horizontal sums. */
static void transpose8(const uint64_t* rows, int64_t n, int32_t W, uint64_t* tb)
{
    const int64_t ng = (n + 7) / 8;
    for (int64_t g = 0; g < ng; ++g)
        for (int32_t l = 0; l < 8; ++l) {
            const int64_t r = 8 * g + l;
            for (int32_t w = 0; w < W; ++w) tb[(g * W + w) * 8 + l] = r < n ? rows[r * W + w] : 0;
        }
}

__attribute__((target("avx512f,avx512vpopcntdq"))) static void groups_avx512(const uint64_t* q, const uint64_t* tb,
                                                                              int64_t ng, int32_t W, int mode,
                                                                              int32_t* out)
{
    for (int64_t g = 0; g < ng; ++g) {
        const uint64_t* t = tb + g * W * 8;
        __m512i acc0 = _mm512_setzero_si512(), acc1 = _mm512_setzero_si512();
        int32_t w = 0;
        if (mode == CP_MIXTURE) {
            for (; w + 2 <= W; w += 2) {
                acc0 = _mm512_add_epi64(acc0, _mm512_popcnt_epi64(_mm512_andnot_si512(
                                                  _mm512_set1_epi64((long long)q[w]), _mm512_loadu_si512(t + 8 * w))));
                acc1 = _mm512_add_epi64(acc1, _mm512_popcnt_epi64(_mm512_andnot_si512(
                                                  _mm512_set1_epi64((long long)q[w + 1]),
                                                  _mm512_loadu_si512(t + 8 * w + 8))));
            }
            if (w < W)
                acc0 = _mm512_add_epi64(acc0, _mm512_popcnt_epi64(_mm512_andnot_si512(
                                                  _mm512_set1_epi64((long long)q[w]), _mm512_loadu_si512(t + 8 * w))));
        } else {
            for (; w + 2 <= W; w += 2) {
                acc0 = _mm512_add_epi64(acc0, _mm512_popcnt_epi64(_mm512_xor_si512(
                                                  _mm512_set1_epi64((long long)q[w]), _mm512_loadu_si512(t + 8 * w))));
                acc1 = _mm512_add_epi64(acc1, _mm512_popcnt_epi64(_mm512_xor_si512(
                                                  _mm512_set1_epi64((long long)q[w + 1]),
                                                  _mm512_loadu_si512(t + 8 * w + 8))));
            }
            if (w < W)
                acc0 = _mm512_add_epi64(acc0, _mm512_popcnt_epi64(_mm512_xor_si512(
                                                  _mm512_set1_epi64((long long)q[w]), _mm512_loadu_si512(t + 8 * w))));
        }
        _mm256_storeu_si256((__m256i*)(out + 8 * g), _mm512_cvtepi64_epi32(_mm512_add_epi64(acc0, acc1)));
    }
}

static int has_avx512(void)
{
    __builtin_cpu_init();
    return __builtin_cpu_supports("avx512f") && __builtin_cpu_supports("avx512vpopcntdq");
}

/* Which inner loop runs on this CPU: 2 AVX-512 vpopcntq, 1 popcnt, 0 plain C. */
int cp_isa(void)
{
    if (has_avx512()) return 2;
    return __builtin_cpu_supports("popcnt") ? 1 : 0;
}

/* A block of references, ready for one query after another. */
typedef struct {
    int isa;
    const uint64_t* rows;  /* row layout */
    uint64_t* tb;          /* transposed groups (AVX-512) */
    int64_t n;
    int32_t W;
} cp_block;

static void block_prepare(cp_block* b, const uint64_t* rows, int64_t n)
{
    b->rows = rows;
    b->n = n;
    if (b->isa == 2) transpose8(rows, n, b->W, b->tb);
}

/* out[j] = count of query q against reference j of the block (room for n
 * rounded up to 8). */
static void block_counts(const cp_block* b, const uint64_t* q, int mode, int32_t* out)
{
    if (b->isa == 2) groups_avx512(q, b->tb, (b->n + 7) / 8, b->W, mode, out);
    else if (b->isa == 1) rows_popcnt(q, b->rows, b->n, b->W, mode, out);
    else rows_plain(q, b->rows, b->n, b->W, mode, out);
}

/* references per cache block: about 256 KiB of reference words, whole groups of 8 */
static int64_t block_refs(int32_t W)
{
    int64_t rb = (256 * 1024) / (8 * (int64_t)W);
    rb = rb / 8 * 8;
    return rb < 8 ? 8 : rb;
}

/* Full count matrix counts[q * n_refs + r]. */
int cp_counts(const uint64_t* refs, int64_t n_refs, const uint64_t* qrys, int32_t n_q, int32_t n_loci, int mode,
              int32_t* counts)
{
    if (mode != CP_MIXTURE && mode != CP_IDENTITY) return -1;
    const int32_t W = cp_words(n_loci);
    const int isa = cp_isa();
    const int64_t rb = block_refs(W);
    const int64_t nb = (n_refs + rb - 1) / rb;
    int rc = 0;
#pragma omp parallel
    {
        cp_block b = {isa, NULL, NULL, 0, W};
        b.tb = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)rb * (size_t)W);
        int32_t* c = (int32_t*)malloc(sizeof(int32_t) * (size_t)rb);
        if (!b.tb || !c) rc = -1;
#pragma omp for schedule(dynamic, 1)
        for (int64_t bi = 0; bi < nb; ++bi) {
            if (!b.tb || !c) continue;
            const int64_t r0 = bi * rb, n = r0 + rb < n_refs ? rb : n_refs - r0;
            block_prepare(&b, refs + r0 * W, n);
            for (int32_t q = 0; q < n_q; ++q) {
                block_counts(&b, qrys + (int64_t)q * W, mode, c);
                memcpy(counts + (int64_t)q * n_refs + r0, c, sizeof(int32_t) * (size_t)n);
            }
        }
        free(b.tb);
        free(c);
    }
    return rc;
}

/* ------------------------------------------------------------ top-k */
/* A bounded max-heap of keys (count << 40 | index) per (thread, query). */
static void heap_push_bounded(uint64_t* h, int32_t* fill, int32_t k, uint64_t key)
{
    int32_t n = *fill;
    if (n < k) {
        int32_t i = n++;
        while (i > 0) {
            const int32_t p = (i - 1) / 2;
            if (h[p] >= key) break;
            h[i] = h[p];
            i = p;
        }
        h[i] = key;
        *fill = n;
        return;
    }
    if (key >= h[0]) return;
    int32_t i = 0;
    for (;;) {
        const int32_t a = 2 * i + 1, b = a + 1;
        int32_t m = i;
        uint64_t mv = key;
        if (a < n && h[a] > mv) { m = a; mv = h[a]; }
        if (b < n && h[b] > mv) { m = b; mv = h[b]; }
        if (m == i) break;
        h[i] = h[m];
        i = m;
    }
    h[i] = key;
}

static int cmp_u64(const void* a, const void* b)
{
    const uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : x > y;
}

/*
 * Top-k of every query over all references.  Threads own contiguous
 * reference ranges; each keeps a bounded heap per query and walks its range
 * in blocks of references small enough to stay in cache while every query
 * meets them; the per-thread heaps are merged at the end.  Returns 0, or -1
 * on bad arguments or allocation failure.
 */
int cp_topk(const uint64_t* refs, int64_t n_refs, const uint64_t* qrys, int32_t n_q, int32_t n_loci, int mode,
            int32_t k, int32_t* cnt, int64_t* idx)
{
    if (mode != CP_MIXTURE && mode != CP_IDENTITY) return -1;
    if (k < 1 || n_q < 0 || n_refs < 0) return -1;
    const int32_t W = cp_words(n_loci);
    const int isa = cp_isa();
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    uint64_t* heaps = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)nt * (size_t)n_q * (size_t)k);
    int32_t* fills = (int32_t*)calloc((size_t)nt * (size_t)n_q, sizeof(int32_t));
    if (!heaps || !fills) {
        free(heaps);
        free(fills);
        return -1;
    }
    const int64_t rb = block_refs(W);
    int bad = 0;
#pragma omp parallel num_threads(nt) reduction(| : bad)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        const int64_t lo = n_refs * t / nt, hi = n_refs * (t + 1) / nt;
        uint64_t* H = heaps + (size_t)t * n_q * k;
        int32_t* F = fills + (size_t)t * n_q;
        cp_block b = {isa, NULL, NULL, 0, W};
        b.tb = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)rb * (size_t)W);
        int32_t* c = (int32_t*)malloc(sizeof(int32_t) * (size_t)rb);
        if (!b.tb || !c) bad = 1;
        for (int64_t b0 = lo; b0 < hi && b.tb && c; b0 += rb) {
            const int64_t n = b0 + rb < hi ? rb : hi - b0;
            block_prepare(&b, refs + b0 * W, n);
            for (int32_t q = 0; q < n_q; ++q) {
                uint64_t* h = H + (size_t)q * k;
                block_counts(&b, qrys + (int64_t)q * W, mode, c);
                /* a full heap admits only keys below its largest; within a
                 * thread references come in increasing index order */
                const uint32_t lim = F[q] < k ? 0xFFFFFFFFu : (uint32_t)(h[0] >> 40) + 1u;
                for (int64_t j = 0; j < n; ++j) {
                    if ((uint32_t)c[j] >= lim) continue;
                    const uint64_t key = ((uint64_t)(uint32_t)c[j] << 40) | (uint64_t)(b0 + j);
                    if (F[q] < k || key < h[0]) heap_push_bounded(h, F + q, k, key);
                }
            }
        }
        free(b.tb);
        free(c);
    }
    if (bad) {
        free(heaps);
        free(fills);
        return -1;
    }
    int rc = 0;
#pragma omp parallel
    {
        uint64_t* all = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)nt * (size_t)k);
        if (!all) rc = -1;
#pragma omp for schedule(static)
        for (int32_t q = 0; q < n_q; ++q) {
            if (!all) continue;
            int64_t n = 0;
            for (int t = 0; t < nt; ++t) {
                const int32_t fl = fills[(size_t)t * n_q + q];
                memcpy(all + n, heaps + ((size_t)t * n_q + q) * k, sizeof(uint64_t) * (size_t)fl);
                n += fl;
            }
            qsort(all, (size_t)n, sizeof(uint64_t), cmp_u64);
            for (int32_t j = 0; j < k; ++j) {
                cnt[(int64_t)q * k + j] = j < n ? (int32_t)(all[j] >> 40) : INT32_MAX;
                idx[(int64_t)q * k + j] = j < n ? (int64_t)(all[j] & ((1ull << 40) - 1)) : -1;
            }
        }
        free(all);
    }
    free(heaps);
    free(fills);
    return rc;
}

int cp_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
