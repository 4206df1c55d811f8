/*
 * Seeded synthetic SNP profiles (CPU side).  Shared input generator: it serves
 * both the oracle and the GPU library's tests/benchmarks, and holds none of
 * the comparison arithmetic.
 *
 * Every random draw is a pure function of (seed, stream, row, col):
 *   key  = seed ^ (stream << 56) ^ (row << 16) ^ col     (row < 2^40, col < 2^16)
 *   draw = splitmix64(key)
 * where splitmix64 is the output function of Steele, Lea and Flood's
 * SplittableRandom (OOPSLA 2014), with the finalizer constants of Vigna's
 * public-domain splitmix64.c.  Being counter-based, any row can be
 * regenerated on its own, on the CPU or on the GPU (fidgen_gpu.hip implements
 * the same function), and the two agree bit for bit.
 *
 * Streams: 0 per-locus minor-allele frequency, 1 reference bits,
 *          2 query composition, 3 query bit flips, 4 jobs / arrivals,
 *          5 sampling of tiles and check points.
 */
#include <stdint.h>
#include <string.h>

uint64_t fg_mix(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t fg_key(uint64_t seed, uint32_t stream, uint64_t row, uint32_t col)
{
    return seed ^ ((uint64_t)stream << 56) ^ (row << 16) ^ (uint64_t)col;
}

static uint32_t fg_u32(uint64_t seed, uint32_t stream, uint64_t row, uint32_t col)
{
    return (uint32_t)(fg_mix(fg_key(seed, stream, row, col)) >> 32);
}

/* floor(p * 2^32) for p in [0, 1) -- a Bernoulli(p) draw is u32 < threshold. */
uint32_t fg_prob_threshold(double p)
{
    if (p <= 0.0) return 0u;
    if (p >= 1.0) return 0xFFFFFFFFu;
    return (uint32_t)(p * 4294967296.0);
}

/* Per-locus minor-allele frequency p_k = lo + (hi - lo) * u53, as thresholds. */
void fg_maf_thresholds(uint64_t seed, int32_t n_loci, double lo, double hi, uint32_t* thr)
{
    for (int32_t k = 0; k < n_loci; ++k) {
        double u = (double)(fg_mix(fg_key(seed, 0, 0, (uint32_t)k)) >> 11) * (1.0 / 9007199254740992.0);
        thr[k] = fg_prob_threshold(lo + (hi - lo) * u);
    }
}

/* Reference r, locus k: minor allele present iff u32(seed, 1, r, k) < thr[k]. */
void fg_ref_bytes(uint64_t seed, const uint32_t* thr, int32_t n_loci,
                  int64_t r0, int64_t n, uint8_t* out)
{
    /* Rows are independent draws: any thread split gives the same bytes. */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int32_t k = 0; k < n_loci; ++k)
            out[i * n_loci + k] = fg_u32(seed, 1, (uint64_t)(r0 + i), (uint32_t)k) < thr[k];
}

/* The same reference rows for an arbitrary list of row numbers. */
void fg_ref_rows(uint64_t seed, const uint32_t* thr, int32_t n_loci, const int64_t* rows, int64_t n,
                 uint8_t* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int32_t k = 0; k < n_loci; ++k)
            out[i * n_loci + k] = fg_u32(seed, 1, (uint64_t)rows[i], (uint32_t)k) < thr[k];
}

/* Distinct draws from [pool_base, pool_base + pool_size) for query row q. */
static int32_t fg_pick(uint64_t seed, uint64_t q, int64_t pool_base, int64_t pool_size,
                       int32_t want, int64_t* picked)
{
    if (want > pool_size) want = (int32_t)pool_size;
    int32_t got = 0;
    for (uint32_t j = 1; got < want; ++j) {
        int64_t c = pool_base + (int64_t)(fg_mix(fg_key(seed, 2, q, j)) % (uint64_t)pool_size);
        int dup = 0;
        for (int32_t i = 0; i < got; ++i) dup |= (picked[i] == c);
        if (!dup) picked[got++] = c;
    }
    return got;
}

/*
 * Mixture queries q0 .. q0+nq-1: the OR of nc in [nc_lo, nc_hi] distinct
 * references drawn from the pool, then every bit flipped independently with
 * probability flip_thr / 2^32.  Records the contributors ([nq][nc_hi], -1
 * padded), their number, and (optionally) the flip mask.
 */
int fg_mixtures(uint64_t seed, const uint32_t* thr, int32_t n_loci,
                int64_t pool_base, int64_t pool_size, int64_t q0, int64_t nq,
                int32_t nc_lo, int32_t nc_hi, uint32_t flip_thr,
                uint8_t* out, int64_t* contrib, int32_t* n_contrib, uint8_t* flips)
{
    if (nc_lo < 1 || nc_hi < nc_lo || nc_hi > 64 || pool_size < 1 || n_loci < 1) return -1;
    int64_t picked[64];
    for (int64_t i = 0; i < nq; ++i) {
        uint64_t q = (uint64_t)(q0 + i);
        int32_t want = nc_lo + (int32_t)(fg_u32(seed, 2, q, 0) % (uint32_t)(nc_hi - nc_lo + 1));
        int32_t got = fg_pick(seed, q, pool_base, pool_size, want, picked);
        uint8_t* row = out + i * n_loci;
        memset(row, 0, (size_t)n_loci);
        for (int32_t c = 0; c < got; ++c)
            for (int32_t k = 0; k < n_loci; ++k)
                row[k] |= (uint8_t)(fg_u32(seed, 1, (uint64_t)picked[c], (uint32_t)k) < thr[k]);
        for (int32_t k = 0; k < n_loci; ++k) {
            uint8_t f = fg_u32(seed, 3, q, (uint32_t)k) < flip_thr;
            row[k] ^= f;
            if (flips) flips[i * n_loci + k] = f;
        }
        if (n_contrib) n_contrib[i] = got;
        if (contrib)
            for (int32_t c = 0; c < nc_hi; ++c) contrib[i * nc_hi + c] = c < got ? picked[c] : -1;
    }
    return 0;
}

/*
 * Single-source (identity) queries: one reference drawn from the pool, with
 * every bit flipped independently with probability flip_thr / 2^32.
 */
int fg_identity(uint64_t seed, const uint32_t* thr, int32_t n_loci,
                int64_t pool_base, int64_t pool_size, int64_t q0, int64_t nq,
                uint32_t flip_thr, uint8_t* out, int64_t* source)
{
    if (pool_size < 1 || n_loci < 1) return -1;
    for (int64_t i = 0; i < nq; ++i) {
        uint64_t q = (uint64_t)(q0 + i);
        int64_t src;
        fg_pick(seed, q, pool_base, pool_size, 1, &src);
        for (int32_t k = 0; k < n_loci; ++k)
            out[i * n_loci + k] = (uint8_t)((fg_u32(seed, 1, (uint64_t)src, (uint32_t)k) < thr[k]) ^
                                            (fg_u32(seed, 3, q, (uint32_t)k) < flip_thr));
        if (source) source[i] = src;
    }
    return 0;
}

/* Raw uniform draws for jobs / arrivals / sampling (streams 4 and 5). */
void fg_u64s(uint64_t seed, uint32_t stream, uint64_t row, uint32_t col0, int64_t n, uint64_t* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = fg_mix(fg_key(seed, stream, row, col0 + (uint32_t)i));
}
