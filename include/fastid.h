/*
 * fastid.h -- C ABI of libfastid, an MI355X (gfx950) implementation of the
 * FastID all-pairs SNP comparison cast as an overloaded matrix multiply
 * (Samsi, Helfer, Kepner, Reuther, Ricke: "A Linear Algebra Approach to Fast
 * DNA Mixture Analysis Using GPUs", arXiv 1707.00516).
 *
 * Problem statement (Section II-A, Algorithm 2; Section II-B): N_R known
 * (reference) profiles and N_Q unknown (query) profiles, each of L SNP loci
 * with one bit per locus (bit set = minor allele present, Section II-A).  The
 * library computes, for every query q and reference r,
 *
 *   FID_MODE_MIXTURE  : C[q][r] = POPCOUNT(AND(XOR(R_r, Q_q), R_r))     (Eq. 1)
 *                                = number of loci where the reference carries
 *                                  a minor allele the query lacks
 *   FID_MODE_IDENTITY : C[q][r] = POPCOUNT(XOR(R_r, Q_q))
 *                                  (Section II-A, individual-to-individual)
 *
 * i.e. the overloaded product C = A B of Section II-B with A the N_R x N_W
 * reference matrix and B the N_W x N_Q query matrix.  C is addressed here
 * query-major, C[q][r] (the transpose of the paper's N_R x N_Q layout; the
 * values are the same).  Counts are exact 32-bit integers, 0 <= C <= L.
 *
 * Conventions shared by every entry point
 *   - Return value: a fid_status (0 = FID_OK, negative = error).  Nothing
 *     throws.  fid_last_error() gives a thread-local message for the last
 *     failing call on the calling thread.
 *   - Memory: every large buffer (profiles, database, workspace, outputs) is
 *     device memory allocated and owned by the caller; the library keeps only
 *     pointers to it for the duration of a call (fid_db keeps db_mem until
 *     fid_db_destroy).  The library itself allocates only small per-context
 *     scratch (staged query words and status words), freed by
 *     fid_ctx_destroy.
 *   - Execution: work is enqueued on the context's HIP stream (borrowed, not
 *     owned) and is asynchronous unless a function says it synchronises.
 *     Results are valid once that stream has been synchronised.  A context
 *     must not be used by two host threads at once.
 *   - Packed profile format ("packed rows"): profile i is row i of a
 *     uint64_t array [n][fid_row_words(L)].  Locus k (0-based) is bit (k & 63)
 *     of word (k >> 6), least significant bit first -- equivalently bit
 *     (k & 7) of byte (k >> 3) on this little-endian device.  Row length is
 *     rounded up to a 16-byte multiple.  Bits at loci >= L are ignored.
 *     (Section II-A maps 32 SNPs to one 32-bit word; the word width and bit
 *     order do not change any count.)
 *   - Indices: 0-based database row numbers, int64_t.
 *   - Limits: 1 <= L <= 65535; 1 <= N_R < 2^40; 1 <= N_Q <= 2^24;
 *     1 <= k <= 1024.  Device pointers must be 16-byte aligned.
 */
#ifndef FASTID_H
#define FASTID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FID_MODE_MIXTURE = 0,  /* Eq. 1: popcount((R ^ Q) & R) == popcount(R & ~Q) */
    FID_MODE_IDENTITY = 1  /* popcount(R ^ Q), the Hamming distance            */
} fid_mode;

typedef enum {
    FID_OK = 0,
    FID_EINVAL = -1,     /* invalid argument; nothing was enqueued                 */
    FID_ENOMEM = -2,     /* library scratch allocation failed, or buffer too small */
    FID_EHIP = -3,       /* a HIP runtime call or kernel launch failed             */
    FID_EOVERFLOW = -4,  /* threshold hits exceed the output capacity              */
    FID_EBUDGET = -5,    /* request exceeds a memory budget                        */
    FID_ETIMEOUT = -6,   /* wait timed out                                         */
    FID_ENOTREADY = -7,  /* result not ready yet                                   */
    FID_ENODEV = -8      /* no usable gfx950 device                                */
} fid_status;

/*
 * Kernel family evaluating the overloaded product (Section II-B).
 * POPCOUNT: bitwise op + population count on the vector ALUs, 32 loci per
 *   pair of instructions (Eq. 1 / XOR as written).
 * MFMA: the exact closed form popcount(R & ~Q) = popcount(R) - R.Q and
 *   popcount(R ^ Q) = popcount(R) + popcount(Q) - 2 R.Q, with the 0/1 dot
 *   product R.Q on the int8 matrix cores (int32 accumulation, exact).
 * MFMA_FP4: the same closed form with 0/1 operands in fp4 (e2m1) on the
 *   f8f6f4 matrix cores, fp32 accumulation (exact: sums stay below 2^24).
 * MFMA covers L <= 2304 (longer rows run POPCOUNT); MFMA_FP4 covers every L
 * (rows over 2048 loci stage the query tile in 2048-locus chunks).  AUTO picks per
 * call from the problem shape (row length, query-tile fill).  Results are
 * identical whatever the family.
 */
typedef enum {
    FID_BACKEND_AUTO = 0,
    FID_BACKEND_POPCOUNT = 1,
    FID_BACKEND_MFMA = 2,
    FID_BACKEND_MFMA_FP4 = 3
} fid_backend;

typedef struct fid_ctx fid_ctx;
typedef struct fid_db fid_db;

/* Static text for a status code. */
const char* fid_status_str(int status);

/* Thread-local description of the last error raised on this thread ("" if none). */
const char* fid_last_error(void);

/* Library ABI version (major * 10000 + minor * 100 + patch). */
int fid_version(void);

/*
 * Create a context on HIP device `device` that enqueues on `stream`
 * (a hipStream_t; NULL = the device's null stream).  The stream is borrowed.
 * Errors: FID_EINVAL (out NULL), FID_ENODEV (no such device, or not gfx950),
 * FID_EHIP.
 */
int fid_ctx_create(fid_ctx** out, int device, void* stream);

/* Release a context and its scratch (synchronises its stream first).  NULL is
 * a no-op.  Batches created on the context must be destroyed before it. */
int fid_ctx_destroy(fid_ctx* ctx);

/* Select the kernel family for later calls on this context (default FID_BACKEND_AUTO). */
int fid_ctx_set_backend(fid_ctx* ctx, int backend);

/*
 * The kernel family (fid_backend, never AUTO) a comparison of n_q queries
 * against db would use on this context now.
 */
int fid_backend_for(fid_ctx* ctx, const fid_db* db, int32_t n_q, int* backend);

/* Change the stream later calls enqueue on (borrowed). */
int fid_ctx_set_stream(fid_ctx* ctx, void* stream);

/* Block until all work enqueued on the context's stream has finished. */
int fid_sync(fid_ctx* ctx);

/*
 * Kernel timing for measurement.  While enabled, every compare call records a
 * pair of HIP events on the context's stream around its main scan kernel (the
 * kernel that evaluates the overloaded product).  fid_ctx_scan_time
 * synchronises on those events and returns the summed milliseconds and the
 * number of timed launches since the last reset; reset != 0 starts a new
 * window.
 */
int fid_ctx_enable_timing(fid_ctx* ctx, int enable);
int fid_ctx_scan_time(fid_ctx* ctx, double* total_ms, int64_t* launches, int reset);

/*
 * Genotype profiles (Section II-A: each locus is one of the genotypes with
 * 0, 1 or 2 copies of the minor allele; comparing them allele by allele is
 * two allele comparisons per locus).  geno_dev is [n_rows][ld_bytes]
 * device bytes with values 0, 1, 2 in the first n_loci of each row
 * (1 <= n_loci <= 32767).  rows_dev receives packed rows of 2 * n_loci loci
 * ([n_rows][fid_row_words(2 * n_loci)], 16-byte aligned): locus k becomes
 * loci 2k (at least one minor allele) and 2k + 1 (two).  A database built
 * from such rows, compared with queries packed the same way (every call
 * above, with n_loci' = 2 * n_loci), gives allele-level counts:
 *   FID_MODE_IDENTITY: sum over loci of |g_r - g_q|
 *   FID_MODE_MIXTURE : sum over loci of max(0, g_r - g_q)
 * Synchronises the context's stream (it reads back the validation flag);
 * FID_EINVAL for a value above 2 (rows_dev is then undefined), NULL or
 * misaligned buffers, or sizes out of range.  n_rows = 0 is a no-op.
 */
int fid_pack_genotypes(fid_ctx* ctx, const uint8_t* geno_dev, int64_t n_rows, int32_t n_loci, int64_t ld_bytes,
                       uint64_t* rows_dev);

/*
 * Streamed database: top-k of n_q queries against n_refs packed rows that
 * stay in HOST memory (the paper's host driver, Section III-C and Section
 * IV, which blocks the references to fit device memory and overlaps the
 * transfers with the comparisons).  The rows (rows_host, [n_refs][
 * fid_row_words(n_loci)], the packed format above) pass through the device
 * block_refs rows at a time: the copy of the next block (on a stream of the
 * call's own) overlaps the database build and top-k scan of the current one
 * (on the context's stream), and every block's top-k folds into a running
 * top-k whose k-th count bounds the scans of the later blocks.  The result
 * (cnt_dev / idx_dev, [n_q][k], global row indices, padding INT32_MAX / -1
 * when k > n_refs) is exactly fid_compare_topk's over the same rows.
 * rows_host should be pinned (hipHostMalloc, torch pin_memory) for the
 * copies to overlap; pageable memory still gives the same result.  ws_dev:
 * fid_stream_workspace_bytes() bytes of device memory (two staging blocks,
 * one database block, one block's top-k workspace, the running top-k).
 * Synchronises the context's stream before returning (the host rows are
 * free to reuse then).  FID_EINVAL for NULL or misaligned pointers, sizes out
 * of range or a bad mode; FID_ENOMEM for a short workspace.
 */
int fid_stream_workspace_bytes(fid_ctx* ctx, int64_t n_refs, int32_t n_loci, int64_t block_refs, int32_t n_q,
                               int32_t k, size_t* bytes);
int fid_compare_topk_streamed(fid_ctx* ctx, const uint64_t* rows_host, int64_t n_refs, int32_t n_loci,
                              int64_t block_refs, const uint64_t* q_dev, int32_t n_q, int mode, int32_t k,
                              void* ws_dev, size_t ws_bytes, int32_t* cnt_dev, int64_t* idx_dev);

/*
 * The full count matrix of a streamed database, the paper's host pipeline
 * (Section III-C): the packed reference rows stay in host memory
 * (rows_host, [n_refs][fid_row_words(n_loci)]) and pass through the device
 * block_refs rows at a time; block b's rows go host -> device on one stream
 * of the call's own and its counts device -> host on another, while the
 * context's stream builds and scans the next block.  counts_host receives
 * C[q][r] for every query q and reference r at counts_host[q * ld + r]
 * (ld >= n_refs), exactly fid_compare_full's values.  Host buffers should be
 * pinned for the copies to overlap.  ws_dev: fid_full_stream_workspace_bytes()
 * bytes of device memory (two staged row blocks, one database block, two
 * [n_q][block_refs] count blocks).  Synchronises before returning.  Errors:
 * FID_EINVAL for NULL or misaligned pointers, ld < n_refs, sizes out of range
 * or a bad mode; FID_ENOMEM for a short workspace.
 */
int fid_full_stream_workspace_bytes(fid_ctx* ctx, int64_t n_refs, int32_t n_loci, int64_t block_refs, int32_t n_q,
                                    size_t* bytes);
int fid_compare_full_streamed(fid_ctx* ctx, const uint64_t* rows_host, int64_t n_refs, int32_t n_loci,
                              int64_t block_refs, const uint64_t* q_dev, int32_t n_q, int mode, void* ws_dev,
                              size_t ws_bytes, int32_t* counts_host, int64_t ld);

/*
 * Threshold hits of a streamed database (rows in host memory as for
 * fid_compare_topk_streamed; Section III-C's blocking with Section IV's
 * reduction on the device): every block is copied in on a stream of the
 * call's own while the previous block is scanned, and scanned with the
 * threshold epilogue into one append buffer; hits are shifted to database
 * rows and sorted once at the end.  Output, thresholds, capacity and
 * FID_EOVERFLOW (with *total_host = the exact number of hits) are as for
 * fid_compare_threshold over the same rows.  ws_dev:
 * fid_threshold_stream_workspace_bytes() bytes.  Synchronises the context's
 * stream (the host rows are free to reuse on return; the CSR is complete
 * once the stream is synchronised again).
 */
int fid_threshold_stream_workspace_bytes(fid_ctx* ctx, int64_t n_refs, int32_t n_loci, int64_t block_refs,
                                         int32_t n_q, int64_t cap, size_t* bytes);
int fid_compare_threshold_streamed(fid_ctx* ctx, const uint64_t* rows_host, int64_t n_refs, int32_t n_loci,
                                   int64_t block_refs, const uint64_t* q_dev, int32_t n_q, int mode,
                                   const int32_t* thr_dev, void* ws_dev, size_t ws_bytes, int64_t cap,
                                   int64_t* offs_dev, int64_t* idx_dev, int32_t* cnt_dev, int64_t* total_host);

/*
 * Peak probes (measurement only; no comparison work).  Each runs a small
 * kernel that saturates one unit the comparison kernels are bound by, on the
 * context's device and stream, and returns its sustained rate (*rate) and
 * the average launch time in ms (*ms), from HIP events over 5 launches after
 * one warm-up.  Synchronises the context's stream.
 *   FID_PROBE_MFMA_FP4  e2m1 16x16x128 matrix-core MACs per second
 *   FID_PROBE_MFMA_I8   int8 32x32x32 matrix-core MACs per second
 *   FID_PROBE_VALU      32-bit VALU lane-ops per second (AND + fused
 *                       count-and-add, the popcount scan's inner pair)
 *   FID_PROBE_HBM_COPY  bytes read + written per second by a 16-byte-per-lane
 *                       copy from the first half of buf_dev to the second
 * buf_dev: caller-owned device memory, 16-byte aligned, contents clobbered;
 * the compute probes need num_CUs * 8192 bytes (8 MiB covers 256 CUs), the
 * copy probe moves buf_bytes / 2 (use >= 2 GiB, well past the last-level
 * cache, for an HBM figure).
 * FID_EINVAL for NULL pointers, an unknown probe or a short buffer.
 */
typedef enum {
    FID_PROBE_MFMA_FP4 = 0,
    FID_PROBE_MFMA_I8 = 1,
    FID_PROBE_VALU = 2,
    FID_PROBE_HBM_COPY = 3
} fid_probe;
int fid_peak_probe(fid_ctx* ctx, int probe, void* buf_dev, size_t buf_bytes, double* rate, double* ms);

/* Number of uint64_t words in one packed row of n_loci loci, or -1 if n_loci is out of range. */
int64_t fid_row_words(int32_t n_loci);

/*
 * Pack profiles (Section II-A encoding): bytes_dev is [n_rows][ld_bytes] device
 * bytes, byte k of a row = locus k, value 0 or 1; rows_dev receives
 * [n_rows][fid_row_words(n_loci)] packed rows (padding bits zero).
 * Synchronises the stream to validate the input: any byte other than 0/1
 * gives FID_EINVAL (rows_dev then holds unspecified values).
 */
int fid_pack(fid_ctx* ctx, const uint8_t* bytes_dev, int64_t n_rows, int32_t n_loci,
             int64_t ld_bytes, uint64_t* rows_dev);

/*
 * Host-side pack (Section II-A encoding), for callers whose profiles are in
 * host memory: bytes is [n_rows][ld_bytes] host bytes, byte k of a row =
 * locus k, value 0 or 1; rows receives [n_rows][fid_row_words(n_loci)]
 * uint64_t words in host memory (the packed format above, padding bits
 * zero), identical to what fid_pack writes on the device.  No GPU work and
 * no context.  FID_EINVAL for NULL buffers, n_rows < 0, n_loci out of range,
 * ld_bytes < n_loci, or any byte other than 0/1 (rows is then unspecified).
 * n_rows = 0 is a no-op.
 */
int fid_pack_host(const uint8_t* bytes, int64_t n_rows, int32_t n_loci, int64_t ld_bytes, uint64_t* rows);

/*
 * Device bytes a database of n_refs profiles of n_loci loci occupies:
 * interleaved reference words, padded with zero rows to a whole number of
 * 1024-reference tiles, four 1 KiB planes of read slack, and the
 * per-reference minor-allele totals (4 bytes per padded row).
 */
int fid_db_bytes(int64_t n_refs, int32_t n_loci, size_t* bytes);

/*
 * Build the resident reference database (the matrix A of Section II-B, laid
 * out on the device for coalesced loads, Section III-B).  rows_dev: [n_refs][fid_row_words(n_loci)] packed rows (may be
 * freed once the build has executed).  db_mem_dev: caller-owned device memory
 * of at least fid_db_bytes() bytes, which the returned handle refers to until
 * fid_db_destroy.  Asynchronous.
 * Errors: FID_EINVAL (sizes, alignment, db_bytes too small), FID_EHIP.
 */
int fid_db_build(fid_ctx* ctx, const uint64_t* rows_dev, int64_t n_refs, int32_t n_loci,
                 void* db_mem_dev, size_t db_bytes, fid_db** out);

/* Release the handle (not the caller's db memory).  NULL is a no-op. */
int fid_db_destroy(fid_db* db);

/* Shape of a database. */
int fid_db_info(const fid_db* db, int64_t* n_refs, int32_t* n_loci);

/* Device pointer to int32_t[n_refs]: minor-allele total popcount(R_r) of each reference. */
int fid_db_popcounts(const fid_db* db, const int32_t** pc_dev);

/*
 * Full count matrix (Algorithm 2 / Section II-B): counts_dev[q * ld + r] =
 * C[q][r] for q < n_q, r < N_R.  q_dev: [n_q][fid_row_words(L)] packed query
 * rows with the database's L.  ld >= N_R.  Asynchronous.
 */
int fid_compare_full(fid_ctx* ctx, const fid_db* db, const uint64_t* q_dev, int32_t n_q,
                     int mode, int32_t* counts_dev, int64_t ld);

/*
 * Full counts for n_tiles sub-blocks of C: tile t covers queries
 * [q0_t, q0_t + th) and references [r0_t, r0_t + tw), with (q0_t, r0_t) =
 * (tiles_host[2t], tiles_host[2t+1]) (host memory); out_dev is
 * [n_tiles][th][tw] row-major.  Every tile must lie inside the matrix.
 */
int fid_compare_tiles(fid_ctx* ctx, const fid_db* db, const uint64_t* q_dev, int32_t n_q,
                      int mode, const int64_t* tiles_host, int32_t n_tiles, int32_t th,
                      int32_t tw, int32_t* out_dev);

/* Workspace bytes fid_compare_topk needs for this database, n_q and k. */
int fid_topk_workspace_bytes(fid_ctx* ctx, const fid_db* db, int32_t n_q, int32_t k,
                             size_t* bytes);

/*
 * Per-query top-k (the GPU-side reduction Section IV recommends instead of
 * shipping C to the host): for each query the k smallest (C[q][r], r) pairs in
 * lexicographic order -- ties in count go to the lowest index -- written
 * ascending to cnt_dev[q * k + j] / idx_dev[q * k + j].  If k > N_R the tail is
 * (INT32_MAX, -1).  The full matrix is never materialised.  ws_dev: caller
 * device memory of fid_topk_workspace_bytes() bytes.  Asynchronous.
 */
int fid_compare_topk(fid_ctx* ctx, const fid_db* db, const uint64_t* q_dev, int32_t n_q,
                     int mode, int32_t k, void* ws_dev, size_t ws_bytes, int32_t* cnt_dev,
                     int64_t* idx_dev);

/*
 * fid_compare_topk for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments and results, without a workspace.  The staged queries and
 * the top-k workspace live in a fixed 256 MiB array that every device holds
 * from the library's load until the process ends; the call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine).  The array must hold
 * fid_topk_workspace_bytes() plus the staged queries (at most n_q x L/2 bytes
 * + 4 n_q, 256-byte aligned): e.g. up to 256 queries against 20M references at
 * 2048 loci and k = 32.  Larger problems return FID_ENOMEM, with the bytes
 * needed in fid_last_error(), before anything is enqueued.  Every call on a
 * device shares that device's array: calls that overlap on one device (two
 * streams, two contexts or two threads) race and must be ordered by the
 * caller.  Nothing in the array needs clearing between calls.  Asynchronous
 * on the context's stream.
 */
int fid_compare_topk_noalloc(fid_ctx* ctx, const fid_db* db, const uint64_t* q_dev, int32_t n_q,
                             int mode, int32_t k, int32_t* cnt_dev, int64_t* idx_dev);

/* Workspace bytes fid_compare_topk_range needs for references [r_lo, r_hi). */
int fid_topk_range_workspace_bytes(fid_ctx* ctx, const fid_db* db, int64_t r_lo, int64_t r_hi,
                                   int32_t n_q, int32_t k, size_t* bytes);

/*
 * fid_compare_topk restricted to the reference rows [r_lo, r_hi) of db (the
 * paper's host driver compares against the reference set block by block,
 * Section IV).  Indices in idx_dev are database rows; if k exceeds the range
 * the tail is (INT32_MAX, -1).  Errors as fid_compare_topk, plus FID_EINVAL
 * for an empty range or one outside the database.
 */
int fid_compare_topk_range(fid_ctx* ctx, const fid_db* db, int64_t r_lo, int64_t r_hi,
                           const uint64_t* q_dev, int32_t n_q, int mode, int32_t k, void* ws_dev,
                           size_t ws_bytes, int32_t* cnt_dev, int64_t* idx_dev);

/* Workspace bytes fid_compare_topk_mixed needs for references [r_lo, r_hi). */
int fid_topk_mixed_workspace_bytes(fid_ctx* ctx, const fid_db* db, int64_t r_lo, int64_t r_hi,
                                   int32_t n_q, int32_t k, size_t* bytes);

/*
 * fid_compare_topk_range for a batch whose queries each carry their own
 * comparison: modes_dev[q] (device int32) is FID_MODE_MIXTURE (Eq. 1) or
 * FID_MODE_IDENTITY (XOR) for query q; identity and mixture unknowns are then
 * compared in the same launches.  Each query's result equals that of a
 * single-mode call.  The modes are checked on the device first (the call
 * synchronises the context's stream once for that): FID_EINVAL, with
 * nothing else enqueued, when any mode is neither FID_MODE_MIXTURE nor
 * FID_MODE_IDENTITY or modes_dev is NULL.  Runs on the fp4 or popcount
 * family.
 */
int fid_compare_topk_mixed(fid_ctx* ctx, const fid_db* db, int64_t r_lo, int64_t r_hi,
                           const uint64_t* q_dev, const int32_t* modes_dev, int32_t n_q, int32_t k,
                           void* ws_dev, size_t ws_bytes, int32_t* cnt_dev, int64_t* idx_dev);

/*
 * fid_compare_topk_mixed with a caller-known bound per query, for callers
 * that block the references themselves and carry a running top-k from block
 * to block (the paper's host driver compares the unknowns against the
 * reference set one block at a time, Section IV).  bound_dev[q] (device
 * uint32) is an exclusive bound on the counts that matter to query q, e.g.
 * the k-th count + 1 of that query's top-k over earlier blocks; any value is
 * valid, 0xFFFFFFFF meaning none.  References with a count >= bound_dev[q]
 * may be left out, so the output is the range's top-k except past the
 * entries below the bound: every entry whose count is below bound_dev[q] is
 * exactly the top-k entry at its position; the entries after them are
 * correct (count, index) pairs with counts >= bound_dev[q], ascending, not
 * necessarily the smallest such, or (INT32_MAX, -1) padding.  use_seed = 0
 * skips the seed pass (the bound alone filters); use_seed != 0 runs it and
 * filters with the tighter of the two.  Workspace: fid_topk_mixed_workspace_
 * bytes().  Modes are checked as in fid_compare_topk_mixed (one
 * synchronisation); FID_EINVAL also for a NULL or unaligned bound pointer.
 */
int fid_compare_topk_bounded(fid_ctx* ctx, const fid_db* db, int64_t r_lo, int64_t r_hi,
                             const uint64_t* q_dev, const int32_t* modes_dev, int32_t n_q, int32_t k,
                             const uint32_t* bound_dev, int use_seed, void* ws_dev, size_t ws_bytes,
                             int32_t* cnt_dev, int64_t* idx_dev);

/* Workspace bytes fid_compare_threshold needs for a hit capacity of cap. */
int fid_threshold_workspace_bytes(const fid_db* db, int32_t n_q, int64_t cap, size_t* bytes);

/*
 * Per-query threshold hits: every (q, r) with C[q][r] <= thr_dev[q], as CSR:
 * offs_dev[n_q + 1] (int64), and for query q the hits
 * idx_dev[offs[q] .. offs[q+1]) in ascending r with their counts in cnt_dev.
 * cap = capacity of idx_dev / cnt_dev.  Synchronises the stream to learn the
 * hit total, which is written to *total_host.  If the total exceeds cap the
 * call returns FID_EOVERFLOW (outputs unspecified; *total_host = the capacity
 * needed).
 */
int fid_compare_threshold(fid_ctx* ctx, const fid_db* db, const uint64_t* q_dev, int32_t n_q,
                          int mode, const int32_t* thr_dev, void* ws_dev, size_t ws_bytes,
                          int64_t cap, int64_t* offs_dev, int64_t* idx_dev, int32_t* cnt_dev,
                          int64_t* total_host);

/*
 * Threshold hits and top-k of the same queries from one pass over the
 * database (Section IV recommends both reductions on the GPU; a large SNP
 * panel wants the candidates under a threshold and the closest k at once).
 * Outputs are exactly those of fid_compare_threshold (offs_dev, hidx_dev,
 * hcnt_dev, cap, *total_host, FID_EOVERFLOW) and fid_compare_topk (cnt_dev,
 * idx_dev: [n_q][k]) for the same arguments.  On the fp4 matrix-core family
 * one scan carries both epilogues; other families, and databases short
 * enough for the direct top-k, run the two comparisons back to back.  The
 * top-k output is complete even when the call returns FID_EOVERFLOW.
 * ws_dev: fid_threshold_topk_workspace_bytes() bytes.  Synchronises the
 * context's stream to learn the hit total (the CSR is complete once the
 * stream is synchronised again).
 */
int fid_threshold_topk_workspace_bytes(fid_ctx* ctx, const fid_db* db, int32_t n_q, int32_t k, int64_t cap,
                                       size_t* bytes);
int fid_compare_threshold_topk(fid_ctx* ctx, const fid_db* db, const uint64_t* q_dev, int32_t n_q, int mode,
                               const int32_t* thr_dev, int32_t k, void* ws_dev, size_t ws_bytes, int64_t cap,
                               int64_t* offs_dev, int64_t* hidx_dev, int32_t* hcnt_dev, int64_t* total_host,
                               int32_t* cnt_dev, int64_t* idx_dev);

/* ------------------------------------------------------------------------
 * Ragged batches: many independent top-k jobs in persistent launches.
 *
 * The paper blocks the reference set to fit device memory and runs one
 * comparison per block (Section IV); a batch instead packs many unrelated
 * jobs -- each with its own queries, reference slice, loci panel and mode --
 * into shared work queues that persistent launches drain, so jobs of every
 * size fill the GPU together: the jobs suited to the fp4 matrix cores in
 * one persistent top-k pass (plus a persistent seed pass and one launch each
 * for staging, selection and merging, for all of them at once), the others
 * in one persistent popcount pass.  Every job's result is exactly what
 * fid_compare_topk gives for that job alone (indices are rows of the job's
 * database, ties go to the lowest index).
 */
typedef struct {
    const fid_db* db;       /* reference panel; its n_loci is the job's L */
    int64_t r_lo, r_hi;     /* reference slice [r_lo, r_hi) of db */
    const uint64_t* q_dev;  /* [n_q][fid_row_words(L)] packed queries, 16-byte aligned */
    int32_t n_q;            /* 1 .. 2^24 */
    int32_t mode;           /* fid_mode */
    int32_t* cnt_dev;       /* out: [n_q][k] counts */
    int64_t* idx_dev;       /* out: [n_q][k] reference indices (-1 past the slice) */
} fid_job;

/*
 * One autotuner row: the work-item shapes for jobs on a panel of n_loci loci
 * (n_loci = 0 matches any panel without a row of its own).  A popcount item
 * is q_per_item (1..32) queries x blocks_per_item (>= 1) 64-reference
 * blocks; a matrix-core (fp4) item is one 128-query tile x at most
 * fp4_tiles (0: 128) 512-reference tiles.
 */
typedef struct {
    int32_t n_loci;
    int32_t q_per_item;
    int32_t blocks_per_item;
    int32_t fp4_tiles;
} fid_tune;

typedef struct fid_batch fid_batch;

/* Device workspace bytes fid_batch_create needs for these jobs (k <= 128). */
int fid_batch_workspace_bytes(fid_ctx* ctx, const fid_job* jobs, int32_t n_jobs, int32_t k,
                              const fid_tune* tune, int32_t n_tune, size_t* bytes);

/*
 * Plan a batch.  Under the AUTO backend every job whose rows the fp4 scan
 * holds (every row length the library accepts) goes to the batched fp4
 * passes, whatever its query count (a query tile of few queries skips its
 * empty 16-query row blocks); a backend forced on the context decides
 * instead (FID_BACKEND_MFMA_FP4: the same; FID_BACKEND_MFMA: the int8
 * kernel where it holds the rows, below; FID_BACKEND_POPCOUNT: the
 * persistent popcount launch, below).  Batched fp4 work
 * items are (job, 128-query tile, run of at most fp4_tiles 512-reference
 * tiles), the items of one reference run queued together on one XCD's
 * queue, the runs dealt largest first to the least-loaded queue.  Jobs sent
 * to the int8 matrix cores run as
 * per-call top-k (fid_compare_topk_range) inside the batch, spread over up to
 * 8 streams the batch creates (each with a context of its own, with the
 * batch context's device and backend, and query scratch reserved here).
 * The others are cut into work items for the persistent popcount launch
 * (q_per_item queries x blocks_per_item blocks; the first reference range
 * of every query block first, then longest first).  tune may be NULL
 * (16 queries x 64 blocks, 128 fp4 tiles; jobs of a panel without a row
 * take the n_loci = 0 row).  The tables go into ws_dev (caller device
 * memory of fid_batch_workspace_bytes() bytes, held until
 * fid_batch_destroy; it includes every fp4 job's staged queries, seed
 * counts and top-k lists).  The jobs' query and output buffers must stay valid
 * for every run.  Synchronises the context's stream once.
 * Errors: FID_EINVAL (any job invalid, k out of range), FID_ENOMEM
 * (workspace too small), FID_EHIP.
 */
int fid_batch_create(fid_ctx* ctx, const fid_job* jobs, int32_t n_jobs, int32_t k,
                     const fid_tune* tune, int32_t n_tune, void* ws_dev, size_t ws_bytes,
                     fid_batch** out);

/*
 * Enqueue the whole batch on the context's stream: the popcount jobs'
 * staging, persistent scan and merge; the fp4 jobs' staging, persistent
 * seed pass, selection, persistent top-k pass and merge; and any per-call
 * jobs' top-k calls on the batch's streams, forked from and joined back to
 * the context's stream by events (no host sync).  With use_graph != 0 the
 * sequence is captured into a HIP graph on the first call and every call
 * replays it.  Asynchronous.  With context timing enabled
 * (fid_ctx_enable_timing), an eager run times its persistent scans (the
 * popcount pass, then the fp4 top-k pass).
 */
int fid_batch_run(fid_batch* b, int use_graph);

/*
 * Work items, item lists and persistent workgroups of the popcount pass of
 * a planned batch, and the number of jobs on the matrix cores (batched fp4
 * passes or per-call).
 */
int fid_batch_info(const fid_batch* b, int64_t* n_items, int64_t* n_lists, int32_t* grid,
                   int32_t* n_routed);

/*
 * Where the plan put job `job` (its index in the array given to
 * fid_batch_create): *routed = 1 for the matrix cores (the batched fp4
 * passes, or a per-call int8 top-k), 0 for the persistent popcount launch.  Host only, no GPU work.  FID_EINVAL for
 * a NULL batch or output or an index outside [0, n_jobs).
 */
int fid_batch_job_routed(const fid_batch* b, int32_t job, int32_t* routed);

/* Release the batch (synchronises the context's stream, which must still
 * exist: destroy batches before their context).  NULL is a no-op. */
int fid_batch_destroy(fid_batch* b);

/* ------------------------------------------------------------------------
 * Serving: a resident database answering a stream of requests.
 *
 * A server owns a worker thread and a stream of its own.  Under
 * FID_SERVE_CONTINUOUS the database is cut into n_chunks reference chunks
 * and the worker runs back-to-back ticks, each comparing every active query
 * (identity and mixture requests mixed in one launch) against a run of
 * consecutive chunks and folding that range's top-k into each query's running
 * top-k; requests are admitted at tick boundaries, in arrival order, as soon
 * as enough query slots are free, and finish once they have met every chunk
 * exactly once.  By default (tick_chunks = 0) a tick spans the whole
 * database: every request waiting at a tick boundary joins one pass and is
 * answered straight from that comparison, so a burst shares one pass instead
 * of queueing for a pass each; tick_chunks = n >= 1 caps a tick at n chunks,
 * so that new requests join mid-pass and complete over later ticks.  Query
 * slots are sized from hbm_budget (slot state, hit buffers and the top-k
 * workspace of a whole-database pass).  FID_SERVE_FIFO answers one request
 * at a time with one whole-database pass.  Either way a request's top-k is
 * identical to fid_compare_topk and its threshold hits to
 * fid_compare_threshold on that request alone (Section IV: the reductions on
 * the GPU, here per request).
 */
typedef enum { FID_SERVE_CONTINUOUS = 0, FID_SERVE_FIFO = 1 } fid_serve_policy;

typedef struct {
    size_t hbm_budget;      /* device bytes for slots, running state, hit buffers and workspace */
    int32_t max_queries;    /* cap on query slots (queries in flight), 1 .. 2^20 */
    int32_t k;              /* top-k depth kept per query, 1 .. 1024 */
    int32_t n_chunks;       /* database chunks per pass (0: 8); FIFO: 1 */
    int32_t policy;         /* fid_serve_policy */
    int32_t tick_chunks;    /* chunks one tick may span: 0 = the whole database, n >= 1 = at most n */
    int32_t hits_per_query; /* threshold hits buffered per query slot and tick (0: 256) */
} fid_server_config;

typedef struct {
    const uint64_t* q_dev;      /* [n_q][fid_row_words(L)] packed queries on the server's
                                   device; read until the request completes */
    int32_t n_q;
    int32_t mode;               /* fid_mode */
    int32_t k;                  /* 1 .. config k */
    int32_t reserved;
    int32_t* cnt_host;          /* out: [n_q][k] host memory, written before completion */
    int64_t* idx_host;          /* out: [n_q][k] */
    /* Threshold hits (optional; thr_host = NULL: none).  thr_host[q] (host,
     * read at submit): a hit is a reference with count <= thr_host[q].  On
     * completion the hits are CSR in reference order: hit_offs_host[n_q + 1],
     * and hit_idx_host / hit_cnt_host [hit_cap] (host).  If they exceed
     * hit_cap the request completes with FID_EOVERFLOW, its top-k valid and
     * hit_offs_host[n_q] = the hits needed; if one tick's hits exceeded the
     * server's buffer (hits_per_query x slots) the request also completes with
     * FID_EOVERFLOW and hit_offs_host[n_q] = -1. */
    const int32_t* thr_host;
    int64_t hit_cap;
    int64_t* hit_offs_host;
    int64_t* hit_idx_host;
    int32_t* hit_cnt_host;
} fid_request;

typedef struct fid_server fid_server;

/*
 * Start a server on db (which must outlive it).  The server allocates its
 * own device memory (at most hbm_budget bytes) and pinned staging.
 * Errors: FID_EINVAL, FID_EBUDGET (the budget holds no query slot),
 * FID_ENOMEM, FID_EHIP.
 */
int fid_server_create(fid_ctx* ctx, const fid_db* db, const fid_server_config* cfg,
                      fid_server** out);

/* Query slots the budget holds, chunks per pass, device bytes allocated. */
int fid_server_info(const fid_server* s, int32_t* max_queries, int32_t* n_chunks,
                    size_t* device_bytes);

/*
 * Queue a request (thread-safe, returns at once).  FID_EBUDGET if it has
 * more queries than the server has slots (it could never be admitted).
 */
int fid_server_submit(fid_server* s, const fid_request* r, uint64_t* ticket);

/*
 * FID_ENOTREADY while the request is in flight; FID_OK once its outputs are
 * written (the ticket is then retired), or FID_EOVERFLOW when its threshold
 * hits did not fit (see fid_request; the top-k outputs are written).
 * times_ns (may be NULL) receives [submit, admit, done] on the steady clock
 * (CLOCK_MONOTONIC) in ns.
 */
int fid_server_poll(fid_server* s, uint64_t ticket, int64_t* times_ns);

/* Block until the request completes (timeout_us < 0: no limit), then poll. */
int fid_server_wait(fid_server* s, uint64_t ticket, int64_t timeout_us, int64_t* times_ns);

/*
 * Counters: stats[0] ticks run, [1] requests completed, [2] most queries in
 * flight at once, [3] summed tick wall time (ns), [4] summed queries in
 * flight over ticks.
 */
int fid_server_stats(const fid_server* s, int64_t* stats);

/* Stop the worker after its current tick and free the server; requests still
 * queued or in flight are dropped.  NULL is a no-op. */
int fid_server_destroy(fid_server* s);

#ifdef __cplusplus
}
#endif

#endif /* FASTID_H */
