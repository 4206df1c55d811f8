// Internal definitions shared by the libfastid kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "fastid.h"

#include <atomic>

namespace fid {

constexpr int kWave = 64;          // CDNA wavefront
constexpr int kWavesPerWG = 4;     // scan workgroups: 4 independent waves
constexpr int kWG = kWave * kWavesPerWG;
constexpr int kIdxBits = 40;       // top-k key = count << 40 | reference index
constexpr uint64_t kIdxMask = (1ull << kIdxBits) - 1;
constexpr uint64_t kSentinel = ~0ull;  // empty top-k slot (larger than every key)
constexpr int64_t kDbTileRefs = 1024;  // database padding granule (references)
constexpr int kMaxK = 1024;
constexpr int kMaxLoci = 65535;
constexpr int kSelectThreads = 256;
constexpr int kSelectSlots = 2048;  // LDS keys of the workgroup top-k (16 KB)
constexpr int kSeedBins = 16384;    // LDS histogram bins of a call's top-k seed bound (64 KB)
constexpr int kSeedBinsBatch = 4096; // the same in ragged batches (16 KB: 8 workgroups per CU)
// Witness levels of a top-k query: the seed bins of its (k/2)-th, (k/4)-th, ...,
// (k/32)-th smallest seed counts (each at least the first), stored [q][kWitLevels].
constexpr int kWitLevels = 5;
constexpr int kMaxListWorkers = 8192;  // top-k workers along references (merge prefix in LDS)
constexpr int kChunkQueries = 60;   // queries per wave when counts span several chunks
                                    // (4 waves x 60 x 64 16-bit partial counts: 30 KiB of LDS)

// EPI_BOTH (fp4 family): the threshold hits and the top-k lists of one scan.
enum Epi { EPI_FULL = 0, EPI_TOPK = 1, EPI_THRESH = 2, EPI_BOTH = 3 };

// Internal mode value: every query carries its own fid_mode in
// ScanParams::qmode (the closed forms and the staging differ per query only).
constexpr int kModePerQuery = 2;

// Resident reference database.  Reference r = 64 * blk + lane; its 16-byte
// unit u (loci 128u .. 128u+127) lives at words[(blk * w4 + u) * 64 + lane],
// so one wave loading unit u of a block reads 1 KiB of contiguous memory.
struct DbView {
    const uint4* words;
    const int32_t* pc;   // popcount of each reference row, [nblk * 64]
    int64_t n_refs;
    int64_t nblk;
    int32_t n_loci;
    int32_t w4;          // 16-byte units per row
};

// One scan launch: references [r_lo, r_hi) x queries [q_lo, q_hi).
struct ScanParams {
    DbView db;
    int32_t qw;            // staged 32-bit words per query (multiple of the chunk width)
    int32_t nchunks;       // chunks of the row held in registers in turn
    int64_t r_lo, r_hi;
    int64_t blk_lo, nblk;  // blocks covering [r_lo, r_hi)
    int32_t q_lo, q_hi;
    int32_t n_rsplit;      // workers along the reference axis
    int32_t q_per_worker;  // queries per worker
    int32_t n_workers;
    int32_t lds_words_per_wave;
    // EPI_FULL: out[(q - out_q_base) * ld + (r - out_r_base)]
    int64_t ld;
    int32_t out_q_base;
    int64_t out_r_base;
    // EPI_TOPK: lists[(q * n_rsplit + worker_r) * k + j]
    int32_t k;
    // EPI_THRESH
    int64_t hit_cap;
    // kModePerQuery: fid_mode of query q at qmode[q]
    const int32_t* qmode;
};

struct ScanBuffers {
    const uint32_t* qs;        // staged queries [.][qw]
    int32_t* out;              // EPI_FULL
    uint64_t* lists;           // EPI_TOPK
    uint32_t* fills;           // EPI_TOPK: filled slots of each list, [q][worker]
    const uint32_t* thr_init;  // EPI_TOPK: accept count < thr_init[q]
    const int32_t* thr;        // EPI_THRESH: hit if count <= thr[q]
    unsigned long long* hit_count;
    uint64_t* hit_keys;        // (q << 40) | r
    int32_t* hit_cnt;
};

// Matrix-core (int8 MFMA) path buffers.
struct MfmaBuffers {
    const uint8_t* qx;         // expanded queries [.][kpad] (0/1 bytes)
    int32_t kpad;
    const int32_t* pcq;        // popcount of each query
    int32_t* out;
    uint64_t* lists;
    uint32_t* fills;
    const uint32_t* thr_init;
    const uint32_t* level;     // top-k witness levels, [q][kWitLevels] (optional)
    uint32_t* wit;             // witnesses counted below each, [q][kWitLevels]
    const int32_t* thr;
    unsigned long long* hit_count;
    uint64_t* hit_keys;
    int32_t* hit_cnt;
};

// Up to kTilesPerLaunch tile origins passed by value (kernel arguments).
constexpr int kTilesPerLaunch = 64;
struct TileTable {
    int32_t n;
    int32_t q0[kTilesPerLaunch];
    int64_t r0[kTilesPerLaunch];
    int32_t out_index[kTilesPerLaunch];
};

// Batched fp4 passes (many query sets -- ragged-batch jobs -- in one
// persistent launch).  A set is one job: its queries (staged for the fp4
// kernel, per-query modes), its reference range and its outputs.
struct Fp4BatchSet {
    DbView db;
    int64_t r_lo, r_hi;
    const uint8_t* qx;           // staged rows, kpad / 2 bytes each
    int32_t kpad;
    int32_t n_slots;             // reference ranges per query tile (list owners: n_slots x 8 waves)
    const int32_t* pcq;
    const int32_t* qmode;
    int32_t n_q;
    int32_t k;
    int32_t* out;                // EPI_FULL: counts [q][ld] of references [out_r_base, ...)
    int64_t ld;
    int64_t out_r_base;
    uint64_t* lists;             // EPI_TOPK
    uint32_t* fills;
    const uint32_t* thr_init;
    const uint32_t* level;
    uint32_t* wit;
};
// One work item: query tile qtile of set `set` against tiles [tb, te) of its range.
struct Fp4BatchItem {
    int32_t set;
    int32_t qtile;
    int32_t slot;
    int32_t pad;
    int64_t tb, te;
};
// Query staging of many jobs in one launch: job j's rows start at global
// query q_off (its pcq / qmode entries) and word w_off (32-locus words over
// all jobs, for the thread split).
struct Fp4ExpandJob {
    const uint64_t* q;
    int32_t n_q, row_words, n_loci, kpad;
    int64_t q_off, w_off;
    uint8_t* qx;
};
// Per-query selection over a seed block of counts (one descriptor per job):
// global query index q_off + i is query i of the job.
struct SelectJob {
    const int32_t* counts;       // [n_q][n_cols]
    int64_t n_cols;
    int64_t q_off;
    int32_t n_q, k;
    int32_t n_loci;
    int32_t pad;
    int64_t idx_base;            // direct top-k: index of column 0
    uint32_t* thr_init;          // seed bound: [n_q], levels / witness counters [n_q][kWitLevels]
    uint32_t* level;
    uint32_t* wit;
    int32_t* cnt;                // direct top-k outputs [n_q][k]
    int64_t* idx;
};

// ---------------------------------------------------------------- launchers
hipError_t launch_pack(const uint8_t* bytes, int64_t n, int32_t n_loci, int64_t ld,
                       int32_t row_words, uint64_t* out, int* bad, hipStream_t s);
// *bad |= 1 when a per-query mode is neither FID_MODE_MIXTURE nor FID_MODE_IDENTITY.
hipError_t launch_check_modes(const int32_t* modes, int32_t n, int* bad, hipStream_t s);
hipError_t launch_db_build(const uint64_t* rows, int64_t n_refs, int32_t row_words,
                           int32_t n_loci, uint4* words, int32_t* pc, int32_t w4, int64_t nblk,
                           hipStream_t s);
hipError_t launch_stage_queries(const uint64_t* q, int32_t n_q, int32_t row_words,
                                int32_t n_loci, int mode, const int32_t* qmode, uint32_t* out,
                                int32_t qw, hipStream_t s);
hipError_t launch_scan(int mode, int nw, int epi, bool chunked, int rpl, const ScanParams& p,
                       const ScanBuffers& b, hipStream_t s);
hipError_t launch_mfma_scan(int mode, int epi, const ScanParams& p, const MfmaBuffers& b,
                            hipStream_t s);
hipError_t launch_tile_counts(int mode, const DbView& db, const uint32_t* qs, int32_t qw,
                              const TileTable& tt, int32_t th, int32_t tw, int32_t* out, hipStream_t s);
hipError_t launch_expand_queries(const uint64_t* q, int32_t n_q, int32_t row_words,
                                 int32_t n_loci, uint8_t* qx, int32_t kpad, int32_t* pcq,
                                 hipStream_t s);
int mfma_kpad(int32_t n_loci);
int mfma_max_loci();
int mfma_refs_per_wg();
int mfma_queries_per_wg();
int mfma_waves_per_wg();
hipError_t launch_fp4_scan(int mode, int epi, const ScanParams& p, const MfmaBuffers& b,
                           hipStream_t s);
// Identity queries (mode, or qmode[i] when mode is kModePerQuery) get
// doubled codes.
hipError_t launch_expand_queries_fp4(const uint64_t* q, int32_t n_q, int32_t row_words,
                                     int32_t n_loci, int mode, const int32_t* qmode, uint8_t* qx,
                                     int32_t kpad, int32_t* pcq, hipStream_t s);
int fp4_kpad(int32_t n_loci);
int fp4_max_kpad();
int fp4_refs_per_wg();
int fp4_queries_per_wg();
int fp4_list_workers_per_wg();
// Persistent fp4 pass over work items taken from 8 queues, one per XCD
// (queue x = items [queue_off[x], queue_off[x + 1]); counters[x] must be 0;
// a workgroup drains its own XCD's queue first, then the others).
// epi: EPI_FULL (sets' out) or EPI_TOPK (sets' lists).  grid = workgroups.
hipError_t launch_fp4_batch(int epi, const Fp4BatchSet* sets, const Fp4BatchItem* items, const int32_t* queue_off,
                            unsigned int* counters, int32_t grid, hipStream_t s);
// Staged fp4 rows and |Q| of every query of n_jobs jobs (per-query modes
// from qmode, indexed by global query); total_words = sum of n_q * kpad / 32.
hipError_t launch_expand_batch_fp4(const Fp4ExpandJob* jobs, int32_t n_jobs, int64_t total_words, int64_t total_q,
                                   const int32_t* qmode, int32_t* pcq, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s);
hipError_t launch_min_bound(uint32_t* thr, const uint32_t* bound, int32_t n, bool keep, int32_t n_loci,
                            uint32_t* level, uint32_t* wit, hipStream_t s);
hipError_t launch_seed_select(const int32_t* counts, int32_t n_q, int64_t n_cols, int32_t k,
                              int32_t n_loci, uint32_t* thr_init, uint32_t* level, uint32_t* wit,
                              hipStream_t s);
hipError_t launch_select_counts(const int32_t* counts, int32_t n_q, int64_t n_cols, int32_t k,
                                int64_t idx_base, int32_t* cnt, int64_t* idx, hipStream_t s);
// The seed bounds (launch_seed_select) of every query of n_jobs jobs, one
// workgroup per query (total_q queries); n_loci_max bounds the histogram.
hipError_t launch_seed_select_batch(const SelectJob* jobs, int32_t n_jobs, int64_t total_q, int32_t n_loci_max,
                                    hipStream_t s);
// The direct top-k (launch_select_counts) of every query of n_jobs jobs.
hipError_t launch_select_counts_batch(const SelectJob* jobs, int32_t n_jobs, int64_t total_q, hipStream_t s);
hipError_t launch_merge_lists(const uint64_t* lists, const uint32_t* fills, int32_t n_q,
                              int32_t n_rsplit, int32_t k, int32_t n_loci, int32_t* cnt, int64_t* idx,
                              hipStream_t s);
hipError_t launch_sort_hits(uint64_t* keys, int32_t* vals, uint64_t* keys2, int32_t* vals2,
                            int64_t n, uint64_t** out_keys, int32_t** out_vals, hipStream_t s);
hipError_t launch_hits_to_csr(const uint64_t* keys, const int32_t* vals, int64_t n, int32_t n_q,
                              int64_t* offs, int64_t* idx, int32_t* cnt, hipStream_t s);

// Genotype rows (0/1/2 per locus) -> 1-bit rows of 2 n_loci loci (two planes).
hipError_t launch_pack_genotypes(const uint8_t* geno, int64_t n, int32_t n_loci, int64_t ld, int32_t row_words,
                                 uint64_t* out, int* bad, hipStream_t s);

// Running top-k per query (serving chunks, streamed blocks): keys
// (count << 40 | index) ascending, kSentinel when empty; bound = k-th count + 1
// (0xFFFFFFFF while not full).  slots maps query i to its row (nullptr: i).
hipError_t launch_reset_running(const int32_t* slots, int32_t n, int32_t k, uint64_t* running, uint32_t* bound,
                                hipStream_t s);
// Fold part results (cnt/idx [n][k], indices + idx_offset) into the rows.
hipError_t launch_fold_topk(const int32_t* cnt, const int64_t* idx, const int32_t* slots, int32_t n, int32_t k,
                            int64_t idx_offset, uint64_t* running, uint32_t* bound, hipStream_t s);
// Rows -> cnt/idx [n][k] (the first k of each row of k_run keys; padding INT32_MAX / -1).
hipError_t launch_finalize_topk(const uint64_t* running, const int32_t* slots, int32_t n, int32_t k_run, int32_t k,
                                int32_t* cnt, int64_t* idx, hipStream_t s);

// After host block b's threshold scan: ends[b + 1] = hits so far, and the
// block's stored hits [ends[b], min(ends[b + 1], cap)) get r0 added to their
// reference index.  ends[0] must be 0.
hipError_t launch_offset_block_hits(const unsigned long long* counter, int64_t* ends, int32_t b, uint64_t* keys,
                                    int64_t cap, int64_t r0, hipStream_t s);

// Opt kernel K in to `bytes` of dynamic LDS (beyond the 64 KiB default) on
// the current device, once per kernel and device (devices 0-63); safe to call
// from several threads.  `bytes` must be the most any launch of K requests.
template <auto K>
hipError_t lds_opt_in(int bytes)
{
    static std::atomic<uint64_t> done{0};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = 1ull << (dev & 63);
    if (done.load(std::memory_order_acquire) & bit) return hipSuccess;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(K), hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess) done.fetch_or(bit, std::memory_order_acq_rel);
    return e;
}

}  // namespace fid
