// libfastid C ABI: argument validation, launch planning and the host side of
// every entry point declared in include/fastid.h.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "fid_internal.hpp"

using namespace fid;

namespace fid {

thread_local std::string g_err;

int fail(int st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(FID_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int env_int(const char* name, int dflt, int lo, int hi)
{
    const char* e = getenv(name);
    if (!e) return dflt;
    const int v = atoi(e);
    return v >= lo && v <= hi ? v : dflt;
}

int set_device(const fid_ctx* ctx)
{
    FID_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    return FID_OK;
}

int timing_begin(fid_ctx* ctx, hipStream_t s, hipEvent_t* end)
{
    *end = nullptr;
    if (!ctx->timing) return FID_OK;
    if (ctx->events_used == ctx->events.size()) {
        std::pair<hipEvent_t, hipEvent_t> ev;
        FID_HIP(hipEventCreate(&ev.first), "hipEventCreate");
        FID_HIP(hipEventCreate(&ev.second), "hipEventCreate");
        ctx->events.push_back(ev);
    }
    FID_HIP(hipEventRecord(ctx->events[ctx->events_used].first, s), "hipEventRecord");
    *end = ctx->events[ctx->events_used].second;
    ++ctx->events_used;
    return FID_OK;
}

}  // namespace fid

// Fixed scratch of fid_compare_topk_noalloc: every device that loads the
// library holds its own copy of this array until the process ends, so that
// call allocates nothing.  Host code never passes the array's name to a
// kernel or a copy: it uses the device address that fixed_scratch_address()
// resolves once per device (kept in each context).
namespace {
constexpr size_t kFixedScratchBytes = (size_t)256 << 20;
}
static __device__ __align__(256) unsigned char scratch[kFixedScratchBytes];

namespace {

std::mutex g_fixed_mu;
std::vector<void*> g_fixed_addr;  // per device, resolved on first use

// The calling thread's current device must be `device`.
int fixed_scratch_address(int device, void** out)
{
    std::lock_guard<std::mutex> lk(g_fixed_mu);
    if ((int)g_fixed_addr.size() <= device) g_fixed_addr.resize((size_t)device + 1, nullptr);
    if (!g_fixed_addr[(size_t)device]) {
        void* p = nullptr;
        FID_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!p) return fail(FID_EHIP, "hipGetSymbolAddress(scratch) returned NULL on device %d", device);
        g_fixed_addr[(size_t)device] = p;
    }
    *out = g_fixed_addr[(size_t)device];
    return FID_OK;
}

}  // namespace

namespace {

constexpr int64_t kMaxRefs = (1ll << kIdxBits) - 1;
constexpr int32_t kMaxQueries = 1 << 24;
constexpr size_t kStatusBytes = 256;

int64_t row_words_of(int32_t n_loci)
{
    if (n_loci < 1 || n_loci > kMaxLoci) return -1;
    return 2 * (((int64_t)n_loci + 127) / 128);
}

// The device database holds whole kDbTileRefs-reference tiles (zero rows
// past n_refs) plus four trailing 16-byte unit planes of slack: the
// matrix-core scans start their tiles on a kDbTileRefs boundary and read up
// to three units past a row, so every load they issue is unconditional and
// in bounds.
int64_t padded_blocks(int64_t n_refs) { return ((n_refs + kDbTileRefs - 1) / kDbTileRefs) * (kDbTileRefs / 64); }

size_t db_words_bytes(int64_t nblk, int64_t row_words)
{
    return align256((size_t)nblk * 64 * (size_t)row_words * 8 + 4 * 64 * 16);
}

// Library scratch: [status words | staged or expanded queries].  Grown on demand.
int ensure_scratch(fid_ctx* ctx, size_t need)
{
    need = align256(need + kStatusBytes);
    if (need <= ctx->scratch_bytes) return FID_OK;
    if (ctx->scratch) {
        FID_HIP(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        FID_HIP(hipFree(ctx->scratch), "hipFree");
        ctx->scratch = nullptr;
        ctx->scratch_bytes = 0;
    }
    hipError_t e = hipMalloc(&ctx->scratch, need);
    if (e != hipSuccess) {
        ctx->scratch = nullptr;
        return fail(FID_ENOMEM, "scratch allocation of %zu bytes failed: %s", need,
                    hipGetErrorString(e));
    }
    ctx->scratch_bytes = need;
    return FID_OK;
}

int* status_words(fid_ctx* ctx) { return static_cast<int*>(ctx->scratch); }

char* query_area(fid_ctx* ctx) { return static_cast<char*>(ctx->scratch) + kStatusBytes; }

// ---------------------------------------------------------------- planning
// Register-resident chunk width (32-bit words per lane) of the popcount scan.
struct Shape {
    int nw;
    int nchunks;
    bool chunked;
    int32_t qw;
};

Shape shape_for(const fid_db* db)
{
    const int32_t w32 = db->v.w4 * 4;
    Shape s{};
    if (w32 <= 16) s.nw = 16;
    else if (w32 <= 32) s.nw = 32;
    else if (w32 <= 64) s.nw = 64;
    else if (w32 <= 128) s.nw = 128;
    else {
        s.nw = 64;
        s.chunked = true;
    }
    s.nchunks = s.chunked ? (w32 + 63) / 64 : 1;
    s.qw = s.nw * s.nchunks;
    return s;
}

// References each lane of the popcount scan holds (two halves the per-query
// overhead per VALU op but doubles the row registers); a tuning switch.
int refs_per_lane(int nw, bool chunked)
{
    if (chunked || nw > 64) return 1;
    return env_int("FASTID_RPL", 1, 1, 2);
}

struct Plan {
    int32_t n_rsplit;            // popcount: waves along references; MFMA: workgroups
    int32_t q_per_worker;
    int32_t n_workers;           // popcount: waves; MFMA: workgroups
    int32_t lds_words_per_wave;
    int32_t list_workers;        // top-k list owners along references
};

constexpr int32_t kTopkQueriesPerWave = 1024;  // LDS: 8 bytes per query per wave

Plan plan_popcount(int num_cus, int64_t nblk, int32_t nq, const Shape& sh, int epi)
{
    const int64_t target = (int64_t)num_cus * env_int("FASTID_WAVES_PER_CU", 24, 1, 64);
    int32_t qmax = nq;
    if (sh.chunked) qmax = kChunkQueries;
    else if (epi == EPI_TOPK) qmax = kTopkQueriesPerWave;
    if (qmax > nq) qmax = nq;
    int64_t qsplit = (nq + qmax - 1) / qmax;
    int64_t rsplit;
    const int64_t rcap = epi == EPI_TOPK ? std::min<int64_t>(target, kMaxListWorkers) : target;
    if (nblk >= rcap) {
        rsplit = rcap;
    } else {
        rsplit = nblk;
        int64_t want = (target + nblk - 1) / nblk;
        if (want > nq) want = nq;
        if (want > qsplit) qsplit = want;
    }
    Plan p{};
    if (rsplit * qsplit > (int64_t)(1 << 30)) return p;  // n_workers == 0: rejected
    p.n_rsplit = (int32_t)rsplit;
    p.q_per_worker = (int32_t)((nq + qsplit - 1) / qsplit);
    p.n_workers = (int32_t)(rsplit * ((nq + p.q_per_worker - 1) / p.q_per_worker));
    int32_t words = 0;
    if (epi == EPI_TOPK) words += 2 * p.q_per_worker;
    if (sh.chunked) words += p.q_per_worker * 32;  // 64 16-bit partial counts per query
    p.lds_words_per_wave = words;
    p.list_workers = p.n_rsplit;
    return p;
}

Plan plan_mfma(int num_cus, int64_t r_lo, int64_t r_hi, int32_t nq, int epi)
{
    const int64_t n_qtiles = (nq + mfma_queries_per_wg() - 1) / mfma_queries_per_wg();
    const int64_t base = (r_lo / kDbTileRefs) * kDbTileRefs;
    const int64_t ntiles = (r_hi - base + mfma_refs_per_wg() - 1) / mfma_refs_per_wg();
    const int64_t target = (int64_t)num_cus * env_int("FASTID_MFMA_WG_PER_CU", 2, 1, 64);
    int64_t rsplit = std::max<int64_t>(1, target / n_qtiles);
    rsplit = std::min(rsplit, ntiles);
    if (epi == EPI_TOPK) rsplit = std::min<int64_t>(rsplit, kMaxListWorkers / mfma_waves_per_wg());
    Plan p{};
    if (rsplit * n_qtiles > (int64_t)(1 << 30)) return p;
    p.n_rsplit = (int32_t)rsplit;
    p.q_per_worker = mfma_queries_per_wg();
    p.n_workers = (int32_t)(rsplit * n_qtiles);
    p.list_workers = p.n_rsplit * mfma_waves_per_wg();
    return p;
}

// One evaluation of the overloaded product on a chosen kernel family.
struct Job {
    int backend;   // FID_BACKEND_POPCOUNT or FID_BACKEND_MFMA (resolved)
    Shape sh;
    int32_t kpad;  // MFMA: expanded query row bytes
};

// The int8 kernel holds a query tile of whole rows in LDS (rows up to
// mfma_max_loci() loci; longer rows use the popcount scan); the fp4 kernel
// stages long rows chunk by chunk and covers every row length.  AUTO weighs each
// family's measured rate at 2048 x 20M x 2048 (comparisons/s relative to the
// popcount scan: int8 x2.2, fp4 x3.2) by how full its query tiles are
// (64 queries for int8, 128 for fp4) and takes the best.
int resolve_backend(const fid_ctx* ctx, const fid_db* db, int32_t n_q)
{
    const bool int8_ok = mfma_kpad(db->v.n_loci) <= mfma_max_loci();
    const bool fp4_ok = fp4_kpad(db->v.n_loci) <= fp4_max_kpad();
    int b = ctx->backend;
    if (b == FID_BACKEND_AUTO) b = env_int("FASTID_BACKEND", FID_BACKEND_AUTO, 0, 3);
    if (b == FID_BACKEND_MFMA_FP4 && !fp4_ok) b = FID_BACKEND_MFMA;
    if (b == FID_BACKEND_MFMA) return int8_ok ? b : FID_BACKEND_POPCOUNT;
    if (b == FID_BACKEND_MFMA_FP4 || b == FID_BACKEND_POPCOUNT) return b;
    auto fill = [&](int tile) {
        const int64_t tiles = (n_q + tile - 1) / tile;
        return (double)n_q / (double)(tiles * tile);
    };
    // Rate of a full 128-query fp4 tile relative to the popcount scan, from
    // measured crossovers (top-32 over 2M-5M references): short rows give
    // the matrix cores little work per tile and its fixed costs dominate.
    const int kp = fp4_kpad(db->v.n_loci);
    const double fp4_rate = kp <= 1024 ? 2.0 : kp <= 2048 ? 5.3 : 6.0;
    // the int8 kernel never beat the fp4 one in the measured sweeps: AUTO
    // takes it only where the fp4 tile cannot hold the rows
    const double r_int8 = int8_ok && !fp4_ok ? 2.2 * fill(mfma_queries_per_wg()) : 0.0;
    const double r_fp4 = fp4_ok ? fp4_rate * fill(fp4_queries_per_wg()) : 0.0;
    if (r_fp4 >= 1.0 && r_fp4 >= r_int8) return FID_BACKEND_MFMA_FP4;
    if (r_int8 >= 1.0) return FID_BACKEND_MFMA;
    return FID_BACKEND_POPCOUNT;
}

// Per-query modes run on the fp4 or popcount kernels only.
Job make_job(const fid_ctx* ctx, const fid_db* db, int32_t n_q, bool per_query_modes = false)
{
    Job j{};
    j.backend = resolve_backend(ctx, db, n_q);
    if (per_query_modes && j.backend == FID_BACKEND_MFMA) j.backend = FID_BACKEND_POPCOUNT;
    j.sh = shape_for(db);
    j.kpad = j.backend == FID_BACKEND_MFMA_FP4 ? fp4_kpad(db->v.n_loci) : mfma_kpad(db->v.n_loci);
    return j;
}

Plan plan_fp4(int num_cus, int64_t r_lo, int64_t r_hi, int32_t nq, int epi)
{
    const int64_t n_qtiles = (nq + fp4_queries_per_wg() - 1) / fp4_queries_per_wg();
    const int64_t base = (r_lo / kDbTileRefs) * kDbTileRefs;
    const int64_t ntiles = (r_hi - base + fp4_refs_per_wg() - 1) / fp4_refs_per_wg();
    const int64_t target = (int64_t)num_cus * env_int("FASTID_MFMA_WG_PER_CU", 2, 1, 64);
    int64_t rsplit = std::max<int64_t>(1, target / n_qtiles);
    rsplit = std::min(rsplit, ntiles);
    if (epi == EPI_TOPK) rsplit = std::min<int64_t>(rsplit, kMaxListWorkers / fp4_list_workers_per_wg());
    Plan p{};
    if (rsplit * n_qtiles > (int64_t)(1 << 30)) return p;
    p.n_rsplit = (int32_t)rsplit;
    p.q_per_worker = fp4_queries_per_wg();
    p.n_workers = (int32_t)(rsplit * n_qtiles);
    p.list_workers = p.n_rsplit * fp4_list_workers_per_wg();
    return p;
}

Plan plan_for(const fid_ctx* ctx, const Job& j, int64_t r_lo, int64_t r_hi, int32_t n_q, int epi)
{
    if (j.backend == FID_BACKEND_MFMA) return plan_mfma(ctx->num_cus, r_lo, r_hi, n_q, epi);
    if (j.backend == FID_BACKEND_MFMA_FP4) return plan_fp4(ctx->num_cus, r_lo, r_hi, n_q, epi);
    const int64_t nblk = (r_hi + 63) / 64 - r_lo / 64;
    return plan_popcount(ctx->num_cus, nblk, n_q, j.sh, epi);
}

ScanParams make_params(const fid_db* db, const Job& j, const Plan& pl, int64_t r_lo, int64_t r_hi,
                       int32_t q_lo, int32_t q_hi)
{
    ScanParams p{};
    p.db = db->v;
    p.qw = j.sh.qw;
    p.nchunks = j.sh.nchunks;
    p.r_lo = r_lo;
    p.r_hi = r_hi;
    p.blk_lo = r_lo / 64;
    p.nblk = (r_hi + 63) / 64 - p.blk_lo;
    p.q_lo = q_lo;
    p.q_hi = q_hi;
    p.n_rsplit = pl.n_rsplit;
    p.q_per_worker = pl.q_per_worker;
    p.n_workers = pl.n_workers;
    p.lds_words_per_wave = pl.lds_words_per_wave;
    return p;
}

int check_mode(int mode)
{
    if (mode != FID_MODE_MIXTURE && mode != FID_MODE_IDENTITY)
        return fail(FID_EINVAL, "mode must be FID_MODE_MIXTURE (0) or FID_MODE_IDENTITY (1), got %d", mode);
    return FID_OK;
}

int check_common(const fid_ctx* ctx, const fid_db* db, const uint64_t* q_dev, int32_t n_q, int mode)
{
    if (!ctx) return fail(FID_EINVAL, "ctx is NULL");
    if (!db) return fail(FID_EINVAL, "db is NULL");
    if (db->device != ctx->device) return fail(FID_EINVAL, "db lives on device %d, ctx on %d", db->device, ctx->device);
    if (!q_dev) return fail(FID_EINVAL, "query pointer is NULL");
    if (!aligned16(q_dev)) return fail(FID_EINVAL, "query pointer not 16-byte aligned");
    if (n_q < 1 || n_q > kMaxQueries) return fail(FID_EINVAL, "n_q=%d out of [1, 2^24]", n_q);
    return check_mode(mode);
}

// Query preparation (step A3): popcount scan -> masked, padded 32-bit words
// (mixture queries inverted); matrix cores -> 0/1 bytes plus popcounts.
struct Prepared {
    const uint32_t* qs;
    const uint8_t* qx;
    const int32_t* pcq;
    const int32_t* qmode;  // kModePerQuery: per-query fid_mode
};

// Staged queries go to the context's scratch (grown on demand), or to
// `area` when the caller provides one (query_scratch_bytes() bytes), which
// allocates nothing.
int prepare_queries(fid_ctx* ctx, const fid_db* db, const Job& j, const uint64_t* q_dev,
                    int32_t n_q, int mode, Prepared* out, const int32_t* qmode = nullptr,
                    char* area = nullptr)
{
    *out = Prepared{};
    out->qmode = qmode;
    auto reserve = [&](size_t bytes) -> int { return area ? FID_OK : ensure_scratch(ctx, bytes); };
    auto qbase = [&]() { return area ? area : query_area(ctx); };
    if (j.backend == FID_BACKEND_MFMA_FP4) {
        const size_t xbytes = align256((size_t)n_q * (size_t)(j.kpad / 2));
        FID_TRY(reserve(xbytes + (size_t)n_q * sizeof(int32_t)));
        uint8_t* qx = reinterpret_cast<uint8_t*>(qbase());
        int32_t* pcq = reinterpret_cast<int32_t*>(qbase() + xbytes);
        FID_HIP(launch_expand_queries_fp4(q_dev, n_q, db->row_words, db->v.n_loci, mode, qmode, qx, j.kpad,
                                          pcq, ctx->stream),
                "expand_queries launch");
        out->qx = qx;
        out->pcq = pcq;
        out->qmode = qmode;
        return FID_OK;
    }
    if (j.backend == FID_BACKEND_MFMA) {
        const size_t xbytes = align256((size_t)n_q * (size_t)j.kpad);
        FID_TRY(reserve(xbytes + (size_t)n_q * sizeof(int32_t)));
        uint8_t* qx = reinterpret_cast<uint8_t*>(qbase());
        int32_t* pcq = reinterpret_cast<int32_t*>(qbase() + xbytes);
        FID_HIP(launch_expand_queries(q_dev, n_q, db->row_words, db->v.n_loci, qx, j.kpad, pcq,
                                      ctx->stream),
                "expand_queries launch");
        out->qx = qx;
        out->pcq = pcq;
        out->qmode = qmode;
        return FID_OK;
    }
    FID_TRY(reserve((size_t)n_q * j.sh.qw * sizeof(uint32_t)));
    uint32_t* qs = reinterpret_cast<uint32_t*>(qbase());
    FID_HIP(launch_stage_queries(q_dev, n_q, db->row_words, db->v.n_loci, mode, qmode, qs, j.sh.qw,
                                 ctx->stream),
            "stage_queries launch");
    out->qs = qs;
    out->qmode = qmode;
    return FID_OK;
}

// Output side of a scan (only the members of the epilogue in use are read).
struct Outputs {
    int32_t* out = nullptr;
    uint64_t* lists = nullptr;
    uint32_t* fills = nullptr;
    const uint32_t* thr_init = nullptr;
    const uint32_t* level = nullptr;
    uint32_t* wit = nullptr;
    const int32_t* thr = nullptr;
    unsigned long long* hit_count = nullptr;
    uint64_t* hit_keys = nullptr;
    int32_t* hit_cnt = nullptr;
};

// Launch one scan; `timed` brackets it with events when timing is on.
int run_scan(fid_ctx* ctx, const Job& j, int mode, int epi, const ScanParams& p_in,
             const Prepared& q, const Outputs& o, bool timed)
{
    ScanParams p = p_in;
    p.qmode = q.qmode;
    if (p.n_workers <= 0) return fail(FID_EINVAL, "problem too large for one launch");
    hipEvent_t e1 = nullptr;
    if (timed) FID_TRY(timing_begin(ctx, ctx->stream, &e1));
    if (j.backend == FID_BACKEND_MFMA || j.backend == FID_BACKEND_MFMA_FP4) {
        MfmaBuffers b{};
        b.qx = q.qx;
        b.kpad = j.kpad;
        b.pcq = q.pcq;
        b.out = o.out;
        b.lists = o.lists;
        b.fills = o.fills;
        b.thr_init = o.thr_init;
        b.level = o.level;
        b.wit = o.wit;
        b.thr = o.thr;
        b.hit_count = o.hit_count;
        b.hit_keys = o.hit_keys;
        b.hit_cnt = o.hit_cnt;
        if (j.backend == FID_BACKEND_MFMA_FP4)
            FID_HIP(launch_fp4_scan(mode, epi, p, b, ctx->stream), "fp4 scan launch");
        else
            FID_HIP(launch_mfma_scan(mode, epi, p, b, ctx->stream), "mfma scan launch");
    } else {
        ScanBuffers b{};
        b.qs = q.qs;
        b.out = o.out;
        b.lists = o.lists;
        b.fills = o.fills;
        b.thr_init = o.thr_init;
        b.thr = o.thr;
        b.hit_count = o.hit_count;
        b.hit_keys = o.hit_keys;
        b.hit_cnt = o.hit_cnt;
        FID_HIP(launch_scan(mode, j.sh.nw, epi, j.sh.chunked, refs_per_lane(j.sh.nw, j.sh.chunked),
                            p, b, ctx->stream),
                "scan launch");
    }
    if (e1) FID_HIP(hipEventRecord(e1, ctx->stream), "hipEventRecord");
    return FID_OK;
}

// Full counts of queries [q_lo, q_hi) x references [r_lo, r_hi) into
// out[(q - q_base) * ld + (r - r_base)].
int run_full(fid_ctx* ctx, const fid_db* db, const Job& j, const Prepared& q, int mode,
             int64_t r_lo, int64_t r_hi, int32_t q_lo, int32_t q_hi, int32_t* out, int64_t ld,
             int32_t q_base, int64_t r_base, bool timed)
{
    const Plan pl = plan_for(ctx, j, r_lo, r_hi, q_hi - q_lo, EPI_FULL);
    ScanParams p = make_params(db, j, pl, r_lo, r_hi, q_lo, q_hi);
    p.ld = ld;
    p.out_q_base = q_base;
    p.out_r_base = r_base;
    Outputs o;
    o.out = out;
    return run_scan(ctx, j, mode, EPI_FULL, p, q, o, timed);
}

// Reference-prefix size whose exact k-th count seeds the top-k filter.  The
// fp4 scan also tightens its bound during the scan with the witness levels
// from the same prefix, so it takes a 4x smaller prefix than the kernels
// that filter with the seed bound alone.  A call of one or two fp4 query
// tiles spreads each query over thousands of list owners (one per wave),
// whose own lists rarely fill: there the starting bound decides how many
// candidates the scan inserts, and a 2x larger prefix pays (2048 x 20M x
// 2048 loci: 128 queries 2.47 -> 2.03 ms per call, 48 queries 2.00 -> 1.77;
// with four or more tiles the larger prefix costs more than it saves).
int64_t seed_refs(int64_t n_refs, int backend, int32_t n_q)
{
    const bool witnessed = backend == FID_BACKEND_MFMA_FP4;
    const bool few_tiles = witnessed && n_q <= 2 * fp4_queries_per_wg();
    const int64_t div = witnessed ? (few_tiles ? 128 : 256) : 64;
    const int64_t cap = witnessed ? (few_tiles ? 131072 : 65536) : 262144;
    int64_t s = ((n_refs / div) + 63) / 64 * 64;
    if (s < 16384) s = 16384;
    if (s > cap) s = cap;
    return s < n_refs ? s : n_refs;
}

struct TopkLayout {
    bool direct;          // whole count block fits: count then select
    Plan plan;
    int64_t seed;         // reference prefix of the seed pass
    size_t off_lists, off_fills, off_counts, off_thr, off_level, off_wit, total;
};

TopkLayout topk_layout(const fid_ctx* ctx, const Job& j, int64_t r_lo, int64_t r_hi, int32_t n_q,
                       int32_t k)
{
    TopkLayout L{};
    const int64_t n = r_hi - r_lo;
    L.seed = seed_refs(n, j.backend, n_q);
    L.direct = L.seed == n;
    size_t off = 0;
    if (L.direct) {
        L.off_counts = off;
        off += align256((size_t)n_q * (size_t)n * sizeof(int32_t));
    } else {
        L.plan = plan_for(ctx, j, r_lo, r_hi, n_q, EPI_TOPK);
        L.off_lists = off;
        off += align256((size_t)n_q * L.plan.list_workers * (size_t)k * sizeof(uint64_t));
        L.off_fills = off;
        off += align256((size_t)n_q * L.plan.list_workers * sizeof(uint32_t));
        L.off_counts = off;
        off += align256((size_t)n_q * (size_t)L.seed * sizeof(int32_t));
        L.off_thr = off;
        off += align256((size_t)n_q * sizeof(uint32_t));
        L.off_level = off;
        off += align256((size_t)n_q * kWitLevels * sizeof(uint32_t));
        L.off_wit = off;
        off += align256((size_t)n_q * kWitLevels * sizeof(uint32_t));
    }
    L.total = off;
    return L;
}

int check_range(const fid_db* db, int64_t r_lo, int64_t r_hi)
{
    if (r_lo < 0 || r_hi <= r_lo || r_hi > db->v.n_refs)
        return fail(FID_EINVAL, "reference range [%lld, %lld) outside [0, %lld) or empty",
                    (long long)r_lo, (long long)r_hi, (long long)db->v.n_refs);
    return FID_OK;
}

// Per-query modes live in device memory: one small check kernel, read back
// synchronously, so that a mode outside {MIXTURE, IDENTITY} is refused
// before any comparison is enqueued.
int check_modes_dev(fid_ctx* ctx, const int32_t* modes_dev, int32_t n_q)
{
    if (!modes_dev) return fail(FID_EINVAL, "modes pointer is NULL");
    if ((reinterpret_cast<uintptr_t>(modes_dev) & 3u) != 0) return fail(FID_EINVAL, "modes pointer not 4-byte aligned");
    FID_TRY(set_device(ctx));
    int* bad = status_words(ctx);
    FID_HIP(launch_fill_u64(reinterpret_cast<uint64_t*>(bad), 1, 0ull, ctx->stream), "fill launch");
    FID_HIP(launch_check_modes(modes_dev, n_q, bad, ctx->stream), "mode check launch");
    int bad_host = 0;
    FID_HIP(hipMemcpyAsync(&bad_host, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream), "hipMemcpyAsync");
    FID_HIP(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    if (bad_host)
        return fail(FID_EINVAL, "modes_dev holds a value other than FID_MODE_MIXTURE (0) or FID_MODE_IDENTITY (1)");
    return FID_OK;
}

// Top-k of queries x references [r_lo, r_hi); indices are database rows.
// mode may be kModePerQuery with qmode[n_q] (device) giving each query's mode.
// bound_dev (optional, device [n_q]): a caller-known exclusive bound per query
// ("count < bound" loses nothing); with seed = false it replaces the seed
// pass, with seed = true the tighter of the two filters.
int topk_range(fid_ctx* ctx, const fid_db* db, int64_t r_lo, int64_t r_hi, const uint64_t* q_dev,
               int32_t n_q, int mode, int32_t k, void* ws_dev, size_t ws_bytes, int32_t* cnt_dev,
               int64_t* idx_dev, const int32_t* qmode = nullptr, const uint32_t* bound_dev = nullptr,
               bool seed = true, char* qarea = nullptr, bool timed = true)
{
    const bool per_query = mode == kModePerQuery;
    FID_TRY(check_common(ctx, db, q_dev, n_q, per_query ? FID_MODE_MIXTURE : mode));
    if (per_query && !qmode) return fail(FID_EINVAL, "modes pointer is NULL");
    FID_TRY(check_range(db, r_lo, r_hi));
    if (k < 1 || k > kMaxK) return fail(FID_EINVAL, "k=%d out of [1, %d]", k, kMaxK);
    if (!cnt_dev || !idx_dev || !ws_dev) return fail(FID_EINVAL, "NULL buffer");
    if (!aligned16(ws_dev)) return fail(FID_EINVAL, "workspace not 16-byte aligned");
    const Job j = make_job(ctx, db, n_q, per_query);
    const TopkLayout L = topk_layout(ctx, j, r_lo, r_hi, n_q, k);
    if (ws_bytes < L.total) return fail(FID_ENOMEM, "workspace %zu bytes < required %zu", ws_bytes, L.total);
    FID_TRY(set_device(ctx));
    Prepared q;
    FID_TRY(prepare_queries(ctx, db, j, q_dev, n_q, mode, &q, qmode, qarea));
    char* ws = static_cast<char*>(ws_dev);
    int32_t* counts = reinterpret_cast<int32_t*>(ws + L.off_counts);

    // Seed (or, for a small range, the whole answer): the full count block of
    // the first L.seed references of the range, then an exact per-query
    // selection.
    if (L.direct || seed || !bound_dev)
        FID_TRY(run_full(ctx, db, j, q, mode, r_lo, r_lo + L.seed, 0, n_q, counts, L.seed, 0, r_lo,
                         L.direct && timed));
    if (L.direct) {
        FID_HIP(launch_select_counts(counts, n_q, L.seed, k, r_lo, cnt_dev, idx_dev, ctx->stream),
                "select launch");
        return FID_OK;
    }
    uint64_t* lists = reinterpret_cast<uint64_t*>(ws + L.off_lists);
    uint32_t* fills = reinterpret_cast<uint32_t*>(ws + L.off_fills);
    uint32_t* thr_init = reinterpret_cast<uint32_t*>(ws + L.off_thr);
    uint32_t* level = reinterpret_cast<uint32_t*>(ws + L.off_level);
    uint32_t* wit = reinterpret_cast<uint32_t*>(ws + L.off_wit);
    if (seed || !bound_dev)
        FID_HIP(launch_seed_select(counts, n_q, L.seed, k, db->v.n_loci, thr_init, level, wit, ctx->stream),
                "seed select launch");
    if (bound_dev)
        FID_HIP(launch_min_bound(thr_init, bound_dev, n_q, seed, db->v.n_loci, level, wit, ctx->stream),
                "bound launch");
    ScanParams p = make_params(db, j, L.plan, r_lo, r_hi, 0, n_q);
    p.k = k;
    Outputs o;
    o.lists = lists;
    o.fills = fills;
    o.thr_init = thr_init;
    o.level = level;
    o.wit = wit;
    FID_TRY(run_scan(ctx, j, mode, EPI_TOPK, p, q, o, timed));
    FID_HIP(launch_merge_lists(lists, fills, n_q, L.plan.list_workers, k, db->v.n_loci, cnt_dev, idx_dev,
                               ctx->stream),
            "merge launch");
    return FID_OK;
}

}  // namespace

namespace fid {

int topk_range_bounded(fid_ctx* ctx, const fid_db* db, int64_t r_lo, int64_t r_hi, const uint64_t* q_dev,
                       const int32_t* modes_dev, int32_t n_q, int32_t k, void* ws_dev, size_t ws_bytes,
                       int32_t* cnt_dev, int64_t* idx_dev, const uint32_t* bound_dev, bool seed)
{
    return topk_range(ctx, db, r_lo, r_hi, q_dev, n_q, kModePerQuery, k, ws_dev, ws_bytes, cnt_dev, idx_dev,
                      modes_dev, bound_dev, seed);
}

int thresh_range(fid_ctx* ctx, const fid_db* db, int64_t r_lo, int64_t r_hi, const uint64_t* q_dev, int32_t n_q,
                 int mode, const int32_t* thr_dev, unsigned long long* counter, uint64_t* keys, int32_t* vals,
                 int64_t cap)
{
    FID_TRY(check_common(ctx, db, q_dev, n_q, mode));
    FID_TRY(check_range(db, r_lo, r_hi));
    if (!thr_dev || !counter || (cap > 0 && (!keys || !vals))) return fail(FID_EINVAL, "NULL buffer");
    FID_TRY(set_device(ctx));
    const Job j = make_job(ctx, db, n_q);
    Prepared q;
    FID_TRY(prepare_queries(ctx, db, j, q_dev, n_q, mode, &q));
    const Plan pl = plan_for(ctx, j, r_lo, r_hi, n_q, EPI_THRESH);
    ScanParams p = make_params(db, j, pl, r_lo, r_hi, 0, n_q);
    p.hit_cap = cap;
    Outputs o;
    o.thr = thr_dev;
    o.hit_count = counter;
    o.hit_keys = keys;
    o.hit_cnt = vals;
    return run_scan(ctx, j, mode, EPI_THRESH, p, q, o, false);
}

int scratch_reserve(fid_ctx* ctx, size_t bytes) { return ensure_scratch(ctx, bytes); }

int64_t seed_prefix(int64_t n_refs, int backend, int32_t n_q) { return seed_refs(n_refs, backend, n_q); }

int auto_family(const fid_ctx* ctx, const fid_db* db, int32_t n_q) { return resolve_backend(ctx, db, n_q); }

// Inside a ragged batch a job either shares the persistent popcount launch
// (no per-job cost) or runs as its own matrix-core top-k call (a fixed cost
// for its seed, merge and launches).  The persistent launch hides the small
// jobs' fixed costs, so the batch routes a job only when a full query tile
// of the matrix cores beats the popcount scan by the query-tile fill: fp4
// rate 3.2 (rows <= 2048 loci) or 2.6 (chunked rows) times the fill, as
// measured on the 400-job ragged batch (413 ms against 425-434 ms for the
// per-call crossovers or a per-job cost model).  A backend forced on the
// context is honoured as it is.
// A batch job runs as a per-call matrix-core top-k exactly when a single call
// would (the routed calls overlap one another on the batch's streams, which
// hides their fixed costs as well as the persistent launch would).
bool batch_routes_to_matrix_cores(const fid_ctx* ctx, const fid_db* db, int32_t n_q)
{
    return resolve_backend(ctx, db, n_q) != FID_BACKEND_POPCOUNT;
}

size_t query_scratch_bytes(const fid_ctx* ctx, const fid_db* db, int32_t n_q)
{
    const Job j = make_job(ctx, db, n_q);
    if (j.backend == FID_BACKEND_MFMA_FP4) return align256((size_t)n_q * (j.kpad / 2)) + (size_t)n_q * 4;
    if (j.backend == FID_BACKEND_MFMA) return align256((size_t)n_q * j.kpad) + (size_t)n_q * 4;
    return (size_t)n_q * j.sh.qw * sizeof(uint32_t);
}

}  // namespace fid

// ====================================================================== C ABI
extern "C" {

const char* fid_status_str(int status)
{
    switch (status) {
        case FID_OK: return "FID_OK";
        case FID_EINVAL: return "FID_EINVAL: invalid argument";
        case FID_ENOMEM: return "FID_ENOMEM: out of memory or buffer too small";
        case FID_EHIP: return "FID_EHIP: HIP runtime error";
        case FID_EOVERFLOW: return "FID_EOVERFLOW: output capacity exceeded";
        case FID_EBUDGET: return "FID_EBUDGET: memory budget exceeded";
        case FID_ETIMEOUT: return "FID_ETIMEOUT: timed out";
        case FID_ENOTREADY: return "FID_ENOTREADY: not ready";
        case FID_ENODEV: return "FID_ENODEV: no usable gfx950 device";
        default: return "unknown fid_status";
    }
}

const char* fid_last_error(void) { return g_err.c_str(); }

int fid_version(void) { return 100; }

int fid_ctx_create(fid_ctx** out, int device, void* stream)
{
    if (!out) return fail(FID_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) return fail(FID_ENODEV, "no HIP device available");
    if (device < 0 || device >= n) return fail(FID_ENODEV, "device %d out of range [0, %d)", device, n);
    hipDeviceProp_t prop;
    FID_HIP(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(FID_ENODEV, "device %d is %s; this library is built for gfx950", device, prop.gcnArchName);
    FID_HIP(hipSetDevice(device), "hipSetDevice");
    fid_ctx* c = new fid_ctx{};
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    c->num_cus = prop.multiProcessorCount;
    c->backend = FID_BACKEND_AUTO;
    c->scratch = nullptr;
    c->scratch_bytes = 0;
    c->timing = false;
    c->events_used = 0;
    c->fixed_scratch = nullptr;
    int st = fixed_scratch_address(device, &c->fixed_scratch);
    if (!st) st = ensure_scratch(c, 0);
    if (st) {
        delete c;
        return st;
    }
    *out = c;
    return FID_OK;
}

int fid_ctx_destroy(fid_ctx* ctx)
{
    if (!ctx) return FID_OK;
    int st = set_device(ctx);
    if (!st) {
        hipStreamSynchronize(ctx->stream);
        if (ctx->scratch) hipFree(ctx->scratch);
        for (auto& ev : ctx->events) {
            hipEventDestroy(ev.first);
            hipEventDestroy(ev.second);
        }
    }
    delete ctx;
    return st;
}

int fid_ctx_set_backend(fid_ctx* ctx, int backend)
{
    if (!ctx) return fail(FID_EINVAL, "ctx is NULL");
    if (backend < FID_BACKEND_AUTO || backend > FID_BACKEND_MFMA_FP4)
        return fail(FID_EINVAL, "unknown backend %d", backend);
    ctx->backend = backend;
    return FID_OK;
}

int fid_backend_for(fid_ctx* ctx, const fid_db* db, int32_t n_q, int* backend)
{
    if (!ctx || !db || !backend) return fail(FID_EINVAL, "NULL argument");
    if (n_q < 1 || n_q > kMaxQueries) return fail(FID_EINVAL, "n_q out of range");
    *backend = resolve_backend(ctx, db, n_q);
    return FID_OK;
}

int fid_ctx_set_stream(fid_ctx* ctx, void* stream)
{
    if (!ctx) return fail(FID_EINVAL, "ctx is NULL");
    ctx->stream = static_cast<hipStream_t>(stream);
    return FID_OK;
}

int fid_sync(fid_ctx* ctx)
{
    if (!ctx) return fail(FID_EINVAL, "ctx is NULL");
    FID_TRY(set_device(ctx));
    FID_HIP(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    return FID_OK;
}

int fid_ctx_enable_timing(fid_ctx* ctx, int enable)
{
    if (!ctx) return fail(FID_EINVAL, "ctx is NULL");
    ctx->timing = enable != 0;
    return FID_OK;
}

int fid_ctx_scan_time(fid_ctx* ctx, double* total_ms, int64_t* launches, int reset)
{
    if (!ctx || !total_ms || !launches) return fail(FID_EINVAL, "NULL argument");
    FID_TRY(set_device(ctx));
    double sum = 0.0;
    for (size_t i = 0; i < ctx->events_used; ++i) {
        FID_HIP(hipEventSynchronize(ctx->events[i].second), "hipEventSynchronize");
        float ms = 0.f;
        FID_HIP(hipEventElapsedTime(&ms, ctx->events[i].first, ctx->events[i].second),
                "hipEventElapsedTime");
        sum += ms;
    }
    *total_ms = sum;
    *launches = (int64_t)ctx->events_used;
    if (reset) ctx->events_used = 0;
    return FID_OK;
}

int64_t fid_row_words(int32_t n_loci) { return row_words_of(n_loci); }

int fid_pack(fid_ctx* ctx, const uint8_t* bytes_dev, int64_t n_rows, int32_t n_loci,
             int64_t ld_bytes, uint64_t* rows_dev)
{
    if (!ctx) return fail(FID_EINVAL, "ctx is NULL");
    const int64_t rw = row_words_of(n_loci);
    if (rw < 0) return fail(FID_EINVAL, "n_loci=%d out of [1, %d]", n_loci, kMaxLoci);
    if (n_rows < 0) return fail(FID_EINVAL, "n_rows < 0");
    if (n_rows == 0) return FID_OK;
    if (!bytes_dev || !rows_dev) return fail(FID_EINVAL, "NULL buffer");
    if (ld_bytes < n_loci) return fail(FID_EINVAL, "ld_bytes < n_loci");
    if (!aligned16(rows_dev)) return fail(FID_EINVAL, "rows_dev not 16-byte aligned");
    FID_TRY(set_device(ctx));
    int* bad = status_words(ctx);
    FID_HIP(launch_fill_u64(reinterpret_cast<uint64_t*>(bad), 1, 0ull, ctx->stream), "fill launch");
    FID_HIP(launch_pack(bytes_dev, n_rows, n_loci, ld_bytes, (int32_t)rw, rows_dev, bad, ctx->stream),
            "pack launch");
    int bad_host = 0;
    FID_HIP(hipMemcpyAsync(&bad_host, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream), "hipMemcpyAsync");
    FID_HIP(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    if (bad_host) return fail(FID_EINVAL, "profile bytes must be 0 or 1");
    return FID_OK;
}

int fid_pack_host(const uint8_t* bytes, int64_t n_rows, int32_t n_loci, int64_t ld_bytes, uint64_t* rows)
{
    const int64_t rw = row_words_of(n_loci);
    if (rw < 0) return fail(FID_EINVAL, "n_loci=%d out of [1, %d]", n_loci, kMaxLoci);
    if (n_rows < 0) return fail(FID_EINVAL, "n_rows < 0");
    if (n_rows == 0) return FID_OK;
    if (!bytes || !rows) return fail(FID_EINVAL, "NULL buffer");
    if (ld_bytes < n_loci) return fail(FID_EINVAL, "ld_bytes < n_loci");
    for (int64_t i = 0; i < n_rows; ++i) {
        const uint8_t* src = bytes + i * ld_bytes;
        uint64_t* dst = rows + i * rw;
        uint8_t badbits = 0;
        for (int64_t w = 0; w < rw; ++w) {
            uint64_t word = 0;
            const int32_t k0 = (int32_t)(w * 64);
            for (int32_t b = 0; b < 64 && k0 + b < n_loci; ++b) {
                badbits |= src[k0 + b] & 0xFEu;
                word |= (uint64_t)(src[k0 + b] & 1u) << b;
            }
            dst[w] = word;
        }
        if (badbits) return fail(FID_EINVAL, "row %lld: profile bytes must be 0 or 1", (long long)i);
    }
    return FID_OK;
}

int fid_pack_genotypes(fid_ctx* ctx, const uint8_t* geno_dev, int64_t n_rows, int32_t n_loci, int64_t ld_bytes,
                       uint64_t* rows_dev)
{
    if (!ctx) return fail(FID_EINVAL, "ctx is NULL");
    if (n_loci < 1 || 2 * (int64_t)n_loci > kMaxLoci)
        return fail(FID_EINVAL, "n_loci=%d out of [1, %d]", n_loci, kMaxLoci / 2);
    const int64_t rw = row_words_of(2 * n_loci);
    if (n_rows < 0) return fail(FID_EINVAL, "n_rows < 0");
    if (n_rows == 0) return FID_OK;
    if (!geno_dev || !rows_dev) return fail(FID_EINVAL, "NULL buffer");
    if (ld_bytes < n_loci) return fail(FID_EINVAL, "ld_bytes < n_loci");
    if (!aligned16(rows_dev)) return fail(FID_EINVAL, "rows_dev not 16-byte aligned");
    FID_TRY(set_device(ctx));
    int* bad = status_words(ctx);
    FID_HIP(launch_fill_u64(reinterpret_cast<uint64_t*>(bad), 1, 0ull, ctx->stream), "fill launch");
    FID_HIP(launch_pack_genotypes(geno_dev, n_rows, n_loci, ld_bytes, (int32_t)rw, rows_dev, bad, ctx->stream),
            "genotype pack launch");
    int bad_host = 0;
    FID_HIP(hipMemcpyAsync(&bad_host, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream), "hipMemcpyAsync");
    FID_HIP(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    if (bad_host) return fail(FID_EINVAL, "genotypes must be 0, 1 or 2");
    return FID_OK;
}

int fid_db_bytes(int64_t n_refs, int32_t n_loci, size_t* bytes)
{
    if (!bytes) return fail(FID_EINVAL, "bytes is NULL");
    const int64_t rw = row_words_of(n_loci);
    if (rw < 0) return fail(FID_EINVAL, "n_loci=%d out of [1, %d]", n_loci, kMaxLoci);
    if (n_refs < 1 || n_refs > kMaxRefs) return fail(FID_EINVAL, "n_refs=%lld out of range", (long long)n_refs);
    *bytes = db_words_bytes(padded_blocks(n_refs), rw) + align256((size_t)padded_blocks(n_refs) * 64 * 4);
    return FID_OK;
}

int fid_db_build(fid_ctx* ctx, const uint64_t* rows_dev, int64_t n_refs, int32_t n_loci,
                 void* db_mem_dev, size_t db_bytes, fid_db** out)
{
    if (!out) return fail(FID_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctx) return fail(FID_EINVAL, "ctx is NULL");
    size_t need = 0;
    FID_TRY(fid_db_bytes(n_refs, n_loci, &need));
    if (!rows_dev || !db_mem_dev) return fail(FID_EINVAL, "NULL buffer");
    if (!aligned16(rows_dev) || !aligned16(db_mem_dev)) return fail(FID_EINVAL, "buffers must be 16-byte aligned");
    if (db_bytes < need) return fail(FID_EINVAL, "db_bytes=%zu < required %zu", db_bytes, need);
    FID_TRY(set_device(ctx));
    const int32_t rw = (int32_t)row_words_of(n_loci);
    fid_db* db = new fid_db{};
    db->device = ctx->device;
    db->row_words = rw;
    db->mem = db_mem_dev;
    db->bytes = db_bytes;
    db->v.n_refs = n_refs;
    db->v.nblk = padded_blocks(n_refs);
    db->v.n_loci = n_loci;
    db->v.w4 = rw / 2;
    db->v.words = static_cast<const uint4*>(db_mem_dev);
    db->v.pc = reinterpret_cast<const int32_t*>(static_cast<char*>(db_mem_dev) +
                                                db_words_bytes(db->v.nblk, rw));
    hipError_t e = launch_db_build(rows_dev, n_refs, rw, n_loci, const_cast<uint4*>(db->v.words),
                                   const_cast<int32_t*>(db->v.pc), db->v.w4, db->v.nblk, ctx->stream);
    if (e != hipSuccess) {
        delete db;
        return hip_fail(e, "db_build launch");
    }
    *out = db;
    return FID_OK;
}

int fid_db_destroy(fid_db* db)
{
    delete db;
    return FID_OK;
}

int fid_db_info(const fid_db* db, int64_t* n_refs, int32_t* n_loci)
{
    if (!db) return fail(FID_EINVAL, "db is NULL");
    if (n_refs) *n_refs = db->v.n_refs;
    if (n_loci) *n_loci = db->v.n_loci;
    return FID_OK;
}

int fid_db_popcounts(const fid_db* db, const int32_t** pc_dev)
{
    if (!db || !pc_dev) return fail(FID_EINVAL, "NULL argument");
    *pc_dev = db->v.pc;
    return FID_OK;
}

int fid_compare_full(fid_ctx* ctx, const fid_db* db, const uint64_t* q_dev, int32_t n_q, int mode,
                     int32_t* counts_dev, int64_t ld)
{
    FID_TRY(check_common(ctx, db, q_dev, n_q, mode));
    if (!counts_dev) return fail(FID_EINVAL, "counts pointer is NULL");
    if (ld < db->v.n_refs) return fail(FID_EINVAL, "ld=%lld < n_refs=%lld", (long long)ld, (long long)db->v.n_refs);
    if ((reinterpret_cast<uintptr_t>(counts_dev) & 3u) != 0) return fail(FID_EINVAL, "counts pointer not 4-byte aligned");
    FID_TRY(set_device(ctx));
    const Job j = make_job(ctx, db, n_q);
    Prepared q;
    FID_TRY(prepare_queries(ctx, db, j, q_dev, n_q, mode, &q));
    return run_full(ctx, db, j, q, mode, 0, db->v.n_refs, 0, n_q, counts_dev, ld, 0, 0, true);
}

int fid_compare_tiles(fid_ctx* ctx, const fid_db* db, const uint64_t* q_dev, int32_t n_q, int mode,
                      const int64_t* tiles_host, int32_t n_tiles, int32_t th, int32_t tw,
                      int32_t* out_dev)
{
    FID_TRY(check_common(ctx, db, q_dev, n_q, mode));
    if (n_tiles < 0) return fail(FID_EINVAL, "n_tiles < 0");
    if (n_tiles == 0) return FID_OK;
    if (!tiles_host || !out_dev) return fail(FID_EINVAL, "NULL buffer");
    if (th < 1 || tw < 1) return fail(FID_EINVAL, "tile shape must be positive");
    for (int32_t t = 0; t < n_tiles; ++t) {
        const int64_t q0 = tiles_host[2 * t], r0 = tiles_host[2 * t + 1];
        if (q0 < 0 || r0 < 0 || q0 + th > n_q || r0 + tw > db->v.n_refs)
            return fail(FID_EINVAL, "tile %d at (%lld, %lld) leaves the %d x %lld matrix", t,
                        (long long)q0, (long long)r0, n_q, (long long)db->v.n_refs);
    }
    FID_TRY(set_device(ctx));
    // all tiles in one launch per kTilesPerLaunch: staged queries in 64-word
    // chunks, tile origins passed as kernel arguments
    const int32_t qw = (int32_t)((((int64_t)db->v.n_loci + 31) / 32 + 63) / 64 * 64);
    FID_TRY(ensure_scratch(ctx, (size_t)n_q * qw * sizeof(uint32_t)));
    uint32_t* qs = reinterpret_cast<uint32_t*>(query_area(ctx));
    FID_HIP(launch_stage_queries(q_dev, n_q, db->row_words, db->v.n_loci, mode, nullptr, qs, qw, ctx->stream),
            "stage_queries launch");
    for (int32_t t0 = 0; t0 < n_tiles; t0 += kTilesPerLaunch) {
        TileTable tt{};
        tt.n = std::min<int32_t>(kTilesPerLaunch, n_tiles - t0);
        for (int32_t i = 0; i < tt.n; ++i) {
            tt.q0[i] = (int32_t)tiles_host[2 * (t0 + i)];
            tt.r0[i] = tiles_host[2 * (t0 + i) + 1];
            tt.out_index[i] = t0 + i;
        }
        FID_HIP(launch_tile_counts(mode, db->v, qs, qw, tt, th, tw, out_dev, ctx->stream), "tile launch");
    }
    return FID_OK;
}

int fid_topk_workspace_bytes(fid_ctx* ctx, const fid_db* db, int32_t n_q, int32_t k, size_t* bytes)
{
    if (!db) return fail(FID_EINVAL, "db is NULL");
    return fid_topk_range_workspace_bytes(ctx, db, 0, db->v.n_refs, n_q, k, bytes);
}

int fid_topk_range_workspace_bytes(fid_ctx* ctx, const fid_db* db, int64_t r_lo, int64_t r_hi,
                                   int32_t n_q, int32_t k, size_t* bytes)
{
    if (!ctx || !db || !bytes) return fail(FID_EINVAL, "NULL argument");
    if (n_q < 1 || n_q > kMaxQueries) return fail(FID_EINVAL, "n_q out of range");
    if (k < 1 || k > kMaxK) return fail(FID_EINVAL, "k=%d out of [1, %d]", k, kMaxK);
    FID_TRY(check_range(db, r_lo, r_hi));
    *bytes = topk_layout(ctx, make_job(ctx, db, n_q), r_lo, r_hi, n_q, k).total;
    return FID_OK;
}

int fid_topk_mixed_workspace_bytes(fid_ctx* ctx, const fid_db* db, int64_t r_lo, int64_t r_hi,
                                   int32_t n_q, int32_t k, size_t* bytes)
{
    if (!ctx || !db || !bytes) return fail(FID_EINVAL, "NULL argument");
    if (n_q < 1 || n_q > kMaxQueries) return fail(FID_EINVAL, "n_q out of range");
    if (k < 1 || k > kMaxK) return fail(FID_EINVAL, "k=%d out of [1, %d]", k, kMaxK);
    FID_TRY(check_range(db, r_lo, r_hi));
    *bytes = topk_layout(ctx, make_job(ctx, db, n_q, true), r_lo, r_hi, n_q, k).total;
    return FID_OK;
}

// ---------------------------------------------------------- streamed database
// The paper's host driver (Section III-C, Section IV): the reference rows stay
// in host memory and pass through the device one block at a time; the copy
// of block b + 1 (on a copy stream) overlaps the build and scan of block b
// (on the context's stream), and each block's top-k folds into a running
// top-k whose k-th count bounds the next blocks' scans.
namespace {

struct StreamLayout {
    size_t off_stage[2], off_db, off_ws, off_tcnt, off_tidx, off_run, off_bound, total;
    size_t stage_bytes, db_bytes, ws_bytes;
};

int stream_layout(const fid_ctx* ctx, int64_t n_refs, int32_t n_loci, int64_t block_refs, int32_t n_q, int32_t k,
                  StreamLayout* L)
{
    const int64_t rw = row_words_of(n_loci);
    if (rw < 0) return fail(FID_EINVAL, "n_loci=%d out of [1, %d]", n_loci, kMaxLoci);
    if (n_refs < 1 || n_refs > kMaxRefs) return fail(FID_EINVAL, "n_refs=%lld out of range", (long long)n_refs);
    if (block_refs < 1) return fail(FID_EINVAL, "block_refs=%lld < 1", (long long)block_refs);
    if (n_q < 1 || n_q > kMaxQueries) return fail(FID_EINVAL, "n_q=%d out of [1, 2^24]", n_q);
    if (k < 1 || k > kMaxK) return fail(FID_EINVAL, "k=%d out of [1, %d]", k, kMaxK);
    const int64_t blk = std::min(block_refs, n_refs);
    L->stage_bytes = align256((size_t)blk * (size_t)rw * sizeof(uint64_t));
    FID_TRY(fid_db_bytes(blk, n_loci, &L->db_bytes));
    // top-k workspace of a full block and of the last, shorter one
    L->ws_bytes = 0;
    for (const int64_t n : {blk, n_refs - (n_refs - 1) / blk * blk}) {
        fid_db v{};
        v.device = ctx->device;
        v.row_words = (int32_t)rw;
        v.v.n_refs = n;
        v.v.nblk = padded_blocks(n);
        v.v.n_loci = n_loci;
        v.v.w4 = (int32_t)(rw / 2);
        L->ws_bytes = std::max(L->ws_bytes, topk_layout(ctx, make_job(ctx, &v, n_q), 0, n, n_q, k).total);
    }
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off += align256(bytes); return o; };
    L->off_stage[0] = take(L->stage_bytes);
    L->off_stage[1] = take(L->stage_bytes);
    L->off_db = take(L->db_bytes);
    L->off_ws = take(L->ws_bytes);
    L->off_tcnt = take((size_t)n_q * k * sizeof(int32_t));
    L->off_tidx = take((size_t)n_q * k * sizeof(int64_t));
    L->off_run = take((size_t)n_q * k * sizeof(uint64_t));
    L->off_bound = take((size_t)n_q * sizeof(uint32_t));
    L->total = off;
    return FID_OK;
}

}  // namespace

int fid_stream_workspace_bytes(fid_ctx* ctx, int64_t n_refs, int32_t n_loci, int64_t block_refs, int32_t n_q,
                               int32_t k, size_t* bytes)
{
    if (!ctx || !bytes) return fail(FID_EINVAL, "NULL argument");
    StreamLayout L;
    FID_TRY(stream_layout(ctx, n_refs, n_loci, block_refs, n_q, k, &L));
    *bytes = L.total;
    return FID_OK;
}

int fid_compare_topk_streamed(fid_ctx* ctx, const uint64_t* rows_host, int64_t n_refs, int32_t n_loci,
                              int64_t block_refs, const uint64_t* q_dev, int32_t n_q, int mode, int32_t k,
                              void* ws_dev, size_t ws_bytes, int32_t* cnt_dev, int64_t* idx_dev)
{
    if (!ctx) return fail(FID_EINVAL, "ctx is NULL");
    if (!rows_host) return fail(FID_EINVAL, "rows_host is NULL");
    if (!q_dev || !aligned16(q_dev)) return fail(FID_EINVAL, "query pointer NULL or not 16-byte aligned");
    FID_TRY(check_mode(mode));
    if (!cnt_dev || !idx_dev || !ws_dev || !aligned16(ws_dev)) return fail(FID_EINVAL, "NULL or unaligned buffer");
    StreamLayout L;
    FID_TRY(stream_layout(ctx, n_refs, n_loci, block_refs, n_q, k, &L));
    if (ws_bytes < L.total) return fail(FID_ENOMEM, "workspace %zu bytes < required %zu", ws_bytes, L.total);
    FID_TRY(set_device(ctx));
    char* ws = static_cast<char*>(ws_dev);
    const int64_t rw = row_words_of(n_loci);
    const int64_t blk = std::min(block_refs, n_refs);
    const int64_t n_blocks = (n_refs + blk - 1) / blk;
    uint64_t* running = reinterpret_cast<uint64_t*>(ws + L.off_run);
    uint32_t* bound = reinterpret_cast<uint32_t*>(ws + L.off_bound);
    int32_t* tcnt = reinterpret_cast<int32_t*>(ws + L.off_tcnt);
    int64_t* tidx = reinterpret_cast<int64_t*>(ws + L.off_tidx);

    hipStream_t copy = nullptr;
    hipEvent_t copied[2] = {nullptr, nullptr}, freed[2] = {nullptr, nullptr};
    int st = FID_OK;
    auto hip = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && !st) st = hip_fail(e, what);
    };
    hip(hipStreamCreateWithFlags(&copy, hipStreamNonBlocking), "hipStreamCreate");
    for (int i = 0; i < 2 && !st; ++i) {
        hip(hipEventCreateWithFlags(&copied[i], hipEventDisableTiming), "hipEventCreate");
        hip(hipEventCreateWithFlags(&freed[i], hipEventDisableTiming), "hipEventCreate");
    }
    if (!st) hip(launch_reset_running(nullptr, n_q, k, running, bound, ctx->stream), "reset launch");
    // the copy stream starts after everything already queued on the context
    if (!st) hip(hipEventRecord(freed[1], ctx->stream), "hipEventRecord");
    if (!st) hip(hipStreamWaitEvent(copy, freed[1], 0), "hipStreamWaitEvent");
    for (int64_t b = 0; b < n_blocks && !st; ++b) {
        const int slot = (int)(b & 1);
        const int64_t r0 = b * blk;
        const int64_t n = std::min(blk, n_refs - r0);
        uint64_t* stage = reinterpret_cast<uint64_t*>(ws + L.off_stage[slot]);
        // block b's copy waits until block b - 2 has been built from this slot
        if (b >= 2) hip(hipStreamWaitEvent(copy, freed[slot], 0), "hipStreamWaitEvent");
        if (!st)
            hip(hipMemcpyAsync(stage, rows_host + r0 * rw, (size_t)n * (size_t)rw * sizeof(uint64_t),
                               hipMemcpyHostToDevice, copy), "block copy");
        if (!st) hip(hipEventRecord(copied[slot], copy), "hipEventRecord");
        if (!st) hip(hipStreamWaitEvent(ctx->stream, copied[slot], 0), "hipStreamWaitEvent");
        if (st) break;
        fid_db* db = nullptr;
        st = fid_db_build(ctx, stage, n, n_loci, ws + L.off_db, L.db_bytes, &db);
        if (st) break;
        if (!st) hip(hipEventRecord(freed[slot], ctx->stream), "hipEventRecord");  // the slot is read
        // every block after the first filters with the running k-th count
        if (!st)
            st = topk_range(ctx, db, 0, n, q_dev, n_q, mode, k, ws + L.off_ws, L.ws_bytes, tcnt, tidx, nullptr,
                            b > 0 ? bound : nullptr, b == 0);
        delete db;  // the host handle only: the launches took its view by value
        if (!st) hip(launch_fold_topk(tcnt, tidx, nullptr, n_q, k, r0, running, bound, ctx->stream), "fold launch");
    }
    if (!st) hip(launch_finalize_topk(running, nullptr, n_q, k, k, cnt_dev, idx_dev, ctx->stream), "finalize launch");
    // the host rows must stay untouched until every copy has run
    if (copy) hip(hipStreamSynchronize(copy), "hipStreamSynchronize");
    hip(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    for (int i = 0; i < 2; ++i) {
        if (copied[i]) (void)hipEventDestroy(copied[i]);
        if (freed[i]) (void)hipEventDestroy(freed[i]);
    }
    if (copy) (void)hipStreamDestroy(copy);
    return st;
}

// The full matrix of a streamed database, as the paper's driver produced it
// (Section III-C): block b's rows go host -> device on one copy stream, its
// counts device -> host on another, while the context's stream builds and
// scans block b + 1; two slots each for staged rows and counts.
namespace {

struct FullStreamLayout {
    size_t off_stage[2], off_db, off_out[2], total;
    size_t stage_bytes, db_bytes, out_bytes;
};

int full_stream_layout(int64_t n_refs, int32_t n_loci, int64_t block_refs, int32_t n_q, FullStreamLayout* L)
{
    const int64_t rw = row_words_of(n_loci);
    if (rw < 0) return fail(FID_EINVAL, "n_loci=%d out of [1, %d]", n_loci, kMaxLoci);
    if (n_refs < 1 || n_refs > kMaxRefs) return fail(FID_EINVAL, "n_refs=%lld out of range", (long long)n_refs);
    if (block_refs < 1) return fail(FID_EINVAL, "block_refs=%lld < 1", (long long)block_refs);
    if (n_q < 1 || n_q > kMaxQueries) return fail(FID_EINVAL, "n_q=%d out of [1, 2^24]", n_q);
    const int64_t blk = std::min(block_refs, n_refs);
    L->stage_bytes = align256((size_t)blk * (size_t)rw * sizeof(uint64_t));
    FID_TRY(fid_db_bytes(blk, n_loci, &L->db_bytes));
    L->out_bytes = align256((size_t)n_q * (size_t)blk * sizeof(int32_t));
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off += align256(bytes); return o; };
    L->off_stage[0] = take(L->stage_bytes);
    L->off_stage[1] = take(L->stage_bytes);
    L->off_db = take(L->db_bytes);
    L->off_out[0] = take(L->out_bytes);
    L->off_out[1] = take(L->out_bytes);
    L->total = off;
    return FID_OK;
}

}  // namespace

int fid_full_stream_workspace_bytes(fid_ctx* ctx, int64_t n_refs, int32_t n_loci, int64_t block_refs, int32_t n_q,
                                    size_t* bytes)
{
    if (!ctx || !bytes) return fail(FID_EINVAL, "NULL argument");
    FullStreamLayout L;
    FID_TRY(full_stream_layout(n_refs, n_loci, block_refs, n_q, &L));
    *bytes = L.total;
    return FID_OK;
}

int fid_compare_full_streamed(fid_ctx* ctx, const uint64_t* rows_host, int64_t n_refs, int32_t n_loci,
                              int64_t block_refs, const uint64_t* q_dev, int32_t n_q, int mode, void* ws_dev,
                              size_t ws_bytes, int32_t* counts_host, int64_t ld)
{
    if (!ctx) return fail(FID_EINVAL, "ctx is NULL");
    if (!rows_host || !counts_host) return fail(FID_EINVAL, "host pointer is NULL");
    if (!q_dev || !aligned16(q_dev)) return fail(FID_EINVAL, "query pointer NULL or not 16-byte aligned");
    FID_TRY(check_mode(mode));
    if (!ws_dev || !aligned16(ws_dev)) return fail(FID_EINVAL, "workspace NULL or not 16-byte aligned");
    if (ld < n_refs) return fail(FID_EINVAL, "ld=%lld < n_refs=%lld", (long long)ld, (long long)n_refs);
    FullStreamLayout L;
    FID_TRY(full_stream_layout(n_refs, n_loci, block_refs, n_q, &L));
    if (ws_bytes < L.total) return fail(FID_ENOMEM, "workspace %zu bytes < required %zu", ws_bytes, L.total);
    FID_TRY(set_device(ctx));
    char* ws = static_cast<char*>(ws_dev);
    const int64_t rw = row_words_of(n_loci);
    const int64_t blk = std::min(block_refs, n_refs);
    const int64_t n_blocks = (n_refs + blk - 1) / blk;

    hipStream_t h2d = nullptr, d2h = nullptr;
    hipEvent_t copied[2] = {}, built[2] = {}, counted[2] = {}, shipped[2] = {}, start = nullptr;
    int st = FID_OK;
    auto hip = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && !st) st = hip_fail(e, what);
    };
    hip(hipStreamCreateWithFlags(&h2d, hipStreamNonBlocking), "hipStreamCreate");
    hip(hipStreamCreateWithFlags(&d2h, hipStreamNonBlocking), "hipStreamCreate");
    hip(hipEventCreateWithFlags(&start, hipEventDisableTiming), "hipEventCreate");
    for (int i = 0; i < 2 && !st; ++i) {
        hip(hipEventCreateWithFlags(&copied[i], hipEventDisableTiming), "hipEventCreate");
        hip(hipEventCreateWithFlags(&built[i], hipEventDisableTiming), "hipEventCreate");
        hip(hipEventCreateWithFlags(&counted[i], hipEventDisableTiming), "hipEventCreate");
        hip(hipEventCreateWithFlags(&shipped[i], hipEventDisableTiming), "hipEventCreate");
    }
    // both copy streams start after everything already queued on the context
    if (!st) hip(hipEventRecord(start, ctx->stream), "hipEventRecord");
    if (!st) hip(hipStreamWaitEvent(h2d, start, 0), "hipStreamWaitEvent");
    if (!st) hip(hipStreamWaitEvent(d2h, start, 0), "hipStreamWaitEvent");
    for (int64_t b = 0; b < n_blocks && !st; ++b) {
        const int slot = (int)(b & 1);
        const int64_t r0 = b * blk;
        const int64_t n = std::min(blk, n_refs - r0);
        uint64_t* stage = reinterpret_cast<uint64_t*>(ws + L.off_stage[slot]);
        int32_t* out = reinterpret_cast<int32_t*>(ws + L.off_out[slot]);
        // rows in: the slot is free once block b - 2 has been built from it
        if (b >= 2) hip(hipStreamWaitEvent(h2d, built[slot], 0), "hipStreamWaitEvent");
        if (!st)
            hip(hipMemcpyAsync(stage, rows_host + r0 * rw, (size_t)n * (size_t)rw * sizeof(uint64_t),
                               hipMemcpyHostToDevice, h2d), "block copy");
        if (!st) hip(hipEventRecord(copied[slot], h2d), "hipEventRecord");
        // build and count: the count slot is free once block b - 2's counts shipped
        if (!st) hip(hipStreamWaitEvent(ctx->stream, copied[slot], 0), "hipStreamWaitEvent");
        if (!st && b >= 2) hip(hipStreamWaitEvent(ctx->stream, shipped[slot], 0), "hipStreamWaitEvent");
        if (st) break;
        fid_db* db = nullptr;
        st = fid_db_build(ctx, stage, n, n_loci, ws + L.off_db, L.db_bytes, &db);
        if (st) break;
        hip(hipEventRecord(built[slot], ctx->stream), "hipEventRecord");
        if (!st) st = fid_compare_full(ctx, db, q_dev, n_q, mode, out, n);
        delete db;  // the host handle only: the launches took its view by value
        if (!st) hip(hipEventRecord(counted[slot], ctx->stream), "hipEventRecord");
        // counts out: [n_q][n] into columns [r0, r0 + n) of the caller's rows
        if (!st) hip(hipStreamWaitEvent(d2h, counted[slot], 0), "hipStreamWaitEvent");
        if (!st)
            hip(hipMemcpy2DAsync(counts_host + r0, (size_t)ld * sizeof(int32_t), out, (size_t)n * sizeof(int32_t),
                                 (size_t)n * sizeof(int32_t), (size_t)n_q, hipMemcpyDeviceToHost, d2h),
                "counts copy");
        if (!st) hip(hipEventRecord(shipped[slot], d2h), "hipEventRecord");
    }
    // every copy has run before the host buffers are handed back
    if (h2d) hip(hipStreamSynchronize(h2d), "hipStreamSynchronize");
    if (d2h) hip(hipStreamSynchronize(d2h), "hipStreamSynchronize");
    hip(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    for (int i = 0; i < 2; ++i)
        for (hipEvent_t e : {copied[i], built[i], counted[i], shipped[i]})
            if (e) (void)hipEventDestroy(e);
    if (start) (void)hipEventDestroy(start);
    if (h2d) (void)hipStreamDestroy(h2d);
    if (d2h) (void)hipStreamDestroy(d2h);
    return st;
}

int fid_compare_topk_mixed(fid_ctx* ctx, const fid_db* db, int64_t r_lo, int64_t r_hi,
                           const uint64_t* q_dev, const int32_t* modes_dev, int32_t n_q, int32_t k,
                           void* ws_dev, size_t ws_bytes, int32_t* cnt_dev, int64_t* idx_dev)
{
    if (!db) return fail(FID_EINVAL, "db is NULL");
    FID_TRY(check_common(ctx, db, q_dev, n_q, FID_MODE_MIXTURE));
    FID_TRY(check_modes_dev(ctx, modes_dev, n_q));
    return topk_range(ctx, db, r_lo, r_hi, q_dev, n_q, kModePerQuery, k, ws_dev, ws_bytes, cnt_dev,
                      idx_dev, modes_dev);
}

int fid_compare_topk_bounded(fid_ctx* ctx, const fid_db* db, int64_t r_lo, int64_t r_hi,
                             const uint64_t* q_dev, const int32_t* modes_dev, int32_t n_q, int32_t k,
                             const uint32_t* bound_dev, int use_seed, void* ws_dev, size_t ws_bytes,
                             int32_t* cnt_dev, int64_t* idx_dev)
{
    if (!db) return fail(FID_EINVAL, "db is NULL");
    if (!bound_dev || (reinterpret_cast<uintptr_t>(bound_dev) & 3u) != 0)
        return fail(FID_EINVAL, "bound pointer NULL or not 4-byte aligned");
    FID_TRY(check_common(ctx, db, q_dev, n_q, FID_MODE_MIXTURE));
    FID_TRY(check_modes_dev(ctx, modes_dev, n_q));
    return topk_range(ctx, db, r_lo, r_hi, q_dev, n_q, kModePerQuery, k, ws_dev, ws_bytes, cnt_dev,
                      idx_dev, modes_dev, bound_dev, use_seed != 0);
}

int fid_compare_topk(fid_ctx* ctx, const fid_db* db, const uint64_t* q_dev, int32_t n_q, int mode,
                     int32_t k, void* ws_dev, size_t ws_bytes, int32_t* cnt_dev, int64_t* idx_dev)
{
    if (!db) return fail(FID_EINVAL, "db is NULL");
    return topk_range(ctx, db, 0, db->v.n_refs, q_dev, n_q, mode, k, ws_dev, ws_bytes, cnt_dev,
                      idx_dev);
}

int fid_compare_topk_noalloc(fid_ctx* ctx, const fid_db* db, const uint64_t* q_dev, int32_t n_q, int mode,
                             int32_t k, int32_t* cnt_dev, int64_t* idx_dev)
{
    FID_TRY(check_common(ctx, db, q_dev, n_q, mode));
    if (k < 1 || k > kMaxK) return fail(FID_EINVAL, "k=%d out of [1, %d]", k, kMaxK);
    if (!cnt_dev || !idx_dev) return fail(FID_EINVAL, "NULL buffer");
    if (!ctx->fixed_scratch) return fail(FID_EHIP, "fixed scratch not resolved on device %d", ctx->device);
    // the same plan, workspace layout and kernels as fid_compare_topk; the
    // staged queries and the workspace both live in the fixed array
    const Job j = make_job(ctx, db, n_q);
    const TopkLayout L = topk_layout(ctx, j, 0, db->v.n_refs, n_q, k);
    const size_t qbytes = align256(query_scratch_bytes(ctx, db, n_q));
    if (qbytes + L.total > kFixedScratchBytes)
        return fail(FID_ENOMEM,
                    "fid_compare_topk_noalloc: %d queries x %lld references at k=%d need %zu bytes of scratch; "
                    "the fixed scratch holds %zu (use fid_compare_topk with a workspace)",
                    n_q, (long long)db->v.n_refs, k, qbytes + L.total, kFixedScratchBytes);
    char* base = static_cast<char*>(ctx->fixed_scratch);
    return topk_range(ctx, db, 0, db->v.n_refs, q_dev, n_q, mode, k, base + qbytes, L.total, cnt_dev, idx_dev,
                      nullptr, nullptr, true, base, false);
}

int fid_compare_topk_range(fid_ctx* ctx, const fid_db* db, int64_t r_lo, int64_t r_hi,
                           const uint64_t* q_dev, int32_t n_q, int mode, int32_t k, void* ws_dev,
                           size_t ws_bytes, int32_t* cnt_dev, int64_t* idx_dev)
{
    if (!db) return fail(FID_EINVAL, "db is NULL");
    return topk_range(ctx, db, r_lo, r_hi, q_dev, n_q, mode, k, ws_dev, ws_bytes, cnt_dev, idx_dev);
}

int fid_threshold_workspace_bytes(const fid_db* db, int32_t n_q, int64_t cap, size_t* bytes)
{
    if (!db || !bytes) return fail(FID_EINVAL, "NULL argument");
    if (n_q < 1 || n_q > kMaxQueries) return fail(FID_EINVAL, "n_q out of range");
    if (cap < 0) return fail(FID_EINVAL, "cap < 0");
    const size_t c = (size_t)(cap > 0 ? cap : 1);
    *bytes = 256 + 2 * align256(c * sizeof(uint64_t)) + 2 * align256(c * sizeof(int32_t));
    return FID_OK;
}

int fid_compare_threshold(fid_ctx* ctx, const fid_db* db, const uint64_t* q_dev, int32_t n_q, int mode,
                          const int32_t* thr_dev, void* ws_dev, size_t ws_bytes, int64_t cap,
                          int64_t* offs_dev, int64_t* idx_dev, int32_t* cnt_dev, int64_t* total_host)
{
    FID_TRY(check_common(ctx, db, q_dev, n_q, mode));
    if (!thr_dev || !ws_dev || !offs_dev || !total_host) return fail(FID_EINVAL, "NULL buffer");
    if (cap > 0 && (!idx_dev || !cnt_dev)) return fail(FID_EINVAL, "NULL output buffer");
    if (!aligned16(ws_dev)) return fail(FID_EINVAL, "workspace not 16-byte aligned");
    size_t need = 0;
    FID_TRY(fid_threshold_workspace_bytes(db, n_q, cap, &need));
    if (ws_bytes < need) return fail(FID_ENOMEM, "workspace %zu bytes < required %zu", ws_bytes, need);
    FID_TRY(set_device(ctx));
    const Job j = make_job(ctx, db, n_q);
    Prepared q;
    FID_TRY(prepare_queries(ctx, db, j, q_dev, n_q, mode, &q));
    const size_t c = (size_t)(cap > 0 ? cap : 1);
    char* ws = static_cast<char*>(ws_dev);
    unsigned long long* counter = reinterpret_cast<unsigned long long*>(ws);
    uint64_t* keys = reinterpret_cast<uint64_t*>(ws + 256);
    uint64_t* keys2 = reinterpret_cast<uint64_t*>(ws + 256 + align256(c * 8));
    int32_t* vals = reinterpret_cast<int32_t*>(ws + 256 + 2 * align256(c * 8));
    int32_t* vals2 = reinterpret_cast<int32_t*>(ws + 256 + 2 * align256(c * 8) + align256(c * 4));
    FID_HIP(launch_fill_u64(reinterpret_cast<uint64_t*>(counter), 1, 0ull, ctx->stream), "fill launch");
    const Plan pl = plan_for(ctx, j, 0, db->v.n_refs, n_q, EPI_THRESH);
    ScanParams p = make_params(db, j, pl, 0, db->v.n_refs, 0, n_q);
    p.hit_cap = cap;
    Outputs o;
    o.thr = thr_dev;
    o.hit_count = counter;
    o.hit_keys = keys;
    o.hit_cnt = vals;
    FID_TRY(run_scan(ctx, j, mode, EPI_THRESH, p, q, o, true));
    unsigned long long total = 0;
    FID_HIP(hipMemcpyAsync(&total, counter, sizeof total, hipMemcpyDeviceToHost, ctx->stream), "hipMemcpyAsync");
    FID_HIP(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    *total_host = (int64_t)total;
    if ((int64_t)total > cap)
        return fail(FID_EOVERFLOW, "%llu threshold hits exceed capacity %lld", total, (long long)cap);
    uint64_t* sk;
    int32_t* sv;
    FID_HIP(launch_sort_hits(keys, vals, keys2, vals2, (int64_t)total, &sk, &sv, ctx->stream), "sort launch");
    FID_HIP(launch_hits_to_csr(sk, sv, (int64_t)total, n_q, offs_dev, idx_dev, cnt_dev, ctx->stream), "csr launch");
    return FID_OK;
}

// Threshold hits and top-k of the same queries in one pass over the
// database (Section IV: both reductions on the GPU).  On the fp4 family one
// scan carries both epilogues -- a reference is looked at when its count is
// below the larger of the threshold + 1 and the top-k bound, then appended
// as a hit and/or inserted into the lists -- so the database is read once
// for both outputs.  Other families, and ranges short enough for the direct
// top-k, run the two calls back to back (identical results).
// Workspace: [top-k workspace | hit counter | keys x 2 | counts x 2].
namespace {

size_t hits_bytes(int64_t cap)
{
    const size_t c = (size_t)(cap > 0 ? cap : 1);
    return 256 + 2 * align256(c * sizeof(uint64_t)) + 2 * align256(c * sizeof(int32_t));
}

}  // namespace

int fid_threshold_topk_workspace_bytes(fid_ctx* ctx, const fid_db* db, int32_t n_q, int32_t k, int64_t cap,
                                       size_t* bytes)
{
    if (!ctx || !db || !bytes) return fail(FID_EINVAL, "NULL argument");
    if (n_q < 1 || n_q > kMaxQueries) return fail(FID_EINVAL, "n_q out of range");
    if (k < 1 || k > kMaxK) return fail(FID_EINVAL, "k=%d out of [1, %d]", k, kMaxK);
    if (cap < 0) return fail(FID_EINVAL, "cap < 0");
    *bytes = align256(topk_layout(ctx, make_job(ctx, db, n_q), 0, db->v.n_refs, n_q, k).total) + hits_bytes(cap);
    return FID_OK;
}

int fid_compare_threshold_topk(fid_ctx* ctx, const fid_db* db, const uint64_t* q_dev, int32_t n_q, int mode,
                               const int32_t* thr_dev, int32_t k, void* ws_dev, size_t ws_bytes, int64_t cap,
                               int64_t* offs_dev, int64_t* hidx_dev, int32_t* hcnt_dev, int64_t* total_host,
                               int32_t* cnt_dev, int64_t* idx_dev)
{
    FID_TRY(check_common(ctx, db, q_dev, n_q, mode));
    if (k < 1 || k > kMaxK) return fail(FID_EINVAL, "k=%d out of [1, %d]", k, kMaxK);
    if (!thr_dev || !ws_dev || !offs_dev || !total_host || !cnt_dev || !idx_dev)
        return fail(FID_EINVAL, "NULL buffer");
    if (cap > 0 && (!hidx_dev || !hcnt_dev)) return fail(FID_EINVAL, "NULL hit output buffer");
    if (cap < 0) return fail(FID_EINVAL, "cap < 0");
    if (!aligned16(ws_dev)) return fail(FID_EINVAL, "workspace not 16-byte aligned");
    const Job j = make_job(ctx, db, n_q);
    const TopkLayout L = topk_layout(ctx, j, 0, db->v.n_refs, n_q, k);
    const size_t tk_bytes = align256(L.total);
    if (ws_bytes < tk_bytes + hits_bytes(cap))
        return fail(FID_ENOMEM, "workspace %zu bytes < required %zu", ws_bytes, tk_bytes + hits_bytes(cap));
    char* ws = static_cast<char*>(ws_dev);
    char* hw = ws + tk_bytes;
    if (j.backend != FID_BACKEND_MFMA_FP4 || L.direct) {
        // two scans; the top-k first, so that its output is complete whatever
        // the threshold call returns
        FID_TRY(topk_range(ctx, db, 0, db->v.n_refs, q_dev, n_q, mode, k, ws, L.total, cnt_dev, idx_dev));
        return fid_compare_threshold(ctx, db, q_dev, n_q, mode, thr_dev, hw, hits_bytes(cap), cap, offs_dev,
                                     hidx_dev, hcnt_dev, total_host);
    }
    FID_TRY(set_device(ctx));
    Prepared q;
    FID_TRY(prepare_queries(ctx, db, j, q_dev, n_q, mode, &q));
    int32_t* counts = reinterpret_cast<int32_t*>(ws + L.off_counts);
    uint64_t* lists = reinterpret_cast<uint64_t*>(ws + L.off_lists);
    uint32_t* fills = reinterpret_cast<uint32_t*>(ws + L.off_fills);
    uint32_t* thr_init = reinterpret_cast<uint32_t*>(ws + L.off_thr);
    uint32_t* level = reinterpret_cast<uint32_t*>(ws + L.off_level);
    uint32_t* wit = reinterpret_cast<uint32_t*>(ws + L.off_wit);
    const size_t c = (size_t)(cap > 0 ? cap : 1);
    unsigned long long* counter = reinterpret_cast<unsigned long long*>(hw);
    uint64_t* keys = reinterpret_cast<uint64_t*>(hw + 256);
    uint64_t* keys2 = reinterpret_cast<uint64_t*>(hw + 256 + align256(c * 8));
    int32_t* vals = reinterpret_cast<int32_t*>(hw + 256 + 2 * align256(c * 8));
    int32_t* vals2 = reinterpret_cast<int32_t*>(hw + 256 + 2 * align256(c * 8) + align256(c * 4));
    // top-k seed: exact counts of the first references give each query's
    // starting bound and witness levels
    FID_TRY(run_full(ctx, db, j, q, mode, 0, L.seed, 0, n_q, counts, L.seed, 0, 0, false));
    FID_HIP(launch_seed_select(counts, n_q, L.seed, k, db->v.n_loci, thr_init, level, wit, ctx->stream),
            "seed select launch");
    FID_HIP(launch_fill_u64(reinterpret_cast<uint64_t*>(counter), 1, 0ull, ctx->stream), "fill launch");
    ScanParams p = make_params(db, j, L.plan, 0, db->v.n_refs, 0, n_q);
    p.k = k;
    p.hit_cap = cap;
    Outputs o;
    o.lists = lists;
    o.fills = fills;
    o.thr_init = thr_init;
    o.level = level;
    o.wit = wit;
    o.thr = thr_dev;
    o.hit_count = counter;
    o.hit_keys = keys;
    o.hit_cnt = vals;
    FID_TRY(run_scan(ctx, j, mode, EPI_BOTH, p, q, o, true));
    FID_HIP(launch_merge_lists(lists, fills, n_q, L.plan.list_workers, k, db->v.n_loci, cnt_dev, idx_dev,
                               ctx->stream),
            "merge launch");
    unsigned long long total = 0;
    FID_HIP(hipMemcpyAsync(&total, counter, sizeof total, hipMemcpyDeviceToHost, ctx->stream), "hipMemcpyAsync");
    FID_HIP(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    *total_host = (int64_t)total;
    if ((int64_t)total > cap)
        return fail(FID_EOVERFLOW, "%llu threshold hits exceed capacity %lld", total, (long long)cap);
    uint64_t* sk;
    int32_t* sv;
    FID_HIP(launch_sort_hits(keys, vals, keys2, vals2, (int64_t)total, &sk, &sv, ctx->stream), "sort launch");
    FID_HIP(launch_hits_to_csr(sk, sv, (int64_t)total, n_q, offs_dev, hidx_dev, hcnt_dev, ctx->stream),
            "csr launch");
    return FID_OK;
}

// Threshold hits of a streamed database (the paper's host driver, Section
// III-C, with the Section IV reduction on the device): every block of rows
// is copied in (on a stream of the call's own, overlapping the previous
// block's scan), built and scanned with the threshold epilogue into one
// shared append buffer; the block's hits are shifted to database rows; one
// sort and CSR pass at the end.
int fid_threshold_stream_workspace_bytes(fid_ctx* ctx, int64_t n_refs, int32_t n_loci, int64_t block_refs,
                                         int32_t n_q, int64_t cap, size_t* bytes)
{
    if (!ctx || !bytes) return fail(FID_EINVAL, "NULL argument");
    const int64_t rw = row_words_of(n_loci);
    if (rw < 0) return fail(FID_EINVAL, "n_loci=%d out of [1, %d]", n_loci, kMaxLoci);
    if (n_refs < 1 || n_refs > kMaxRefs) return fail(FID_EINVAL, "n_refs=%lld out of range", (long long)n_refs);
    if (block_refs < 1) return fail(FID_EINVAL, "block_refs=%lld < 1", (long long)block_refs);
    if (n_q < 1 || n_q > kMaxQueries) return fail(FID_EINVAL, "n_q=%d out of [1, 2^24]", n_q);
    if (cap < 0) return fail(FID_EINVAL, "cap < 0");
    const int64_t blk = std::min(block_refs, n_refs);
    size_t db_bytes = 0;
    FID_TRY(fid_db_bytes(blk, n_loci, &db_bytes));
    const size_t c = (size_t)(cap > 0 ? cap : 1);
    const int64_t n_blocks = (n_refs + blk - 1) / blk;
    *bytes = 2 * align256((size_t)blk * (size_t)rw * sizeof(uint64_t)) + align256(db_bytes) + 256 +
             2 * align256(c * sizeof(uint64_t)) + 2 * align256(c * sizeof(int32_t)) +
             align256((size_t)(n_blocks + 1) * sizeof(int64_t));
    return FID_OK;
}

int fid_compare_threshold_streamed(fid_ctx* ctx, const uint64_t* rows_host, int64_t n_refs, int32_t n_loci,
                                   int64_t block_refs, const uint64_t* q_dev, int32_t n_q, int mode,
                                   const int32_t* thr_dev, void* ws_dev, size_t ws_bytes, int64_t cap,
                                   int64_t* offs_dev, int64_t* idx_dev, int32_t* cnt_dev, int64_t* total_host)
{
    if (!ctx) return fail(FID_EINVAL, "ctx is NULL");
    if (!rows_host || !total_host) return fail(FID_EINVAL, "host pointer is NULL");
    if (!q_dev || !aligned16(q_dev)) return fail(FID_EINVAL, "query pointer NULL or not 16-byte aligned");
    FID_TRY(check_mode(mode));
    if (!thr_dev || !offs_dev || !ws_dev || !aligned16(ws_dev)) return fail(FID_EINVAL, "NULL or unaligned buffer");
    if (cap > 0 && (!idx_dev || !cnt_dev)) return fail(FID_EINVAL, "NULL output buffer");
    size_t need = 0;
    FID_TRY(fid_threshold_stream_workspace_bytes(ctx, n_refs, n_loci, block_refs, n_q, cap, &need));
    if (ws_bytes < need) return fail(FID_ENOMEM, "workspace %zu bytes < required %zu", ws_bytes, need);
    FID_TRY(set_device(ctx));
    const int64_t rw = row_words_of(n_loci);
    const int64_t blk = std::min(block_refs, n_refs);
    const int64_t n_blocks = (n_refs + blk - 1) / blk;
    size_t db_bytes = 0;
    FID_TRY(fid_db_bytes(blk, n_loci, &db_bytes));
    const size_t c = (size_t)(cap > 0 ? cap : 1);
    char* ws = static_cast<char*>(ws_dev);
    size_t off = 0;
    auto take = [&](size_t bytes) { char* p = ws + off; off += align256(bytes); return p; };
    uint64_t* stage[2];
    stage[0] = reinterpret_cast<uint64_t*>(take((size_t)blk * (size_t)rw * sizeof(uint64_t)));
    stage[1] = reinterpret_cast<uint64_t*>(take((size_t)blk * (size_t)rw * sizeof(uint64_t)));
    void* dbmem = take(db_bytes);
    unsigned long long* counter = reinterpret_cast<unsigned long long*>(take(256));
    uint64_t* keys = reinterpret_cast<uint64_t*>(take(c * sizeof(uint64_t)));
    uint64_t* keys2 = reinterpret_cast<uint64_t*>(take(c * sizeof(uint64_t)));
    int32_t* vals = reinterpret_cast<int32_t*>(take(c * sizeof(int32_t)));
    int32_t* vals2 = reinterpret_cast<int32_t*>(take(c * sizeof(int32_t)));
    int64_t* ends = reinterpret_cast<int64_t*>(take((size_t)(n_blocks + 1) * sizeof(int64_t)));

    hipStream_t copy = nullptr;
    hipEvent_t copied[2] = {}, freed[2] = {};
    int st = FID_OK;
    auto hip = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && !st) st = hip_fail(e, what);
    };
    hip(hipStreamCreateWithFlags(&copy, hipStreamNonBlocking), "hipStreamCreate");
    for (int i = 0; i < 2 && !st; ++i) {
        hip(hipEventCreateWithFlags(&copied[i], hipEventDisableTiming), "hipEventCreate");
        hip(hipEventCreateWithFlags(&freed[i], hipEventDisableTiming), "hipEventCreate");
    }
    if (!st) hip(launch_fill_u64(reinterpret_cast<uint64_t*>(counter), 1, 0ull, ctx->stream), "fill launch");
    if (!st) hip(launch_fill_u64(reinterpret_cast<uint64_t*>(ends), 1, 0ull, ctx->stream), "fill launch");
    if (!st) hip(hipEventRecord(freed[1], ctx->stream), "hipEventRecord");
    if (!st) hip(hipStreamWaitEvent(copy, freed[1], 0), "hipStreamWaitEvent");
    Prepared q;
    Job j{};
    for (int64_t b = 0; b < n_blocks && !st; ++b) {
        const int slot = (int)(b & 1);
        const int64_t r0 = b * blk;
        const int64_t n = std::min(blk, n_refs - r0);
        if (b >= 2) hip(hipStreamWaitEvent(copy, freed[slot], 0), "hipStreamWaitEvent");
        if (!st)
            hip(hipMemcpyAsync(stage[slot], rows_host + r0 * rw, (size_t)n * (size_t)rw * sizeof(uint64_t),
                               hipMemcpyHostToDevice, copy), "block copy");
        if (!st) hip(hipEventRecord(copied[slot], copy), "hipEventRecord");
        if (!st) hip(hipStreamWaitEvent(ctx->stream, copied[slot], 0), "hipStreamWaitEvent");
        if (st) break;
        fid_db* db = nullptr;
        st = fid_db_build(ctx, stage[slot], n, n_loci, dbmem, db_bytes, &db);
        if (st) break;
        hip(hipEventRecord(freed[slot], ctx->stream), "hipEventRecord");
        if (!st && b == 0) {
            // every block has the same row length: one query preparation
            j = make_job(ctx, db, n_q);
            st = prepare_queries(ctx, db, j, q_dev, n_q, mode, &q);
        }
        if (!st) {
            const Plan pl = plan_for(ctx, j, 0, n, n_q, EPI_THRESH);
            ScanParams p = make_params(db, j, pl, 0, n, 0, n_q);
            p.hit_cap = cap;
            Outputs o;
            o.thr = thr_dev;
            o.hit_count = counter;
            o.hit_keys = keys;
            o.hit_cnt = vals;
            st = run_scan(ctx, j, mode, EPI_THRESH, p, q, o, true);
        }
        delete db;  // the host handle only: the launches took its view by value
        if (!st)
            hip(launch_offset_block_hits(counter, ends, (int32_t)b, keys, cap, r0, ctx->stream), "offset launch");
    }
    unsigned long long total = 0;
    if (!st) hip(hipMemcpyAsync(&total, counter, sizeof total, hipMemcpyDeviceToHost, ctx->stream), "hipMemcpyAsync");
    if (copy) hip(hipStreamSynchronize(copy), "hipStreamSynchronize");
    hip(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    if (!st) {
        *total_host = (int64_t)total;
        if ((int64_t)total > cap) {
            st = fail(FID_EOVERFLOW, "%llu threshold hits exceed capacity %lld", total, (long long)cap);
        } else {
            uint64_t* sk;
            int32_t* sv;
            hip(launch_sort_hits(keys, vals, keys2, vals2, (int64_t)total, &sk, &sv, ctx->stream), "sort launch");
            if (!st)
                hip(launch_hits_to_csr(sk, sv, (int64_t)total, n_q, offs_dev, idx_dev, cnt_dev, ctx->stream),
                    "csr launch");
        }
    }
    for (int i = 0; i < 2; ++i) {
        if (copied[i]) (void)hipEventDestroy(copied[i]);
        if (freed[i]) (void)hipEventDestroy(freed[i]);
    }
    if (copy) (void)hipStreamDestroy(copy);
    return st;
}

}  // extern "C"
