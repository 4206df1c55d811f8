// libfastid C ABI: argument validation, launch planning and the host side of
// every entry point declared in include/fastid.h.
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <algorithm>
#include <utility>
#include <vector>

#include "fid_common.hpp"

using namespace fid;

struct fid_ctx {
    int device;
    hipStream_t stream;
    int num_cus;
    void* scratch;       // staged queries, status words
    size_t scratch_bytes;
    bool timing;         // record events around each call's main scan kernel
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    size_t events_used;
};

struct fid_db {
    int device;
    DbView v;
    int32_t row_words;
    void* mem;
    size_t bytes;
};

namespace {

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

#define FID_HIP(call, what)                         \
    do {                                            \
        hipError_t e_ = (call);                     \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

constexpr int64_t kMaxRefs = (1ll << kIdxBits) - 1;
constexpr int32_t kMaxQueries = 1 << 24;
constexpr size_t kStatusBytes = 256;

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t row_words_of(int32_t n_loci)
{
    if (n_loci < 1 || n_loci > kMaxLoci) return -1;
    return 2 * (((int64_t)n_loci + 127) / 128);
}

int set_device(const fid_ctx* ctx)
{
    FID_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    return FID_OK;
}

// Library scratch: [status words | staged queries].  Grown on demand.
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

uint32_t* staged_queries(fid_ctx* ctx)
{
    return reinterpret_cast<uint32_t*>(static_cast<char*>(ctx->scratch) + kStatusBytes);
}

// Register-resident chunk width (32-bit words per lane) for a row of w32 words.
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

// Waves per CU the scan aims for; overridable for tuning sweeps.
int waves_per_cu()
{
    const char* e = getenv("FASTID_WAVES_PER_CU");
    const int v = e ? atoi(e) : 0;
    return v > 0 && v <= 64 ? v : 24;
}

// References each lane holds (two halves the per-query overhead per VALU op
// but doubles the row registers); overridable for tuning sweeps.
int refs_per_lane(int nw, bool chunked)
{
    if (chunked || nw > 64) return 1;
    const char* e = getenv("FASTID_RPL");
    return (e && atoi(e) == 2) ? 2 : 1;
}

struct Plan {
    int32_t n_rsplit;
    int32_t q_per_worker;
    int32_t n_workers;
    int32_t lds_words_per_wave;
};

constexpr int32_t kTopkQueriesPerWave = 1024;  // LDS: 8 bytes per query per wave

Plan plan_scan(int num_cus, int64_t nblk, int32_t nq, const Shape& sh, int epi)
{
    const int64_t target = (int64_t)num_cus * waves_per_cu();
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
    if (rsplit * qsplit > (int64_t)(1 << 30)) return p;  // n_workers == 0: caller rejects
    p.n_rsplit = (int32_t)rsplit;
    p.q_per_worker = (int32_t)((nq + qsplit - 1) / qsplit);
    p.n_workers = (int32_t)(rsplit * ((nq + p.q_per_worker - 1) / p.q_per_worker));
    int32_t words = 0;
    if (epi == EPI_TOPK) words += 2 * p.q_per_worker;
    if (sh.chunked) words += p.q_per_worker * 64;
    p.lds_words_per_wave = words;
    return p;
}

ScanParams base_params(const fid_db* db, const Shape& sh, const Plan& pl, int64_t r_lo,
                       int64_t r_hi, int32_t q_lo, int32_t q_hi)
{
    ScanParams p{};
    p.db = db->v;
    p.qw = sh.qw;
    p.nchunks = sh.nchunks;
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

int stage(fid_ctx* ctx, const fid_db* db, const uint64_t* q_dev, int32_t n_q, int mode,
          const Shape& sh)
{
    int st = ensure_scratch(ctx, (size_t)n_q * sh.qw * sizeof(uint32_t));
    if (st) return st;
    FID_HIP(launch_stage_queries(q_dev, n_q, db->row_words, db->v.n_loci, mode,
                                 staged_queries(ctx), sh.qw, ctx->stream),
            "stage_queries launch");
    return FID_OK;
}

// The dominant kernel of a call; bracketed by events when timing is on.
int main_scan(fid_ctx* ctx, int mode, int nw, int epi, bool chunked, const ScanParams& p,
              const ScanBuffers& b)
{
    if (p.n_workers <= 0) return fail(FID_EINVAL, "problem too large for one launch");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->timing) {
        if (ctx->events_used == ctx->events.size()) {
            std::pair<hipEvent_t, hipEvent_t> ev;
            FID_HIP(hipEventCreate(&ev.first), "hipEventCreate");
            FID_HIP(hipEventCreate(&ev.second), "hipEventCreate");
            ctx->events.push_back(ev);
        }
        e0 = ctx->events[ctx->events_used].first;
        e1 = ctx->events[ctx->events_used].second;
        ++ctx->events_used;
        FID_HIP(hipEventRecord(e0, ctx->stream), "hipEventRecord");
    }
    FID_HIP(launch_scan(mode, nw, epi, chunked, refs_per_lane(nw, chunked), p, b, ctx->stream),
            "scan launch");
    if (e1) FID_HIP(hipEventRecord(e1, ctx->stream), "hipEventRecord");
    return FID_OK;
}

// Reference-prefix size whose exact k-th count seeds the top-k filter.
int64_t seed_refs(int64_t n_refs)
{
    int64_t s = ((n_refs / 64) + 63) / 64 * 64;
    if (s < 16384) s = 16384;
    if (s > 262144) s = 262144;
    return s < n_refs ? s : n_refs;
}

struct TopkLayout {
    bool direct;          // whole count matrix fits: count then select
    Plan plan;
    int64_t seed;         // reference prefix of the seed pass
    size_t off_lists, off_fills, off_counts, off_thr, total;
};

TopkLayout topk_layout(const fid_ctx* ctx, const fid_db* db, int32_t n_q, int32_t k)
{
    TopkLayout L{};
    const Shape sh = shape_for(db);
    L.seed = seed_refs(db->v.n_refs);
    L.direct = L.seed == db->v.n_refs;
    size_t off = 0;
    if (L.direct) {
        L.off_counts = off;
        off += align256((size_t)n_q * (size_t)db->v.n_refs * sizeof(int32_t));
    } else {
        L.plan = plan_scan(ctx->num_cus, db->v.nblk, n_q, sh, EPI_TOPK);
        L.off_lists = off;
        off += align256((size_t)n_q * L.plan.n_rsplit * (size_t)k * sizeof(uint64_t));
        L.off_fills = off;
        off += align256((size_t)n_q * L.plan.n_rsplit * sizeof(uint32_t));
        L.off_counts = off;
        off += align256((size_t)n_q * (size_t)L.seed * sizeof(int32_t));
        L.off_thr = off;
        off += align256((size_t)n_q * sizeof(uint32_t));
    }
    L.total = off;
    return L;
}

}  // namespace

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
    c->scratch = nullptr;
    c->scratch_bytes = 0;
    c->timing = false;
    c->events_used = 0;
    const int st = ensure_scratch(c, 0);
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

int fid_ctx_set_stream(fid_ctx* ctx, void* stream)
{
    if (!ctx) return fail(FID_EINVAL, "ctx is NULL");
    ctx->stream = static_cast<hipStream_t>(stream);
    return FID_OK;
}

int fid_sync(fid_ctx* ctx)
{
    if (!ctx) return fail(FID_EINVAL, "ctx is NULL");
    int st = set_device(ctx);
    if (st) return st;
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
    int st = set_device(ctx);
    if (st) return st;
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
    int st = set_device(ctx);
    if (st) return st;
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

int fid_db_bytes(int64_t n_refs, int32_t n_loci, size_t* bytes)
{
    if (!bytes) return fail(FID_EINVAL, "bytes is NULL");
    const int64_t rw = row_words_of(n_loci);
    if (rw < 0) return fail(FID_EINVAL, "n_loci=%d out of [1, %d]", n_loci, kMaxLoci);
    if (n_refs < 1 || n_refs > kMaxRefs) return fail(FID_EINVAL, "n_refs=%lld out of range", (long long)n_refs);
    const int64_t nblk = (n_refs + 63) / 64;
    *bytes = align256((size_t)nblk * 64 * (size_t)rw * 8) + align256((size_t)nblk * 64 * 4);
    return FID_OK;
}

int fid_db_build(fid_ctx* ctx, const uint64_t* rows_dev, int64_t n_refs, int32_t n_loci,
                 void* db_mem_dev, size_t db_bytes, fid_db** out)
{
    if (!out) return fail(FID_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctx) return fail(FID_EINVAL, "ctx is NULL");
    size_t need = 0;
    int st = fid_db_bytes(n_refs, n_loci, &need);
    if (st) return st;
    if (!rows_dev || !db_mem_dev) return fail(FID_EINVAL, "NULL buffer");
    if (!aligned16(rows_dev) || !aligned16(db_mem_dev)) return fail(FID_EINVAL, "buffers must be 16-byte aligned");
    if (db_bytes < need) return fail(FID_EINVAL, "db_bytes=%zu < required %zu", db_bytes, need);
    st = set_device(ctx);
    if (st) return st;
    const int32_t rw = (int32_t)row_words_of(n_loci);
    fid_db* db = new fid_db{};
    db->device = ctx->device;
    db->row_words = rw;
    db->mem = db_mem_dev;
    db->bytes = db_bytes;
    db->v.n_refs = n_refs;
    db->v.nblk = (n_refs + 63) / 64;
    db->v.n_loci = n_loci;
    db->v.w4 = rw / 2;
    db->v.words = static_cast<const uint4*>(db_mem_dev);
    db->v.pc = reinterpret_cast<const int32_t*>(
        static_cast<char*>(db_mem_dev) + align256((size_t)db->v.nblk * 64 * (size_t)rw * 8));
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
    int st = check_common(ctx, db, q_dev, n_q, mode);
    if (st) return st;
    if (!counts_dev) return fail(FID_EINVAL, "counts pointer is NULL");
    if (ld < db->v.n_refs) return fail(FID_EINVAL, "ld=%lld < n_refs=%lld", (long long)ld, (long long)db->v.n_refs);
    if ((reinterpret_cast<uintptr_t>(counts_dev) & 3u) != 0) return fail(FID_EINVAL, "counts pointer not 4-byte aligned");
    if ((st = set_device(ctx))) return st;
    const Shape sh = shape_for(db);
    if ((st = stage(ctx, db, q_dev, n_q, mode, sh))) return st;
    const Plan pl = plan_scan(ctx->num_cus, db->v.nblk, n_q, sh, EPI_FULL);
    ScanParams p = base_params(db, sh, pl, 0, db->v.n_refs, 0, n_q);
    p.ld = ld;
    p.out_q_base = 0;
    p.out_r_base = 0;
    ScanBuffers b{};
    b.qs = staged_queries(ctx);
    b.out = counts_dev;
    return main_scan(ctx, mode, sh.nw, EPI_FULL, sh.chunked, p, b);
}

int fid_compare_tiles(fid_ctx* ctx, const fid_db* db, const uint64_t* q_dev, int32_t n_q, int mode,
                      const int64_t* tiles_host, int32_t n_tiles, int32_t th, int32_t tw,
                      int32_t* out_dev)
{
    int st = check_common(ctx, db, q_dev, n_q, mode);
    if (st) return st;
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
    if ((st = set_device(ctx))) return st;
    const Shape sh = shape_for(db);
    if ((st = stage(ctx, db, q_dev, n_q, mode, sh))) return st;
    ScanBuffers b{};
    b.qs = staged_queries(ctx);
    for (int32_t t = 0; t < n_tiles; ++t) {
        const int64_t q0 = tiles_host[2 * t], r0 = tiles_host[2 * t + 1];
        const int64_t nblk = (r0 + tw + 63) / 64 - r0 / 64;
        const Plan pl = plan_scan(ctx->num_cus, nblk, th, sh, EPI_FULL);
        ScanParams p = base_params(db, sh, pl, r0, r0 + tw, (int32_t)q0, (int32_t)(q0 + th));
        p.ld = tw;
        p.out_q_base = (int32_t)q0;
        p.out_r_base = r0;
        b.out = out_dev + (size_t)t * th * tw;
        FID_HIP(launch_scan(mode, sh.nw, EPI_FULL, sh.chunked, refs_per_lane(sh.nw, sh.chunked), p,
                            b, ctx->stream),
                "scan launch");
    }
    return FID_OK;
}

int fid_topk_workspace_bytes(fid_ctx* ctx, const fid_db* db, int32_t n_q, int32_t k, size_t* bytes)
{
    if (!ctx || !db || !bytes) return fail(FID_EINVAL, "NULL argument");
    if (n_q < 1 || n_q > kMaxQueries) return fail(FID_EINVAL, "n_q out of range");
    if (k < 1 || k > kMaxK) return fail(FID_EINVAL, "k=%d out of [1, %d]", k, kMaxK);
    *bytes = topk_layout(ctx, db, n_q, k).total;
    return FID_OK;
}

int fid_compare_topk(fid_ctx* ctx, const fid_db* db, const uint64_t* q_dev, int32_t n_q, int mode,
                     int32_t k, void* ws_dev, size_t ws_bytes, int32_t* cnt_dev, int64_t* idx_dev)
{
    int st = check_common(ctx, db, q_dev, n_q, mode);
    if (st) return st;
    if (k < 1 || k > kMaxK) return fail(FID_EINVAL, "k=%d out of [1, %d]", k, kMaxK);
    if (!cnt_dev || !idx_dev || !ws_dev) return fail(FID_EINVAL, "NULL buffer");
    if (!aligned16(ws_dev)) return fail(FID_EINVAL, "workspace not 16-byte aligned");
    const TopkLayout L = topk_layout(ctx, db, n_q, k);
    if (ws_bytes < L.total) return fail(FID_ENOMEM, "workspace %zu bytes < required %zu", ws_bytes, L.total);
    if ((st = set_device(ctx))) return st;
    const Shape sh = shape_for(db);
    if ((st = stage(ctx, db, q_dev, n_q, mode, sh))) return st;
    char* ws = static_cast<char*>(ws_dev);
    int32_t* counts = reinterpret_cast<int32_t*>(ws + L.off_counts);
    ScanBuffers b{};
    b.qs = staged_queries(ctx);

    // Seed (or, for a small database, the whole answer): the full count block
    // of the first L.seed references, then an exact per-query selection.
    {
        const int64_t nblk = (L.seed + 63) / 64;
        const Plan pl = plan_scan(ctx->num_cus, nblk, n_q, sh, EPI_FULL);
        ScanParams p = base_params(db, sh, pl, 0, L.seed, 0, n_q);
        p.ld = L.seed;
        b.out = counts;
        if (L.direct) {
            if ((st = main_scan(ctx, mode, sh.nw, EPI_FULL, sh.chunked, p, b))) return st;
        } else {
            FID_HIP(launch_scan(mode, sh.nw, EPI_FULL, sh.chunked, refs_per_lane(sh.nw, sh.chunked),
                                p, b, ctx->stream),
                    "seed scan launch");
        }
    }
    if (L.direct) {
        FID_HIP(launch_select_counts(counts, n_q, L.seed, k, cnt_dev, idx_dev, ctx->stream), "select launch");
        return FID_OK;
    }
    uint64_t* lists = reinterpret_cast<uint64_t*>(ws + L.off_lists);
    uint32_t* fills = reinterpret_cast<uint32_t*>(ws + L.off_fills);
    uint32_t* thr_init = reinterpret_cast<uint32_t*>(ws + L.off_thr);
    FID_HIP(launch_seed_select(counts, n_q, L.seed, k, db->v.n_loci, thr_init, ctx->stream),
            "seed select launch");
    ScanParams p = base_params(db, sh, L.plan, 0, db->v.n_refs, 0, n_q);
    p.k = k;
    b.out = nullptr;
    b.lists = lists;
    b.fills = fills;
    b.thr_init = thr_init;
    if ((st = main_scan(ctx, mode, sh.nw, EPI_TOPK, sh.chunked, p, b))) return st;
    FID_HIP(launch_merge_lists(lists, fills, n_q, L.plan.n_rsplit, k, cnt_dev, idx_dev, ctx->stream),
            "merge launch");
    return FID_OK;
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
    int st = check_common(ctx, db, q_dev, n_q, mode);
    if (st) return st;
    if (!thr_dev || !ws_dev || !offs_dev || !total_host) return fail(FID_EINVAL, "NULL buffer");
    if (cap > 0 && (!idx_dev || !cnt_dev)) return fail(FID_EINVAL, "NULL output buffer");
    if (!aligned16(ws_dev)) return fail(FID_EINVAL, "workspace not 16-byte aligned");
    size_t need = 0;
    if ((st = fid_threshold_workspace_bytes(db, n_q, cap, &need))) return st;
    if (ws_bytes < need) return fail(FID_ENOMEM, "workspace %zu bytes < required %zu", ws_bytes, need);
    if ((st = set_device(ctx))) return st;
    const Shape sh = shape_for(db);
    if ((st = stage(ctx, db, q_dev, n_q, mode, sh))) return st;
    const size_t c = (size_t)(cap > 0 ? cap : 1);
    char* ws = static_cast<char*>(ws_dev);
    unsigned long long* counter = reinterpret_cast<unsigned long long*>(ws);
    uint64_t* keys = reinterpret_cast<uint64_t*>(ws + 256);
    uint64_t* keys2 = reinterpret_cast<uint64_t*>(ws + 256 + align256(c * 8));
    int32_t* vals = reinterpret_cast<int32_t*>(ws + 256 + 2 * align256(c * 8));
    int32_t* vals2 = reinterpret_cast<int32_t*>(ws + 256 + 2 * align256(c * 8) + align256(c * 4));
    FID_HIP(launch_fill_u64(reinterpret_cast<uint64_t*>(counter), 1, 0ull, ctx->stream), "fill launch");
    const Plan pl = plan_scan(ctx->num_cus, db->v.nblk, n_q, sh, EPI_THRESH);
    ScanParams p = base_params(db, sh, pl, 0, db->v.n_refs, 0, n_q);
    p.hit_cap = cap;
    ScanBuffers b{};
    b.qs = staged_queries(ctx);
    b.thr = thr_dev;
    b.hit_count = counter;
    b.hit_keys = keys;
    b.hit_cnt = vals;
    if ((st = main_scan(ctx, mode, sh.nw, EPI_THRESH, sh.chunked, p, b))) return st;
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

}  // extern "C"
