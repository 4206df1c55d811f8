// libfastid serving: a resident reference database answering a stream of
// requests (mixed identity and mixture queries, per-query top-k and, on
// request, threshold hits) with continuous batching.
//
// The database is cut into C chunks of references.  A worker thread runs
// ticks back to back; a tick compares every query in flight against a run of
// consecutive chunks (one top-k call over all of them, gathered into a
// contiguous block, each query with its own mode) and folds each query's
// result into its running top-k.  A request is admitted at a tick boundary
// as soon as enough query slots are free (slots are sized from an HBM
// budget), joins the batch at whatever chunk is current, and completes once
// it has met every chunk exactly once -- so requests that arrive while others
// run share their launches instead of queueing behind them.  By default a
// tick spans the whole database: every request waiting at a tick boundary
// joins one pass, answered straight from the comparison with nothing
// folded, and a burst of requests shares one pass instead of queueing for a
// pass each.  A configured span of fewer chunks lets new requests join
// mid-pass instead (measured slower at every load tried: the extra ticks'
// fixed costs outweigh the earlier start).  Keys (count << 40 | index) are a total order,
// so the fold of per-range top-k lists is exactly the top-k of the whole
// database: every result is bit-identical to fid_compare_topk on that
// request alone.  Threshold hits (count <= the query's threshold) of every
// tick's range are collected per request and handed out as CSR in
// reference order, exactly fid_compare_threshold's.
//
// The FIFO policy is the plain alternative: one request at a time, each a
// full-database comparison.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "fid_device.hpp"
#include "fid_internal.hpp"

namespace fid {
namespace {

__global__ void scatter_rows_kernel(const uint64_t* __restrict__ src, const int32_t* __restrict__ slots,
                                    int32_t n, int32_t rw, uint64_t* __restrict__ dst)
{
    const int64_t total = (int64_t)n * rw;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / rw;
        const int32_t w = (int32_t)(t - i * rw);
        dst[(int64_t)slots[i] * rw + w] = src[t];
    }
}

__global__ void gather_rows_kernel(const uint64_t* __restrict__ src, const int32_t* __restrict__ slots,
                                   int32_t n, int32_t rw, uint64_t* __restrict__ dst)
{
    const int64_t total = (int64_t)n * rw;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / rw;
        const int32_t w = (int32_t)(t - i * rw);
        dst[t] = src[(int64_t)slots[i] * rw + w];
    }
}

__global__ void gather_u32_kernel(const uint32_t* __restrict__ src, const int32_t* __restrict__ slots, int32_t n,
                                  uint32_t* __restrict__ dst)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) dst[i] = src[slots[i]];
}

unsigned grid_for(int64_t n)
{
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    return (unsigned)(b < 1 ? 1 : b);
}

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    uint64_t ticket;
    fid_request r;
    std::vector<int32_t> thr;        // per-query thresholds (empty: no threshold output)
    std::vector<int32_t> slots;
    int32_t chunks_left = 0;         // chunks still to meet
    std::vector<uint64_t> hits;      // (query << 40 | reference) of the hits so far
    std::vector<int32_t> hit_counts;
    bool hits_lost = false;          // a tick's hit buffer overflowed while this request was in flight
    int status = FID_ENOTREADY;      // FID_OK when done, an error code on failure
    int64_t submit_ns = 0, admit_ns = 0, done_ns = 0;
};

}  // namespace
}  // namespace fid

using namespace fid;

struct fid_server {
    fid_ctx* ctx = nullptr;          // the worker's own context (own stream)
    hipStream_t stream = nullptr;
    const fid_db* db = nullptr;
    fid_server_config cfg{};
    int32_t rw = 0;                  // packed words per query row
    int32_t max_slots = 0;
    int32_t n_chunks = 0;
    int64_t chunk_refs = 0;
    size_t device_bytes = 0;
    // device memory (one allocation)
    void* mem = nullptr;
    uint64_t* slot_rows = nullptr;   // [max_slots][rw]
    uint64_t* running = nullptr;     // [max_slots][k]
    uint32_t* bound = nullptr;       // [max_slots] exclusive count bound from the running top-k
    uint32_t* tbound = nullptr;      // [max_slots] the in-flight queries' bounds, gathered
    uint64_t* gathered = nullptr;    // [max_slots][rw] the tick's query rows
    uint64_t* trows = nullptr;       // [max_slots][rw] the tick's threshold queries, mixture first
    int32_t* tcnt = nullptr;         // [max_slots][k]
    int64_t* tidx = nullptr;         // [max_slots][k]
    int32_t* dslots = nullptr;       // [kTables][max_slots] tables of one tick
    unsigned long long* hcounter = nullptr;  // hit counter of a tick, then 3 int64 block ends
    uint64_t* hkeys = nullptr;       // [hcap] (threshold query << 40 | reference)
    int32_t* hvals = nullptr;        // [hcap]
    int64_t hcap = 0;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    // pinned host staging
    int32_t* hslots = nullptr;       // [kTables][max_slots]
    int32_t* hcnt = nullptr;         // [max_slots][k]
    int64_t* hidx = nullptr;
    unsigned long long* hcount_host = nullptr;
    uint64_t* hkeys_host = nullptr;  // [hcap]
    int32_t* hvals_host = nullptr;
    // state
    std::mutex mu;
    std::condition_variable cv;      // wakes the worker
    std::condition_variable done_cv; // wakes waiters
    std::deque<uint64_t> pending;
    std::vector<uint64_t> active;
    std::unordered_map<uint64_t, Request> reqs;
    std::vector<int32_t> free_slots;
    uint64_t next_ticket = 1;
    int32_t pos = 0;                 // first chunk of the next tick
    int64_t tick = 0;
    int64_t tick_ns = 0;             // summed wall time of the ticks
    int64_t tick_queries = 0;        // summed queries in flight per tick
    int64_t completed = 0;
    int32_t peak_active_queries = 0;
    int fatal = FID_OK;
    std::string fatal_msg;
    bool stop = false;
    std::thread worker;
};

namespace {

// tables of one tick: [0] fresh slots, [1] in-flight slots (gathered order),
// [2] their modes, [3] finishing slots, [4] threshold queries (gathered
// index, mixture ones first), [5] their thresholds
constexpr int kTables = 6;
constexpr int32_t kDefaultHitsPerQuery = 256;

int64_t chunk_lo(const fid_server* s, int64_t c) { return std::min<int64_t>(s->db->v.n_refs, c * s->chunk_refs); }

// Chunks the next tick may span: the configured span, else the whole database.
int32_t span_cap(const fid_server* s) { return s->cfg.tick_chunks > 0 ? s->cfg.tick_chunks : s->n_chunks; }

// Device work of one tick over chunks [c0, c0 + m): every request in act,
// the newly admitted ones (fresh, a prefix of act) included.  Called by the
// worker with the lock released; touches only slots owned by act.  Results
// of requests that finish (meet their last chunk) are handed out here, with
// each request's own status in rstat.
int run_tick(fid_server* s, const std::vector<Request*>& act, const std::vector<Request*>& fresh, int32_t c0,
             int32_t m, std::vector<int>& rstat)
{
    const int32_t k = s->cfg.k;
    const int32_t M = s->max_slots;
    int32_t* hs = s->hslots;
    const int64_t r_lo = chunk_lo(s, c0), r_hi = chunk_lo(s, c0 + m);
    // every request in flight starts and ends here: one comparison, no running state
    const bool whole = fresh.size() == act.size() && c0 == 0 && m == s->n_chunks;
    int32_t n_fresh = 0, n_act = 0, n_fin = 0, n_mix = 0, n_thr = 0;
    bool one_mode = true;
    for (Request* r : act) {
        one_mode = one_mode && r->r.mode == act[0]->r.mode;
        for (int32_t q = 0; q < r->r.n_q; ++q) {
            hs[M + n_act] = r->slots[q];
            hs[2 * M + n_act] = r->r.mode;
            ++n_act;
        }
        if (r->chunks_left == m)
            for (int32_t sl : r->slots) hs[3 * M + n_fin++] = sl;
    }
    for (Request* r : fresh)
        for (int32_t sl : r->slots) hs[n_fresh++] = sl;
    // threshold queries: mixture ones first, then identity ones
    for (int pass = 0; pass < 2; ++pass) {
        int32_t g = 0;
        for (Request* r : act) {
            const bool want = r->r.mode == (pass == 0 ? FID_MODE_MIXTURE : FID_MODE_IDENTITY);
            for (int32_t q = 0; q < r->r.n_q; ++q, ++g) {
                if (!want || r->thr.empty()) continue;
                hs[4 * M + n_thr] = g;
                hs[5 * M + n_thr] = r->thr[q];
                ++n_thr;
            }
        }
        if (pass == 0) n_mix = n_thr;
    }
    FID_HIP(hipMemcpyAsync(s->dslots, hs, sizeof(int32_t) * kTables * (size_t)M, hipMemcpyHostToDevice, s->stream),
            "slot table upload");
    const int32_t* tbl = s->dslots + (size_t)M;
    const int32_t* modes = s->dslots + 2 * (size_t)M;

    // the tick's query rows, in gathered order
    const uint64_t* qsrc = s->gathered;
    if (whole && act.size() == 1) {
        qsrc = act[0]->r.q_dev;
    } else if (whole) {
        size_t off = 0;
        for (Request* r : act) {
            FID_HIP(hipMemcpyAsync(s->gathered + off, r->r.q_dev, sizeof(uint64_t) * (size_t)r->r.n_q * s->rw,
                                   hipMemcpyDeviceToDevice, s->stream), "query copy");
            off += (size_t)r->r.n_q * s->rw;
        }
    } else {
        // newly admitted requests: their queries into their slots, state cleared
        int32_t off = 0;
        for (Request* r : fresh) {
            const int32_t n = r->r.n_q;
            hipLaunchKernelGGL(scatter_rows_kernel, dim3(grid_for((int64_t)n * s->rw)), dim3(256), 0, s->stream,
                               r->r.q_dev, s->dslots + off, n, s->rw, s->slot_rows);
            FID_HIP(hipGetLastError(), "scatter launch");
            off += n;
        }
        if (n_fresh) FID_HIP(launch_reset_running(s->dslots, n_fresh, k, s->running, s->bound, s->stream), "reset launch");
        hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_for((int64_t)n_act * s->rw)), dim3(256), 0, s->stream,
                           s->slot_rows, tbl, n_act, s->rw, s->gathered);
        FID_HIP(hipGetLastError(), "gather launch");
    }

    // top-k of every query in flight over the tick's references
    if (whole && one_mode) {
        FID_TRY(fid_compare_topk_range(s->ctx, s->db, r_lo, r_hi, qsrc, n_act, act[0]->r.mode, k, s->ws,
                                       s->ws_bytes, s->tcnt, s->tidx));
    } else if (whole) {
        FID_TRY(topk_range_bounded(s->ctx, s->db, r_lo, r_hi, qsrc, modes, n_act, k, s->ws, s->ws_bytes, s->tcnt,
                                   s->tidx, nullptr, true));
    } else {
        // queries past their first chunk are filtered by their running k-th
        // count; only a tick that admits new queries pays the seed pass
        hipLaunchKernelGGL(gather_u32_kernel, dim3((unsigned)((n_act + 255) / 256)), dim3(256), 0, s->stream,
                           s->bound, tbl, n_act, s->tbound);
        FID_HIP(hipGetLastError(), "gather launch");
        FID_TRY(topk_range_bounded(s->ctx, s->db, r_lo, r_hi, qsrc, modes, n_act, k, s->ws, s->ws_bytes, s->tcnt,
                                   s->tidx, s->tbound, n_fresh > 0));
        FID_HIP(launch_fold_topk(s->tcnt, s->tidx, tbl, n_act, k, 0, s->running, s->bound, s->stream),
                "fold launch");
        if (n_fin)
            FID_HIP(launch_finalize_topk(s->running, s->dslots + 3 * (size_t)M, n_fin, k, k, s->tcnt, s->tidx,
                                         s->stream), "finalize launch");
    }
    const int32_t n_out = whole ? n_act : n_fin;
    if (n_out) {
        FID_HIP(hipMemcpyAsync(s->hcnt, s->tcnt, sizeof(int32_t) * (size_t)n_out * k, hipMemcpyDeviceToHost,
                               s->stream), "result copy");
        FID_HIP(hipMemcpyAsync(s->hidx, s->tidx, sizeof(int64_t) * (size_t)n_out * k, hipMemcpyDeviceToHost,
                               s->stream), "result copy");
    }

    // threshold hits of the tick's references: one scan per mode
    if (n_thr) {
        unsigned long long* counter = s->hcounter;
        int64_t* ends = reinterpret_cast<int64_t*>(s->hcounter + 1);
        FID_HIP(launch_fill_u64(reinterpret_cast<uint64_t*>(s->hcounter), 4, 0ull, s->stream), "fill launch");
        hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_for((int64_t)n_thr * s->rw)), dim3(256), 0, s->stream, qsrc,
                           s->dslots + 4 * (size_t)M, n_thr, s->rw, s->trows);
        FID_HIP(hipGetLastError(), "gather launch");
        const int32_t* tthr = s->dslots + 5 * (size_t)M;
        if (n_mix) {
            FID_TRY(thresh_range(s->ctx, s->db, r_lo, r_hi, s->trows, n_mix, FID_MODE_MIXTURE, tthr, counter,
                                 s->hkeys, s->hvals, s->hcap));
            FID_HIP(launch_offset_block_hits(counter, ends, 0, s->hkeys, s->hcap, 0, s->stream), "hit offsets");
        }
        if (n_thr > n_mix) {
            // identity hits carry their block-local query index + n_mix
            FID_TRY(thresh_range(s->ctx, s->db, r_lo, r_hi, s->trows + (size_t)n_mix * s->rw, n_thr - n_mix,
                                 FID_MODE_IDENTITY, tthr + n_mix, counter, s->hkeys, s->hvals, s->hcap));
            FID_HIP(launch_offset_block_hits(counter, ends, n_mix ? 1 : 0, s->hkeys, s->hcap, (int64_t)n_mix << kIdxBits,
                                             s->stream), "hit offsets");
        }
        FID_HIP(hipMemcpyAsync(s->hcount_host, counter, sizeof(unsigned long long), hipMemcpyDeviceToHost, s->stream),
                "hit count copy");
    }
    FID_HIP(hipStreamSynchronize(s->stream), "hipStreamSynchronize");

    if (n_thr) {
        const unsigned long long total = *s->hcount_host;
        const int64_t stored = std::min<int64_t>((int64_t)total, s->hcap);
        if (stored > 0) {
            FID_HIP(hipMemcpy(s->hkeys_host, s->hkeys, sizeof(uint64_t) * (size_t)stored, hipMemcpyDeviceToHost),
                    "hit copy");
            FID_HIP(hipMemcpy(s->hvals_host, s->hvals, sizeof(int32_t) * (size_t)stored, hipMemcpyDeviceToHost),
                    "hit copy");
        }
        // threshold query t -> (request, query): the order the table was built in
        std::vector<std::pair<Request*, int32_t>> owner((size_t)n_thr);
        {
            std::vector<std::pair<Request*, int32_t>> by_g((size_t)n_act);
            int32_t g = 0;
            for (Request* r : act)
                for (int32_t q = 0; q < r->r.n_q; ++q) by_g[(size_t)g++] = {r, q};
            for (int32_t t = 0; t < n_thr; ++t) owner[(size_t)t] = by_g[(size_t)hs[4 * M + t]];
        }
        for (int64_t i = 0; i < stored; ++i) {
            const uint64_t key = s->hkeys_host[i];
            const auto& o = owner[(size_t)(key >> kIdxBits)];
            o.first->hits.push_back(((uint64_t)o.second << kIdxBits) | (key & kIdxMask));
            o.first->hit_counts.push_back(s->hvals_host[i]);
        }
        if ((int64_t)total > s->hcap)
            for (Request* r : act)
                if (!r->thr.empty()) r->hits_lost = true;
    }

    // hand finished results to their callers (request k may be below the server's)
    int32_t row = 0;
    rstat.assign(act.size(), FID_OK);
    for (size_t a = 0; a < act.size(); ++a) {
        Request* r = act[a];
        if (r->chunks_left != m) continue;
        const int32_t kr = r->r.k;
        for (int32_t q = 0; q < r->r.n_q; ++q, ++row) {
            memcpy(r->r.cnt_host + (size_t)q * kr, s->hcnt + (size_t)row * k, sizeof(int32_t) * kr);
            memcpy(r->r.idx_host + (size_t)q * kr, s->hidx + (size_t)row * k, sizeof(int64_t) * kr);
        }
        if (r->thr.empty()) continue;
        // hits in (query, reference) order, as CSR
        std::vector<size_t> order(r->hits.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = i;
        std::sort(order.begin(), order.end(), [&](size_t x, size_t y) { return r->hits[x] < r->hits[y]; });
        const int64_t total = (int64_t)order.size();
        int64_t* offs = r->r.hit_offs_host;
        if (r->hits_lost || total > r->r.hit_cap) {
            for (int32_t q = 0; q < r->r.n_q; ++q) offs[q] = 0;
            offs[r->r.n_q] = r->hits_lost ? -1 : total;
            rstat[a] = FID_EOVERFLOW;
            continue;
        }
        int64_t j = 0;
        for (int32_t q = 0; q < r->r.n_q; ++q) {
            offs[q] = j;
            while (j < total && (int32_t)(r->hits[order[(size_t)j]] >> kIdxBits) == q) {
                r->r.hit_idx_host[j] = (int64_t)(r->hits[order[(size_t)j]] & kIdxMask);
                r->r.hit_cnt_host[j] = r->hit_counts[order[(size_t)j]];
                ++j;
            }
        }
        offs[r->r.n_q] = total;
    }
    return FID_OK;
}

void worker_main(fid_server* s)
{
    hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    std::vector<int> rstat;
    for (;;) {
        s->cv.wait(lk, [&] { return s->stop || !s->pending.empty() || !s->active.empty(); });
        if (s->stop) break;
        const bool idle = s->active.empty();
        // admit in arrival order while slots last (FIFO: one request at a time)
        std::vector<Request*> fresh;
        while (!s->pending.empty() && (s->cfg.policy != FID_SERVE_FIFO || (s->active.empty() && fresh.empty()))) {
            Request* r = &s->reqs[s->pending.front()];
            if ((size_t)r->r.n_q > s->free_slots.size()) break;
            s->pending.pop_front();
            for (int32_t q = 0; q < r->r.n_q; ++q) {
                r->slots.push_back(s->free_slots.back());
                s->free_slots.pop_back();
            }
            r->chunks_left = s->n_chunks;
            r->admit_ns = now_ns();
            s->active.push_back(r->ticket);
            fresh.push_back(r);
        }
        if (idle) s->pos = 0;
        std::vector<Request*> act;
        int32_t nq = 0;
        int32_t m = s->n_chunks - s->pos;
        for (uint64_t t : s->active) {
            act.push_back(&s->reqs[t]);
            nq += act.back()->r.n_q;
            m = std::min(m, act.back()->chunks_left);
        }
        m = std::min(m, span_cap(s));
        if (nq > s->peak_active_queries) s->peak_active_queries = nq;
        const int32_t c0 = s->pos;
        lk.unlock();
        const int64_t t_start = now_ns();
        const int st = run_tick(s, act, fresh, c0, m, rstat);
        const std::string msg = st ? fid_last_error() : "";
        lk.lock();
        ++s->tick;
        const int64_t t_done = now_ns();
        s->tick_ns += t_done - t_start;
        s->tick_queries += nq;
        s->pos = (c0 + m) % s->n_chunks;
        std::vector<uint64_t> still;
        for (size_t a = 0; a < act.size(); ++a) {
            Request* r = act[a];
            r->chunks_left -= m;
            if (st || r->chunks_left == 0) {
                r->status = st ? st : (a < rstat.size() ? rstat[a] : FID_OK);
                r->done_ns = t_done;
                for (int32_t sl : r->slots) s->free_slots.push_back(sl);
                r->slots.clear();
                r->hits.clear();
                r->hit_counts.clear();
                ++s->completed;
            } else {
                still.push_back(r->ticket);
            }
        }
        s->active.swap(still);
        if (st && !s->fatal) {
            s->fatal = st;
            s->fatal_msg = msg;
        }
        s->done_cv.notify_all();
    }
}

size_t server_bytes(int32_t slots, int32_t rw, int32_t k, size_t ws, int64_t hcap)
{
    const size_t n = (size_t)slots;
    return align256(n * rw * 8) * 3 + align256(n * k * 8) * 2 + align256(n * k * 4) +
           align256((size_t)kTables * n * 4) + 2 * align256(n * 4) + align256(4 * 8) +
           align256((size_t)hcap * 8) + align256((size_t)hcap * 4) + align256(ws);
}

}  // namespace

extern "C" {

int fid_server_create(fid_ctx* ctx, const fid_db* db, const fid_server_config* cfg, fid_server** out)
{
    if (!out) return fail(FID_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctx || !db || !cfg) return fail(FID_EINVAL, "NULL argument");
    if (db->device != ctx->device) return fail(FID_EINVAL, "db and ctx on different devices");
    if (cfg->k < 1 || cfg->k > kMaxK) return fail(FID_EINVAL, "k=%d out of [1, %d]", cfg->k, kMaxK);
    if (cfg->policy != FID_SERVE_CONTINUOUS && cfg->policy != FID_SERVE_FIFO)
        return fail(FID_EINVAL, "unknown policy %d", cfg->policy);
    if (cfg->max_queries < 1 || cfg->max_queries > (1 << 20))
        return fail(FID_EINVAL, "max_queries=%d out of [1, 2^20]", cfg->max_queries);
    if (cfg->n_chunks < 0 || cfg->n_chunks > 4096) return fail(FID_EINVAL, "n_chunks out of [0, 4096]");
    if (cfg->tick_chunks < 0) return fail(FID_EINVAL, "tick_chunks < 0");
    if (cfg->hits_per_query < 0 || cfg->hits_per_query > (1 << 20))
        return fail(FID_EINVAL, "hits_per_query out of [0, 2^20]");
    FID_TRY(set_device(ctx));
    fid_server* s = new fid_server{};
    s->db = db;
    s->cfg = *cfg;
    if (s->cfg.hits_per_query == 0) s->cfg.hits_per_query = kDefaultHitsPerQuery;
    s->rw = db->row_words;
    // chunks: whole 1024-reference tiles; FIFO scans the database in one call
    int32_t C = cfg->policy == FID_SERVE_FIFO ? 1 : (cfg->n_chunks ? cfg->n_chunks : 8);
    s->chunk_refs = ((db->v.n_refs + C - 1) / C + kDbTileRefs - 1) / kDbTileRefs * kDbTileRefs;
    s->n_chunks = (int32_t)((db->v.n_refs + s->chunk_refs - 1) / s->chunk_refs);
    auto cleanup = [&](int st) {
        if (s->ctx) fid_ctx_destroy(s->ctx);
        if (s->stream) (void)hipStreamDestroy(s->stream);
        if (s->mem) (void)hipFree(s->mem);
        for (void* h : {(void*)s->hslots, (void*)s->hcnt, (void*)s->hidx, (void*)s->hcount_host,
                        (void*)s->hkeys_host, (void*)s->hvals_host})
            if (h) (void)hipHostFree(h);
        delete s;
        return st;
    };
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return cleanup(hip_fail(e, "hipStreamCreate"));
    int st = fid_ctx_create(&s->ctx, ctx->device, s->stream);
    if (st) return cleanup(st);
    s->ctx->backend = ctx->backend;
    // workspace: the largest top-k any tick may run -- a range of up to the
    // whole database, with one mode or per-query modes
    auto ws_for = [&](int32_t n, size_t* bytes) -> int {
        size_t best = 0;
        for (int32_t m = 1; m <= n; m = m < 64 ? m + 1 : m + 64) {  // the family (and layout) depends on m
            size_t a = 0, b = 0;
            FID_TRY(fid_topk_workspace_bytes(s->ctx, db, m, cfg->k, &a));
            FID_TRY(fid_topk_mixed_workspace_bytes(s->ctx, db, 0, db->v.n_refs, m, cfg->k, &b));
            best = std::max(best, std::max(a, b));
            if (m == n) break;
            if (m >= 64 && m + 64 > n) m = n - 64;
        }
        *bytes = best;
        return FID_OK;
    };
    auto total_for = [&](int32_t n, size_t w) {
        return server_bytes(n, s->rw, cfg->k, w, (int64_t)n * s->cfg.hits_per_query);
    };
    int32_t lo = 0, hi = cfg->max_queries;
    size_t ws = 0;
    while (lo < hi) {  // largest slot count whose state + workspace fit the budget
        const int32_t mid = lo + (hi - lo + 1) / 2;
        size_t w = 0;
        st = ws_for(mid, &w);
        if (st) return cleanup(st);
        if (total_for(mid, w) <= cfg->hbm_budget) lo = mid;
        else hi = mid - 1;
    }
    if (lo < 1) return cleanup(fail(FID_EBUDGET, "hbm_budget %zu holds no query slot", cfg->hbm_budget));
    s->max_slots = lo;
    st = ws_for(lo, &ws);
    if (st) return cleanup(st);
    s->ws_bytes = ws;
    s->hcap = (int64_t)lo * s->cfg.hits_per_query;
    s->device_bytes = total_for(lo, ws);
    e = hipMalloc(&s->mem, s->device_bytes);
    if (e != hipSuccess) return cleanup(fail(FID_ENOMEM, "server memory (%zu bytes): %s", s->device_bytes,
                                             hipGetErrorString(e)));
    char* p = static_cast<char*>(s->mem);
    const size_t n = (size_t)lo;
    auto take = [&](size_t bytes) { char* q = p; p += align256(bytes); return q; };
    s->slot_rows = reinterpret_cast<uint64_t*>(take(n * s->rw * 8));
    s->gathered = reinterpret_cast<uint64_t*>(take(n * s->rw * 8));
    s->trows = reinterpret_cast<uint64_t*>(take(n * s->rw * 8));
    s->running = reinterpret_cast<uint64_t*>(take(n * cfg->k * 8));
    s->tidx = reinterpret_cast<int64_t*>(take(n * cfg->k * 8));
    s->tcnt = reinterpret_cast<int32_t*>(take(n * cfg->k * 4));
    s->dslots = reinterpret_cast<int32_t*>(take((size_t)kTables * n * 4));
    s->bound = reinterpret_cast<uint32_t*>(take(n * 4));
    s->tbound = reinterpret_cast<uint32_t*>(take(n * 4));
    s->hcounter = reinterpret_cast<unsigned long long*>(take(4 * 8));
    s->hkeys = reinterpret_cast<uint64_t*>(take((size_t)s->hcap * 8));
    s->hvals = reinterpret_cast<int32_t*>(take((size_t)s->hcap * 4));
    s->ws = take(ws);
    if ((e = hipHostMalloc((void**)&s->hslots, (size_t)kTables * n * 4, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void**)&s->hcnt, n * cfg->k * 4, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void**)&s->hidx, n * cfg->k * 8, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void**)&s->hcount_host, 8, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void**)&s->hkeys_host, (size_t)s->hcap * 8, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void**)&s->hvals_host, (size_t)s->hcap * 4, hipHostMallocDefault)) != hipSuccess)
        return cleanup(fail(FID_ENOMEM, "pinned staging: %s", hipGetErrorString(e)));
    for (int32_t i = lo - 1; i >= 0; --i) s->free_slots.push_back(i);
    s->worker = std::thread(worker_main, s);
    *out = s;
    return FID_OK;
}

int fid_server_info(const fid_server* s, int32_t* max_queries, int32_t* n_chunks, size_t* device_bytes)
{
    if (!s) return fail(FID_EINVAL, "server is NULL");
    if (max_queries) *max_queries = s->max_slots;
    if (n_chunks) *n_chunks = s->n_chunks;
    if (device_bytes) *device_bytes = s->device_bytes;
    return FID_OK;
}

int fid_server_submit(fid_server* s, const fid_request* r, uint64_t* ticket)
{
    if (!s || !r || !ticket) return fail(FID_EINVAL, "NULL argument");
    if (r->n_q < 1) return fail(FID_EINVAL, "n_q=%d", r->n_q);
    if (r->mode != FID_MODE_MIXTURE && r->mode != FID_MODE_IDENTITY) return fail(FID_EINVAL, "bad mode %d", r->mode);
    if (r->k < 1 || r->k > s->cfg.k) return fail(FID_EINVAL, "k=%d out of [1, %d]", r->k, s->cfg.k);
    if (!r->q_dev || !aligned16(r->q_dev)) return fail(FID_EINVAL, "query pointer NULL or unaligned");
    if (!r->cnt_host || !r->idx_host) return fail(FID_EINVAL, "NULL output");
    if (r->thr_host && (!r->hit_offs_host || r->hit_cap < 0 || (r->hit_cap > 0 && (!r->hit_idx_host ||
                                                                                   !r->hit_cnt_host))))
        return fail(FID_EINVAL, "threshold request without its hit outputs");
    if (r->n_q > s->max_slots)
        return fail(FID_EBUDGET, "request of %d queries exceeds the %d query slots the budget holds", r->n_q,
                    s->max_slots);
    Request q;
    q.r = *r;
    if (r->thr_host) q.thr.assign(r->thr_host, r->thr_host + r->n_q);
    std::lock_guard<std::mutex> g(s->mu);
    if (s->fatal) return fail(s->fatal, "server failed: %s", s->fatal_msg.c_str());
    const uint64_t t = s->next_ticket++;
    q.ticket = t;
    q.submit_ns = now_ns();
    s->reqs.emplace(t, std::move(q));
    s->pending.push_back(t);
    *ticket = t;
    s->cv.notify_one();
    return FID_OK;
}

int fid_server_poll(fid_server* s, uint64_t ticket, int64_t* times_ns)
{
    if (!s) return fail(FID_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(FID_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Request& r = it->second;
    if (r.status == FID_ENOTREADY) return FID_ENOTREADY;
    if (times_ns) {
        times_ns[0] = r.submit_ns;
        times_ns[1] = r.admit_ns;
        times_ns[2] = r.done_ns;
    }
    const int st = r.status;
    s->reqs.erase(it);
    if (st) return fail(st, "request failed");
    return FID_OK;
}

int fid_server_wait(fid_server* s, uint64_t ticket, int64_t timeout_us, int64_t* times_ns)
{
    if (!s) return fail(FID_EINVAL, "server is NULL");
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto ready = [&] {
            auto it = s->reqs.find(ticket);
            return it == s->reqs.end() || it->second.status != FID_ENOTREADY;
        };
        if (timeout_us < 0) s->done_cv.wait(lk, ready);
        else if (!s->done_cv.wait_for(lk, std::chrono::microseconds(timeout_us), ready))
            return fail(FID_ETIMEOUT, "request %llu not done after %lld us", (unsigned long long)ticket,
                        (long long)timeout_us);
    }
    return fid_server_poll(s, ticket, times_ns);
}

int fid_server_stats(const fid_server* s, int64_t* stats)
{
    if (!s || !stats) return fail(FID_EINVAL, "NULL argument");
    fid_server* m = const_cast<fid_server*>(s);
    std::lock_guard<std::mutex> g(m->mu);
    stats[0] = s->tick;
    stats[1] = s->completed;
    stats[2] = s->peak_active_queries;
    stats[3] = s->tick_ns;
    stats[4] = s->tick_queries;
    return FID_OK;
}

int fid_server_destroy(fid_server* s)
{
    if (!s) return FID_OK;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->ctx->device);
    (void)hipStreamSynchronize(s->stream);
    fid_ctx_destroy(s->ctx);
    (void)hipStreamDestroy(s->stream);
    (void)hipFree(s->mem);
    for (void* h : {(void*)s->hslots, (void*)s->hcnt, (void*)s->hidx, (void*)s->hcount_host, (void*)s->hkeys_host,
                    (void*)s->hvals_host})
        (void)hipHostFree(h);
    delete s;
    return FID_OK;
}

}  // extern "C"
