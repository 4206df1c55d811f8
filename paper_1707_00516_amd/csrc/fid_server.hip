// libfastid serving: a resident reference database answering a stream of
// top-k requests (mixed identity and mixture queries) with continuous
// batching.
//
// The database is cut into C chunks of references.  A worker thread runs
// ticks back to back; tick t compares every active query against chunk
// t mod C (one top-k call over all of them, gathered into a contiguous
// block, each query with its own mode) and folds each query's chunk result
// into its running top-k.  A request is admitted at a tick boundary
// as soon as enough query slots are free (slots are sized from an HBM
// budget), joins the batch at whatever chunk is current, and completes
// after C ticks -- it has then met every chunk exactly once -- so requests
// that arrive while others run share their launches instead of queueing
// behind them.  Keys (count << 40 | index) are a total order, so the fold of
// per-chunk top-k lists is exactly the top-k of the whole database: every
// result is bit-identical to fid_compare_topk on that request alone.
//
// The FIFO policy is the plain alternative: one request at a time, each a
// full-database fid_compare_topk call.
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
    std::vector<int32_t> slots;
    int32_t chunks_done = 0;
    int status = FID_ENOTREADY;  // FID_OK when done, an error code on failure
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
    uint64_t* gathered = nullptr;    // [max_slots][rw]
    int32_t* tcnt = nullptr;         // [max_slots][k]
    int64_t* tidx = nullptr;         // [max_slots][k]
    int32_t* dslots = nullptr;       // [4][max_slots] slot tables of one tick
    void* ws = nullptr;
    size_t ws_bytes = 0;
    // pinned host staging
    int32_t* hslots = nullptr;       // [4][max_slots]
    int32_t* hcnt = nullptr;         // [max_slots][k]
    int64_t* hidx = nullptr;
    // state
    std::mutex mu;
    std::condition_variable cv;      // wakes the worker
    std::condition_variable done_cv; // wakes waiters
    std::deque<uint64_t> pending;
    std::vector<uint64_t> active;
    std::unordered_map<uint64_t, Request> reqs;
    std::vector<int32_t> free_slots;
    uint64_t next_ticket = 1;
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

// Per-tick device work of the continuous-batching policy.  Called by the
// worker with the lock released; touches only slots owned by `act`.
int run_tick(fid_server* s, const std::vector<Request*>& act, const std::vector<Request*>& fresh,
             int64_t chunk)
{
    const int32_t k = s->cfg.k;
    int32_t* hs = s->hslots;
    const int32_t M = s->max_slots;
    // tables: [0] fresh slots, [1] in-flight slots, [2] their modes, [3] finishing slots
    int32_t n_fresh = 0, n_act = 0, n_fin = 0;
    for (Request* r : fresh)
        for (int32_t sl : r->slots) hs[n_fresh++] = sl;
    for (Request* r : act) {
        for (int32_t sl : r->slots) {
            hs[M + n_act] = sl;
            hs[2 * M + n_act] = r->r.mode;
            ++n_act;
        }
        if (r->chunks_done + 1 == s->n_chunks)
            for (int32_t sl : r->slots) hs[3 * M + n_fin++] = sl;
    }
    FID_HIP(hipMemcpyAsync(s->dslots, hs, sizeof(int32_t) * 4 * (size_t)M, hipMemcpyHostToDevice, s->stream),
            "slot table upload");
    // newly admitted requests: copy their queries into their slots, clear state
    int32_t off = 0;
    for (Request* r : fresh) {
        const int32_t n = r->r.n_q;
        hipLaunchKernelGGL(scatter_rows_kernel, dim3(grid_for((int64_t)n * s->rw)), dim3(256), 0, s->stream,
                           r->r.q_dev, s->dslots + off, n, s->rw, s->slot_rows);
        FID_HIP(hipGetLastError(), "scatter launch");
        off += n;
    }
    if (n_fresh) {
        FID_HIP(launch_reset_running(s->dslots, n_fresh, k, s->running, s->bound, s->stream), "reset launch");
    }
    // every in-flight query, identity and mixture alike, against this chunk
    const int64_t r_lo = chunk * s->chunk_refs;
    const int64_t r_hi = std::min<int64_t>(s->db->v.n_refs, r_lo + s->chunk_refs);
    if (n_act) {
        const int32_t* tbl = s->dslots + (size_t)M;
        hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_for((int64_t)n_act * s->rw)), dim3(256), 0, s->stream,
                           s->slot_rows, tbl, n_act, s->rw, s->gathered);
        FID_HIP(hipGetLastError(), "gather launch");
        // queries past their first chunk are filtered by their running k-th
        // count; only a tick that admits new queries pays the seed pass
        hipLaunchKernelGGL(gather_u32_kernel, dim3((unsigned)((n_act + 255) / 256)), dim3(256), 0, s->stream,
                           s->bound, tbl, n_act, s->tbound);
        FID_HIP(hipGetLastError(), "gather launch");
        FID_TRY(topk_range_bounded(s->ctx, s->db, r_lo, r_hi, s->gathered, s->dslots + 2 * (size_t)M, n_act, k,
                                   s->ws, s->ws_bytes, s->tcnt, s->tidx, s->tbound, n_fresh > 0));
        FID_HIP(launch_fold_topk(s->tcnt, s->tidx, tbl, n_act, k, 0, s->running, s->bound, s->stream),
                "fold launch");
    }
    if (n_fin) {
        FID_HIP(launch_finalize_topk(s->running, s->dslots + 3 * (size_t)M, n_fin, k, k, s->tcnt, s->tidx,
                                     s->stream), "finalize launch");
        FID_HIP(hipMemcpyAsync(s->hcnt, s->tcnt, sizeof(int32_t) * (size_t)n_fin * k, hipMemcpyDeviceToHost,
                               s->stream), "result copy");
        FID_HIP(hipMemcpyAsync(s->hidx, s->tidx, sizeof(int64_t) * (size_t)n_fin * k, hipMemcpyDeviceToHost,
                               s->stream), "result copy");
    }
    FID_HIP(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    // hand finished results to their callers (request k may be below the server's)
    int32_t row = 0;
    for (Request* r : act) {
        if (r->chunks_done + 1 != s->n_chunks) continue;
        const int32_t kr = r->r.k;
        for (int32_t q = 0; q < r->r.n_q; ++q, ++row) {
            memcpy(r->r.cnt_host + (size_t)q * kr, s->hcnt + (size_t)row * k, sizeof(int32_t) * kr);
            memcpy(r->r.idx_host + (size_t)q * kr, s->hidx + (size_t)row * k, sizeof(int64_t) * kr);
        }
    }
    return FID_OK;
}

// FIFO policy: one request, one full-database call.
int run_fifo(fid_server* s, Request* r)
{
    const int32_t k = s->cfg.k;
    const int32_t n = r->r.n_q;
    FID_TRY(fid_compare_topk(s->ctx, s->db, r->r.q_dev, n, r->r.mode, k, s->ws, s->ws_bytes, s->tcnt,
                             s->tidx));
    FID_HIP(hipMemcpyAsync(s->hcnt, s->tcnt, sizeof(int32_t) * (size_t)n * k, hipMemcpyDeviceToHost, s->stream),
            "result copy");
    FID_HIP(hipMemcpyAsync(s->hidx, s->tidx, sizeof(int64_t) * (size_t)n * k, hipMemcpyDeviceToHost, s->stream),
            "result copy");
    FID_HIP(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    const int32_t kr = r->r.k;
    for (int32_t q = 0; q < n; ++q) {
        memcpy(r->r.cnt_host + (size_t)q * kr, s->hcnt + (size_t)q * k, sizeof(int32_t) * kr);
        memcpy(r->r.idx_host + (size_t)q * kr, s->hidx + (size_t)q * k, sizeof(int64_t) * kr);
    }
    return FID_OK;
}

void worker_main(fid_server* s)
{
    hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv.wait(lk, [&] { return s->stop || !s->pending.empty() || !s->active.empty(); });
        if (s->stop) break;
        if (s->cfg.policy == FID_SERVE_FIFO) {
            const uint64_t t = s->pending.front();
            s->pending.pop_front();
            Request* r = &s->reqs[t];
            r->admit_ns = now_ns();
            lk.unlock();
            const int st = run_fifo(s, r);
            const std::string msg = st ? fid_last_error() : "";
            lk.lock();
            r->status = st;
            r->done_ns = now_ns();
            if (st && !s->fatal) {
                s->fatal = st;
                s->fatal_msg = msg;
            }
            ++s->completed;
            s->done_cv.notify_all();
            continue;
        }
        // admit in arrival order while slots last
        std::vector<Request*> fresh;
        while (!s->pending.empty()) {
            Request* r = &s->reqs[s->pending.front()];
            if ((size_t)r->r.n_q > s->free_slots.size()) break;
            s->pending.pop_front();
            for (int32_t q = 0; q < r->r.n_q; ++q) {
                r->slots.push_back(s->free_slots.back());
                s->free_slots.pop_back();
            }
            r->admit_ns = now_ns();
            s->active.push_back(r->ticket);
            fresh.push_back(r);
        }
        std::vector<Request*> act;
        int32_t nq = 0;
        for (uint64_t t : s->active) {
            act.push_back(&s->reqs[t]);
            nq += act.back()->r.n_q;
        }
        if (nq > s->peak_active_queries) s->peak_active_queries = nq;
        const int64_t chunk = s->tick % s->n_chunks;
        lk.unlock();
        const int64_t t_start = now_ns();
        const int st = run_tick(s, act, fresh, chunk);
        const std::string msg = st ? fid_last_error() : "";
        lk.lock();
        ++s->tick;
        const int64_t t_done = now_ns();
        s->tick_ns += t_done - t_start;
        s->tick_queries += nq;
        std::vector<uint64_t> still;
        for (Request* r : act) {
            ++r->chunks_done;
            if (st || r->chunks_done == s->n_chunks) {
                r->status = st ? st : FID_OK;
                r->done_ns = t_done;
                for (int32_t sl : r->slots) s->free_slots.push_back(sl);
                r->slots.clear();
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

size_t server_bytes(int32_t slots, int32_t rw, int32_t k, size_t ws)
{
    const size_t n = (size_t)slots;
    return align256(n * rw * 8) * 2 + align256(n * k * 8) * 2 + align256(n * k * 4) +
           align256(4 * n * 4) + 2 * align256(n * 4) + align256(ws);
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
    FID_TRY(set_device(ctx));
    fid_server* s = new fid_server{};
    s->db = db;
    s->cfg = *cfg;
    s->rw = db->row_words;
    // chunks: whole 1024-reference tiles; FIFO scans the database in one call
    int32_t C = cfg->policy == FID_SERVE_FIFO ? 1 : (cfg->n_chunks ? cfg->n_chunks : 8);
    s->chunk_refs = ((db->v.n_refs + C - 1) / C + kDbTileRefs - 1) / kDbTileRefs * kDbTileRefs;
    s->n_chunks = (int32_t)((db->v.n_refs + s->chunk_refs - 1) / s->chunk_refs);
    auto cleanup = [&](int st) {
        if (s->ctx) fid_ctx_destroy(s->ctx);
        if (s->stream) (void)hipStreamDestroy(s->stream);
        if (s->mem) (void)hipFree(s->mem);
        if (s->hslots) (void)hipHostFree(s->hslots);
        if (s->hcnt) (void)hipHostFree(s->hcnt);
        if (s->hidx) (void)hipHostFree(s->hidx);
        delete s;
        return st;
    };
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return cleanup(hip_fail(e, "hipStreamCreate"));
    int st = fid_ctx_create(&s->ctx, ctx->device, s->stream);
    if (st) return cleanup(st);
    s->ctx->backend = ctx->backend;
    // slots: as many as the budget holds (workspace of one chunk's top-k included)
    const int64_t r_hi0 = std::min<int64_t>(db->v.n_refs, s->chunk_refs);
    auto ws_for = [&](int32_t n, size_t* bytes) -> int {
        size_t best = 0;
        for (int32_t m = 1; m <= n; m = m < 64 ? m + 1 : m + 64) {  // the family (and layout) depends on n
            size_t b = 0;
            FID_TRY(cfg->policy == FID_SERVE_FIFO ? fid_topk_workspace_bytes(s->ctx, db, m, cfg->k, &b)
                                                 : fid_topk_mixed_workspace_bytes(s->ctx, db, 0, r_hi0, m,
                                                                                  cfg->k, &b));
            best = std::max(best, b);
            if (m == n) break;
            if (m >= 64 && m + 64 > n) m = n - 64;
        }
        *bytes = best;
        return FID_OK;
    };
    int32_t lo = 0, hi = cfg->max_queries;
    size_t ws = 0;
    while (lo < hi) {  // largest slot count whose state + workspace fit the budget
        const int32_t mid = lo + (hi - lo + 1) / 2;
        size_t w = 0;
        st = ws_for(mid, &w);
        if (st) return cleanup(st);
        if (server_bytes(mid, s->rw, cfg->k, w) <= cfg->hbm_budget) lo = mid;
        else hi = mid - 1;
    }
    if (lo < 1) return cleanup(fail(FID_EBUDGET, "hbm_budget %zu holds no query slot", cfg->hbm_budget));
    s->max_slots = lo;
    st = ws_for(lo, &ws);
    if (st) return cleanup(st);
    s->ws_bytes = ws;
    s->device_bytes = server_bytes(lo, s->rw, cfg->k, ws);
    e = hipMalloc(&s->mem, s->device_bytes);
    if (e != hipSuccess) return cleanup(fail(FID_ENOMEM, "server memory (%zu bytes): %s", s->device_bytes,
                                             hipGetErrorString(e)));
    char* p = static_cast<char*>(s->mem);
    const size_t n = (size_t)lo;
    auto take = [&](size_t bytes) { char* q = p; p += align256(bytes); return q; };
    s->slot_rows = reinterpret_cast<uint64_t*>(take(n * s->rw * 8));
    s->gathered = reinterpret_cast<uint64_t*>(take(n * s->rw * 8));
    s->running = reinterpret_cast<uint64_t*>(take(n * cfg->k * 8));
    s->tidx = reinterpret_cast<int64_t*>(take(n * cfg->k * 8));
    s->tcnt = reinterpret_cast<int32_t*>(take(n * cfg->k * 4));
    s->dslots = reinterpret_cast<int32_t*>(take(4 * n * 4));
    s->bound = reinterpret_cast<uint32_t*>(take(n * 4));
    s->tbound = reinterpret_cast<uint32_t*>(take(n * 4));
    s->ws = take(ws);
    if ((e = hipHostMalloc((void**)&s->hslots, 4 * n * 4, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void**)&s->hcnt, n * cfg->k * 4, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void**)&s->hidx, n * cfg->k * 8, hipHostMallocDefault)) != hipSuccess)
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
    if (r->n_q > s->max_slots)
        return fail(FID_EBUDGET, "request of %d queries exceeds the %d query slots the budget holds", r->n_q,
                    s->max_slots);
    std::lock_guard<std::mutex> g(s->mu);
    if (s->fatal) return fail(s->fatal, "server failed: %s", s->fatal_msg.c_str());
    const uint64_t t = s->next_ticket++;
    Request q;
    q.ticket = t;
    q.r = *r;
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
    (void)hipHostFree(s->hslots);
    (void)hipHostFree(s->hcnt);
    (void)hipHostFree(s->hidx);
    delete s;
    return FID_OK;
}

}  // extern "C"
