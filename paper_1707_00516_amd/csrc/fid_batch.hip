// libfastid ragged batches: many independent top-k comparison jobs (each with
// its own queries, reference slice, loci panel and mode) run as persistent
// launches over shared work queues.
//
// Jobs with enough queries for the matrix cores run on the fp4 kernel in a
// handful of batched launches for all of them together: one staging launch,
// a persistent pass counting each job's seed prefix exactly, one launch
// selecting every query's seed bound (or, for jobs no longer than their
// seed, its top-k), a persistent top-k pass, and one merge launch.  Their
// work items are (job, 128-query tile, run of 512-reference tiles); the
// items of one reference run sit together in the queue of one XCD, so the
// query tiles scanning that run share the XCD's L2.  The remaining jobs
// share the persistent popcount pass described next.
//
// The work of job j is cut into items = (block of <= 16 queries) x (range of
// 64-reference database blocks); item shapes come from a tuning table per
// loci panel.  Every wave of the persistent grid repeatedly takes the next
// item from an atomic counter and runs the popcount scan of Section III-B on
// it (reference words in VGPRs, wave-uniform query words in SGPRs, one logic
// op and one v_bcnt per 32 loci), in 1024-locus chunks with partial counts in
// LDS, so one kernel serves every panel length.  Each (item, query) keeps its
// own k-slot list in LDS; a per-query bound shared through global memory
// (atomicMin of a full list's worst count + 1) lets every item filter with
// the best bound found so far by any item of that query.  The first reference
// range of each query block is queued ahead of the rest so the shared bounds
// tighten early.  A second launch merges the item lists of every query.
#include <algorithm>
#include <cstring>
#include <numeric>

#include "fid_device.hpp"
#include "fid_internal.hpp"

namespace fid {

namespace {

constexpr int kRoutedLanes = 8;        // streams the routed per-call jobs spread over
constexpr int kBatchNW = 32;          // 32-bit words per chunk (1024 loci)
constexpr int kBatchMaxQ = 32;        // queries per item (LDS per wave grows with the largest)
constexpr int kBatchDefaultQ = 16;
constexpr int kBatchMaxK = 128;       // k of a batch (lists live in LDS)
constexpr int kBatchRefreshBlocks = 8;  // blocks between reads of the shared bounds

struct BJob {
    const uint4* words;       // database of the job's panel
    const uint64_t* qsrc;     // packed queries [n_q][row_words]
    int64_t r_lo, r_hi;
    int64_t stage_off;        // first staged word of the job
    int32_t w4;               // 16-byte units per reference row
    int32_t nch;              // 1024-locus chunks
    int32_t qw;               // staged words per query (nch * 32)
    int32_t mode;
    int32_t n_loci;
    int32_t row_words;        // u64 words per packed query row
    int32_t n_q;
    int32_t g0;               // global index of the job's first query
};

struct BItem {
    int64_t b0, b1;           // database blocks [b0, b1)
    int32_t job;
    int32_t q0, q1;           // job-local queries [q0, q1)
    int32_t slot;             // reference range index within the query block
};

struct BQuery {
    int64_t lbase;            // first list key of the query ([slot][k])
    int64_t fbase;            // first fill count of the query ([slot])
    int32_t* cnt;
    int64_t* idx;
    int32_t nslot;
    int32_t n_loci;
};

__device__ __forceinline__ uint32_t load_bound(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Staging of every job's queries: masked 32-bit words, zero padded to whole
// chunks, mixture queries inverted (Eq. 1 as R AND NOT Q).
__global__ void batch_stage_kernel(const BJob* __restrict__ jobs, int32_t n_jobs,
                                   const int64_t* __restrict__ job_word_off, int64_t total,
                                   uint32_t* __restrict__ qs)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        int a = 0, b = n_jobs;  // largest job with job_word_off[job] <= t
        while (b - a > 1) {
            const int m = (a + b) >> 1;
            if (job_word_off[m] <= t) a = m;
            else b = m;
        }
        const BJob& j = jobs[a];
        const int64_t rel = t - job_word_off[a];
        const int64_t i = rel / j.qw;
        const int32_t w = (int32_t)(rel - i * j.qw);
        const int32_t l32 = (j.n_loci + 31) / 32;
        uint32_t v = 0;
        if (w < l32) {
            v = reinterpret_cast<const uint32_t*>(j.qsrc + i * j.row_words)[w];
            if (w == l32 - 1 && (j.n_loci & 31)) v &= (1u << (j.n_loci & 31)) - 1u;
        }
        if (j.mode == FID_MODE_MIXTURE) v = ~v;
        qs[t] = v;
    }
}

template <int MODE>
__device__ void batch_item(const BJob& jb, const BItem& it, const uint32_t* __restrict__ qs,
                           const BQuery* __restrict__ qmeta, uint64_t* __restrict__ lists,
                           uint32_t* __restrict__ fills, uint32_t* __restrict__ gbound, int k,
                           uint64_t* llist, uint16_t* lacc, uint32_t* lthr, uint32_t* lfill)
{
    const int lane = lane_id();
    const int nq = it.q1 - it.q0;
    const int gq0 = jb.g0 + it.q0;
    if (lane < nq) {
        lthr[lane] = load_bound(gbound + gq0 + lane);
        lfill[lane] = 0u;
    }
    wave_lds_sync();
    // (block, chunk) steps in order; the next chunk's reference words are
    // always in flight while the current one is compared
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    // the database pointer comes from a table: name its address space so the
    // loads are global (not flat) loads
    typedef const __attribute__((address_space(1))) u32x4* gptr_u4;
    auto load_chunk = [&](u32x4 (&dst)[kBatchNW / 4], int64_t blk, int c) {
        const gptr_u4 src = (gptr_u4)(jb.words + (size_t)blk * jb.w4 * 64 + lane);
#pragma unroll
        for (int i = 0; i < kBatchNW / 4; ++i) {
            const int u = c * (kBatchNW / 4) + i;
            dst[i] = u < jb.w4 ? src[(size_t)u * 64] : u32x4{0u, 0u, 0u, 0u};
        }
    };
    u32x4 cur[kBatchNW / 4];
    load_chunk(cur, it.b0, 0);
    int since = 0;
    int c = 0;
    for (int64_t blk = it.b0; blk < it.b1;) {
        int cn = c + 1;
        int64_t bn = blk;
        if (cn == jb.nch) {
            cn = 0;
            ++bn;
        }
        u32x4 nxt[kBatchNW / 4];
        if (bn < it.b1) load_chunk(nxt, bn, cn);
        if (c == 0 && ++since == kBatchRefreshBlocks) {
            since = 0;
            if (lane < nq) {
                const uint32_t g = load_bound(gbound + gq0 + lane);
                if (g < lthr[lane]) lthr[lane] = g;
            }
            wave_lds_sync();
        }
        const int64_t r = blk * 64 + lane;
        const bool rin = r >= jb.r_lo && r < jb.r_hi;
        const bool last = c + 1 == jb.nch;
        kptr_u32 qrow = (kptr_u32)(qs + jb.stage_off + (int64_t)it.q0 * jb.qw + c * kBatchNW);
        for (int q = 0; q < nq; ++q, qrow += jb.qw) {
            uint32_t acc = c > 0 ? lacc[q * 64 + lane] : 0u;
#pragma unroll
            for (int g = 0; g < kBatchNW / 16; ++g) {
                const u32x16 qg = ((kptr_u32x16)qrow)[g];  // one 16-dword scalar load
#pragma unroll
                for (int w2 = 0; w2 < 16; ++w2) {
                    const int w = g * 16 + w2;
                    const uint32_t rv = cur[w >> 2][w & 3];
                    const uint32_t x = MODE == FID_MODE_MIXTURE ? (rv & qg[w2]) : (rv ^ qg[w2]);
                    acc = popc_acc(x, acc);
                }
            }
            if (!last) {
                lacc[q * 64 + lane] = (uint16_t)acc;  // a count is at most L < 2^16
                continue;
            }
            const uint64_t m = __builtin_amdgcn_ballot_w64(rin && acc < lthr[q]);
            if (m) {
                topk_insert(llist + q * k, k, blk * 64, acc, m, lthr + q, lfill + q);
                wave_lds_sync();
                // a full list proves k keys with count <= its worst: publish
                if (lane == 0 && lfill[q] == (uint32_t)k)
                    atomicMin(gbound + gq0 + q, lthr[q] + 1u);
            }
        }
        if (bn < it.b1) {
#pragma unroll
            for (int i = 0; i < kBatchNW / 4; ++i) cur[i] = nxt[i];
        }
        blk = bn;
        c = cn;
    }
    wave_lds_sync();
    for (int q = 0; q < nq; ++q) {
        const BQuery& qm = qmeta[gq0 + q];
        const uint32_t fill = lfill[q];
        uint64_t* dst = lists + qm.lbase + (int64_t)it.slot * k;
        for (int i = lane; i < (int)fill; i += 64) dst[i] = llist[q * k + i];
        if (lane == 0) fills[qm.fbase + it.slot] = fill;
    }
    wave_lds_sync();
}

// Persistent scan: every wave takes items from the queue until it is empty.
__global__ __launch_bounds__(kWG) void batch_scan_kernel(
    const BJob* __restrict__ jobs, const BItem* __restrict__ items, int32_t n_items,
    unsigned int* __restrict__ counter, const uint32_t* __restrict__ qs,
    const BQuery* __restrict__ qmeta, uint64_t* __restrict__ lists, uint32_t* __restrict__ fills,
    uint32_t* __restrict__ gbound, int32_t k, int32_t qmax, int32_t lds_bytes_per_wave)
{
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    uint8_t* base = smem + (size_t)wv * lds_bytes_per_wave;
    uint64_t* llist = reinterpret_cast<uint64_t*>(base);
    uint16_t* lacc = reinterpret_cast<uint16_t*>(base + (size_t)qmax * k * 8);
    uint32_t* lthr = reinterpret_cast<uint32_t*>(lacc + qmax * 64);
    uint32_t* lfill = lthr + qmax;
    for (;;) {
        unsigned int n = 0;
        if (lane == 0) n = atomicAdd(counter, 1u);
        const int i = __builtin_amdgcn_readfirstlane((int)__shfl((int)n, 0));
        if (i >= n_items) break;
        const BItem it = items[i];
        const BJob jb = jobs[it.job];
        if (jb.mode == FID_MODE_MIXTURE)
            batch_item<FID_MODE_MIXTURE>(jb, it, qs, qmeta, lists, fills, gbound, k, llist, lacc,
                                         lthr, lfill);
        else
            batch_item<FID_MODE_IDENTITY>(jb, it, qs, qmeta, lists, fills, gbound, k, llist, lacc,
                                          lthr, lfill);
    }
}

__global__ __launch_bounds__(kSelectThreads) void batch_merge_kernel(
    const BQuery* __restrict__ qmeta, const uint64_t* __restrict__ lists,
    const uint32_t* __restrict__ fills, int32_t k)
{
    __shared__ uint64_t s[kSelectSlots];
    __shared__ int nb;
    __shared__ uint32_t part[kSelectThreads];
    extern __shared__ uint32_t off[];  // [nslot + 1] prefix of the fill counts
    const BQuery qm = qmeta[blockIdx.x];
    merge_query_lists(lists + qm.lbase, fills + qm.fbase, qm.nslot, k, qm.n_loci, qm.cnt, qm.idx, s,
                      &nb, part, off);
}

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Per wave: k-slot lists, 16-bit partial counts [q][64], bound and fill per query.
size_t batch_lds_per_wave(int k, int qmax)
{
    return (size_t)qmax * k * 8 + (size_t)qmax * 64 * 2 + 2 * (size_t)qmax * 4;
}

}  // namespace
}  // namespace fid

using namespace fid;

struct fid_batch {
    fid_ctx* ctx;
    int32_t k;
    int32_t n_jobs;
    int64_t n_items;
    int64_t n_queries;
    int64_t n_lists;
    int32_t max_slots;
    int64_t staged_words;
    int32_t grid;
    size_t lds_per_wave;
    int32_t qmax;                    // most queries of one item
    // workspace views
    unsigned int* counter;
    BJob* jobs;
    int64_t* job_word_off;
    BItem* items;
    BQuery* qmeta;
    uint32_t* gbound;
    uint32_t* fills;
    uint32_t* qs;
    uint64_t* lists;
    // jobs routed to the per-call matrix-core path
    std::vector<fid_job> routed;
    std::vector<uint8_t> is_routed;  // per job: 1 = per-call matrix-core top-k
    void* routed_ws;
    size_t routed_ws_bytes;          // one lane's share
    size_t routed_scratch;
    // Routed jobs run on n_lanes streams of their own (job j on lane j mod
    // n_lanes), each with a context, query scratch and workspace share of its
    // own, forked from and joined back to the batch's stream by events, so
    // one job's small kernels (seed, select, merge) overlap another's scan.
    int n_lanes;
    fid_ctx* lane_ctx[kRoutedLanes];
    hipStream_t lane_stream[kRoutedLanes];
    hipEvent_t fork;
    hipEvent_t join[kRoutedLanes];
    hipStream_t capture;
    hipGraph_t graph;
    hipGraphExec_t exec;
    // matrix-core (fp4) jobs, batched
    int32_t f4_jobs;                 // jobs on the batched fp4 passes
    int32_t f4_grid;                 // persistent workgroups
    int32_t f4_loci_max;
    int32_t f4_max_slots;            // most list owners of one query
    int64_t f4_queries, f4_words;    // staged queries, their 32-locus words
    int32_t n_f4_seed_sel, n_f4_direct_sel;
    int64_t f4_seed_q, f4_direct_q;  // queries of each selection
    int64_t f4_merge_q;
    unsigned int* f4_counters;       // [16]: seed pass queues, then scan pass queues
    Fp4BatchSet* f4_seed_sets;
    Fp4BatchSet* f4_scan_sets;
    Fp4BatchItem* f4_seed_items;
    Fp4BatchItem* f4_scan_items;
    int32_t* f4_seed_qoff;           // [9]
    int32_t* f4_scan_qoff;           // [9]
    int64_t n_f4_seed_items, n_f4_scan_items;
    Fp4ExpandJob* f4_expand;
    SelectJob* f4_sel_seed;
    SelectJob* f4_sel_direct;
    BQuery* f4_merge;
    int32_t* f4_qmode;
    int32_t* f4_pcq;
    uint64_t* f4_lists;
    uint32_t* f4_fills;
};

namespace {

struct BatchPlan {
    std::vector<fid_job> routed;
    std::vector<uint8_t> is_routed;      // [n_jobs]
    size_t routed_ws = 0, routed_scratch = 0;
    std::vector<BJob> jobs;
    std::vector<int64_t> job_word_off;  // [n_jobs + 1]
    std::vector<BItem> items;
    std::vector<BQuery> qmeta;
    int64_t n_lists = 0;
    int32_t max_slots = 0;
    int32_t qmax = 1;
    size_t off_counter, off_jobs, off_jwo, off_items, off_qmeta, off_gbound, off_fills, off_qs,
        off_lists, off_routed, total;
    // batched fp4 jobs
    struct F4 {
        int32_t job;                 // index in the caller's job array
        int32_t n_q, n_loci, kpad, tiles, n_slots, qtiles;
        int64_t seed;                // seed prefix (== the slice: counted directly)
        bool direct;
        int64_t g_off, w_off;        // first global query / staged word
        int64_t lbase, fbase;        // first list key / fill of the job in the fp4 lists
        size_t off_qx, off_counts, off_bounds;
    };
    std::vector<F4> f4;
    std::vector<Fp4BatchItem> f4_seed_items, f4_scan_items;
    std::vector<int32_t> f4_seed_qoff, f4_scan_qoff;  // [9] each
    int64_t f4_queries = 0, f4_words = 0, f4_keys = 0, f4_fills = 0;
    int32_t f4_loci_max = 1, f4_max_slots = 0;
    int32_t n_seed_sel = 0, n_direct_sel = 0;
    int64_t seed_q = 0, direct_q = 0, merge_q = 0;
    size_t off_f4_counters, off_f4_sets, off_f4_items, off_f4_qoff, off_f4_expand, off_f4_sel, off_f4_merge,
        off_f4_qmode, off_f4_pcq, off_f4_lists, off_f4_fills;
};

constexpr int32_t kFp4DefaultTiles = 128;  // 512-reference tiles per fp4 work item

// Deal the groups of items (a group: every query tile of one reference run)
// to the 8 XCD queues, largest first onto the least-loaded queue; within a
// queue the groups keep that order and each group's items stay together.
void deal_to_queues(std::vector<std::vector<Fp4BatchItem>>& groups, const std::vector<int64_t>& cost,
                    std::vector<Fp4BatchItem>& items, std::vector<int32_t>& qoff)
{
    std::vector<size_t> order(groups.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
    std::vector<std::vector<size_t>> q(8);
    int64_t load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (size_t g : order) {
        const int x = (int)(std::min_element(load, load + 8) - load);
        q[x].push_back(g);
        load[x] += cost[g];
    }
    items.clear();
    qoff.assign(9, 0);
    for (int x = 0; x < 8; ++x) {
        qoff[x] = (int32_t)items.size();
        for (size_t g : q[x]) items.insert(items.end(), groups[g].begin(), groups[g].end());
    }
    qoff[8] = (int32_t)items.size();
}

const fid_tune* find_tune(const fid_tune* tune, int32_t n_tune, int32_t n_loci)
{
    const fid_tune* any = nullptr;
    for (int32_t i = 0; i < n_tune; ++i) {
        if (tune[i].n_loci == n_loci) return &tune[i];
        if (tune[i].n_loci == 0 && !any) any = &tune[i];
    }
    return any;
}

int plan_batch(const fid_ctx* ctx, const fid_job* jobs, int32_t n_jobs, int32_t k,
               const fid_tune* tune, int32_t n_tune, BatchPlan* P)
{
    if (!ctx) return fail(FID_EINVAL, "ctx is NULL");
    if (!jobs || n_jobs < 1) return fail(FID_EINVAL, "no jobs");
    if (k < 1 || k > kBatchMaxK) return fail(FID_EINVAL, "batch k=%d out of [1, %d]", k, kBatchMaxK);
    if (n_tune < 0 || (n_tune > 0 && !tune)) return fail(FID_EINVAL, "bad tuning table");
    for (int32_t i = 0; i < n_tune; ++i)
        if (tune[i].q_per_item < 1 || tune[i].q_per_item > kBatchMaxQ || tune[i].blocks_per_item < 1 ||
            tune[i].fp4_tiles < 0)
            return fail(FID_EINVAL, "tuning entry %d: q_per_item in [1, %d], blocks_per_item >= 1, fp4_tiles >= 0",
                        i, kBatchMaxQ);
    P->jobs.resize(n_jobs);
    P->job_word_off.assign(n_jobs + 1, 0);
    P->is_routed.assign(n_jobs, 0);
    int64_t g = 0, words = 0;
    struct Seg { BItem it; int64_t cost; bool seed; };
    std::vector<Seg> segs;
    for (int32_t j = 0; j < n_jobs; ++j) {
        const fid_job& J = jobs[j];
        if (!J.db) return fail(FID_EINVAL, "job %d: db is NULL", j);
        if (J.db->device != ctx->device) return fail(FID_EINVAL, "job %d: db on another device", j);
        if (J.r_lo < 0 || J.r_hi <= J.r_lo || J.r_hi > J.db->v.n_refs)
            return fail(FID_EINVAL, "job %d: reference slice [%lld, %lld) outside [0, %lld)", j,
                        (long long)J.r_lo, (long long)J.r_hi, (long long)J.db->v.n_refs);
        if (!J.q_dev || !aligned16(J.q_dev)) return fail(FID_EINVAL, "job %d: query pointer NULL or unaligned", j);
        if (J.n_q < 1 || J.n_q > (1 << 24)) return fail(FID_EINVAL, "job %d: n_q=%d", j, J.n_q);
        if (J.mode != FID_MODE_MIXTURE && J.mode != FID_MODE_IDENTITY)
            return fail(FID_EINVAL, "job %d: bad mode %d", j, J.mode);
        if (!J.cnt_dev || !J.idx_dev) return fail(FID_EINVAL, "job %d: NULL output", j);
        // Every job whose rows the fp4 scan holds joins the batched fp4
        // passes, whatever its query count (the family AUTO picks for a
        // full query tile): a tile of few queries skips its empty row
        // blocks, and the persistent passes overlap such jobs' database-
        // bound items with the compute-bound ones.  A backend forced on the
        // context decides instead: int8 jobs run as per-call top-k inside
        // the batch, popcount jobs share the persistent popcount launch.
        if (auto_family(ctx, J.db, std::max(J.n_q, fp4_queries_per_wg())) == FID_BACKEND_MFMA_FP4) {
            BatchPlan::F4 f{};
            f.job = j;
            f.n_q = J.n_q;
            f.n_loci = J.db->v.n_loci;
            f.kpad = fp4_kpad(f.n_loci);
            const fid_tune* t = find_tune(tune, n_tune, f.n_loci);
            f.tiles = t && t->fp4_tiles > 0 ? t->fp4_tiles : kFp4DefaultTiles;
            f.seed = seed_prefix(J.r_hi - J.r_lo, FID_BACKEND_MFMA_FP4, J.n_q);
            f.direct = f.seed == J.r_hi - J.r_lo;
            f.qtiles = (f.n_q + fp4_queries_per_wg() - 1) / fp4_queries_per_wg();
            const int64_t base = (J.r_lo / kDbTileRefs) * kDbTileRefs;
            const int64_t ntiles = (J.r_hi - base + fp4_refs_per_wg() - 1) / fp4_refs_per_wg();
            f.n_slots = f.direct ? 0 : (int32_t)std::min<int64_t>((ntiles + f.tiles - 1) / f.tiles,
                                                                kMaxListWorkers / fp4_list_workers_per_wg());
            f.g_off = P->f4_queries;
            f.w_off = P->f4_words;
            P->f4_queries += f.n_q;
            P->f4_words += (int64_t)f.n_q * (f.kpad / 32);
            P->f4_loci_max = std::max(P->f4_loci_max, f.n_loci);
            if (!f.direct) {
                const int32_t owners = f.n_slots * fp4_list_workers_per_wg();
                f.lbase = P->f4_keys;
                f.fbase = P->f4_fills;
                P->f4_keys += (int64_t)f.n_q * owners * k;
                P->f4_fills += (int64_t)f.n_q * owners;
                P->f4_max_slots = std::max(P->f4_max_slots, owners);
                P->n_seed_sel++;
                P->seed_q += f.n_q;
                P->merge_q += f.n_q;
            } else {
                P->n_direct_sel++;
                P->direct_q += f.n_q;
            }
            P->f4.push_back(f);
            P->is_routed[j] = 1;
            P->job_word_off[j] = words;  // an empty popcount staging segment
            continue;
        }
        if (batch_routes_to_matrix_cores(ctx, J.db, J.n_q)) {
            size_t w = 0;
            FID_TRY(fid_topk_range_workspace_bytes(const_cast<fid_ctx*>(ctx), J.db, J.r_lo, J.r_hi, J.n_q, k, &w));
            P->routed_ws = std::max(P->routed_ws, w);
            P->routed_scratch = std::max(P->routed_scratch, query_scratch_bytes(ctx, J.db, J.n_q));
            P->routed.push_back(J);
            P->is_routed[j] = 1;
            P->job_word_off[j] = words;  // an empty staging segment
            continue;
        }
        BJob& b = P->jobs[j];
        b.words = J.db->v.words;
        b.qsrc = J.q_dev;
        b.r_lo = J.r_lo;
        b.r_hi = J.r_hi;
        b.w4 = J.db->v.w4;
        b.n_loci = J.db->v.n_loci;
        b.nch = (b.n_loci + 32 * kBatchNW - 1) / (32 * kBatchNW);
        b.qw = b.nch * kBatchNW;
        b.mode = J.mode;
        b.row_words = J.db->row_words;
        b.n_q = J.n_q;
        b.g0 = (int32_t)g;
        b.stage_off = words;
        P->job_word_off[j] = words;
        words += (int64_t)J.n_q * b.qw;
        const fid_tune* t = find_tune(tune, n_tune, b.n_loci);
        const int qpi = t ? t->q_per_item : kBatchDefaultQ;
        const int64_t bpi = t ? t->blocks_per_item : 64;
        const int64_t blk_lo = J.r_lo / 64, blk_hi = (J.r_hi + 63) / 64, nblk = blk_hi - blk_lo;
        int64_t nsplit = (nblk + bpi - 1) / bpi;
        if (nsplit > kMaxListWorkers) nsplit = kMaxListWorkers;
        const int nqb = (J.n_q + qpi - 1) / qpi;
        for (int qb = 0; qb < nqb; ++qb) {
            const int q0 = (int)((int64_t)J.n_q * qb / nqb), q1 = (int)((int64_t)J.n_q * (qb + 1) / nqb);
            P->qmax = std::max(P->qmax, q1 - q0);
            for (int64_t s = 0; s < nsplit; ++s) {
                Seg sg;
                sg.it.b0 = blk_lo + nblk * s / nsplit;
                sg.it.b1 = blk_lo + nblk * (s + 1) / nsplit;
                sg.it.job = j;
                sg.it.q0 = q0;
                sg.it.q1 = q1;
                sg.it.slot = (int32_t)s;
                sg.cost = (int64_t)(q1 - q0) * (sg.it.b1 - sg.it.b0) * b.nch;
                sg.seed = s == 0;
                segs.push_back(sg);
            }
        }
        for (int32_t q = 0; q < J.n_q; ++q) {
            BQuery m{};
            m.nslot = (int32_t)nsplit;
            m.n_loci = b.n_loci;
            m.lbase = P->n_lists * k;
            m.fbase = P->n_lists;
            m.cnt = J.cnt_dev + (size_t)q * k;
            m.idx = J.idx_dev + (size_t)q * k;
            P->qmeta.push_back(m);
            P->n_lists += nsplit;
        }
        P->max_slots = std::max<int32_t>(P->max_slots, (int32_t)nsplit);
        g += J.n_q;
    }
    P->job_word_off[n_jobs] = words;
    if (segs.size() > (size_t)INT32_MAX) return fail(FID_EINVAL, "too many work items");
    // seed ranges first, then longest-processing-time order
    std::stable_sort(segs.begin(), segs.end(), [](const Seg& a, const Seg& b) {
        if (a.seed != b.seed) return a.seed;
        return a.cost > b.cost;
    });
    P->items.resize(segs.size());
    for (size_t i = 0; i < segs.size(); ++i) P->items[i] = segs[i].it;
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off += align256(bytes); return o; };
    P->off_counter = take(256);
    P->off_jobs = take(P->jobs.size() * sizeof(BJob));
    P->off_jwo = take(P->job_word_off.size() * sizeof(int64_t));
    P->off_items = take(P->items.size() * sizeof(BItem));
    P->off_qmeta = take(P->qmeta.size() * sizeof(BQuery));
    P->off_gbound = take((size_t)g * sizeof(uint32_t));
    P->off_fills = take((size_t)P->n_lists * sizeof(uint32_t));
    P->off_qs = take((size_t)words * sizeof(uint32_t));
    P->off_lists = take((size_t)P->n_lists * k * sizeof(uint64_t));
    P->routed_ws = align256(P->routed_ws);  // each lane's share starts 256-byte aligned
    P->off_routed = take(P->routed_ws * (size_t)std::min<size_t>(kRoutedLanes, P->routed.size()));
    // batched fp4 jobs: tables, then per-job staged queries, seed counts and
    // bounds, then the lists
    const size_t nf = P->f4.size();
    if (nf) {
        std::vector<std::vector<Fp4BatchItem>> groups;
        std::vector<int64_t> cost;
        auto add_runs = [&](int32_t set, const BatchPlan::F4& f, int64_t ntiles, int32_t n_slots) {
            for (int32_t sl = 0; sl < n_slots; ++sl) {
                std::vector<Fp4BatchItem> g;
                const int64_t tb = ntiles * sl / n_slots, te = ntiles * (sl + 1) / n_slots;
                for (int32_t qt = 0; qt < f.qtiles; ++qt) g.push_back(Fp4BatchItem{set, qt, sl, 0, tb, te});
                groups.push_back(std::move(g));
                cost.push_back((int64_t)f.qtiles * (te - tb) * f.kpad);
            }
        };
        for (size_t i = 0; i < nf; ++i) {  // seed pass: each job's seed prefix
            const BatchPlan::F4& f = P->f4[i];
            const fid_job& J = jobs[f.job];
            const int64_t base = (J.r_lo / kDbTileRefs) * kDbTileRefs;
            const int64_t ntiles = (J.r_lo + f.seed - base + fp4_refs_per_wg() - 1) / fp4_refs_per_wg();
            add_runs((int32_t)i, f, ntiles, (int32_t)((ntiles + f.tiles - 1) / f.tiles));
        }
        deal_to_queues(groups, cost, P->f4_seed_items, P->f4_seed_qoff);
        groups.clear();
        cost.clear();
        for (size_t i = 0; i < nf; ++i) {  // top-k pass
            const BatchPlan::F4& f = P->f4[i];
            if (f.direct) continue;
            const fid_job& J = jobs[f.job];
            const int64_t base = (J.r_lo / kDbTileRefs) * kDbTileRefs;
            const int64_t ntiles = (J.r_hi - base + fp4_refs_per_wg() - 1) / fp4_refs_per_wg();
            add_runs((int32_t)i, f, ntiles, f.n_slots);
        }
        deal_to_queues(groups, cost, P->f4_scan_items, P->f4_scan_qoff);
        if (P->f4_seed_items.size() + P->f4_scan_items.size() > (size_t)INT32_MAX)
            return fail(FID_EINVAL, "too many fp4 work items");
        P->off_f4_counters = take(16 * sizeof(uint32_t));
        P->off_f4_sets = take(2 * nf * sizeof(Fp4BatchSet));
        P->off_f4_items = take((P->f4_seed_items.size() + P->f4_scan_items.size()) * sizeof(Fp4BatchItem));
        P->off_f4_qoff = take(18 * sizeof(int32_t));
        P->off_f4_expand = take(nf * sizeof(Fp4ExpandJob));
        P->off_f4_sel = take(nf * sizeof(SelectJob));
        P->off_f4_merge = take((size_t)P->merge_q * sizeof(BQuery));
        P->off_f4_qmode = take((size_t)P->f4_queries * sizeof(int32_t));
        P->off_f4_pcq = take((size_t)P->f4_queries * sizeof(int32_t));
        for (BatchPlan::F4& f : P->f4) {
            f.off_qx = take((size_t)f.n_q * (f.kpad / 2));
            f.off_counts = take((size_t)f.n_q * (size_t)f.seed * sizeof(int32_t));
            f.off_bounds = f.direct ? 0 : take((size_t)f.n_q * (1 + 2 * kWitLevels) * sizeof(uint32_t));
        }
        P->off_f4_lists = take((size_t)P->f4_keys * sizeof(uint64_t));
        P->off_f4_fills = take((size_t)P->f4_fills * sizeof(uint32_t));
    }
    P->total = off;
    return FID_OK;
}

int enqueue_persistent(fid_batch* b, hipStream_t s, bool timed);

int enqueue_fp4(fid_batch* b, hipStream_t s, bool timed);

int enqueue_batch(fid_batch* b, hipStream_t s, bool timed)
{
    if (b->n_items > 0) FID_TRY(enqueue_persistent(b, s, timed));
    if (b->f4_jobs > 0) FID_TRY(enqueue_fp4(b, s, timed));
    if (b->routed.empty()) return FID_OK;
    // routed jobs: per-call top-k, spread over the lanes (forked from s after
    // the persistent launch, so the lanes fill the machine around it)
    FID_HIP(hipEventRecord(b->fork, s), "hipEventRecord");
    for (int l = 0; l < b->n_lanes; ++l)
        FID_HIP(hipStreamWaitEvent(b->lane_stream[l], b->fork, 0), "hipStreamWaitEvent");
    int st = FID_OK;
    for (size_t i = 0; i < b->routed.size() && !st; ++i) {
        const fid_job& J = b->routed[i];
        const int l = (int)(i % (size_t)b->n_lanes);
        st = fid_compare_topk_range(b->lane_ctx[l], J.db, J.r_lo, J.r_hi, J.q_dev, J.n_q, J.mode, b->k,
                                    static_cast<char*>(b->routed_ws) + (size_t)l * b->routed_ws_bytes,
                                    b->routed_ws_bytes, J.cnt_dev, J.idx_dev);
    }
    // join every lane back, also after a failure (nothing is left forked)
    for (int l = 0; l < b->n_lanes; ++l) {
        hipError_t e = hipEventRecord(b->join[l], b->lane_stream[l]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, b->join[l], 0);
        if (e != hipSuccess && !st) st = hip_fail(e, "lane join");
    }
    return st;
}

// The batched fp4 passes (no host synchronisation, so a graph can hold them).
int enqueue_fp4(fid_batch* b, hipStream_t s, bool timed)
{
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, s, b->f4_counters, (int64_t)16, 0u);
    FID_HIP(hipGetLastError(), "fill launch");
    FID_HIP(launch_expand_batch_fp4(b->f4_expand, b->f4_jobs, b->f4_words, b->f4_queries, b->f4_qmode, b->f4_pcq, s),
            "batched staging launch");
    FID_HIP(launch_fp4_batch(EPI_FULL, b->f4_seed_sets, b->f4_seed_items, b->f4_seed_qoff, b->f4_counters,
                             b->f4_grid, s), "batched seed pass launch");
    FID_HIP(launch_seed_select_batch(b->f4_sel_seed, b->n_f4_seed_sel, b->f4_seed_q, b->f4_loci_max, s),
            "batched seed select launch");
    FID_HIP(launch_select_counts_batch(b->f4_sel_direct, b->n_f4_direct_sel, b->f4_direct_q, s),
            "batched direct select launch");
    if (b->n_f4_scan_items > 0) {
        hipEvent_t e1 = nullptr;
        if (timed) FID_TRY(timing_begin(b->ctx, s, &e1));
        FID_HIP(launch_fp4_batch(EPI_TOPK, b->f4_scan_sets, b->f4_scan_items, b->f4_scan_qoff, b->f4_counters + 8,
                                 b->f4_grid, s), "batched top-k pass launch");
        if (e1) FID_HIP(hipEventRecord(e1, s), "hipEventRecord");
        hipLaunchKernelGGL(batch_merge_kernel, dim3((unsigned)b->f4_merge_q), dim3(kSelectThreads),
                           (size_t)(b->f4_max_slots + 1) * sizeof(uint32_t), s, b->f4_merge, b->f4_lists,
                           b->f4_fills, b->k);
        FID_HIP(hipGetLastError(), "batched merge launch");
    }
    return FID_OK;
}

int enqueue_persistent(fid_batch* b, hipStream_t s, bool timed)
{
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, s, b->counter, (int64_t)1, 0u);
    FID_HIP(hipGetLastError(), "fill launch");
    int64_t blocks = std::min<int64_t>((b->n_queries + 255) / 256, 65536);
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, s,
                       b->gbound, b->n_queries, 0xFFFFFFFFu);
    FID_HIP(hipGetLastError(), "fill launch");
    blocks = std::min<int64_t>((b->staged_words + 255) / 256, 65536);
    hipLaunchKernelGGL(batch_stage_kernel, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, s,
                       b->jobs, b->n_jobs, b->job_word_off, b->staged_words, b->qs);
    FID_HIP(hipGetLastError(), "batch stage launch");
    hipEvent_t e1 = nullptr;
    if (timed) FID_TRY(timing_begin(b->ctx, s, &e1));
    hipLaunchKernelGGL(batch_scan_kernel, dim3(b->grid), dim3(kWG), b->lds_per_wave * kWavesPerWG, s,
                       b->jobs, b->items, (int32_t)b->n_items, b->counter, b->qs, b->qmeta, b->lists,
                       b->fills, b->gbound, b->k, b->qmax, (int32_t)b->lds_per_wave);
    FID_HIP(hipGetLastError(), "batch scan launch");
    if (e1) FID_HIP(hipEventRecord(e1, s), "hipEventRecord");
    hipLaunchKernelGGL(batch_merge_kernel, dim3((unsigned)b->n_queries), dim3(kSelectThreads),
                       (size_t)(b->max_slots + 1) * sizeof(uint32_t), s, b->qmeta, b->lists, b->fills,
                       b->k);
    FID_HIP(hipGetLastError(), "batch merge launch");
    return FID_OK;
}

}  // namespace

extern "C" {

int fid_batch_workspace_bytes(fid_ctx* ctx, const fid_job* jobs, int32_t n_jobs, int32_t k,
                              const fid_tune* tune, int32_t n_tune, size_t* bytes)
{
    if (!bytes) return fail(FID_EINVAL, "bytes is NULL");
    BatchPlan P;
    FID_TRY(plan_batch(ctx, jobs, n_jobs, k, tune, n_tune, &P));
    *bytes = P.total;
    return FID_OK;
}

int fid_batch_create(fid_ctx* ctx, const fid_job* jobs, int32_t n_jobs, int32_t k,
                     const fid_tune* tune, int32_t n_tune, void* ws_dev, size_t ws_bytes,
                     fid_batch** out)
{
    if (!out) return fail(FID_EINVAL, "out is NULL");
    *out = nullptr;
    BatchPlan P;
    FID_TRY(plan_batch(ctx, jobs, n_jobs, k, tune, n_tune, &P));
    if (!ws_dev || !aligned16(ws_dev)) return fail(FID_EINVAL, "workspace NULL or not 16-byte aligned");
    if (ws_bytes < P.total) return fail(FID_ENOMEM, "workspace %zu bytes < required %zu", ws_bytes, P.total);
    if ((int64_t)P.qmeta.size() > INT32_MAX) return fail(FID_EINVAL, "too many queries");
    FID_TRY(set_device(ctx));
    char* ws = static_cast<char*>(ws_dev);
    fid_batch* b = new fid_batch{};
    b->ctx = ctx;
    b->k = k;
    b->n_jobs = n_jobs;
    b->n_items = (int64_t)P.items.size();
    b->n_queries = (int64_t)P.qmeta.size();
    b->n_lists = P.n_lists;
    b->max_slots = P.max_slots;
    b->staged_words = P.job_word_off.back();
    b->qmax = P.qmax;
    b->lds_per_wave = batch_lds_per_wave(k, P.qmax);
    // persistent grid: as many workgroups as can be resident at once
    const int wpc = env_int("FASTID_BATCH_WAVES_PER_CU", 24, 4, 64);
    const int by_lds = (int)(163840 / (b->lds_per_wave * kWavesPerWG));
    b->grid = std::max(1, ctx->num_cus * std::max(1, std::min(wpc / kWavesPerWG, by_lds)));
    b->counter = reinterpret_cast<unsigned int*>(ws + P.off_counter);
    b->jobs = reinterpret_cast<BJob*>(ws + P.off_jobs);
    b->job_word_off = reinterpret_cast<int64_t*>(ws + P.off_jwo);
    b->items = reinterpret_cast<BItem*>(ws + P.off_items);
    b->qmeta = reinterpret_cast<BQuery*>(ws + P.off_qmeta);
    b->gbound = reinterpret_cast<uint32_t*>(ws + P.off_gbound);
    b->fills = reinterpret_cast<uint32_t*>(ws + P.off_fills);
    b->qs = reinterpret_cast<uint32_t*>(ws + P.off_qs);
    b->lists = reinterpret_cast<uint64_t*>(ws + P.off_lists);
    b->routed = P.routed;
    b->is_routed = P.is_routed;
    b->routed_ws = ws + P.off_routed;
    b->routed_ws_bytes = P.routed_ws;
    b->routed_scratch = P.routed_scratch;
    auto up = [&](void* dst, const void* src, size_t n) -> int {
        if (n) FID_HIP(hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, ctx->stream), "table upload");
        return FID_OK;
    };
    // batched fp4 jobs: device tables with this workspace's addresses
    b->f4_jobs = (int32_t)P.f4.size();
    std::vector<Fp4BatchSet> f4_sets;
    std::vector<Fp4ExpandJob> f4_expand;
    std::vector<SelectJob> f4_sel;
    std::vector<BQuery> f4_merge;
    std::vector<int32_t> f4_qmode, f4_qoff;
    if (b->f4_jobs) {
        b->f4_grid = ctx->num_cus;  // one workgroup per CU: the tile's LDS and registers fill it
        b->f4_loci_max = P.f4_loci_max;
        b->f4_max_slots = P.f4_max_slots;
        b->f4_queries = P.f4_queries;
        b->f4_words = P.f4_words;
        b->f4_counters = reinterpret_cast<unsigned int*>(ws + P.off_f4_counters);
        b->f4_seed_sets = reinterpret_cast<Fp4BatchSet*>(ws + P.off_f4_sets);
        b->f4_scan_sets = b->f4_seed_sets + P.f4.size();
        b->f4_seed_items = reinterpret_cast<Fp4BatchItem*>(ws + P.off_f4_items);
        b->f4_scan_items = b->f4_seed_items + P.f4_seed_items.size();
        b->n_f4_seed_items = (int64_t)P.f4_seed_items.size();
        b->n_f4_scan_items = (int64_t)P.f4_scan_items.size();
        b->f4_seed_qoff = reinterpret_cast<int32_t*>(ws + P.off_f4_qoff);
        b->f4_scan_qoff = b->f4_seed_qoff + 9;
        b->f4_expand = reinterpret_cast<Fp4ExpandJob*>(ws + P.off_f4_expand);
        b->f4_qmode = reinterpret_cast<int32_t*>(ws + P.off_f4_qmode);
        b->f4_pcq = reinterpret_cast<int32_t*>(ws + P.off_f4_pcq);
        b->f4_lists = reinterpret_cast<uint64_t*>(ws + P.off_f4_lists);
        b->f4_fills = reinterpret_cast<uint32_t*>(ws + P.off_f4_fills);
        b->f4_merge = reinterpret_cast<BQuery*>(ws + P.off_f4_merge);
        b->f4_merge_q = P.merge_q;
        f4_sets.resize(2 * P.f4.size());
        std::vector<SelectJob> seed_sel, direct_sel;
        int64_t seed_q = 0, direct_q = 0;
        for (size_t i = 0; i < P.f4.size(); ++i) {
            const BatchPlan::F4& f = P.f4[i];
            const fid_job& J = jobs[f.job];
            uint8_t* qx = reinterpret_cast<uint8_t*>(ws + f.off_qx);
            int32_t* counts = reinterpret_cast<int32_t*>(ws + f.off_counts);
            uint32_t* bounds = f.direct ? nullptr : reinterpret_cast<uint32_t*>(ws + f.off_bounds);
            Fp4BatchSet S{};
            S.db = J.db->v;
            S.r_lo = J.r_lo;
            S.qx = qx;
            S.kpad = f.kpad;
            S.pcq = b->f4_pcq + f.g_off;
            S.qmode = b->f4_qmode + f.g_off;
            S.n_q = f.n_q;
            S.k = k;
            Fp4BatchSet seed = S;  // exact counts of the seed prefix
            seed.r_hi = J.r_lo + f.seed;
            seed.out = counts;
            seed.ld = f.seed;
            seed.out_r_base = J.r_lo;
            f4_sets[i] = seed;
            Fp4BatchSet scan = S;  // top-k of the whole slice
            scan.r_hi = J.r_hi;
            scan.n_slots = f.n_slots;
            if (!f.direct) {
                scan.lists = b->f4_lists + f.lbase;
                scan.fills = b->f4_fills + f.fbase;
                scan.thr_init = bounds;
                scan.level = bounds + f.n_q;
                scan.wit = bounds + (size_t)(1 + kWitLevels) * f.n_q;
            }
            f4_sets[P.f4.size() + i] = scan;
            f4_expand.push_back(Fp4ExpandJob{J.q_dev, f.n_q, J.db->row_words, f.n_loci, f.kpad, f.g_off, f.w_off, qx});
            for (int32_t q = 0; q < f.n_q; ++q) f4_qmode.push_back(J.mode);
            SelectJob sj{};
            sj.counts = counts;
            sj.n_cols = f.seed;
            sj.n_q = f.n_q;
            sj.k = k;
            sj.n_loci = f.n_loci;
            if (f.direct) {
                sj.q_off = direct_q;
                sj.idx_base = J.r_lo;
                sj.cnt = J.cnt_dev;
                sj.idx = J.idx_dev;
                direct_q += f.n_q;
                direct_sel.push_back(sj);
            } else {
                sj.q_off = seed_q;
                sj.thr_init = bounds;
                sj.level = bounds + f.n_q;
                sj.wit = bounds + (size_t)(1 + kWitLevels) * f.n_q;
                seed_q += f.n_q;
                seed_sel.push_back(sj);
                const int32_t owners = f.n_slots * fp4_list_workers_per_wg();
                for (int32_t q = 0; q < f.n_q; ++q) {
                    BQuery m{};
                    m.lbase = f.lbase + (int64_t)q * owners * k;
                    m.fbase = f.fbase + (int64_t)q * owners;
                    m.cnt = J.cnt_dev + (size_t)q * k;
                    m.idx = J.idx_dev + (size_t)q * k;
                    m.nslot = owners;
                    m.n_loci = f.n_loci;
                    f4_merge.push_back(m);
                }
            }
        }
        b->n_f4_seed_sel = (int32_t)seed_sel.size();
        b->n_f4_direct_sel = (int32_t)direct_sel.size();
        b->f4_seed_q = seed_q;
        b->f4_direct_q = direct_q;
        b->f4_sel_seed = reinterpret_cast<SelectJob*>(ws + P.off_f4_sel);
        b->f4_sel_direct = b->f4_sel_seed + seed_sel.size();
        f4_sel = seed_sel;
        f4_sel.insert(f4_sel.end(), direct_sel.begin(), direct_sel.end());
        f4_qoff = P.f4_seed_qoff;
        f4_qoff.insert(f4_qoff.end(), P.f4_scan_qoff.begin(), P.f4_scan_qoff.end());
    }
    int st = up(b->jobs, P.jobs.data(), P.jobs.size() * sizeof(BJob));
    if (!st && b->f4_jobs) {
        st = up(b->f4_seed_sets, f4_sets.data(), f4_sets.size() * sizeof(Fp4BatchSet));
        if (!st) st = up(b->f4_seed_items, P.f4_seed_items.data(), P.f4_seed_items.size() * sizeof(Fp4BatchItem));
        if (!st) st = up(b->f4_scan_items, P.f4_scan_items.data(), P.f4_scan_items.size() * sizeof(Fp4BatchItem));
        if (!st) st = up(b->f4_seed_qoff, f4_qoff.data(), f4_qoff.size() * sizeof(int32_t));
        if (!st) st = up(b->f4_expand, f4_expand.data(), f4_expand.size() * sizeof(Fp4ExpandJob));
        if (!st) st = up(b->f4_sel_seed, f4_sel.data(), f4_sel.size() * sizeof(SelectJob));
        if (!st) st = up(b->f4_merge, f4_merge.data(), f4_merge.size() * sizeof(BQuery));
        if (!st) st = up(b->f4_qmode, f4_qmode.data(), f4_qmode.size() * sizeof(int32_t));
    }
    if (!st) st = up(b->job_word_off, P.job_word_off.data(), P.job_word_off.size() * sizeof(int64_t));
    if (!st) st = up(b->items, P.items.data(), P.items.size() * sizeof(BItem));
    if (!st) st = up(b->qmeta, P.qmeta.data(), P.qmeta.size() * sizeof(BQuery));
    if (!st) {
        const hipError_t e = hipStreamSynchronize(ctx->stream);  // host tables go out of scope
        if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
    }
    // routed lanes: their own streams (default priority), contexts with the
    // batch context's device and backend, and query scratch reserved now, so
    // that nothing allocates while the batch runs or is captured
    b->n_lanes = (int)std::min<size_t>(kRoutedLanes, b->routed.size());
    if (!st && b->n_lanes > 0) {
        hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
        if (e != hipSuccess) st = hip_fail(e, "hipEventCreate");
    }
    for (int l = 0; l < b->n_lanes && !st; ++l) {
        hipError_t e = hipStreamCreateWithFlags(&b->lane_stream[l], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[l], hipEventDisableTiming);
        if (e != hipSuccess) {
            st = hip_fail(e, "lane stream");
            break;
        }
        st = fid_ctx_create(&b->lane_ctx[l], ctx->device, b->lane_stream[l]);
        if (!st) {
            b->lane_ctx[l]->backend = ctx->backend;
            st = scratch_reserve(b->lane_ctx[l], b->routed_scratch);
        }
    }
    if (st) {
        (void)fid_batch_destroy(b);
        return st;
    }
    // the opt-in covers the whole 160 KiB, so that no later batch lowers the
    // limit an earlier one's launches need
    const hipError_t e = lds_opt_in<&batch_scan_kernel>(163840);
    if (e != hipSuccess) {
        (void)fid_batch_destroy(b);
        return hip_fail(e, "hipFuncSetAttribute");
    }
    *out = b;
    return FID_OK;
}

int fid_batch_run(fid_batch* b, int use_graph)
{
    if (!b) return fail(FID_EINVAL, "batch is NULL");
    fid_ctx* ctx = b->ctx;
    FID_TRY(set_device(ctx));
    if (!use_graph) return enqueue_batch(b, ctx->stream, true);
    if (!b->exec) {
        // Capture the whole batch once (on a private stream; the null stream
        // cannot be captured), then replay it on the context's stream.
        if (!b->capture)
            FID_HIP(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking), "hipStreamCreate");
        // relaxed: the routed calls may set kernel attributes while capturing
        // (their scratch was reserved at creation, so nothing allocates)
        FID_HIP(hipStreamBeginCapture(b->capture, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
        const int st = enqueue_batch(b, b->capture, false);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->capture, &g);
        if (st) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        FID_HIP(e, "hipStreamEndCapture");
        b->graph = g;
        FID_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    }
    FID_HIP(hipGraphLaunch(b->exec, ctx->stream), "hipGraphLaunch");
    return FID_OK;
}

int fid_batch_info(const fid_batch* b, int64_t* n_items, int64_t* n_lists, int32_t* grid,
                   int32_t* n_routed)
{
    if (!b) return fail(FID_EINVAL, "batch is NULL");
    if (n_items) *n_items = b->n_items;
    if (n_lists) *n_lists = b->n_lists;
    if (grid) *grid = b->grid;
    if (n_routed) *n_routed = (int32_t)b->routed.size() + b->f4_jobs;
    return FID_OK;
}

int fid_batch_job_routed(const fid_batch* b, int32_t job, int32_t* routed)
{
    if (!b || !routed) return fail(FID_EINVAL, "batch or output is NULL");
    if (job < 0 || job >= b->n_jobs) return fail(FID_EINVAL, "job %d outside [0, %d)", job, b->n_jobs);
    *routed = b->is_routed[job];
    return FID_OK;
}

int fid_batch_destroy(fid_batch* b)
{
    if (!b) return FID_OK;
    (void)set_device(b->ctx);
    (void)hipStreamSynchronize(b->ctx->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    for (int l = 0; l < kRoutedLanes; ++l) {
        if (b->lane_stream[l]) (void)hipStreamSynchronize(b->lane_stream[l]);
        if (b->lane_ctx[l]) (void)fid_ctx_destroy(b->lane_ctx[l]);
        if (b->lane_stream[l]) (void)hipStreamDestroy(b->lane_stream[l]);
        if (b->join[l]) (void)hipEventDestroy(b->join[l]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    delete b;
    return FID_OK;
}

}  // extern "C"
