// Host-side internals of libfastid shared by the C-ABI translation units:
// the context and database handles, error reporting and small utilities.
#pragma once

#include <string>
#include <utility>
#include <vector>

#include "fid_common.hpp"

struct fid_ctx {
    int device;
    hipStream_t stream;
    int num_cus;
    int backend;         // fid_backend
    void* scratch;       // status words, staged or expanded queries
    size_t scratch_bytes;
    bool timing;         // record events around each call's main scan kernel
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    size_t events_used;
    void* fixed_scratch;  // this device's address of the library's fixed scratch array
};

struct fid_db {
    int device;
    fid::DbView v;
    int32_t row_words;
    void* mem;
    size_t bytes;
};

namespace fid {

// Record a printf-style message as the thread's last error; returns st.
int fail(int st, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int env_int(const char* name, int dflt, int lo, int hi);
int set_device(const fid_ctx* ctx);
// With timing enabled, record the start event of one timed kernel on s and
// return the end event to record after it (else *end = nullptr).
int timing_begin(fid_ctx* ctx, hipStream_t s, hipEvent_t* end);

// fid_compare_topk_mixed with a caller-known exclusive bound per query
// (bound_dev, device [n_q]); seed = false skips the seed pass and filters
// with the bound alone, seed = true takes the tighter of the two.
int topk_range_bounded(fid_ctx* ctx, const fid_db* db, int64_t r_lo, int64_t r_hi, const uint64_t* q_dev,
                       const int32_t* modes_dev, int32_t n_q, int32_t k, void* ws_dev, size_t ws_bytes,
                       int32_t* cnt_dev, int64_t* idx_dev, const uint32_t* bound_dev, bool seed);
// Threshold hits of queries x references [r_lo, r_hi) appended to (keys,
// vals) with the shared counter (keys q << 40 | r, q the query's index in
// q_dev; hits past cap are counted, not stored).  No sort, no sync.
int thresh_range(fid_ctx* ctx, const fid_db* db, int64_t r_lo, int64_t r_hi, const uint64_t* q_dev, int32_t n_q,
                 int mode, const int32_t* thr_dev, unsigned long long* counter, uint64_t* keys, int32_t* vals,
                 int64_t cap);
// References whose exact counts seed a top-k filter of n_q queries over a
// range of n_refs (n_refs itself: the range is counted directly).
int64_t seed_prefix(int64_t n_refs, int backend, int32_t n_q);
// Grow the context's scratch to hold `bytes` of staged queries (may allocate).
int scratch_reserve(fid_ctx* ctx, size_t bytes);
// The kernel family (fid_backend) a call with n_q queries on db resolves to.
int auto_family(const fid_ctx* ctx, const fid_db* db, int32_t n_q);
bool batch_routes_to_matrix_cores(const fid_ctx* ctx, const fid_db* db, int32_t n_q);
// Scratch bytes the query preparation of such a call needs.
size_t query_scratch_bytes(const fid_ctx* ctx, const fid_db* db, int32_t n_q);

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace fid

#define FID_HIP(call, what)                                   \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return fid::hip_fail(e_, what); \
    } while (0)

#define FID_TRY(call)                  \
    do {                               \
        const int st_ = (call);        \
        if (st_ != FID_OK) return st_; \
    } while (0)
