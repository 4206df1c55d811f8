// Device helpers shared by the libfastid kernels: lane and wave utilities,
// the per-wave top-k list primitives and the workgroup top-k selection.
#pragma once

#include "fid_common.hpp"

namespace fid {

// Scalar (constant address space) view of a wave-uniform pointer: loads
// through it become s_load_dwordxN into SGPRs.
typedef const __attribute__((address_space(4))) uint32_t* kptr_u32;
typedef uint32_t u32x16 __attribute__((ext_vector_type(16)));
typedef const __attribute__((address_space(4))) u32x16* kptr_u32x16;

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

// acc + popcount(x) as one v_bcnt_u32_b32 with its accumulator operand.  The
// compiler would otherwise rebalance a long run of these sums into trees of
// popcounts and three-way adds (2.5 VALU per word instead of 2).
__device__ __forceinline__ uint32_t popc_acc(uint32_t x, uint32_t acc)
{
    __asm__("v_bcnt_u32_b32 %0, %1, %2" : "=v"(acc) : "v"(x), "v"(acc));
    return acc;
}

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Largest key of a k-slot list and its position (ties: the last position).
template <typename ListPtr>
__device__ __forceinline__ void list_max(ListPtr list, int k, uint64_t& mx, int& mpos)
{
    const int lane = lane_id();
    uint64_t v = 0;
    int pos = -1;
    for (int i = lane; i < k; i += 64) {
        const uint64_t x = list[i];
        if (pos < 0 || x > v) {
            v = x;
            pos = i;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t ov = __shfl_xor(v, off);
        const int op = __shfl_xor(pos, off);
        if (ov > v || (ov == v && op > pos)) {
            v = ov;
            pos = op;
        }
    }
    mx = v;
    mpos = pos;
}

// Per-wave top-k list of one query, k slots in global memory or LDS.  A worker
// scans its references in increasing index order, so a new candidate whose
// count equals the list's worst count has a larger index and is never better:
// once the list is full the filter is "count < worst count".  Entry i of a
// list is only ever read or written by lane (i & 63) of the owning wave, so
// program order makes every update visible to the next scan.

__device__ __forceinline__ void topk_insert(uint64_t* __restrict__ list, int k, int64_t rbase,
                                            uint32_t acc, uint64_t m, uint32_t* lthr_q,
                                            uint32_t* lfill_q)
{
    const int lane = lane_id();
    uint32_t t = *lthr_q;
    uint32_t fill = *lfill_q;
    while (m) {
        const int src = __builtin_ctzll(m);
        m &= m - 1;
        const uint32_t c = (uint32_t)__shfl((int)acc, src);
        if (c >= t) continue;
        const uint64_t key = ((uint64_t)c << kIdxBits) | (uint64_t)(rbase + src);
        uint64_t mx;
        int mpos;
        if (fill < (uint32_t)k) {
            if (lane == (int)(fill & 63u)) list[fill] = key;
            ++fill;
            if (fill < (uint32_t)k) continue;
            list_max(list, k, mx, mpos);
        } else {
            list_max(list, k, mx, mpos);
            if (key >= mx) continue;
            if (lane == (mpos & 63)) list[mpos] = key;
            list_max(list, k, mx, mpos);
        }
        const uint32_t worst = (uint32_t)(mx >> kIdxBits);
        if (worst < t) t = worst;
    }
    if (lane == 0) {
        *lthr_q = t;
        *lfill_q = fill;
    }
}

// Ascending bitonic sort of kSelectSlots keys in LDS by the NT threads of a
// workgroup (NT unless a kernel says otherwise).
template <int NT = kSelectThreads>
__device__ void bitonic_sort_slots(uint64_t* s)
{
    for (int size = 2; size <= kSelectSlots; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = (int)threadIdx.x; t < kSelectSlots / 2; t += NT) {
                const int i = 2 * t - (t & (stride - 1));
                const int j = i + stride;
                const bool asc = (i & size) == 0;
                const uint64_t a = s[i], b = s[j];
                if ((a > b) == asc) {
                    s[i] = b;
                    s[j] = a;
                }
            }
            __syncthreads();
        }
    }
}

// Exact k smallest of n_in keys (k <= kSelectSlots / 2).  On return s[0..k)
// holds them ascending (kSentinel where fewer than k keys exist).  Keys below
// the current k-th best (and below `below`, which the caller guarantees every
// member of the answer is) are gathered in s[half..) and merged by a full
// sort whenever some arrived, so the work tracks the number of improving keys.
template <int NT = kSelectThreads, class Load>
__device__ void wg_topk(Load load, int64_t n_in, int k, uint64_t* s, int* nb, uint64_t below = kSentinel)
{
    constexpr int half = kSelectSlots / 2;
    for (int i = (int)threadIdx.x; i < kSelectSlots; i += NT) s[i] = kSentinel;
    if (threadIdx.x == 0) *nb = 0;
    __syncthreads();
    for (int64_t base = 0; base < n_in; base += half) {
        const uint64_t kth = s[k - 1] < below ? s[k - 1] : below;
        for (int j = 0; j < half / NT; ++j) {
            const int64_t i = base + j * NT + threadIdx.x;
            if (i < n_in) {
                const uint64_t key = load(i);
                if (key < kth) s[half + atomicAdd(nb, 1)] = key;
            }
        }
        __syncthreads();
        const int n = *nb;
        __syncthreads();
        if (n > 0) {
            bitonic_sort_slots<NT>(s);
            for (int i = (int)threadIdx.x; i < half; i += NT) s[half + i] = kSentinel;
            if (threadIdx.x == 0) *nb = 0;
            __syncthreads();
        }
    }
}

template <int NT = kSelectThreads>
__device__ __forceinline__ void write_topk(const uint64_t* s, int k, int32_t* cnt, int64_t* idx)
{
    for (int j = (int)threadIdx.x; j < k; j += NT) {
        const uint64_t key = s[j];
        cnt[j] = key == kSentinel ? INT32_MAX : (int32_t)(key >> kIdxBits);
        idx[j] = key == kSentinel ? -1 : (int64_t)(key & kIdxMask);
    }
}

// Exact top-k of one query from n_rsplit lists of k slots, of which only the
// first fills[w] of list w are valid.  A prefix over the fill counts (in
// LDS, off[n_rsplit + 1]) gives the filled total.  Densely filled lists are
// streamed slot by slot with coalesced loads (unfilled slots skipped); sparse
// ones are gathered (a dense position maps to (list, slot) by binary search
// over the prefix).  A histogram of the counts (bins of 2^shift counts, in
// the space of s) first gives the bin holding the k-th smallest count; only
// keys up to that bin's upper edge can be in the answer, so the selection
// sorts little more than k keys.  Called by all NT threads of a
// workgroup.
template <int NT = kSelectThreads>
__device__ inline void merge_query_lists(const uint64_t* __restrict__ lists_in,
                                         const uint32_t* __restrict__ fills, int32_t n_rsplit,
                                         int32_t k, int32_t n_loci, int32_t* __restrict__ cnt,
                                         int64_t* __restrict__ idx, uint64_t* s, int* nb,
                                         uint32_t* part, uint32_t* off)
{
    typedef const __attribute__((address_space(1))) uint64_t* gptr_u64;
    const gptr_u64 lists = (gptr_u64)lists_in;  // global: never aliases the LDS below
    const int tid = (int)threadIdx.x;
    const int seg = (n_rsplit + NT - 1) / NT;
    const int lo = min(n_rsplit, tid * seg), hi = min(n_rsplit, (tid + 1) * seg);
    uint32_t sum = 0;
    for (int i = lo; i < hi; ++i) sum += fills[i];
    part[tid] = sum;
    __syncthreads();
    for (int o = 1; o < NT; o <<= 1) {
        const uint32_t v = tid >= o ? part[tid - o] : 0u;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    uint32_t run = tid > 0 ? part[tid - 1] : 0u;
    for (int i = lo; i < hi; ++i) {
        off[i] = run;
        run += fills[i];
    }
    if (tid == NT - 1) off[n_rsplit] = part[NT - 1];
    __syncthreads();
    const int64_t total = off[n_rsplit];
    const int64_t n_slots = (int64_t)n_rsplit * k;  // < 2^31 (n_rsplit <= 8192, k <= 1024)
    const bool dense = total * 4 >= n_slots;
    const int64_t n_in = dense ? n_slots : total;
    auto load = [&](int64_t i) -> uint64_t {
        if (dense) {
            const int32_t w = (int32_t)i / k;
            return (uint32_t)((int32_t)i - w * k) < off[w + 1] - off[w] ? lists[i] : kSentinel;
        }
        int a = 0, b = n_rsplit;  // largest w with off[w] <= i
        while (b - a > 1) {
            const int m = (a + b) >> 1;
            if ((int64_t)off[m] <= i) a = m;
            else b = m;
        }
        return lists[(size_t)a * k + (size_t)(i - off[a])];
    };
    uint64_t below = kSentinel;
    if (total > k) {
        constexpr int kBins = 2 * kSelectSlots;  // uint32 bins in the space of s
        constexpr int kUnroll = 4;               // independent loads in flight per thread
        int shift = 0;
        while ((n_loci >> shift) + 1 > kBins) ++shift;
        const int nbins = (n_loci >> shift) + 1;
        uint32_t* hist = reinterpret_cast<uint32_t*>(s);
        __shared__ uint32_t edge;
        for (int i = tid; i < nbins; i += NT) hist[i] = 0u;
        if (tid == 0) edge = 0xFFFFFFFFu;
        __syncthreads();
        for (int64_t b0 = 0; b0 < n_in; b0 += kUnroll * NT) {
            uint64_t key[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int64_t i = b0 + u * NT + tid;
                key[u] = i < n_in ? load(i) : kSentinel;
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
                if (key[u] != kSentinel)
                    atomicAdd(&hist[min((uint32_t)(key[u] >> kIdxBits) >> shift, (uint32_t)(nbins - 1))], 1u);
        }
        __syncthreads();
        const int bseg = (nbins + NT - 1) / NT;
        uint32_t bsum = 0;
        for (int i = tid * bseg; i < min(nbins, (tid + 1) * bseg); ++i) bsum += hist[i];
        part[tid] = bsum;
        __syncthreads();
        for (int o = 1; o < NT; o <<= 1) {
            const uint32_t v = tid >= o ? part[tid - o] : 0u;
            __syncthreads();
            part[tid] += v;
            __syncthreads();
        }
        const uint32_t before = tid > 0 ? part[tid - 1] : 0u;
        if (before < (uint32_t)k && part[tid] >= (uint32_t)k) {
            uint32_t acc = before;
            for (int i = tid * bseg; i < min(nbins, (tid + 1) * bseg); ++i) {
                acc += hist[i];
                if (acc >= (uint32_t)k) {
                    edge = (uint32_t)i;
                    break;
                }
            }
        }
        __syncthreads();
        if (edge != 0xFFFFFFFFu) below = (uint64_t)((edge + 1u) << shift) << kIdxBits;
        __syncthreads();
    }
    wg_topk<NT>(load, n_in, k, s, nb, below);
    write_topk<NT>(s, k, cnt, idx);
}

}  // namespace fid
