// libfastid: the int8 matrix-core formulation of the overloaded product.
//
// For 0/1 profiles the Eq. 1 count has a closed form in the ordinary dot
// product D[q][r] = sum_k Q_k R_k (an exact int32 sum of 0/1 int8 products):
//   mixture : popcount(R & ~Q) = popcount(R) - D
//   identity: popcount(R ^ Q)  = popcount(R) + popcount(Q) - 2 D
// so the all-pairs comparison becomes a dense int8 GEMM on the MFMA units
// (v_mfma_i32_32x32x32_i8), with the reference bits expanded to bytes in
// registers and the query tile held as bytes in LDS.
//
// Workgroup = 8 waves (2 per SIMD) sharing one 64-query tile held in LDS as
// bytes for the kernel's whole lifetime (rows padded by 16 bytes so the 32
// rows a wave reads at one column hit distinct banks); each wave streams its
// own 128 references (4 MFMA column blocks) against both 32-query row
// blocks: 8 accumulators of 32x32 int32 per wave.  Per 32-locus step a lane
// expands 4 x 16 reference bits (3 VALU ops per 4 loci) and issues 8 MFMAs;
// the next 128-locus unit of reference bits is prefetched.
#include "fid_device.hpp"

namespace fid {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

namespace {

constexpr int kWavesM = 8;
constexpr int kWGM = kWavesM * kWave;
constexpr int kQB = 64;                 // queries per workgroup tile
constexpr int kNBW = 4;                 // 32-reference column blocks per wave
constexpr int kRefsPerWave = 32 * kNBW;
constexpr int kRefsPerWG = kRefsPerWave * kWavesM;
static_assert(kDbTileRefs % kRefsPerWG == 0, "tiles must not cross the database padding granule");
constexpr int kMaxKpad = 2304;          // 64 x (2304 + 16) B of query tile fits the 160 KiB LDS

// 16 bits of w starting at bit sh -> 16 bytes of 0/1: a nibble x times
// 0x204081 puts bit i at bit 8i of the product (the four shifted copies do not
// overlap, so there are no carries).  3 VALU ops per 4 loci.
__device__ __forceinline__ v4i expand16(uint32_t w, uint32_t sh)
{
    v4i r;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        r[j] = (int)((__builtin_amdgcn_ubfe(w, sh + 4u * j, 4u) * 0x204081u) & 0x01010101u);
    return r;
}

// Workgroups are dealt to the 8 XCDs round-robin; renumber them so that the
// workgroups resident on one XCD at a time are consecutive, i.e. share a
// reference range and hit in that XCD's L2.
__device__ __forceinline__ int xcd_local_index(int wg, int n_wg)
{
    const int x = wg & 7, s = wg >> 3;
    const int per = n_wg >> 3, rem = n_wg & 7;
    return x < rem ? x * (per + 1) + s : rem * (per + 1) + (x - rem) * per + s;
}

typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(1))) uint64_t glb_u64;
typedef __attribute__((address_space(1))) uint32_t glb_u32;

// Insert the candidates of one ballot into the wave's lists (entry i of a
// list is only touched by lane i & 63).  Candidates arrive in no particular
// index order, so the decision compares full (count, index) keys, and the
// filter bound of a full list is its worst count plus one (an equal count
// may still win on index).  The address spaces are explicit: this out-of-line
// helper would otherwise reach the LDS bounds and the global lists through
// flat accesses.
__device__ __noinline__ void mfma_insert(uint64_t mask, uint32_t c, int64_t r, int m,
                                         glb_u64* __restrict__ lists, int64_t qstride, int k,
                                         lds_u32* lthr, lds_u32* lfill)
{
    const int lane = lane_id();
    while (mask) {
        // src is wave-uniform: the candidate's fields are read straight from its lane
        const int src = __builtin_ctzll(mask);
        mask &= mask - 1;
        const int ms = __builtin_amdgcn_readlane(m, src);
        const uint32_t cs = (uint32_t)__builtin_amdgcn_readlane((int)c, src);
        const uint32_t rlo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)r, src);
        const uint32_t rhi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)r >> 32), src);
        uint32_t t = lthr[ms];
        if (cs >= t) continue;
        const uint64_t key = ((uint64_t)cs << kIdxBits) | ((uint64_t)rhi << 32) | rlo;
        glb_u64* list = lists + (size_t)ms * qstride;
        uint32_t fill = lfill[ms];
        uint64_t mx;
        int mpos;
        bool changed = false;
        if (fill < (uint32_t)k) {
            if (lane == (int)(fill & 63u)) list[fill] = key;
            ++fill;
            changed = fill == (uint32_t)k;
        } else {
            list_max(list, k, mx, mpos);
            if (key < mx) {
                if (lane == (mpos & 63)) list[mpos] = key;
                changed = true;
            }
        }
        if (changed) {
            list_max(list, k, mx, mpos);
            const uint32_t bound = (uint32_t)(mx >> kIdxBits) + 1u;
            if (bound < t) t = bound;
        }
        if (lane == 0) {
            lthr[ms] = t;
            lfill[ms] = fill;
        }
        wave_lds_sync();
    }
}

// Candidates of one fp4 tile epilogue wait in a per-wave LDS queue of
// kCandQ4 entries.  An entry packs tile query m (7 bits), reference 16 j + n16
// of the wave's 64 (6 bits) and the count (at most 65535, 16 bits):
// m | ref << 7 | c << 13.  An out-of-line call waits for every memory
// operation of the wave on entry and again before it returns, so in the
// single-call scans the drain at the end of a tile leaves its global writes
// to the caller: the call decides where each candidate goes (the bound, fill
// and list updates live in LDS), and the caller then issues the list stores
// inline, where nothing waits for them (witness counts collect in LDS and
// reach global memory every 4th tile).  The persistent batch kernel, whose
// registers leave no room for those inline stores, and a queue that fills up
// mid-tile use a call that writes everything itself.
constexpr int kCandQ4 = 64;
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;

// Drain the queue: every lane takes one entry, so the bound, fill and witness
// lookups of up to 64 candidates happen at once; the witness counters take
// every queued candidate below a level (each is a distinct reference of its
// query: the scan meets a (query, reference) pair once); then the entries of
// each query are appended or merged in queue order, with only readlanes
// between list updates.
__device__ __noinline__ void mfma_insert_queue(const lds_u32* cq, int n, int64_t rbase,
                                               glb_u64* __restrict__ lists, int64_t qstride, int k,
                                               lds_u32* lthr, lds_u32* lfill, const lds_u32* tlvl,
                                               glb_u32* wit)
{
    const int lane = lane_id();
    for (int e0 = 0; e0 < n; e0 += 64) {
        const bool act = lane < n - e0;
        const uint32_t v = act ? cq[e0 + lane] : 0u;
        const int m = (int)(v & 127u);
        const uint32_t c = v >> 13;
        const int ref = (int)((v >> 7) & 63u);
        const uint32_t t0 = act ? lthr[m] : 0u;
        const uint32_t f0 = act ? lfill[m] : 0u;
        if (wit && act) {
            // levels decrease with l: a count at or above one is above the rest
            for (int l = 0; l < kWitLevels; ++l) {
                if (c >= tlvl[kWitLevels * m + l]) break;
                __hip_atomic_fetch_add(wit + kWitLevels * m + l, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        const bool keep = act && c < t0;
        uint64_t rem = __builtin_amdgcn_ballot_w64(keep);
        while (rem) {
            const int lead = __builtin_ctzll(rem);
            const int ms = __builtin_amdgcn_readlane(m, lead);
            uint64_t sel = __builtin_amdgcn_ballot_w64(keep && m == ms);
            rem &= ~sel;
            // this query's bound and fill, as read above (no entry of this
            // chunk has touched them yet)
            uint32_t t = (uint32_t)__builtin_amdgcn_readlane((int)t0, lead);
            uint32_t fill = (uint32_t)__builtin_amdgcn_readlane((int)f0, lead);
            glb_u64* list = lists + (size_t)ms * qstride;
            while (sel) {
                const int src = __builtin_ctzll(sel);
                sel &= sel - 1;
                const uint32_t cs = (uint32_t)__builtin_amdgcn_readlane((int)c, src);
                if (cs >= t) continue;
                const uint64_t key =
                    ((uint64_t)cs << kIdxBits) | (uint64_t)(rbase + __builtin_amdgcn_readlane(ref, src));
                uint64_t mx;
                int mpos;
                bool changed = false;
                if (fill < (uint32_t)k) {
                    if (lane == (int)(fill & 63u)) list[fill] = key;
                    ++fill;
                    changed = fill == (uint32_t)k;
                } else {
                    list_max(list, k, mx, mpos);
                    if (key < mx) {
                        if (lane == (mpos & 63)) list[mpos] = key;
                        changed = true;
                    }
                }
                if (changed) {
                    list_max(list, k, mx, mpos);
                    const uint32_t bound = (uint32_t)(mx >> kIdxBits) + 1u;
                    if (bound < t) t = bound;
                }
            }
            if (lane == 0) {
                lthr[ms] = t;
                lfill[ms] = fill;
            }
        }
        wave_lds_sync();
    }
}

// End-of-tile drain of n <= 64 queued candidates (lane e takes entry e).  The
// entries of one query are kept in queue order while below its bound; as long
// as its list does not fill, they are appended at the next free slots, and the
// slot of entry e goes to cpos[e] for the caller to store (kNoSlot: nothing to
// store).  A list that fills takes its entries one by one here, with
// immediate stores, since its new bound needs the list's worst key.  Witness
// counts go to the workgroup's LDS counters wloc, which the waves add to the
// global ones every 4th tile.
__device__ __noinline__ void mfma_drain_decide(const lds_u32* cq, lds_u32* cpos, int n, int64_t rbase,
                                               glb_u64* __restrict__ lists, int64_t qstride, int k,
                                               lds_u32* lthr, lds_u32* lfill, const lds_u32* tlvl,
                                               lds_u32* wloc)
{
    const int lane = lane_id();
    const bool act = lane < n;
    const uint32_t v = act ? cq[lane] : 0u;
    const int m = (int)(v & 127u);
    const uint32_t c = v >> 13;
    const int ref = (int)((v >> 7) & 63u);
    const uint32_t t0 = act ? lthr[m] : 0u;
    const uint32_t f0 = act ? lfill[m] : 0u;
    if (wloc && act) {
        // witness counts of every queued candidate below a level, into the
        // workgroup's LDS counters (each is a distinct reference of its query:
        // the scan meets a pair once)
        for (int l = 0; l < kWitLevels; ++l)
            if (c < tlvl[kWitLevels * m + l])
                __hip_atomic_fetch_add(wloc + kWitLevels * m + l, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    uint32_t slot = kNoSlot;
    const bool keep = act && c < t0;
    uint64_t rem = __builtin_amdgcn_ballot_w64(keep);
    while (rem) {
        const int lead = __builtin_ctzll(rem);
        const int ms = __builtin_amdgcn_readlane(m, lead);
        const bool mine = keep && m == ms;
        uint64_t sel = __builtin_amdgcn_ballot_w64(mine);
        rem &= ~sel;
        const uint32_t nsel = (uint32_t)__popcll(sel);
        uint32_t t = (uint32_t)__builtin_amdgcn_readlane((int)t0, lead);
        uint32_t fill = (uint32_t)__builtin_amdgcn_readlane((int)f0, lead);
        if (fill + nsel < (uint32_t)k) {
            // appends only: every entry is below the bound, which stays put
            if (mine)
                slot = fill + (uint32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(sel >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)sel, 0u));
            fill += nsel;
        } else {
            glb_u64* list = lists + (size_t)ms * qstride;
            while (sel) {
                const int src = __builtin_ctzll(sel);
                sel &= sel - 1;
                const uint32_t cs = (uint32_t)__builtin_amdgcn_readlane((int)c, src);
                if (cs >= t) continue;
                const uint64_t key =
                    ((uint64_t)cs << kIdxBits) | (uint64_t)(rbase + __builtin_amdgcn_readlane(ref, src));
                uint64_t mx;
                int mpos;
                bool changed = false;
                if (fill < (uint32_t)k) {
                    if (lane == (int)(fill & 63u)) list[fill] = key;
                    ++fill;
                    changed = fill == (uint32_t)k;
                } else {
                    list_max(list, k, mx, mpos);
                    if (key < mx) {
                        if (lane == (mpos & 63)) list[mpos] = key;
                        changed = true;
                    }
                }
                if (changed) {
                    list_max(list, k, mx, mpos);
                    const uint32_t bound = (uint32_t)(mx >> kIdxBits) + 1u;
                    if (bound < t) t = bound;
                }
            }
        }
        if (lane == 0) {
            lthr[ms] = t;
            lfill[ms] = fill;
        }
    }
    if (act) cpos[lane] = slot;
    wave_lds_sync();
}

__device__ __noinline__ void mfma_append_hits(uint64_t mask, bool hit, int32_t c, int64_t r, int q,
                                              unsigned long long* __restrict__ hit_count,
                                              uint64_t* __restrict__ hit_keys,
                                              int32_t* __restrict__ hit_cnt, int64_t cap)
{
    const int lane = lane_id();
    const int first = __builtin_ctzll(mask);
    unsigned long long base = 0;
    if (lane == first) base = atomicAdd(hit_count, (unsigned long long)__popcll(mask));
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)base, first);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(base >> 32), first);
    base = ((unsigned long long)hi << 32) | lo;
    if (hit) {
        const unsigned long long pos =
            base + (unsigned long long)__popcll(mask & ((1ull << lane) - 1ull));
        if (pos < (unsigned long long)cap) {
            hit_keys[pos] = ((uint64_t)q << kIdxBits) | (uint64_t)r;
            hit_cnt[pos] = c;
        }
    }
}

}  // namespace

// LDS layout: [query tile 64 x (kpad + 16)] [per-wave bound 8 x 64] [per-wave
// fill 8 x 64] [tile query popcounts 64] [tile thresholds 64].
template <int MODE, int EPI>
__global__ __launch_bounds__(kWGM) void mfma_scan_kernel(
    const ScanParams p, const uint8_t* __restrict__ qx, int32_t kpad,
    const int32_t* __restrict__ pcq, int32_t* __restrict__ out, uint64_t* __restrict__ lists,
    uint32_t* __restrict__ fills, const uint32_t* __restrict__ thr_init,
    const int32_t* __restrict__ thr, unsigned long long* __restrict__ hit_count,
    uint64_t* __restrict__ hit_keys, int32_t* __restrict__ hit_cnt)
{
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    const int row_bytes = kpad + 16;
    uint8_t* qt = smem;
    uint32_t* lthr_all = reinterpret_cast<uint32_t*>(smem + kQB * row_bytes);
    uint32_t* lfill_all = lthr_all + kWavesM * kQB;
    int32_t* tpcq = reinterpret_cast<int32_t*>(lfill_all + kWavesM * kQB);
    int32_t* tthr = tpcq + kQB;

    const int lane = lane_id();
    const int tid = (int)threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int g = lane >> 5;       // MFMA k half
    const int n32 = lane & 31;     // MFMA row / column within a 32-block

    // Workgroup -> (query tile, reference range).
    const int n_qtiles = (p.q_hi - p.q_lo + kQB - 1) / kQB;
    const int wg = xcd_local_index((int)blockIdx.x, (int)gridDim.x);
    const int qt_idx = wg % n_qtiles;
    const int wr_g = wg / n_qtiles;
    const int q0 = p.q_lo + qt_idx * kQB;
    const int nq_tile = min(kQB, p.q_hi - q0);
    const int64_t base = (p.r_lo / kDbTileRefs) * kDbTileRefs;
    const int64_t ntiles = (p.r_hi - base + kRefsPerWG - 1) / kRefsPerWG;
    const int64_t tb = (ntiles * wr_g) / p.n_rsplit;
    const int64_t te = (ntiles * (wr_g + 1)) / p.n_rsplit;
    const int worker = wr_g * kWavesM + wv;  // list owner along references
    const int n_workers_r = p.n_rsplit * kWavesM;

    // Resident query tile (bytes) and per-query side data.
    const int vec_per_row = kpad / 16;
    for (int i = tid; i < kQB * vec_per_row; i += kWGM) {
        const int row = i / vec_per_row;
        const int col = (i - row * vec_per_row) * 16;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (row < nq_tile) v = *reinterpret_cast<const uint4*>(qx + (size_t)(q0 + row) * kpad + col);
        *reinterpret_cast<uint4*>(qt + row * row_bytes + col) = v;
    }
    if (tid < kQB) {
        tpcq[tid] = (MODE == FID_MODE_IDENTITY && tid < nq_tile) ? pcq[q0 + tid] : 0;
        tthr[tid] = (EPI == EPI_THRESH && tid < nq_tile) ? thr[q0 + tid] : -1;
    }
    uint32_t* lthr = lthr_all + wv * kQB;
    uint32_t* lfill = lfill_all + wv * kQB;
    if constexpr (EPI == EPI_TOPK) {
        for (int i = lane; i < kQB; i += 64) {
            lthr[i] = i < nq_tile ? thr_init[q0 + i] : 0u;
            lfill[i] = 0u;
        }
    }
    __syncthreads();

    const int nunits = kpad / 128;
    const int w4 = p.db.w4;
    const uint8_t* arow0 = qt + n32 * row_bytes + g * 16;
    const uint8_t* arow1 = qt + (32 + n32) * row_bytes + g * 16;
    for (int64_t tile = tb; tile < te; ++tile) {
        const int64_t rbase = base + tile * kRefsPerWG + (int64_t)wv * kRefsPerWave;
        // Reference words: one uniform base per tile plus a 32-bit lane
        // offset; the database is padded to whole tiles, so every load is
        // unconditional (references past r_hi are never read by the epilogue).
        const char* tbase = reinterpret_cast<const char*>(p.db.words) + (size_t)(rbase >> 6) * w4 * 1024;
        const uint32_t loff = (uint32_t)n32 * 16u;
        auto load_unit = [&](uint4 (&dst)[kNBW], int u) {
#pragma unroll
            for (int j = 0; j < kNBW; ++j)
                dst[j] = *reinterpret_cast<const uint4*>(
                    tbase + ((size_t)(j >> 1) * w4 * 64 + 32 * (j & 1)) * 16 + (size_t)u * 1024 + loff);
        };
        v16i acc[2][kNBW];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int j = 0; j < kNBW; ++j) acc[a][j] = v16i{0};

        // One 16-byte unit (128 loci) of each reference feeds 4 MFMA steps.
        auto step_unit = [&](const uint4 (&bits)[kNBW], int u) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int kofs = u * 128 + s * 32;
                const v4i a0 = *reinterpret_cast<const v4i*>(arow0 + kofs);
                const v4i a1 = *reinterpret_cast<const v4i*>(arow1 + kofs);
#pragma unroll
                for (int j = 0; j < kNBW; ++j) {
                    const uint32_t w = s == 0 ? bits[j].x : s == 1 ? bits[j].y : s == 2 ? bits[j].z : bits[j].w;
                    const v4i b = expand16(w, 16u * (uint32_t)g);
                    acc[0][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, b, acc[0][j], 0, 0, 0);
                    acc[1][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, b, acc[1][j], 0, 0, 0);
                }
            }
        };
        uint4 ba[kNBW], bb[kNBW];
        load_unit(ba, 0);
#pragma unroll 1
        for (int u = 0; u < nunits; u += 2) {
            load_unit(bb, u + 1);
            step_unit(ba, u);
            load_unit(ba, u + 2);  // last pass: up to two units past the row, never used
            step_unit(bb, u + 1);
        }

        // ---- epilogue: lane holds reference rbase + 32 j + n32 and, in
        // register i of block a, tile query m = 32 a + (i & 3) + 8 (i >> 2) + 4 g.
#pragma unroll
        for (int j = 0; j < kNBW; ++j) {
            const int64_t r = rbase + 32 * j + n32;
            const bool rin = r >= p.r_lo && r < p.r_hi;
            const int32_t pr = rin ? p.db.pc[r] : 0;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                int32_t cv[16];
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int m = 32 * a + (i & 3) + 8 * (i >> 2) + 4 * g;
                    const int32_t d = acc[a][j][i];
                    cv[i] = MODE == FID_MODE_MIXTURE ? pr - d : pr + tpcq[m] - 2 * d;
                }
                if constexpr (EPI == EPI_FULL) {
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const int m = 32 * a + (i & 3) + 8 * (i >> 2) + 4 * g;
                        if (rin && m < nq_tile)
                            out[(size_t)(q0 + m - p.out_q_base) * p.ld + (r - p.out_r_base)] = cv[i];
                    }
                } else if constexpr (EPI == EPI_TOPK) {
                    bool any = false;
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const int m = 32 * a + (i & 3) + 8 * (i >> 2) + 4 * g;
                        any |= (uint32_t)cv[i] < lthr[m];
                    }
                    if (__builtin_amdgcn_ballot_w64(any && rin)) {
#pragma unroll
                        for (int i = 0; i < 16; ++i) {
                            const int m = 32 * a + (i & 3) + 8 * (i >> 2) + 4 * g;
                            const bool cand = rin && (uint32_t)cv[i] < lthr[m];
                            const uint64_t bm = __builtin_amdgcn_ballot_w64(cand);
                            if (bm)
                                mfma_insert(bm, (uint32_t)cv[i], r, m,
                                            (glb_u64*)(lists + ((size_t)q0 * n_workers_r + worker) * p.k),
                                            (int64_t)n_workers_r * p.k, p.k, (lds_u32*)lthr, (lds_u32*)lfill);
                        }
                    }
                } else {
                    bool any = false;
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const int m = 32 * a + (i & 3) + 8 * (i >> 2) + 4 * g;
                        any |= cv[i] <= tthr[m];
                    }
                    if (__builtin_amdgcn_ballot_w64(any && rin)) {
#pragma unroll
                        for (int i = 0; i < 16; ++i) {
                            const int m = 32 * a + (i & 3) + 8 * (i >> 2) + 4 * g;
                            const bool hit = rin && cv[i] <= tthr[m];
                            const uint64_t bm = __builtin_amdgcn_ballot_w64(hit);
                            if (bm)
                                mfma_append_hits(bm, hit, cv[i], r, q0 + m, hit_count, hit_keys,
                                                 hit_cnt, p.hit_cap);
                        }
                    }
                }
            }
        }
    }
    if constexpr (EPI == EPI_TOPK) {
        wave_lds_sync();
        for (int i = lane; i < nq_tile; i += 64)
            fills[(size_t)(q0 + i) * n_workers_r + worker] = lfill[i];
    }
}

// Expanded queries for the matrix-core path: byte k of row q = locus k of
// query q (0/1), zero padded to kpad; plus popcount(Q_q) for identity mode.
__global__ void expand_queries_kernel(const uint64_t* __restrict__ q, int32_t n_q,
                                      int32_t row_words, int32_t n_loci, uint8_t* __restrict__ qx,
                                      int32_t kpad, int32_t* __restrict__ pcq)
{
    const int64_t total = (int64_t)n_q * (kpad / 4);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / (kpad / 4);
        const int32_t k0 = (int32_t)(t - i * (kpad / 4)) * 4;
        uint32_t v = 0;
        if (k0 < n_loci) {
            const uint64_t w = q[i * row_words + (k0 >> 6)];
            uint32_t nib = (uint32_t)(w >> (k0 & 63)) & 0xFu;
            if (k0 + 4 > n_loci) nib &= (1u << (n_loci - k0)) - 1u;
            v = (nib * 0x204081u) & 0x01010101u;
        }
        reinterpret_cast<uint32_t*>(qx + i * kpad)[k0 >> 2] = v;
    }
    // popcounts: one thread per query
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_q;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t s = 0;
        const int32_t full = n_loci >> 6;
        for (int32_t w = 0; w < full; ++w) s += __popcll(q[i * row_words + w]);
        if (n_loci & 63) s += __popcll(q[i * row_words + full] & ((1ull << (n_loci & 63)) - 1ull));
        pcq[i] = s;
    }
}

hipError_t launch_expand_queries(const uint64_t* q, int32_t n_q, int32_t row_words,
                                 int32_t n_loci, uint8_t* qx, int32_t kpad, int32_t* pcq,
                                 hipStream_t s)
{
    const int64_t total = (int64_t)n_q * (kpad / 4);
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(expand_queries_kernel, dim3((unsigned)blocks), dim3(256), 0, s, q, n_q,
                       row_words, n_loci, qx, kpad, pcq);
    return hipGetLastError();
}

// Loci padded to whole pairs of 128-locus units (the unit loop is unrolled by
// two); the padding is zero on the query side, so whatever the reference
// side holds there adds nothing.
int mfma_kpad(int32_t n_loci) { return ((n_loci + 255) / 256) * 256; }
int mfma_max_loci() { return kMaxKpad; }
int mfma_refs_per_wg() { return kRefsPerWG; }
int mfma_queries_per_wg() { return kQB; }
int mfma_waves_per_wg() { return kWavesM; }

static size_t mfma_lds_bytes(int32_t kpad)
{
    return (size_t)kQB * (kpad + 16) + 2 * (size_t)kWavesM * kQB * 4 + 2 * (size_t)kQB * 4;
}

template <int MODE, int EPI>
static hipError_t launch_mfma_t(const ScanParams& p, const MfmaBuffers& b, hipStream_t s)
{
    if (b.kpad > kMaxKpad) return hipErrorInvalidValue;
    const int n_qtiles = (p.q_hi - p.q_lo + kQB - 1) / kQB;
    const int64_t blocks = (int64_t)n_qtiles * p.n_rsplit;
    const size_t lds = mfma_lds_bytes(b.kpad);
    const hipError_t e = lds_opt_in<&mfma_scan_kernel<MODE, EPI>>((int)mfma_lds_bytes(kMaxKpad));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((mfma_scan_kernel<MODE, EPI>), dim3((unsigned)blocks), dim3(kWGM), lds, s,
                       p, b.qx, b.kpad, b.pcq, b.out, b.lists, b.fills, b.thr_init, b.thr,
                       b.hit_count, b.hit_keys, b.hit_cnt);
    return hipGetLastError();
}

hipError_t launch_mfma_scan(int mode, int epi, const ScanParams& p, const MfmaBuffers& b,
                            hipStream_t s)
{
    if (p.n_rsplit <= 0) return hipSuccess;
    if (mode == kModePerQuery) return hipErrorInvalidValue;  // per-query modes: fp4 or popcount
    if (mode == FID_MODE_MIXTURE) {
        if (epi == EPI_FULL) return launch_mfma_t<FID_MODE_MIXTURE, EPI_FULL>(p, b, s);
        if (epi == EPI_TOPK) return launch_mfma_t<FID_MODE_MIXTURE, EPI_TOPK>(p, b, s);
        return launch_mfma_t<FID_MODE_MIXTURE, EPI_THRESH>(p, b, s);
    }
    if (epi == EPI_FULL) return launch_mfma_t<FID_MODE_IDENTITY, EPI_FULL>(p, b, s);
    if (epi == EPI_TOPK) return launch_mfma_t<FID_MODE_IDENTITY, EPI_TOPK>(p, b, s);
    return launch_mfma_t<FID_MODE_IDENTITY, EPI_THRESH>(p, b, s);
}

// ======================================================================
// fp4 (e2m1) matrix-core variant: v_mfma_f32_16x16x128_f8f6f4 with both
// operands in e2m1 and the fp32 accumulation of at most 65536 unit products,
// which is exact.  It runs the same closed forms as the int8 kernel at twice
// the MAC rate per instruction.
//
// Element order and values: a dot product does not depend on the order of k
// as long as both operands use the same one.  Each 32-locus word w of a
// reference is spread into 4 dwords, dword d holding locus 4j + d in nibble
// j.  A set bit need not be 1.0 on both sides, only the product of the two
// codes must be: the reference keeps loci 4j, 4j+1, 4j+2 where they are (e2m1
// 0x1 = 0.5, 0x2 = 1.0, 0x4 = 2.0: dword d = w & (0x11111111 << d)) and moves
// locus 4j+3 down one bit (2.0), 5 VALU ops per 32 loci; the queries, staged
// once, carry the reciprocals (2.0, 1.0, 0.5, 0.5), so every product of two
// set bits is exactly 1.  The k index of an
// MFMA is permuted further so that each lane loads whole 16-byte units:
// within a group of 4 units (512 loci), lane group kg (k quarter of the
// MFMA operand) holds unit 4g + kg and feeds its word t to step t, so one
// dwordx4 load per lane and 16-reference block covers 4 MFMA steps.
//
// Workgroup = 8 waves sharing a 128-query tile that lives in LDS for the
// kernel's lifetime (rows padded by 16 bytes).  Each wave computes all 128
// queries against its own 64-reference database block (8 x 4 blocks of
// 16x16 fp32 accumulators, 32 MFMAs per 128 loci); the next group of units
// (possibly of the next reference tile) is always in flight.  Accumulators
// start at zero; the top-k and threshold epilogues apply the closed forms
// and the bounds to D afterwards, with the tile's reference popcounts moved
// into LDS by the DMA engine while the tile is scanned.  Nothing that the
// epilogue computes lives across the scan loop, which keeps the whole tile
// in registers without spills.
namespace {

constexpr int kQB4 = 128;               // queries per workgroup (and per wave)
constexpr int kQA4 = kQB4 / 16;         // 16-query row blocks per wave
constexpr int kNB4 = 4;                 // 16-reference column blocks per wave
constexpr int kRefsPerWave4 = 16 * kNB4;
constexpr int kRefsPerWG4 = kRefsPerWave4 * kWavesM;
constexpr int kUnitsPerGroup4 = 4;      // 16-byte units per load group
constexpr int kKChunk4 = 2048;          // loci of the query tile resident in LDS at a time:
                                        // 128 x (1024 + 16) B of queries + 13 KiB fit the LDS
constexpr int kMaxKpad4 = 65536;
constexpr int kRowBytes4 = kKChunk4 / 2 + 16;  // LDS stride of a staged query row
constexpr int kWaitVm0 = 0x0F70;        // s_waitcnt vmcnt(0), other counters untouched
static_assert(kRefsPerWave4 == 64, "a wave covers exactly one database block");
static_assert(kDbTileRefs % kRefsPerWG4 == 0, "tiles must not cross the database padding granule");

typedef float v4f __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));

__device__ __forceinline__ v8i spread_fp4(uint32_t w)
{
    v8i r;
    r[0] = (int)(w & 0x11111111u);          // locus 4j     -> 0.5
    r[1] = (int)(w & 0x22222222u);          // locus 4j + 1 -> 1.0
    r[2] = (int)(w & 0x44444444u);          // locus 4j + 2 -> 2.0
    r[3] = (int)((w >> 1) & 0x44444444u);   // locus 4j + 3 -> 2.0
    r[4] = 0;
    r[5] = 0;
    r[6] = 0;
    r[7] = 0;
    return r;
}

__device__ __forceinline__ uint32_t word_of(const uint4& v, int t)
{
    return t == 0 ? v.x : t == 1 ? v.y : t == 2 ? v.z : v.w;
}

}  // namespace

// One work item of the fp4 scan (see fp4_work).
struct Fp4Work {
    DbView db;
    int64_t r_lo, r_hi;            // the query set's reference range (others compare as +inf)
    int64_t base;                  // r_lo rounded down to a database tile
    int64_t tb, te;                // 512-reference tiles [tb, te) from base
    const uint8_t* qx;             // staged queries of the set, row q at qx + q * kpad / 2
    int32_t kpad;
    bool multi_chunk;              // rows span several LDS chunks (restaged per tile)
    const int32_t* pcq;            // |Q| per query of the set
    const int32_t* qmode;          // per-query fid_mode (kModePerQuery)
    int32_t q0, nq_tile;           // query tile of the set
    int32_t slot, n_slots;         // this item's reference range among the set's ranges
    int32_t k;
    int32_t* out;                  // EPI_FULL: out[(q - out_q_base) * ld + (r - out_r_base)]
    int64_t ld;
    int32_t out_q_base;
    int64_t out_r_base;
    uint64_t* lists;               // top-k lists [q][n_slots * waves][k], fills [q][n_slots * waves]
    uint32_t* fills;
    const uint32_t* thr_init;      // per-query starting bound, witness levels and counters
    const uint32_t* level;
    uint32_t* wit;
    const int32_t* thr;            // threshold hits
    unsigned long long* hit_count;
    uint64_t* hit_keys;
    int32_t* hit_cnt;
    int64_t hit_cap;
};

// Rows longer than one LDS chunk: stage loci [c * kKChunk4, (c + 1) * kKChunk4)
// of every query of the tile, straight from global memory into LDS
// (global_load_lds moves no data through registers, so a tile's accumulators
// stay live across a restage).  One wave instruction moves one row's chunk of
// <= 1 KiB; rows past the tile's queries are zeroed once by the caller.
__device__ __forceinline__ void fp4_stage_chunk(const uint8_t* __restrict__ qx, int qrow, int cbytes,
                                                int row_bytes, int q0, int nq_tile, int wv, int lane,
                                                int c, uint8_t* qt)
{
    typedef __attribute__((address_space(3))) uint8_t lds_u8;
    const int bytes = min(cbytes, qrow - c * cbytes);
    for (int r = wv; r < nq_tile; r += kWavesM)
        if (lane * 16 < bytes)
            __builtin_amdgcn_global_load_lds(qx + (size_t)(q0 + r) * qrow + (size_t)c * cbytes + lane * 16,
                                             (lds_u8*)(qt + r * row_bytes), 16, 0, 0);
    __builtin_amdgcn_s_waitcnt(0);
}

// Witness counts gathered in LDS since the last flush go to the global
// counters: wave wv takes an eighth of the tile's (query, level) counters,
// swapping each with zero (other waves may be adding to it meanwhile).
__device__ __forceinline__ void fp4_flush_witness(uint32_t* wloc, uint32_t* __restrict__ wit_tile, int n, int wv,
                                                  int lane)
{
    constexpr int kPer = kWitLevels * kQB4 / kWavesM;
#pragma unroll
    for (int h = 0; h < (kPer + 63) / 64; ++h) {
        const int i = kPer * wv + 64 * h + lane;
        if (64 * h + lane < kPer && i < n) {
            const uint32_t cnt = __hip_atomic_exchange((lds_u32*)(wloc + i), 0u, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            if (cnt) __hip_atomic_fetch_add(wit_tile + i, cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// LDS: [query tile 128 x kRowBytes4] [bound 8 x 128] [fill 8 x 128]
// [staged reference popcounts 8 x 2 x 64] [tile popcounts 128]
// [tile thresholds 128] [tile modes 128] [witness levels 128 x kWitLevels]
// [staged witness counts 128 x kWitLevels, shared by the waves]
// [combined bound 8 x 128] [candidate queues 8 x kCandQ4] [their list slots 8 x kCandQ4]
// [witness counts not yet flushed 128 x kWitLevels].
// One work item of the fp4 scan: query tile [q0, q0 + nq_tile) of a query
// set against tiles [tb, te) of a reference range (the kernels below take
// their items from the launch geometry or from a queue).  Every wave of the
// workgroup calls it with the same item.  PARTIAL: the tile holds fewer than
// 113 queries, and the MFMAs of its 16-query row blocks past the last query
// are skipped (their accumulators keep their start value, which is what the
// zero rows of those queries would leave).  DEFER: the end-of-tile drain only
// decides where candidates go and this code issues the list stores, with
// witness counts collected in LDS (else one call writes everything).
template <int MODE, int EPI, bool KCHUNKS, bool PARTIAL, bool DEFER>
__device__ __forceinline__ void fp4_work(const Fp4Work& w)
{
    typedef __attribute__((address_space(3))) int32_t lds_i32;
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    constexpr bool kLists = EPI == EPI_TOPK || EPI == EPI_BOTH;    // top-k lists
    constexpr bool kHits = EPI == EPI_THRESH || EPI == EPI_BOTH;   // threshold hits
    // Rows longer than kKChunk4 loci are staged chunk by chunk: the LDS tile
    // holds loci [c * kKChunk4, (c + 1) * kKChunk4) of every query while the
    // accumulators collect all chunks of a reference tile.
    const uint8_t* __restrict__ qx = w.qx;
    const int32_t kpad = w.kpad;
    const int32_t* __restrict__ pcq = w.pcq;
    int32_t* __restrict__ out = w.out;
    uint64_t* __restrict__ lists = w.lists;
    uint32_t* __restrict__ fills = w.fills;
    const uint32_t* __restrict__ thr_init = w.thr_init;
    const uint32_t* __restrict__ level = w.level;
    uint32_t* __restrict__ wit = w.wit;
    const int32_t* __restrict__ thr = w.thr;
    unsigned long long* __restrict__ hit_count = w.hit_count;
    uint64_t* __restrict__ hit_keys = w.hit_keys;
    int32_t* __restrict__ hit_cnt = w.hit_cnt;
    const int q0 = w.q0;
    const int nq_tile = w.nq_tile;
    const int64_t base = w.base;
    const int64_t tb = w.tb;
    const int64_t te = w.te;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int worker = w.slot * kWavesM + wv;
    const int n_workers_r = w.n_slots * kWavesM;
    const bool multi_chunk = w.multi_chunk;
    const int qrow = kpad / 2;             // expanded bytes per query
    const int cbytes = KCHUNKS ? kKChunk4 / 2 : qrow;  // staged bytes per query and chunk
    uint8_t* qt = smem;
    uint32_t* lthr_all = reinterpret_cast<uint32_t*>(smem + kQB4 * kRowBytes4);
    uint32_t* lfill_all = lthr_all + kWavesM * kQB4;
    int32_t* pcst_all = reinterpret_cast<int32_t*>(lfill_all + kWavesM * kQB4);
    int32_t* tpcq = pcst_all + kWavesM * 128;
    int32_t* tthr = tpcq + kQB4;
    int32_t* tmode = tthr + kQB4;
    uint32_t* tlvl = reinterpret_cast<uint32_t*>(tmode + kQB4);
    uint32_t* wst = tlvl + kWitLevels * kQB4;
    uint32_t* lbnd_all = wst + kWitLevels * kQB4;
    uint32_t* cq_all = lbnd_all + kWavesM * kQB4;
    uint32_t* cpos_all = cq_all + kWavesM * kCandQ4;
    uint32_t* wloc = cpos_all + kWavesM * kCandQ4;  // witness counts not yet in global memory

    const int lane = lane_id();
    const int tid = (int)threadIdx.x;
    const int kg = lane >> 4;      // MFMA k quarter = output row group
    const int n16 = lane & 15;


    if constexpr (KCHUNKS) {
        for (int i = tid; i < (kQB4 - nq_tile) * (cbytes / 16); i += kWGM) {
            const int row = nq_tile + i / (cbytes / 16);
            const int col = (i % (cbytes / 16)) * 16;
            *reinterpret_cast<uint4*>(qt + row * kRowBytes4 + col) = make_uint4(0u, 0u, 0u, 0u);
        }
        fp4_stage_chunk(qx, qrow, cbytes, kRowBytes4, q0, nq_tile, wv, lane, 0, qt);
    } else {
        // the whole row fits: one plain copy for the kernel's lifetime
        const int vec_per_row = qrow / 16;
        for (int i = tid; i < kQB4 * vec_per_row; i += kWGM) {
            const int row = i / vec_per_row;
            const int col = (i - row * vec_per_row) * 16;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (row < nq_tile) v = *reinterpret_cast<const uint4*>(qx + (size_t)(q0 + row) * qrow + col);
            *reinterpret_cast<uint4*>(qt + row * kRowBytes4 + col) = v;
        }
    }
    if (tid < kQB4) {
        // tmode: 0 mixture, 1 identity; tpcq: |Q| of identity queries, 0 else.
        // A count is then c = |R| + tpcq - (1 + tmode) D in every mode.
        const int md = MODE != kModePerQuery ? MODE : (tid < nq_tile ? w.qmode[q0 + tid] : FID_MODE_MIXTURE);
        tmode[tid] = md;
        tpcq[tid] = (md == FID_MODE_IDENTITY && tid < nq_tile) ? pcq[q0 + tid] : 0;
        // threshold hit "count <= thr" is "count < thr + 1"; thr is clamped to
        // [-1, L] first (counts lie in [0, L]), which keeps every fp32 value exact
        int32_t tq = ((EPI == EPI_THRESH || EPI == EPI_BOTH) && tid < nq_tile) ? thr[q0 + tid] : -1;
        tq = tq < -1 ? -1 : (tq > w.db.n_loci ? w.db.n_loci : tq);
        tthr[tid] = tq + 1;
        for (int l = 0; l < kWitLevels; ++l) {
            tlvl[kWitLevels * tid + l] =
                (kLists && wit && tid < nq_tile) ? level[(size_t)kWitLevels * (q0 + tid) + l] : 0u;
            // staged witness counts start at zero for every item: a wave may
            // read rows whose staging another wave issues
            wst[kWitLevels * tid + l] = 0u;
            wloc[kWitLevels * tid + l] = 0u;
        }
    }
    uint32_t* lthr = lthr_all + wv * kQB4;
    uint32_t* lfill = lfill_all + wv * kQB4;
    int32_t* pcst = pcst_all + wv * 128;
    // EPI_BOTH: per row, the larger of the top-k bound and threshold + 1 --
    // the bound the accumulators start from, so that a reference is looked
    // at when either output may want it; refreshed whenever lthr changes
    uint32_t* lbnd = lbnd_all + wv * kQB4;
    lds_u32* cq = (lds_u32*)(cq_all + wv * kCandQ4);   // the wave's candidate queue
    lds_u32* cpos = (lds_u32*)(cpos_all + wv * kCandQ4);  // list slots the drain assigns
    auto refresh_lbnd = [&]() {
        if constexpr (EPI == EPI_BOTH) {
            wave_lds_sync();
            for (int i = lane_id(); i < kQB4; i += 64) lbnd[i] = max(lthr[i], (uint32_t)tthr[i]);
            wave_lds_sync();
        }
    };
    const bool witness = kLists && wit != nullptr;
    if constexpr (kLists) {
        // rows past the tile's queries get bound 0: no count is below it.
        // A caller's bound may be anything up to 0xFFFFFFFF ("no bound yet");
        // counts never exceed L, so min(bound, L + 1) filters exactly the
        // same and keeps every accumulator start an integer below 2^18,
        // exact in fp32.
        const uint32_t cap = (uint32_t)w.db.n_loci + 1u;
        for (int i = lane; i < kQB4; i += 64) {
            lthr[i] = i < nq_tile ? min(thr_init[q0 + i], cap) : 0u;
            lfill[i] = 0u;
        }
    }
    __syncthreads();
    refresh_lbnd();

    // Unit group g of reference tile t for this wave: its database block is
    // (base + 512 t + 64 wv) / 64; lane (kg, n16) loads unit 4 g + kg of
    // reference 16 j + n16 of that block.  Groups past the row (kpad may
    // exceed the row's units by up to 3) read the next block or the
    // database's slack: the matching query loci are zero.
    const int ngroups = kpad / (128 * kUnitsPerGroup4);
    const int na = (nq_tile + 15) >> 4;     // row blocks holding queries (PARTIAL)
    const int w4 = w.db.w4;
    const char* words = reinterpret_cast<const char*>(w.db.words);
    const int64_t blk0 = (base >> 6) + wv;
    const uint32_t loff = (uint32_t)kg * 1024u + (uint32_t)n16 * 16u;
    // Byte offsets of the wave's group g of tile t: wave-uniform, so a load
    // is a scalar base plus the lane's 32-bit offset.
    const char* wbase = words + blk0 * w4 * 1024;
    const int64_t tile_bytes = (int64_t)kWavesM * w4 * 1024;
    auto load_at = [&](uint4 (&dst)[kNB4], int64_t off) {
        const char* gp = wbase + off;
#pragma unroll
        for (int j = 0; j < kNB4; ++j)
            dst[j] = *reinterpret_cast<const uint4*>(gp + (loff + (uint32_t)j * 256u));
    };
    // A operand of step t of group g: query row 16 a + n16, 32-locus word
    // 4 (4 g + kg) + t of the staged row (a compile-time row stride).
    const uint8_t* arow = qt + n16 * kRowBytes4 + kg * 64;

    uint4 cur[kNB4], nxt[kNB4];
    // tiles are counted from the range start in 32 bits (a range is far
    // shorter than 2^31 tiles), which keeps the loop state in scalar registers
    const int nt = (int)(te - tb);
    if (nt > 0) load_at(cur, tb * tile_bytes);
    int64_t toff = tb * tile_bytes;
    for (int it = 0; it < nt; ++it, toff += tile_bytes) {
        const int64_t tile = tb + it;
        const int64_t rbase = base + tile * kRefsPerWG4 + (int64_t)wv * kRefsPerWave4;
        // This tile's 64 reference popcounts go to LDS while the tile is
        // scanned (two buffers: the previous tile's epilogue read the other).
        // The database popcounts are padded like its words, so every
        // reference of a tile is readable.
        int32_t* pcs = pcst + (it & 1) * 64;
        __builtin_amdgcn_global_load_lds(w.db.pc + rbase + lane, (lds_i32*)pcs, 4, 0, 0);
        // every 4th tile: the query tile's witness counts, read by the
        // epilogue; the workgroup's waves share them, each staging an eighth
        // (any value read is a count some time during the scan, and counts
        // only grow; rows past the tile's queries repeat its last query)
        if (witness && (it & 3) == 0) {
            constexpr int kPer = kWitLevels * kQB4 / kWavesM;
#pragma unroll
            for (int h = 0; h < (kPer + 63) / 64; ++h) {
                const int o = kPer * wv + 64 * h;
                if (64 * h + lane < kPer)
                    __builtin_amdgcn_global_load_lds(
                        wit + kWitLevels * q0 + min(o + lane, kWitLevels * nq_tile - 1), (lds_u32*)(wst + o), 4,
                        0, 0);
            }
        }
        // Accumulator start: 0 for full counts; for top-k and threshold the
        // row's bound (or threshold + 1) minus |Q| for identity queries, so
        // that the scan leaves x = mul D + bound - |Q| (mul = 2 for identity
        // queries, whose staged codes are doubled) and a candidate is x > |R|.
        // The values sit in the accumulator registers themselves, which keeps
        // one loop body for every tile.
        v4f acc[kQA4][kNB4];
#pragma unroll
        for (int a = 0; a < kQA4; ++a) {
            v4f init = v4f{0.f, 0.f, 0.f, 0.f};
            if constexpr (EPI != EPI_FULL) {
                const int o = 16 * a + 4 * kg;
                const uint4 bv = *reinterpret_cast<const uint4*>(
                    (EPI == EPI_THRESH ? reinterpret_cast<const uint32_t*>(tthr) : EPI == EPI_BOTH ? lbnd : lthr) +
                    o);
                const uint4 pv = *reinterpret_cast<const uint4*>(tpcq + o);
#pragma unroll
                for (int i = 0; i < 4; ++i) init[i] = (float)word_of(bv, i) - (float)word_of(pv, i);
            }
#pragma unroll
            for (int j = 0; j < kNB4; ++j) {
                acc[a][j] = init;
                __asm__ volatile("" : "+v"(acc[a][j]));
            }
        }

        // One group: prefetch the next (tile, group) into dst while the
        // MFMAs consume src.  Groups alternate between the two register sets,
        // so nothing is copied between them.
        const int64_t next_tile_off = it + 1 < nt ? toff + tile_bytes : toff;  // the last re-reads itself
        auto group = [&](const uint4 (&src)[kNB4], uint4 (&dst)[kNB4], int g) {
            if constexpr (KCHUNKS) {
                // next query chunk (every workgroup wave reaches these barriers
                // equally often: the tile range is the workgroup's)
                if ((g & 3) == 0 && (g > 0 || it > 0) && multi_chunk) {
                    __syncthreads();
                    fp4_stage_chunk(qx, qrow, cbytes, kRowBytes4, q0, nq_tile, wv, lane, g >> 2, qt);
                    __syncthreads();
                }
            }
            load_at(dst, g + 1 < ngroups ? toff + (int64_t)(g + 1) * (kUnitsPerGroup4 * 1024) : next_tile_off);
            // keep the prefetch ahead of this group's MFMAs (the scheduler
            // would otherwise sink it to its use to save registers)
            __builtin_amdgcn_sched_barrier(0);
            const uint8_t* ga = arow + (KCHUNKS ? (g & 3) : g) * 256;
#pragma unroll
            for (int t = 0; t < kUnitsPerGroup4; ++t) {
                v8i b[kNB4];
#pragma unroll
                for (int j = 0; j < kNB4; ++j) b[j] = spread_fp4(word_of(src[j], t));
#pragma unroll
                for (int a = 0; a < kQA4; ++a) {
                    if (PARTIAL && a >= na) continue;
                    const uint4 x = *reinterpret_cast<const uint4*>(ga + a * 16 * kRowBytes4 + t * 16);
                    const v8i av = v8i{(int)x.x, (int)x.y, (int)x.z, (int)x.w, 0, 0, 0, 0};
#pragma unroll
                    for (int j = 0; j < kNB4; ++j)
                        acc[a][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                            av, b[j], acc[a][j], 4, 4, 0, 0, 0, 0);
                }
            }
        };
        int g = 0;
        // a wave in its scan loop outranks one in its epilogue, so the
        // matrix-core pipe keeps being fed while the other wave selects
        __builtin_amdgcn_s_setprio(1);
#pragma unroll 1
        for (; g + 1 < ngroups; g += 2) {
            group(cur, nxt, g);
            group(nxt, cur, g + 1);
        }
        if (g < ngroups) {
            group(cur, nxt, g);
#pragma unroll
            for (int j = 0; j < kNB4; ++j) cur[j] = nxt[j];
        }
        __builtin_amdgcn_s_setprio(0);

        // ---- epilogue: lane holds D = |R AND Q'| (or |R AND Q|) of reference
        // rbase + 16 j + n16 and, in element i of row block a, tile query
        // 16 a + 4 kg + i.  The lane coordinates are re-derived here, so that
        // values computed from them stay local to the epilogue instead of
        // living (or spilling) across the scan loop.
        int lane_e = lane;
        __asm__ volatile("" : "+v"(lane_e));
        const int kg_e = lane_e >> 4;
        const int n16_e = lane_e & 15;
        if constexpr (EPI == EPI_FULL) {
            const int kg = kg_e;
            const int n16 = n16_e;
            __builtin_amdgcn_s_waitcnt(kWaitVm0);
            __asm__ volatile("" ::: "memory");
#pragma unroll
            for (int j = 0; j < kNB4; ++j) {
                const int64_t r = rbase + 16 * j + n16;
                const bool rin = r >= w.r_lo && r < w.r_hi;
                const int32_t pr = pcs[16 * j + n16];
                int32_t* col = out + (r - w.out_r_base);
#pragma unroll
                for (int a = 0; a < kQA4; ++a)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int m = 16 * a + 4 * kg + i;
                        // acc = mul D (identity codes are doubled); tpcq is 0
                        // for mixture queries
                        const int32_t c = pr + tpcq[m] - (int32_t)acc[a][j][i];
                        if (rin && m < nq_tile) col[(size_t)(q0 + m - w.out_q_base) * w.ld] = c;
                    }
            }
        } else {
            // The staged popcounts landed once every load issued before the
            // newest group prefetch has (loads complete in order).
            __builtin_amdgcn_s_waitcnt(kWaitVm0);
            __asm__ volatile("" ::: "memory");
            const int kg = kg_e;
            const int n16 = n16_e;
            // A count c = |R| + |Q| - mul D (|Q| = 0 for mixture queries) is a
            // candidate when c < bound, i.e. when the accumulator x = mul D +
            // bound - |Q| exceeds |R|.  References outside [r_lo, r_hi) compare
            // against +inf.  Every operand is an integer below 2^18, so x is
            // exact in fp32.
            const uint32_t* bnd =
                EPI == EPI_THRESH ? reinterpret_cast<const uint32_t*>(tthr) : EPI == EPI_BOTH ? lbnd : lthr;
            float prj[kNB4];
#pragma unroll
            for (int j = 0; j < kNB4; ++j) {
                const int64_t r = rbase + 16 * j + n16;
                const bool rin = r >= w.r_lo && r < w.r_hi;
                prj[j] = rin ? (float)pcs[16 * j + n16] : __builtin_huge_valf();
            }
            bool any = false;
#pragma unroll
            for (int j = 0; j < kNB4; ++j) {
                float mx = acc[0][j][0];
#pragma unroll
                for (int a = 0; a < kQA4; ++a)
#pragma unroll
                    for (int i = (a == 0 ? 1 : 0); i < 4; ++i) mx = fmaxf(mx, acc[a][j][i]);
                any |= mx > prj[j];
            }
            if (__builtin_amdgcn_ballot_w64(any)) {
                // rare.  c = |R| + bound - x with the bound the accumulators
                // started from: inserts only tighten the bounds of their own
                // row block, so each block reads its bounds before any of its
                // candidates is inserted (a full queue is drained mid-tile with
                // entries of this and earlier blocks only).
                int qn = 0;  // queued candidates (wave-uniform)
                glb_u64* wlists = (glb_u64*)(lists + ((size_t)q0 * n_workers_r + worker) * w.k);
                glb_u32* wwit = witness ? (glb_u32*)(wit + kWitLevels * q0) : nullptr;
#pragma unroll
                for (int a = 0; a < kQA4; ++a) {
                    const uint4 b0 = *reinterpret_cast<const uint4*>(bnd + 16 * a + 4 * kg);
                    // list bounds of the block (EPI_BOTH; read before any of its inserts)
                    uint4 lt = b0;
                    if constexpr (EPI == EPI_BOTH) lt = *reinterpret_cast<const uint4*>(lthr + 16 * a + 4 * kg);
#pragma unroll
                    for (int j = 0; j < kNB4; ++j) {
                        const float bmx = fmaxf(fmaxf(acc[a][j][0], acc[a][j][1]), fmaxf(acc[a][j][2], acc[a][j][3]));
                        if (!__builtin_amdgcn_ballot_w64(bmx > prj[j])) continue;
                        const int64_t r = rbase + 16 * j + n16;
                        const bool rin = prj[j] < 1.0e30f;
                        const int32_t pr = rin ? pcs[16 * j + n16] : 0;
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int m = 16 * a + 4 * kg + i;
                            const int32_t c = pr + (int32_t)word_of(b0, i) - (int32_t)acc[a][j][i];
                            if constexpr (kHits) {
                                const bool hit = rin && c < tthr[m];
                                const uint64_t hm = __builtin_amdgcn_ballot_w64(hit);
                                if (hm)
                                    mfma_append_hits(hm, hit, c, r, q0 + m, hit_count, hit_keys, hit_cnt,
                                                     w.hit_cap);
                            }
                            if constexpr (kLists) {
                                // top-k alone: the accumulators started from lthr,
                                // so c < lthr is x > |R|, with no LDS read
                                const bool cand = EPI == EPI_TOPK ? acc[a][j][i] > prj[j]
                                                                  : rin && (uint32_t)c < word_of(lt, i);
                                const uint64_t bm = __builtin_amdgcn_ballot_w64(cand);
                                if (bm) {
                                    const int nb = __popcll(bm);
                                    if (qn + nb > kCandQ4) {
                                        wave_lds_sync();
                                        mfma_insert_queue(cq, qn, rbase, wlists, (int64_t)n_workers_r * w.k, w.k,
                                                          (lds_u32*)lthr, (lds_u32*)lfill, (const lds_u32*)tlvl,
                                                          wwit);
                                        qn = 0;
                                    }
                                    if (cand) {
                                        const int pos = qn + (int)__builtin_amdgcn_mbcnt_hi(
                                                                 (uint32_t)(bm >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u));
                                        cq[pos] = (uint32_t)m | ((uint32_t)(16 * j + n16) << 7) |
                                                  ((uint32_t)c << 13);
                                    }
                                    qn += nb;
                                }
                            }
                        }
                    }
                }
                if constexpr (kLists && !DEFER) {
                    if (qn > 0) {
                        wave_lds_sync();
                        mfma_insert_queue(cq, qn, rbase, wlists, (int64_t)n_workers_r * w.k, w.k, (lds_u32*)lthr,
                                          (lds_u32*)lfill, (const lds_u32*)tlvl, wwit);
                    }
                }
                if constexpr (kLists && DEFER) {
                    if (qn > 0) {
                        wave_lds_sync();
                        const int64_t qstride = (int64_t)n_workers_r * w.k;
                        mfma_drain_decide(cq, cpos, qn, rbase, wlists, qstride, w.k, (lds_u32*)lthr,
                                          (lds_u32*)lfill, (const lds_u32*)tlvl, witness ? (lds_u32*)wloc : nullptr);
                        // the drain's list appends, issued here with nothing
                        // waiting for them, each by the lane owning its slot
                        const bool act = lane_e < qn;
                        const uint32_t v = act ? cq[lane_e] : 0u;
                        const uint32_t slot = act ? cpos[lane_e] : kNoSlot;
                        uint64_t dm = __builtin_amdgcn_ballot_w64(slot != kNoSlot);
                        while (dm) {
                            const int src = __builtin_ctzll(dm);
                            dm &= dm - 1;
                            const uint32_t ss = (uint32_t)__builtin_amdgcn_readlane((int)slot, src);
                            const uint32_t vs = (uint32_t)__builtin_amdgcn_readlane((int)v, src);
                            const uint64_t key = ((uint64_t)(vs >> 13) << kIdxBits) |
                                                 (uint64_t)(rbase + ((vs >> 7) & 63u));
                            if (lane_e == (int)(ss & 63u))
                                wlists[(size_t)(vs & 127u) * qstride + ss] = key;
                        }
                    }
                }
                refresh_lbnd();
            }
            if (witness && (it & 3) == 0) {
                if constexpr (DEFER) fp4_flush_witness(wloc, wit + kWitLevels * q0, kWitLevels * nq_tile, wv, lane_e);
                // k distinct references below one of a query's witness
                // levels make that level a bound (applied after the inserts:
                // the candidate counts above need the bounds this tile started
                // from)
#pragma unroll
                for (int h = 0; h < kQB4 / 64; ++h) {
                    const int i = lane_e + 64 * h;
                    uint32_t b = lthr[i];
#pragma unroll
                    for (int l = 0; l < kWitLevels; ++l)
                        if (wst[kWitLevels * i + l] >= (uint32_t)w.k && tlvl[kWitLevels * i + l] < b)
                            b = tlvl[kWitLevels * i + l];
                    lthr[i] = b;
                }
                wave_lds_sync();
                refresh_lbnd();
            }
        }
    }
    if constexpr (kLists) {
        wave_lds_sync();
        for (int i = lane; i < nq_tile; i += 64)
            fills[(size_t)(q0 + i) * n_workers_r + worker] = lfill[i];
        if (DEFER && witness) fp4_flush_witness(wloc, wit + kWitLevels * q0, kWitLevels * nq_tile, wv, lane);
    }
}


template <int MODE, int EPI, bool KCHUNKS>
__global__ __launch_bounds__(kWGM) void fp4_scan_kernel(
    const ScanParams p, const uint8_t* __restrict__ qx, int32_t kpad,
    const int32_t* __restrict__ pcq, int32_t* __restrict__ out, uint64_t* __restrict__ lists,
    uint32_t* __restrict__ fills, const uint32_t* __restrict__ thr_init,
    const uint32_t* __restrict__ level, uint32_t* __restrict__ wit,
    const int32_t* __restrict__ thr, unsigned long long* __restrict__ hit_count,
    uint64_t* __restrict__ hit_keys, int32_t* __restrict__ hit_cnt)
{
    const int n_qtiles = (p.q_hi - p.q_lo + kQB4 - 1) / kQB4;
    const int wg = xcd_local_index((int)blockIdx.x, (int)gridDim.x);
    const int qt_idx = wg % n_qtiles;
    const int wr_g = wg / n_qtiles;
    Fp4Work w;
    w.db = p.db;
    w.r_lo = p.r_lo;
    w.r_hi = p.r_hi;
    w.base = (p.r_lo / kDbTileRefs) * kDbTileRefs;
    const int64_t ntiles = (p.r_hi - w.base + kRefsPerWG4 - 1) / kRefsPerWG4;
    w.tb = (ntiles * wr_g) / p.n_rsplit;
    w.te = (ntiles * (wr_g + 1)) / p.n_rsplit;
    w.qx = qx;
    w.kpad = kpad;
    w.pcq = pcq;
    w.qmode = p.qmode;
    w.q0 = p.q_lo + qt_idx * kQB4;
    w.nq_tile = min(kQB4, p.q_hi - w.q0);
    w.slot = wr_g;
    w.n_slots = p.n_rsplit;
    w.k = p.k;
    w.out = out;
    w.ld = p.ld;
    w.out_q_base = p.out_q_base;
    w.out_r_base = p.out_r_base;
    w.lists = lists;
    w.fills = fills;
    w.thr_init = thr_init;
    w.level = level;
    w.wit = wit;
    w.thr = thr;
    w.hit_count = hit_count;
    w.hit_keys = hit_keys;
    w.hit_cnt = hit_cnt;
    w.hit_cap = p.hit_cap;
    w.multi_chunk = kpad > kKChunk4;
    // (the full-count epilogue keeps one instance: its partial tiles are
    // rare, and a second instance costs its loop register spills)
    if (EPI == EPI_FULL || w.nq_tile > kQB4 - 16) fp4_work<MODE, EPI, KCHUNKS, false, true>(w);
    else fp4_work<MODE, EPI, KCHUNKS, EPI != EPI_FULL, true>(w);
}

// The staged codes of one 32-locus query word: the reciprocals of the
// reference values, so that every product is 1; doubled for identity
// queries (products 2: the scan then accumulates 2 D, the XOR count's
// multiple of D).  (e2m1 codes: 0x1 = 0.5, 0x2 = 1.0, 0x4 = 2.0, 0x6 = 4.0;
// a code times a 0/1 nibble is that code or 0.)
__device__ __forceinline__ uint4 fp4_query_codes(uint32_t w, bool dbl)
{
    uint4 v;
    v.x = (w & 0x11111111u) * (dbl ? 0x6u : 0x4u);          // 2.0 (4.0)
    v.y = ((w >> 1) & 0x11111111u) * (dbl ? 0x4u : 0x2u);   // 1.0 (2.0)
    v.z = ((w >> 2) & 0x11111111u) * (dbl ? 0x2u : 0x1u);   // 0.5 (1.0)
    v.w = ((w >> 3) & 0x11111111u) * (dbl ? 0x2u : 0x1u);   // 0.5 (1.0)
    return v;
}

// Staged queries for the fp4 kernel: for every 32-locus word, 4 dwords in the
// element order above (loci >= L cleared), plus popcount(Q_q).
__global__ void expand_queries_fp4_kernel(const uint64_t* __restrict__ q, int32_t n_q,
                                          int32_t row_words, int32_t n_loci, int mode,
                                          const int32_t* __restrict__ qmode,
                                          uint8_t* __restrict__ qx, int32_t kpad,
                                          int32_t* __restrict__ pcq)
{
    const int32_t words = kpad / 32;
    const int64_t total = (int64_t)n_q * words;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / words;
        const int32_t wi = (int32_t)(t - i * words);
        const int32_t k0 = wi * 32;
        uint32_t w = 0;
        if (k0 < n_loci) {
            w = reinterpret_cast<const uint32_t*>(q + i * row_words)[wi];
            if (k0 + 32 > n_loci) w &= (1u << (n_loci - k0)) - 1u;
        }
        const int md = mode == kModePerQuery ? qmode[i] : mode;
        reinterpret_cast<uint4*>(qx + i * (kpad / 2))[wi] = fp4_query_codes(w, md == FID_MODE_IDENTITY);
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_q;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t s = 0;
        const int32_t full = n_loci >> 6;
        for (int32_t w = 0; w < full; ++w) s += __popcll(q[i * row_words + w]);
        if (n_loci & 63) s += __popcll(q[i * row_words + full] & ((1ull << (n_loci & 63)) - 1ull));
        pcq[i] = s;
    }
}

hipError_t launch_expand_queries_fp4(const uint64_t* q, int32_t n_q, int32_t row_words,
                                     int32_t n_loci, int mode, const int32_t* qmode, uint8_t* qx,
                                     int32_t kpad, int32_t* pcq, hipStream_t s)
{
    const int64_t total = (int64_t)n_q * (kpad / 32);
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(expand_queries_fp4_kernel, dim3((unsigned)blocks), dim3(256), 0, s, q, n_q,
                       row_words, n_loci, mode, qmode, qx, kpad, pcq);
    return hipGetLastError();
}

// ---------------------------------------------------------- batched passes
static size_t fp4_lds_bytes(int32_t kpad);

// Persistent fp4 pass: every workgroup takes work items from the queue of
// its own XCD (workgroups are dealt to the 8 XCDs round-robin, so those of
// one XCD -- and the items of one queue, which the planner fills range by
// range -- share that XCD's L2), then from the other queues, until all are
// empty.  An item is one query tile of one job against a run of reference
// tiles; the job's queries carry their own modes.
template <int EPI>
__global__ __launch_bounds__(kWGM) void fp4_batch_kernel(const Fp4BatchSet* __restrict__ sets,
                                                         const Fp4BatchItem* __restrict__ items,
                                                         const int32_t* __restrict__ queue_off,
                                                         unsigned int* __restrict__ counters)
{
    __shared__ int s_item;
    const int home = (int)(blockIdx.x & 7u);
    for (int h = 0; h < 8; ++h) {
        const int qi = (home + h) & 7;
        const int32_t first = queue_off[qi];
        const uint32_t n_in = (uint32_t)(queue_off[qi + 1] - first);
        for (;;) {
            if (threadIdx.x == 0) {
                const uint32_t t = atomicAdd(counters + qi, 1u);
                s_item = t < n_in ? first + (int)t : -1;
            }
            __syncthreads();
            const int it = __builtin_amdgcn_readfirstlane(s_item);
            __syncthreads();  // every wave has read s_item before the next item overwrites it
            if (it < 0) break;
            const Fp4BatchItem item = items[it];
            const Fp4BatchSet& S = sets[item.set];
            Fp4Work w;
            w.db = S.db;
            w.r_lo = S.r_lo;
            w.r_hi = S.r_hi;
            w.base = (S.r_lo / kDbTileRefs) * kDbTileRefs;
            w.tb = item.tb;
            w.te = item.te;
            w.qx = S.qx;
            w.kpad = S.kpad;
            w.multi_chunk = S.kpad > kKChunk4;
            w.pcq = S.pcq;
            w.qmode = S.qmode;
            w.q0 = item.qtile * kQB4;
            w.nq_tile = min(kQB4, S.n_q - w.q0);
            w.slot = item.slot;
            w.n_slots = S.n_slots;
            w.k = S.k;
            w.out = S.out;
            w.ld = S.ld;
            w.out_q_base = 0;
            w.out_r_base = S.out_r_base;
            w.lists = S.lists;
            w.fills = S.fills;
            w.thr_init = S.thr_init;
            w.level = S.level;
            w.wit = S.wit;
            w.thr = nullptr;
            w.hit_count = nullptr;
            w.hit_keys = nullptr;
            w.hit_cnt = nullptr;
            w.hit_cap = 0;
            // the end-of-tile drain writes its lists itself here: with two
            // copies of the scan in the persistent kernel, the inline stores
            // of the deferred form leave too few registers (spills inside the
            // scan loop), and a single copy that skips empty row blocks costs
            // full tiles 8%
            if (EPI == EPI_FULL || w.nq_tile > kQB4 - 16) fp4_work<kModePerQuery, EPI, true, false, false>(w);
            else fp4_work<kModePerQuery, EPI, true, EPI != EPI_FULL, false>(w);
            __syncthreads();  // the next item restages the LDS tile
        }
    }
}

hipError_t launch_fp4_batch(int epi, const Fp4BatchSet* sets, const Fp4BatchItem* items, const int32_t* queue_off,
                            unsigned int* counters, int32_t grid, hipStream_t s)
{
    if (grid <= 0) return hipSuccess;
    const size_t lds = fp4_lds_bytes(kKChunk4);
    if (epi == EPI_FULL) {
        const hipError_t e = lds_opt_in<&fp4_batch_kernel<EPI_FULL>>((int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(fp4_batch_kernel<EPI_FULL>, dim3((unsigned)grid), dim3(kWGM), lds, s, sets, items,
                           queue_off, counters);
    } else if (epi == EPI_TOPK) {
        const hipError_t e = lds_opt_in<&fp4_batch_kernel<EPI_TOPK>>((int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(fp4_batch_kernel<EPI_TOPK>, dim3((unsigned)grid), dim3(kWGM), lds, s, sets, items,
                           queue_off, counters);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

__global__ void expand_batch_fp4_kernel(const Fp4ExpandJob* __restrict__ jobs, int32_t n_jobs, int64_t total_words,
                                        int64_t total_q, const int32_t* __restrict__ qmode,
                                        int32_t* __restrict__ pcq)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total_words;
         t += (int64_t)gridDim.x * blockDim.x) {
        int a = 0, b = n_jobs;  // the last job with w_off <= t
        while (b - a > 1) {
            const int m = (a + b) >> 1;
            if (jobs[m].w_off <= t) a = m;
            else b = m;
        }
        const Fp4ExpandJob& J = jobs[a];
        const int32_t words = J.kpad / 32;
        const int64_t rel = t - J.w_off;
        const int64_t i = rel / words;
        const int32_t wi = (int32_t)(rel - i * words);
        const int32_t k0 = wi * 32;
        uint32_t w = 0;
        if (k0 < J.n_loci) {
            w = reinterpret_cast<const uint32_t*>(J.q + i * J.row_words)[wi];
            if (k0 + 32 > J.n_loci) w &= (1u << (J.n_loci - k0)) - 1u;
        }
        reinterpret_cast<uint4*>(J.qx + i * (J.kpad / 2))[wi] =
            fp4_query_codes(w, qmode[J.q_off + i] == FID_MODE_IDENTITY);
    }
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total_q;
         g += (int64_t)gridDim.x * blockDim.x) {
        int a = 0, b = n_jobs;  // the last job with q_off <= g
        while (b - a > 1) {
            const int m = (a + b) >> 1;
            if (jobs[m].q_off <= g) a = m;
            else b = m;
        }
        const Fp4ExpandJob& J = jobs[a];
        const uint64_t* row = J.q + (g - J.q_off) * J.row_words;
        int32_t c = 0;
        const int32_t full = J.n_loci >> 6;
        for (int32_t w = 0; w < full; ++w) c += __popcll(row[w]);
        if (J.n_loci & 63) c += __popcll(row[full] & ((1ull << (J.n_loci & 63)) - 1ull));
        pcq[g] = c;
    }
}

hipError_t launch_expand_batch_fp4(const Fp4ExpandJob* jobs, int32_t n_jobs, int64_t total_words, int64_t total_q,
                                   const int32_t* qmode, int32_t* pcq, hipStream_t s)
{
    if (n_jobs <= 0) return hipSuccess;
    int64_t blocks = ((total_words > total_q ? total_words : total_q) + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(expand_batch_fp4_kernel, dim3((unsigned)blocks), dim3(256), 0, s, jobs, n_jobs, total_words,
                       total_q, qmode, pcq);
    return hipGetLastError();
}

// Loci padded to whole 4-unit load groups (512 loci); zero on the query side.
int fp4_kpad(int32_t n_loci) { return ((n_loci + 511) / 512) * 512; }
int fp4_max_kpad() { return kMaxKpad4; }
int fp4_refs_per_wg() { return kRefsPerWG4; }
int fp4_queries_per_wg() { return kQB4; }
int fp4_list_workers_per_wg() { return kWavesM; }

static size_t fp4_lds_bytes(int32_t kpad)
{
    (void)kpad;
    return (size_t)kQB4 * kRowBytes4 + 2 * (size_t)kWavesM * kQB4 * 4 + (size_t)kWavesM * 128 * 4 +
           3 * (size_t)kQB4 * 4 + 2 * (size_t)kWitLevels * kQB4 * 4 + (size_t)kWavesM * kQB4 * 4 +
           2 * (size_t)kWavesM * kCandQ4 * 4 + (size_t)kWitLevels * kQB4 * 4;
}
// (the persistent batch kernel adds one static int for its work queue)
static_assert(kQB4 * kRowBytes4 + 2 * kWavesM * kQB4 * 4 + kWavesM * 128 * 4 + 3 * kQB4 * 4 +
                      2 * kWitLevels * kQB4 * 4 + kWavesM * kQB4 * 4 + 2 * kWavesM * kCandQ4 * 4 +
                      kWitLevels * kQB4 * 4 + 16 <= 163840,
              "fp4 query tile and epilogue state must fit the 160 KiB LDS");
static_assert(kKChunk4 % 512 == 0, "chunks hold whole 4-unit load groups");

template <int MODE, int EPI, bool KCHUNKS>
static hipError_t launch_fp4_t(const ScanParams& p, const MfmaBuffers& b, hipStream_t s)
{
    if (b.kpad > kMaxKpad4 || b.kpad % 512 != 0) return hipErrorInvalidValue;
    const int n_qtiles = (p.q_hi - p.q_lo + kQB4 - 1) / kQB4;
    const int64_t blocks = (int64_t)n_qtiles * p.n_rsplit;
    const hipError_t e = lds_opt_in<&fp4_scan_kernel<MODE, EPI, KCHUNKS>>((int)fp4_lds_bytes(kKChunk4));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((fp4_scan_kernel<MODE, EPI, KCHUNKS>), dim3((unsigned)blocks), dim3(kWGM),
                       fp4_lds_bytes(b.kpad), s, p, b.qx, b.kpad, b.pcq, b.out, b.lists, b.fills,
                       b.thr_init, b.level, b.wit, b.thr, b.hit_count, b.hit_keys, b.hit_cnt);
    return hipGetLastError();
}

template <bool KCHUNKS>
static hipError_t launch_fp4_k(int mode, int epi, const ScanParams& p, const MfmaBuffers& b, hipStream_t s)
{
    if (mode == kModePerQuery) {
        if (epi == EPI_FULL) return launch_fp4_t<kModePerQuery, EPI_FULL, KCHUNKS>(p, b, s);
        if (epi == EPI_TOPK) return launch_fp4_t<kModePerQuery, EPI_TOPK, KCHUNKS>(p, b, s);
        return hipErrorInvalidValue;
    }
    if (mode == FID_MODE_MIXTURE) {
        if (epi == EPI_FULL) return launch_fp4_t<FID_MODE_MIXTURE, EPI_FULL, KCHUNKS>(p, b, s);
        if (epi == EPI_TOPK) return launch_fp4_t<FID_MODE_MIXTURE, EPI_TOPK, KCHUNKS>(p, b, s);
        if (epi == EPI_BOTH) return launch_fp4_t<FID_MODE_MIXTURE, EPI_BOTH, KCHUNKS>(p, b, s);
        return launch_fp4_t<FID_MODE_MIXTURE, EPI_THRESH, KCHUNKS>(p, b, s);
    }
    if (epi == EPI_FULL) return launch_fp4_t<FID_MODE_IDENTITY, EPI_FULL, KCHUNKS>(p, b, s);
    if (epi == EPI_TOPK) return launch_fp4_t<FID_MODE_IDENTITY, EPI_TOPK, KCHUNKS>(p, b, s);
    if (epi == EPI_BOTH) return launch_fp4_t<FID_MODE_IDENTITY, EPI_BOTH, KCHUNKS>(p, b, s);
    return launch_fp4_t<FID_MODE_IDENTITY, EPI_THRESH, KCHUNKS>(p, b, s);
}

hipError_t launch_fp4_scan(int mode, int epi, const ScanParams& p, const MfmaBuffers& b,
                           hipStream_t s)
{
    if (p.n_rsplit <= 0) return hipSuccess;
    if (b.kpad > kKChunk4) return launch_fp4_k<true>(mode, epi, p, b, s);
    return launch_fp4_k<false>(mode, epi, p, b, s);
}

}  // namespace fid
