// libfastid device code for gfx950 (CDNA4, wave64).
//
// The comparison is the overloaded matrix product of Section II-B: for query
// q and reference r, C[q][r] = sum over 32-locus words w of
// popcount(op(R_r[w], Q_q[w])), where op is AND-NOT (Eq. 1, mixture) or XOR
// (identity).  Every count is an exact integer.
//
// Scan kernel layout (bound: the VALU, 2 ops per 32 loci of a query-reference pair):
//   * one wave = one worker; each lane owns one reference of a 64-reference
//     block and keeps a chunk of its words in VGPRs (register blocking,
//     Section III-B);
//   * the worker walks its query range; a query's words are wave-uniform and
//     are fetched with scalar loads into SGPRs, so the inner loop is exactly
//     one VALU logic op (v_and_b32 against the pre-inverted query word, or
//     v_xor_b32) and one v_bcnt_u32_b32 (popcount fused with the
//     accumulate) per 32 loci;
//   * the count is consumed in registers by the epilogue: a store (full
//     matrix / tiles), a filter into per-worker top-k lists, or a threshold
//     hit append; the query x reference matrix is never written for top-k or
//     threshold output (the reduction-on-GPU Section IV proposes).
#include <type_traits>

#include "fid_device.hpp"

namespace fid {

__device__ __forceinline__ uint64_t bits_below(int64_t word_index, int32_t n_loci)
{
    const int64_t base = word_index * 64;
    if (base >= n_loci) return 0ull;
    if (base + 64 <= n_loci) return ~0ull;
    return (1ull << (n_loci - base)) - 1ull;
}

// ------------------------------------------------------------------ pack
// Section II-A encoding: locus k of a row -> bit (k & 63) of 64-bit word k >> 6.
__global__ void pack_kernel(const uint8_t* __restrict__ bytes, int64_t n, int32_t n_loci,
                            int64_t ld, int32_t row_words, uint64_t* __restrict__ out,
                            int* __restrict__ bad)
{
    const int64_t total = n * row_words;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / row_words;
        const int32_t k0 = (int32_t)(t - i * row_words) * 64;
        const uint8_t* src = bytes + i * ld + k0;
        uint64_t word = 0;
        uint32_t badbits = 0;
        if (k0 + 64 <= n_loci && ((reinterpret_cast<uintptr_t>(src) & 15u) == 0)) {
            const uint4* s4 = reinterpret_cast<const uint4*>(src);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint4 v = s4[j];
                const uint32_t xs[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    // bytes b0..b3 in {0,1}: x * 0x204081 places b_j at bit 21 + j
                    // with no carries, gathering the four bits into a nibble.
                    badbits |= xs[h] & 0xFEFEFEFEu;
                    const uint32_t nib = ((xs[h] * 0x204081u) >> 21) & 0xFu;
                    word |= (uint64_t)nib << (16 * j + 4 * h);
                }
            }
        } else {
            for (int32_t b = 0; b < 64 && k0 + b < n_loci; ++b) {
                const uint8_t x = src[b];
                badbits |= x & 0xFEu;
                word |= (uint64_t)(x & 1u) << b;
            }
        }
        out[t] = word;
        if (badbits) atomicOr(bad, 1);
    }
}

// Per-query modes must be FID_MODE_MIXTURE or FID_MODE_IDENTITY.
__global__ void check_modes_kernel(const int32_t* __restrict__ modes, int32_t n, int* __restrict__ bad)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t m = modes[i];
        if (m != FID_MODE_MIXTURE && m != FID_MODE_IDENTITY) atomicOr(bad, 1);
    }
}

hipError_t launch_check_modes(const int32_t* modes, int32_t n, int* bad, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = ((int64_t)n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(check_modes_kernel, dim3((unsigned)blocks), dim3(256), 0, s, modes, n, bad);
    return hipGetLastError();
}

hipError_t launch_pack(const uint8_t* bytes, int64_t n, int32_t n_loci, int64_t ld,
                       int32_t row_words, uint64_t* out, int* bad, hipStream_t s)
{
    const int64_t total = n * row_words;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)blocks), dim3(256), 0, s, bytes, n, n_loci,
                       ld, row_words, out, bad);
    return hipGetLastError();
}

// ------------------------------------------------------------------ genotype pack
// Genotype profiles (Section II-A: 0, 1 or 2 copies of the minor allele per
// locus) -> 1-bit rows of 2 L loci: locus k becomes bits 2k (at least one
// minor allele) and 2k + 1 (two).  On these planes popcount(R XOR Q) counts
// the minor alleles by which two genotypes differ and popcount(R AND NOT Q)
// the reference's minor-allele copies beyond the query's, so every
// comparison kernel applies unchanged.  One thread per output word (32 loci).
__global__ void pack_genotypes_kernel(const uint8_t* __restrict__ geno, int64_t n, int32_t n_loci, int64_t ld,
                                      int32_t row_words, uint64_t* __restrict__ out, int* __restrict__ bad)
{
    const int64_t total = n * row_words;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / row_words;
        const int32_t w = (int32_t)(t - i * row_words);
        const int32_t k0 = w * 32;
        const uint8_t* src = geno + i * ld;
        uint64_t word = 0;
        uint32_t over = 0;
        for (int32_t j = 0; j < 32 && k0 + j < n_loci; ++j) {
            const uint32_t g = src[k0 + j];
            over |= g > 2u ? 1u : 0u;
            word |= (uint64_t)(g >= 1u) << (2 * j);
            word |= (uint64_t)(g >= 2u) << (2 * j + 1);
        }
        out[t] = word;
        if (over) *bad = 1;
    }
}

hipError_t launch_pack_genotypes(const uint8_t* geno, int64_t n, int32_t n_loci, int64_t ld, int32_t row_words,
                                 uint64_t* out, int* bad, hipStream_t s)
{
    int64_t blocks = (n * row_words + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(pack_genotypes_kernel, dim3((unsigned)blocks), dim3(256), 0, s, geno, n, n_loci, ld,
                       row_words, out, bad);
    return hipGetLastError();
}

// ------------------------------------------------------------------ database build
// Row-major packed rows -> interleaved 16-byte units (coalesced per wave),
// loci >= L cleared; then per-reference minor-allele totals.
__global__ void db_build_kernel(const uint64_t* __restrict__ rows, int64_t n_refs,
                                int32_t row_words, int32_t n_loci, uint4* __restrict__ words,
                                int32_t w4, int64_t nblk)
{
    const int64_t total = nblk * w4 * 64;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int lane = (int)(t & 63);
        const int64_t rest = t >> 6;
        const int32_t u = (int32_t)(rest % w4);
        const int64_t blk = rest / w4;
        const int64_t r = blk * 64 + lane;
        uint64_t a = 0, b = 0;
        if (r < n_refs) {
            const uint64_t* src = rows + r * row_words + 2 * u;
            a = src[0] & bits_below(2 * u, n_loci);
            b = src[1] & bits_below(2 * u + 1, n_loci);
        }
        words[t] = make_uint4((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32));
    }
}

__global__ void db_popcount_kernel(const uint4* __restrict__ words, int32_t w4, int64_t nblk,
                                   int32_t* __restrict__ pc)
{
    const int64_t total = nblk * 64;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t blk = t >> 6;
        const int lane = (int)(t & 63);
        const uint4* src = words + blk * w4 * 64 + lane;
        int32_t sum = 0;
        for (int32_t u = 0; u < w4; ++u) {
            const uint4 v = src[(int64_t)u * 64];
            sum += __builtin_popcount(v.x) + __builtin_popcount(v.y) + __builtin_popcount(v.z) +
                   __builtin_popcount(v.w);
        }
        pc[t] = sum;
    }
}

hipError_t launch_db_build(const uint64_t* rows, int64_t n_refs, int32_t row_words,
                           int32_t n_loci, uint4* words, int32_t* pc, int32_t w4, int64_t nblk,
                           hipStream_t s)
{
    int64_t total = nblk * w4 * 64;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(db_build_kernel, dim3((unsigned)blocks), dim3(256), 0, s, rows, n_refs,
                       row_words, n_loci, words, w4, nblk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    total = nblk * 64;
    blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(db_popcount_kernel, dim3((unsigned)blocks), dim3(256), 0, s, words, w4,
                       nblk, pc);
    return hipGetLastError();
}

// ------------------------------------------------------------------ query staging
// Packed query rows -> [n_q][qw] 32-bit words, loci >= L cleared, zero padded
// to the scan's chunk width.  Mixture queries are stored inverted so that
// Eq. 1 becomes a plain AND: (R ^ Q) & R == R & ~Q.
__global__ void stage_kernel(const uint64_t* __restrict__ q, int32_t n_q, int32_t row_words,
                             int32_t n_loci, int mode, const int32_t* __restrict__ qmode,
                             uint32_t* __restrict__ out, int32_t qw)
{
    const int64_t total = (int64_t)n_q * qw;
    const int32_t l32 = (n_loci + 31) / 32;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / qw;
        const int32_t w = (int32_t)(t - i * qw);
        uint32_t v = 0;
        if (w < l32) {
            v = reinterpret_cast<const uint32_t*>(q + i * row_words)[w];
            if (w == l32 - 1 && (n_loci & 31)) v &= (1u << (n_loci & 31)) - 1u;
        }
        if ((mode == kModePerQuery ? qmode[i] : mode) == FID_MODE_MIXTURE) v = ~v;
        out[t] = v;
    }
}

hipError_t launch_stage_queries(const uint64_t* q, int32_t n_q, int32_t row_words,
                                int32_t n_loci, int mode, const int32_t* qmode, uint32_t* out,
                                int32_t qw, hipStream_t s)
{
    const int64_t total = (int64_t)n_q * qw;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(stage_kernel, dim3((unsigned)blocks), dim3(256), 0, s, q, n_q, row_words,
                       n_loci, mode, qmode, out, qw);
    return hipGetLastError();
}

__device__ __noinline__ void thresh_append(uint64_t m, int q, int64_t rbase, uint32_t acc,
                                           unsigned long long* __restrict__ hit_count,
                                           uint64_t* __restrict__ hit_keys,
                                           int32_t* __restrict__ hit_cnt, int64_t cap)
{
    const int lane = lane_id();
    const int first = __ffsll((unsigned long long)m) - 1;
    unsigned long long base = 0;
    if (lane == first) base = atomicAdd(hit_count, (unsigned long long)__popcll(m));
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)base, first);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(base >> 32), first);
    base = ((unsigned long long)hi << 32) | lo;
    if ((m >> lane) & 1ull) {
        const unsigned long long pos = base + (unsigned long long)__popcll(m & ((1ull << lane) - 1ull));
        if (pos < (unsigned long long)cap) {
            hit_keys[pos] = ((uint64_t)q << kIdxBits) | (uint64_t)(rbase + lane);
            hit_cnt[pos] = (int32_t)acc;
        }
    }
}

// ------------------------------------------------------------------ the scan
template <int MODE, int NW, int EPI, bool CHUNKED, int RPL>
__global__ __launch_bounds__(kWG) void scan_kernel(
    const ScanParams p, const uint32_t* __restrict__ qs, int32_t* __restrict__ out,
    uint64_t* __restrict__ lists, uint32_t* __restrict__ fills,
    const uint32_t* __restrict__ thr_init, const int32_t* __restrict__ thr,
    unsigned long long* __restrict__ hit_count, uint64_t* __restrict__ hit_keys,
    int32_t* __restrict__ hit_cnt)
{
    static_assert(!CHUNKED || RPL == 1, "chunked rows keep one reference per lane");
    static_assert(NW % 16 == 0, "query rows are read in 16-dword groups");
    extern __shared__ uint32_t lds[];
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int worker = (int)blockIdx.x * kWavesPerWG + wv;
    if (worker >= p.n_workers) return;
    const int wr = worker % p.n_rsplit;
    const int wq = worker / p.n_rsplit;
    const int q0 = p.q_lo + wq * p.q_per_worker;
    const int q1 = min(q0 + p.q_per_worker, p.q_hi);
    if (q0 >= q1) return;
    const int64_t b0 = p.blk_lo + (p.nblk * wr) / p.n_rsplit;
    const int64_t b1 = p.blk_lo + (p.nblk * (wr + 1)) / p.n_rsplit;

    uint32_t* wl = lds + wv * p.lds_words_per_wave;
    uint32_t* lthr = wl;                                        // EPI_TOPK: [q_per_worker]
    uint32_t* lfill = wl + p.q_per_worker;                      // EPI_TOPK: [q_per_worker]
    // CHUNKED: partial counts [q][64] as 16-bit values (a count is at most L < 2^16)
    uint16_t* lacc = reinterpret_cast<uint16_t*>(wl + (EPI == EPI_TOPK ? 2 * p.q_per_worker : 0));
    if constexpr (EPI == EPI_TOPK) {
        for (int i = lane; i < q1 - q0; i += 64) {
            lthr[i] = thr_init[q0 + i];
            lfill[i] = 0u;
        }
        wave_lds_sync();
    }

    const int nch = CHUNKED ? p.nchunks : 1;
    for (int64_t blk = b0; blk < b1; blk += RPL) {
        bool rin[RPL];
        const uint4* src[RPL];
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
            const int64_t r = (blk + j) * 64 + lane;
            rin[j] = (blk + j < b1) && (r >= p.r_lo) && (r < p.r_hi);
            src[j] = p.db.words + (size_t)(blk + j) * p.db.w4 * 64 + lane;
        }
        for (int c = 0; c < nch; ++c) {
            uint32_t R[RPL][NW];
#pragma unroll
            for (int j = 0; j < RPL; ++j) {
#pragma unroll
                for (int i = 0; i < NW / 4; ++i) {
                    const int u = c * (NW / 4) + i;
                    uint4 v = make_uint4(0u, 0u, 0u, 0u);
                    if (u < p.db.w4 && blk + j < b1) v = src[j][(size_t)u * 64];
                    R[j][4 * i + 0] = v.x;
                    R[j][4 * i + 1] = v.y;
                    R[j][4 * i + 2] = v.z;
                    R[j][4 * i + 3] = v.w;
                }
            }
            kptr_u32 qrow = (kptr_u32)(qs + (size_t)q0 * p.qw + c * NW);
            for (int q = q0; q < q1; ++q, qrow += p.qw) {
                uint32_t acc[RPL];
#pragma unroll
                for (int j = 0; j < RPL; ++j)
                    acc[j] = (CHUNKED && c > 0) ? lacc[(q - q0) * 64 + lane] : 0u;
                // one logic op per 32 loci: AND with the inverted query (Eq. 1) or XOR
                // the query row comes in 16-dword scalar loads (a 64-byte-aligned row chunk)
                auto accumulate = [&](auto is_mix) {
#pragma unroll
                    for (int g = 0; g < NW / 16; ++g) {
                        const u32x16 qg = ((kptr_u32x16)qrow)[g];
#pragma unroll
                        for (int w2 = 0; w2 < 16; ++w2) {
                            const int w = g * 16 + w2;
                            const uint32_t qv = qg[w2];
#pragma unroll
                            for (int j = 0; j < RPL; ++j) {
                                const uint32_t x = decltype(is_mix)::value ? (R[j][w] & qv) : (R[j][w] ^ qv);
                                acc[j] = popc_acc(x, acc[j]);
                            }
                        }
                    }
                };
                if (MODE == FID_MODE_MIXTURE || (MODE == kModePerQuery && p.qmode[q] == FID_MODE_MIXTURE))
                    accumulate(std::true_type{});
                else
                    accumulate(std::false_type{});
                if (CHUNKED && c + 1 < nch) {
                    lacc[(q - q0) * 64 + lane] = (uint16_t)acc[0];
                    continue;
                }
#pragma unroll
                for (int j = 0; j < RPL; ++j) {
                    const int64_t rb = (blk + j) * 64;
                    if constexpr (EPI == EPI_FULL) {
                        if (rin[j])
                            out[(size_t)(q - p.out_q_base) * p.ld + (rb + lane - p.out_r_base)] = (int32_t)acc[j];
                    } else if constexpr (EPI == EPI_TOPK) {
                        const uint32_t t = lthr[q - q0];
                        const uint64_t m = __builtin_amdgcn_ballot_w64(rin[j] && acc[j] < t);
                        if (m)
                            topk_insert(lists + ((size_t)q * p.n_rsplit + wr) * p.k, p.k, rb,
                                        acc[j], m, lthr + (q - q0), lfill + (q - q0));
                    } else {
                        const int32_t t = thr[q];
                        const uint64_t m = __builtin_amdgcn_ballot_w64(rin[j] && (int32_t)acc[j] <= t);
                        if (m) thresh_append(m, q, rb, acc[j], hit_count, hit_keys, hit_cnt, p.hit_cap);
                    }
                }
            }
        }
    }
    if constexpr (EPI == EPI_TOPK) {
        wave_lds_sync();
        for (int i = lane; i < q1 - q0; i += 64)
            fills[(size_t)(q0 + i) * p.n_rsplit + wr] = lfill[i];
    }
}

template <int MODE, int NW, int EPI, bool CH, int RPL>
static hipError_t launch_scan_t(const ScanParams& p, const ScanBuffers& b, hipStream_t s)
{
    const int blocks = (p.n_workers + kWavesPerWG - 1) / kWavesPerWG;
    const size_t lds = (size_t)p.lds_words_per_wave * kWavesPerWG * sizeof(uint32_t);
    hipLaunchKernelGGL((scan_kernel<MODE, NW, EPI, CH, RPL>), dim3(blocks), dim3(kWG), lds, s, p,
                       b.qs, b.out, b.lists, b.fills, b.thr_init, b.thr, b.hit_count, b.hit_keys,
                       b.hit_cnt);
    return hipGetLastError();
}

template <int MODE, int EPI>
static hipError_t launch_scan_m(int nw, bool chunked, int rpl, const ScanParams& p,
                                const ScanBuffers& b, hipStream_t s)
{
    if (chunked) return launch_scan_t<MODE, 64, EPI, true, 1>(p, b, s);
    if (rpl == 2) {
        switch (nw) {
            case 16: return launch_scan_t<MODE, 16, EPI, false, 2>(p, b, s);
            case 32: return launch_scan_t<MODE, 32, EPI, false, 2>(p, b, s);
            case 64: return launch_scan_t<MODE, 64, EPI, false, 2>(p, b, s);
            default: break;
        }
    }
    switch (nw) {
        case 16: return launch_scan_t<MODE, 16, EPI, false, 1>(p, b, s);
        case 32: return launch_scan_t<MODE, 32, EPI, false, 1>(p, b, s);
        case 64: return launch_scan_t<MODE, 64, EPI, false, 1>(p, b, s);
        case 128: return launch_scan_t<MODE, 128, EPI, false, 1>(p, b, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_scan(int mode, int nw, int epi, bool chunked, int rpl, const ScanParams& p,
                       const ScanBuffers& b, hipStream_t s)
{
    if (p.n_workers <= 0) return hipSuccess;
    if (mode == kModePerQuery) {
        if (epi == EPI_FULL) return launch_scan_m<kModePerQuery, EPI_FULL>(nw, chunked, rpl, p, b, s);
        if (epi == EPI_TOPK) return launch_scan_m<kModePerQuery, EPI_TOPK>(nw, chunked, rpl, p, b, s);
        return hipErrorInvalidValue;
    }
    if (mode == FID_MODE_MIXTURE) {
        if (epi == EPI_FULL) return launch_scan_m<FID_MODE_MIXTURE, EPI_FULL>(nw, chunked, rpl, p, b, s);
        if (epi == EPI_TOPK) return launch_scan_m<FID_MODE_MIXTURE, EPI_TOPK>(nw, chunked, rpl, p, b, s);
        return launch_scan_m<FID_MODE_MIXTURE, EPI_THRESH>(nw, chunked, rpl, p, b, s);
    }
    if (epi == EPI_FULL) return launch_scan_m<FID_MODE_IDENTITY, EPI_FULL>(nw, chunked, rpl, p, b, s);
    if (epi == EPI_TOPK) return launch_scan_m<FID_MODE_IDENTITY, EPI_TOPK>(nw, chunked, rpl, p, b, s);
    return launch_scan_m<FID_MODE_IDENTITY, EPI_THRESH>(nw, chunked, rpl, p, b, s);
}

// ------------------------------------------------------------------ tiles in one launch
// Full counts of many th x tw tiles at arbitrary (q0, r0): one wave per
// (tile, 64-reference column block, group of <= kTileQueries queries).  Each
// lane owns one reference (a tile's columns need not be block aligned) and
// holds a 64-word chunk of its row in VGPRs; query words come through scalar
// loads and partial counts of longer rows wait in LDS.
constexpr int kTileQueries = 16;
constexpr int kTileNW = 64;

template <int MODE>
__global__ __launch_bounds__(kWG) void tile_counts_kernel(const DbView db, const uint32_t* __restrict__ qs,
                                                          int32_t qw, TileTable tt, int32_t th, int32_t tw,
                                                          int32_t* __restrict__ out)
{
    __shared__ uint32_t lacc_all[kWavesPerWG][kTileQueries * 64];
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    uint32_t* lacc = lacc_all[wv];
    const int nrb = (tw + 63) / 64, nqg = (th + kTileQueries - 1) / kTileQueries;
    const int64_t w = (int64_t)blockIdx.x * kWavesPerWG + wv;
    if (w >= (int64_t)tt.n * nrb * nqg) return;
    const int t = (int)(w / (nrb * nqg));
    const int rem = (int)(w - (int64_t)t * nrb * nqg);
    const int rb = rem / nqg, qg = rem - rb * nqg;
    const int col = rb * 64 + lane;
    const bool cin = col < tw;
    const int64_t r = tt.r0[t] + (cin ? col : 0);
    const uint4* src = db.words + (size_t)(r >> 6) * db.w4 * 64 + (r & 63);
    const int q0 = (int)tt.q0[t] + qg * kTileQueries;
    const int nq = min(kTileQueries, th - qg * kTileQueries);
    const int nch = qw / kTileNW;
    int32_t* dst = out + ((size_t)tt.out_index[t] * th + qg * kTileQueries) * tw + col;
    for (int c = 0; c < nch; ++c) {
        uint32_t R[kTileNW];
#pragma unroll
        for (int i = 0; i < kTileNW / 4; ++i) {
            const int u = c * (kTileNW / 4) + i;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (u < db.w4) v = src[(size_t)u * 64];
            R[4 * i + 0] = v.x;
            R[4 * i + 1] = v.y;
            R[4 * i + 2] = v.z;
            R[4 * i + 3] = v.w;
        }
        kptr_u32 qrow = (kptr_u32)(qs + (size_t)q0 * qw + c * kTileNW);
        for (int q = 0; q < nq; ++q, qrow += qw) {
            uint32_t acc = c > 0 ? lacc[q * 64 + lane] : 0u;
#pragma unroll
            for (int i = 0; i < kTileNW; ++i) {
                const uint32_t x = MODE == FID_MODE_MIXTURE ? (R[i] & qrow[i]) : (R[i] ^ qrow[i]);
                acc = popc_acc(x, acc);
            }
            if (c + 1 < nch) lacc[q * 64 + lane] = acc;
            else if (cin) dst[(size_t)q * tw] = (int32_t)acc;
        }
    }
}

hipError_t launch_tile_counts(int mode, const DbView& db, const uint32_t* qs, int32_t qw,
                              const TileTable& tt, int32_t th, int32_t tw, int32_t* out, hipStream_t s)
{
    const int64_t waves = (int64_t)tt.n * ((tw + 63) / 64) * ((th + kTileQueries - 1) / kTileQueries);
    const int64_t blocks = (waves + kWavesPerWG - 1) / kWavesPerWG;
    if (blocks <= 0) return hipSuccess;
    if (mode == FID_MODE_MIXTURE)
        hipLaunchKernelGGL(tile_counts_kernel<FID_MODE_MIXTURE>, dim3((unsigned)blocks), dim3(kWG), 0, s, db,
                           qs, qw, tt, th, tw, out);
    else
        hipLaunchKernelGGL(tile_counts_kernel<FID_MODE_IDENTITY>, dim3((unsigned)blocks), dim3(kWG), 0, s, db,
                           qs, qw, tt, th, tw, out);
    return hipGetLastError();
}

// thr[i] = min(thr[i], bound[i]) (or = bound[i] when there is no seed bound),
// never above n_loci + 1: counts lie in [0, n_loci], so a larger bound
// (0xFFFFFFFF = "none yet") filters exactly as n_loci + 1 does.
__global__ void min_bound_kernel(uint32_t* __restrict__ thr, const uint32_t* __restrict__ bound, int32_t n,
                                 int keep, uint32_t cap, uint32_t* __restrict__ level, uint32_t* __restrict__ wit)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) {
        thr[i] = min(keep ? min(thr[i], bound[i]) : bound[i], cap);
        // without a seed block there is no witness level
        if (!keep && level) {
            for (int l = 0; l < kWitLevels; ++l) {
                level[(size_t)kWitLevels * i + l] = 0u;
                wit[(size_t)kWitLevels * i + l] = 0u;
            }
        }
    }
}

hipError_t launch_min_bound(uint32_t* thr, const uint32_t* bound, int32_t n, bool keep, int32_t n_loci,
                            uint32_t* level, uint32_t* wit, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(min_bound_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, thr, bound, n,
                       keep ? 1 : 0, (uint32_t)n_loci + 1u, level, wit);
    return hipGetLastError();
}

// ------------------------------------------------------------------ workgroup top-k
__global__ void fill_u64_kernel(uint64_t* __restrict__ p, int64_t n, uint64_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// Per-query bound for the top-k filter from the seed block of counts: a
// histogram of count >> shift in LDS gives the bin b holding the k-th
// smallest count; every top-k member of the whole database has a count no
// larger than the k-th count of any k references, hence no larger than the
// bin's upper edge, so "count < (b + 1) << shift" loses nothing.
//
// The same histogram gives kWitLevels lower witness levels: the upper edges of
// the bins holding the (k / 2)-th, (k / 4)-th, ... (k / 32)-th (each at least
// the first) smallest seed counts, stored as level[kWitLevels q + l].  The scan
// counts the distinct references it meets below each level; once there are k
// of them, that level is a valid bound too (k references beat anything at or
// above it).  Halving from level to level, each level passes about as many
// candidates before the next one takes over as there are top-k slots.
template <int NT>
__device__ __forceinline__ void seed_select_one(const int32_t* __restrict__ row, int64_t n_cols, int32_t k,
                                                int32_t shift, int32_t nbins, uint32_t* __restrict__ thr_q,
                                                uint32_t* __restrict__ level_q, uint32_t* __restrict__ wit_q)
{
    extern __shared__ uint32_t hist[];           // [nbins]
    __shared__ uint32_t part[NT];
    __shared__ uint32_t found, found_w[kWitLevels];
    const int tid = (int)threadIdx.x;
    uint32_t kw[kWitLevels];
    for (int l = 0; l < kWitLevels; ++l) kw[l] = (uint32_t)k >> (l + 1) > 0u ? (uint32_t)k >> (l + 1) : 1u;
    for (int i = tid; i < nbins; i += NT) hist[i] = 0u;
    if (tid == 0) {
        found = 0xFFFFFFFFu;
        for (int l = 0; l < kWitLevels; ++l) found_w[l] = 0xFFFFFFFFu;
    }
    __syncthreads();
    for (int64_t i = tid; i < n_cols; i += NT)
        atomicAdd(&hist[(uint32_t)row[i] >> shift], 1u);
    __syncthreads();
    const int seg = (nbins + NT - 1) / NT;
    uint32_t sum = 0;
    for (int i = tid * seg; i < min(nbins, (tid + 1) * seg); ++i) sum += hist[i];
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {  // inclusive scan of the segment sums
        const uint32_t v = tid >= off ? part[tid - off] : 0u;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    const uint32_t before = tid > 0 ? part[tid - 1] : 0u;
    // the bin where the running count first reaches `target`
    auto crossing = [&](uint32_t target, uint32_t& out) {
        if (before < target && part[tid] >= target) {
            uint32_t run = before;
            for (int i = tid * seg; i < min(nbins, (tid + 1) * seg); ++i) {
                run += hist[i];
                if (run >= target) {
                    out = (uint32_t)i;
                    break;
                }
            }
        }
    };
    crossing((uint32_t)k, found);
    if (level_q)
        for (int l = 0; l < kWitLevels; ++l) crossing(kw[l], found_w[l]);
    __syncthreads();
    if (tid == 0) {
        *thr_q = found == 0xFFFFFFFFu ? 0xFFFFFFFFu : (found + 1u) << shift;
        if (level_q) {
            for (int l = 0; l < kWitLevels; ++l) {
                level_q[l] = found_w[l] == 0xFFFFFFFFu || kw[l] >= (uint32_t)k ? 0u : (found_w[l] + 1u) << shift;
                wit_q[l] = 0u;
            }
        }
    }
}


// One workgroup of kSeedSelectThreads per query: a call's seed rows are long
// (up to 131,072 counts) and its queries few (a serving tick holds about 130),
// so the histogram takes wide workgroups rather than many.
constexpr int kSeedSelectThreads = 1024;

__global__ __launch_bounds__(kSeedSelectThreads) void seed_select_kernel(
    const int32_t* __restrict__ counts, int64_t n_cols, int32_t k, int32_t shift, int32_t nbins,
    uint32_t* __restrict__ thr_init, uint32_t* __restrict__ level, uint32_t* __restrict__ wit)
{
    const int q = blockIdx.x;
    seed_select_one<kSeedSelectThreads>(counts + (size_t)q * n_cols, n_cols, k, shift, nbins, thr_init + q,
                    level ? level + (size_t)kWitLevels * q : nullptr, wit ? wit + (size_t)kWitLevels * q : nullptr);
}

hipError_t launch_seed_select(const int32_t* counts, int32_t n_q, int64_t n_cols, int32_t k,
                              int32_t n_loci, uint32_t* thr_init, uint32_t* level, uint32_t* wit,
                              hipStream_t s)
{
    int32_t shift = 0;
    while ((n_loci >> shift) + 1 > kSeedBins) ++shift;
    const int32_t nbins = (n_loci >> shift) + 1;
    hipLaunchKernelGGL(seed_select_kernel, dim3(n_q), dim3(kSeedSelectThreads),
                       (size_t)nbins * sizeof(uint32_t), s, counts, n_cols, k, shift, nbins,
                       thr_init, level, wit);
    return hipGetLastError();
}

// The job holding global query g (jobs ordered by q_off).
__device__ __forceinline__ int select_job_of(const SelectJob* __restrict__ jobs, int32_t n_jobs, int64_t g)
{
    int a = 0, b = n_jobs;
    while (b - a > 1) {
        const int m = (a + b) >> 1;
        if (jobs[m].q_off <= g) a = m;
        else b = m;
    }
    return a;
}

__global__ __launch_bounds__(kSelectThreads) void seed_select_batch_kernel(const SelectJob* __restrict__ jobs,
                                                                           int32_t n_jobs)
{
    const int64_t g = blockIdx.x;
    const SelectJob& J = jobs[select_job_of(jobs, n_jobs, g)];
    const int64_t q = g - J.q_off;
    int32_t shift = 0;
    while ((J.n_loci >> shift) + 1 > kSeedBinsBatch) ++shift;
    seed_select_one<kSelectThreads>(J.counts + q * J.n_cols, J.n_cols, J.k, shift, (J.n_loci >> shift) + 1, J.thr_init + q,
                    J.level + kWitLevels * q, J.wit + kWitLevels * q);
}

hipError_t launch_seed_select_batch(const SelectJob* jobs, int32_t n_jobs, int64_t total_q, int32_t n_loci_max,
                                    hipStream_t s)
{
    if (n_jobs <= 0 || total_q <= 0) return hipSuccess;
    // each job bins its own counts (a shorter row may need more bins than
    // the longest one): room for the most any row can use
    const int32_t nbins = n_loci_max < kSeedBinsBatch ? n_loci_max + 1 : kSeedBinsBatch;
    hipLaunchKernelGGL(seed_select_batch_kernel, dim3((unsigned)total_q), dim3(kSelectThreads),
                       (size_t)nbins * sizeof(uint32_t), s, jobs, n_jobs);
    return hipGetLastError();
}

__global__ __launch_bounds__(kSelectThreads) void select_counts_kernel(
    const int32_t* __restrict__ counts, int64_t n_cols, int32_t k, int64_t idx_base,
    int32_t* __restrict__ cnt, int64_t* __restrict__ idx)
{
    __shared__ uint64_t s[kSelectSlots];
    __shared__ int nb;
    const int q = blockIdx.x;
    const int32_t* row = counts + (size_t)q * n_cols;
    wg_topk([&](int64_t i) { return ((uint64_t)(uint32_t)row[i] << kIdxBits) | (uint64_t)(idx_base + i); },
            n_cols, k, s, &nb);
    write_topk(s, k, cnt + (size_t)q * k, idx + (size_t)q * k);
}

hipError_t launch_select_counts(const int32_t* counts, int32_t n_q, int64_t n_cols, int32_t k,
                                int64_t idx_base, int32_t* cnt, int64_t* idx, hipStream_t s)
{
    hipLaunchKernelGGL(select_counts_kernel, dim3(n_q), dim3(kSelectThreads), 0, s, counts,
                       n_cols, k, idx_base, cnt, idx);
    return hipGetLastError();
}

__global__ __launch_bounds__(kSelectThreads) void select_counts_batch_kernel(const SelectJob* __restrict__ jobs,
                                                                             int32_t n_jobs)
{
    __shared__ uint64_t s[kSelectSlots];
    __shared__ int nb;
    const int64_t g = blockIdx.x;
    const SelectJob& J = jobs[select_job_of(jobs, n_jobs, g)];
    const int64_t q = g - J.q_off;
    const int32_t* row = J.counts + q * J.n_cols;
    const int64_t base = J.idx_base;
    wg_topk([&](int64_t i) { return ((uint64_t)(uint32_t)row[i] << kIdxBits) | (uint64_t)(base + i); }, J.n_cols, J.k,
            s, &nb);
    write_topk(s, J.k, J.cnt + q * J.k, J.idx + q * J.k);
}

hipError_t launch_select_counts_batch(const SelectJob* jobs, int32_t n_jobs, int64_t total_q, hipStream_t s)
{
    if (n_jobs <= 0 || total_q <= 0) return hipSuccess;
    hipLaunchKernelGGL(select_counts_batch_kernel, dim3((unsigned)total_q), dim3(kSelectThreads), 0, s, jobs,
                       n_jobs);
    return hipGetLastError();
}

// Merge of the per-worker lists of one query (one workgroup of NT threads
// per query).
template <int NT>
__global__ __launch_bounds__(NT) void merge_lists_kernel(
    const uint64_t* __restrict__ lists, const uint32_t* __restrict__ fills, int32_t n_rsplit,
    int32_t k, int32_t n_loci, int32_t* __restrict__ cnt, int64_t* __restrict__ idx)
{
    __shared__ uint64_t s[kSelectSlots];
    __shared__ int nb;
    __shared__ uint32_t part[NT];
    extern __shared__ uint32_t off[];  // [n_rsplit + 1] prefix of the fill counts
    const int q = blockIdx.x;
    merge_query_lists<NT>(lists + (size_t)q * n_rsplit * k, fills + (size_t)q * n_rsplit, n_rsplit, k, n_loci,
                          cnt + (size_t)q * k, idx + (size_t)q * k, s, &nb, part, off);
}

// Calls of a few query tiles (a serving tick holds about 130 queries) spread
// each query over thousands of lists: wide workgroups, as in the seed
// selection; many queries fill the device with narrow ones.
constexpr int kMergeWideThreads = 1024;
constexpr int32_t kMergeWideMaxQ = 512;
static_assert(kSelectSlots / 2 % kMergeWideThreads == 0, "the workgroup top-k takes whole rounds of keys");

hipError_t launch_merge_lists(const uint64_t* lists, const uint32_t* fills, int32_t n_q,
                              int32_t n_rsplit, int32_t k, int32_t n_loci, int32_t* cnt, int64_t* idx,
                              hipStream_t s)
{
    if (n_q <= kMergeWideMaxQ)
        hipLaunchKernelGGL(merge_lists_kernel<kMergeWideThreads>, dim3(n_q), dim3(kMergeWideThreads),
                           (size_t)(n_rsplit + 1) * sizeof(uint32_t), s, lists, fills, n_rsplit, k, n_loci,
                           cnt, idx);
    else
        hipLaunchKernelGGL(merge_lists_kernel<kSelectThreads>, dim3(n_q), dim3(kSelectThreads),
                           (size_t)(n_rsplit + 1) * sizeof(uint32_t), s, lists, fills, n_rsplit, k, n_loci,
                           cnt, idx);
    return hipGetLastError();
}

// ------------------------------------------------------------------ threshold hits -> CSR
// Hits are (q << 40 | r, count) pairs in arrival order; a merge sort on the
// (unique) keys puts them in (query, reference) order.
constexpr int kSortTile = 2048;

__global__ __launch_bounds__(kSelectThreads) void block_sort_kv_kernel(
    uint64_t* __restrict__ keys, int32_t* __restrict__ vals, int64_t n)
{
    __shared__ uint64_t sk[kSortTile];
    __shared__ int32_t sv[kSortTile];
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int i = (int)threadIdx.x; i < kSortTile; i += kSelectThreads) {
        const int64_t g = base + i;
        sk[i] = g < n ? keys[g] : kSentinel;
        sv[i] = g < n ? vals[g] : 0;
    }
    __syncthreads();
    for (int size = 2; size <= kSortTile; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = (int)threadIdx.x; t < kSortTile / 2; t += kSelectThreads) {
                const int i = 2 * t - (t & (stride - 1));
                const int j = i + stride;
                const bool asc = (i & size) == 0;
                const uint64_t a = sk[i], b = sk[j];
                if ((a > b) == asc) {
                    sk[i] = b;
                    sk[j] = a;
                    const int32_t va = sv[i];
                    sv[i] = sv[j];
                    sv[j] = va;
                }
            }
            __syncthreads();
        }
    }
    for (int i = (int)threadIdx.x; i < kSortTile; i += kSelectThreads) {
        const int64_t g = base + i;
        if (g < n) {
            keys[g] = sk[i];
            vals[g] = sv[i];
        }
    }
}

__device__ __forceinline__ int64_t lower_bound_u64(const uint64_t* a, int64_t n, uint64_t key)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ void merge_pass_kernel(const uint64_t* __restrict__ ki, const int32_t* __restrict__ vi,
                                  uint64_t* __restrict__ ko, int32_t* __restrict__ vo, int64_t n,
                                  int64_t width)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t run = i / width;
        const int64_t a0 = (run & ~1ll) * width;
        const int64_t a1 = min(a0 + width, n);
        const int64_t b1 = min(a0 + 2 * width, n);
        const uint64_t key = ki[i];
        int64_t pos;
        if ((run & 1) == 0) pos = i + lower_bound_u64(ki + a1, b1 - a1, key);
        else pos = a0 + lower_bound_u64(ki + a0, a1 - a0, key) + (i - a1);
        ko[pos] = key;
        vo[pos] = vi[i];
    }
}

hipError_t launch_sort_hits(uint64_t* keys, int32_t* vals, uint64_t* keys2, int32_t* vals2,
                            int64_t n, uint64_t** out_keys, int32_t** out_vals, hipStream_t s)
{
    *out_keys = keys;
    *out_vals = vals;
    if (n <= 1) return hipSuccess;
    const int64_t tiles = (n + kSortTile - 1) / kSortTile;
    hipLaunchKernelGGL(block_sort_kv_kernel, dim3((unsigned)tiles), dim3(kSelectThreads), 0, s,
                       keys, vals, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint64_t* ka = keys;
    int32_t* va = vals;
    uint64_t* kb = keys2;
    int32_t* vb = vals2;
    for (int64_t width = kSortTile; width < n; width *= 2) {
        int64_t blocks = (n + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(merge_pass_kernel, dim3((unsigned)blocks), dim3(256), 0, s, ka, va, kb,
                           vb, n, width);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint64_t* tk = ka; ka = kb; kb = tk;
        int32_t* tv = va; va = vb; vb = tv;
    }
    *out_keys = ka;
    *out_vals = va;
    return hipSuccess;
}

__global__ void csr_offsets_kernel(const uint64_t* __restrict__ keys, int64_t n, int32_t n_q,
                                   int64_t* __restrict__ offs)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q <= n_q;
         q += (int64_t)gridDim.x * blockDim.x)
        offs[q] = lower_bound_u64(keys, n, (uint64_t)q << kIdxBits);
}

__global__ void csr_values_kernel(const uint64_t* __restrict__ keys, const int32_t* __restrict__ vals,
                                  int64_t n, int64_t* __restrict__ idx, int32_t* __restrict__ cnt)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        idx[i] = (int64_t)(keys[i] & kIdxMask);
        cnt[i] = vals[i];
    }
}

hipError_t launch_hits_to_csr(const uint64_t* keys, const int32_t* vals, int64_t n, int32_t n_q,
                              int64_t* offs, int64_t* idx, int32_t* cnt, hipStream_t s)
{
    int64_t blocks = ((int64_t)n_q + 1 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(csr_offsets_kernel, dim3((unsigned)blocks), dim3(256), 0, s, keys, n, n_q,
                       offs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n == 0) return e;
    blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(csr_values_kernel, dim3((unsigned)blocks), dim3(256), 0, s, keys, vals, n,
                       idx, cnt);
    return hipGetLastError();
}

// ------------------------------------------------------------ running top-k
// A running top-k per query (row `slot` of `running`, k ascending keys
// (count << 40 | index), kSentinel for empty) and its bound: the k-th count
// + 1, or 0xFFFFFFFF while fewer than k keys are held.  Queries map to rows
// through `slots` (nullptr: query i is row i).  Used by the serving loop
// (database chunks) and the streamed database (host blocks).
namespace {

__device__ __forceinline__ int64_t slot_of(const int32_t* slots, int i) { return slots ? slots[i] : i; }

__global__ void reset_running_kernel(const int32_t* __restrict__ slots, int32_t n, int32_t k,
                                     uint64_t* __restrict__ running, uint32_t* __restrict__ bound)
{
    const int64_t total = (int64_t)n * k;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / k;
        running[slot_of(slots, (int)i) * k + (t - i * k)] = kSentinel;
        if (t - i * k == 0) bound[slot_of(slots, (int)i)] = 0xFFFFFFFFu;
    }
}

// Number of keys in the ascending array s[0..n) smaller than x.
__device__ __forceinline__ int rank_below(const uint64_t* s, int n, uint64_t x)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int m = (lo + hi) >> 1;
        if (s[m] < x) lo = m + 1;
        else hi = m;
    }
    return lo;
}

// running[slot] <- k smallest of (running[slot] U the part result of query
// i, whose indices are offset by idx_offset).  Both inputs are ascending;
// real keys are unique (a reference belongs to one part), so each lands at
// (own position + rank in the other list).  The new k-th key also gives the
// slot's bound for its next parts: a reference of another part enters only
// with a count <= the k-th count (an equal count may still win on index).
__global__ __launch_bounds__(256) void fold_topk_kernel(const int32_t* __restrict__ cnt,
                                                        const int64_t* __restrict__ idx,
                                                        const int32_t* __restrict__ slots, int32_t k,
                                                        int64_t idx_offset, uint64_t* __restrict__ running,
                                                        uint32_t* __restrict__ bound)
{
    extern __shared__ uint64_t sh[];  // [2k]
    uint64_t* a = sh;
    uint64_t* b = sh + k;
    const int i = blockIdx.x;
    const int64_t slot = slot_of(slots, i);
    uint64_t* run = running + slot * k;
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
        a[j] = run[j];
        const int64_t r = idx[(int64_t)i * k + j];
        b[j] = r < 0 ? kSentinel
                     : (((uint64_t)(uint32_t)cnt[(int64_t)i * k + j] << kIdxBits) | (uint64_t)(r + idx_offset));
    }
    __syncthreads();
    auto put = [&](int pos, uint64_t key) {
        if (pos >= k) return;
        run[pos] = key;
        if (pos == k - 1) bound[slot] = key == kSentinel ? 0xFFFFFFFFu : (uint32_t)(key >> kIdxBits) + 1u;
    };
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
        put(j + rank_below(b, k, a[j]), a[j]);
        put(j + rank_below(a, k, b[j]), b[j]);
    }
}

__global__ void finalize_topk_kernel(const uint64_t* __restrict__ running, const int32_t* __restrict__ slots,
                                     int32_t n, int32_t k_run, int32_t k, int32_t* __restrict__ cnt,
                                     int64_t* __restrict__ idx)
{
    const int64_t total = (int64_t)n * k;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / k;
        const uint64_t key = running[slot_of(slots, (int)i) * k_run + (t - i * k)];
        cnt[t] = key == kSentinel ? INT32_MAX : (int32_t)(key >> kIdxBits);
        idx[t] = key == kSentinel ? -1 : (int64_t)(key & kIdxMask);
    }
}

unsigned grid_256(int64_t n)
{
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

hipError_t launch_reset_running(const int32_t* slots, int32_t n, int32_t k, uint64_t* running, uint32_t* bound,
                                hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(reset_running_kernel, dim3(grid_256((int64_t)n * k)), dim3(256), 0, s, slots, n, k,
                       running, bound);
    return hipGetLastError();
}

hipError_t launch_fold_topk(const int32_t* cnt, const int64_t* idx, const int32_t* slots, int32_t n, int32_t k,
                            int64_t idx_offset, uint64_t* running, uint32_t* bound, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fold_topk_kernel, dim3((unsigned)n), dim3(256), 2 * (size_t)k * sizeof(uint64_t), s, cnt,
                       idx, slots, k, idx_offset, running, bound);
    return hipGetLastError();
}

hipError_t launch_finalize_topk(const uint64_t* running, const int32_t* slots, int32_t n, int32_t k_run, int32_t k,
                                int32_t* cnt, int64_t* idx, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_topk_kernel, dim3(grid_256((int64_t)n * k)), dim3(256), 0, s, running, slots, n,
                       k_run, k, cnt, idx);
    return hipGetLastError();
}

// --------------------------------------------------- streamed threshold hits
// Threshold hits of successive host blocks share one append buffer; after
// block b, its hits [ends[b], ends[b + 1]) carry block-local reference
// indices, which are shifted to database rows by adding the block's first
// row r0 (key = q << 40 | r, r + r0 < 2^40).
namespace {

__global__ void snapshot_hits_kernel(const unsigned long long* __restrict__ counter, int64_t* __restrict__ ends,
                                     int32_t b)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) ends[b + 1] = (int64_t)*counter;
}

__global__ void offset_hits_kernel(uint64_t* __restrict__ keys, const int64_t* __restrict__ ends, int32_t b,
                                   int64_t cap, int64_t r0)
{
    const int64_t lo = ends[b];
    const int64_t hi = ends[b + 1] < cap ? ends[b + 1] : cap;
    for (int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi;
         i += (int64_t)gridDim.x * blockDim.x)
        keys[i] += (uint64_t)r0;
}

}  // namespace

hipError_t launch_offset_block_hits(const unsigned long long* counter, int64_t* ends, int32_t b, uint64_t* keys,
                                    int64_t cap, int64_t r0, hipStream_t s)
{
    hipLaunchKernelGGL(snapshot_hits_kernel, dim3(1), dim3(64), 0, s, counter, ends, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || r0 == 0) return e;
    hipLaunchKernelGGL(offset_hits_kernel, dim3(1024), dim3(256), 0, s, keys, ends, b, cap, r0);
    return hipGetLastError();
}

}  // namespace fid
