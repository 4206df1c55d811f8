// libfastid peak probes: sustained rates of the units the comparison
// kernels are bound by, measured on the device the context runs on, so that
// the roofline fractions can be read against the chip as it runs as well as
// against its published peaks.
//
//   FID_PROBE_MFMA_FP4  v_mfma_scale_f32_16x16x128_f8f6f4 with e2m1 operands
//                       (the fp4 scan's instruction); rate in MAC/s
//   FID_PROBE_MFMA_I8   v_mfma_i32_32x32x32_i8 (the int8 scan's); MAC/s
//   FID_PROBE_VALU      AND + fused count-and-add, the popcount scan's inner
//                       pair; 32-bit VALU lane-ops/s
//   FID_PROBE_HBM_COPY  16-byte-per-lane grid-stride copy over the caller's
//                       buffer (read half, write half); bytes moved/s
//
// Each compute probe keeps 8 independent accumulator chains per wave in
// registers for a fixed number of iterations and stores one value per lane,
// so nothing is dead code and no memory traffic competes with the unit.
#include "fid_device.hpp"
#include "fid_internal.hpp"

namespace fid {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeBlocksPerCU = 8;
constexpr int kChains = 8;

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kProbeThreads) void probe_fp4_kernel(int iters, int32_t* __restrict__ out)
{
    const int t = (int)threadIdx.x;
    const v8i a = {t, 0x22222222, 0x11111111, t ^ 0x5555, 0, 0, 0, 0};
    const v8i b = {0x11111111, t, 0x44444444, 0x22222222, 0, 0, 0, 0};
    v4f acc[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) acc[j] = v4f{0.f, 0.f, 0.f, 0.f};
    const v4i a4 = {a[0], a[1], a[2], a[3]}, b4 = {b[0], b[1], b[2], b[3]};
    // each accumulator stays in one AGPR tuple (source = destination), as in
    // the scan; through the builtin the compiler rotates the tuples every
    // iteration with register moves that would be charged to the probe
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kChains; ++j)
            __asm__ volatile("v_mfma_f32_16x16x128_f8f6f4 %0, %1, %2, %0 cbsz:4 blgp:4"
                             : "+a"(acc[j]) : "v"(a4), "v"(b4));
    }
    // the compiler does not see the asm's latency: wait it out (64 wait
    // states, above the instruction's 16 passes) before reading the results
    __asm__ volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7\n\ts_nop 7\n\ts_nop 7\n\ts_nop 7\n\ts_nop 7\n\ts_nop 7" ::: "memory");
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
    out[(size_t)blockIdx.x * kProbeThreads + t] = (int32_t)s;
}

__global__ __launch_bounds__(kProbeThreads) void probe_i8_kernel(int iters, int32_t* __restrict__ out)
{
    const int t = (int)threadIdx.x;
    const v4i a = {t, 0x01010101, 0x00010001, 0x01000100};
    const v4i b = {0x01000001, t, 0x00000101, 0x01010000};
    v16i acc[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) acc[j] = v16i{0};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) acc[j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[j], 0, 0, 0);
    }
    int s = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += acc[j][0] + acc[j][15];
    out[(size_t)blockIdx.x * kProbeThreads + t] = s;
}

__global__ __launch_bounds__(kProbeThreads) void probe_valu_kernel(int iters, uint32_t mask,
                                                                   int32_t* __restrict__ out)
{
    const uint32_t t = threadIdx.x;
    uint32_t acc[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) acc[j] = t * 2654435761u + (uint32_t)j;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) acc[j] = popc_acc(acc[j] & mask, acc[j]);
    }
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s ^= acc[j];
    out[(size_t)blockIdx.x * kProbeThreads + t] = (int32_t)s;
}

// four independent 16-byte loads in flight per lane before their stores
__global__ __launch_bounds__(kProbeThreads) void probe_copy_kernel(const v4i* __restrict__ src,
                                                                   v4i* __restrict__ dst, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
    int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        v4i v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

}  // namespace
}  // namespace fid

extern "C" int fid_peak_probe(fid_ctx* ctx, int probe, void* buf_dev, size_t buf_bytes, double* rate,
                              double* ms)
{
    using namespace fid;
    if (!ctx || !buf_dev || !rate || !ms) return fail(FID_EINVAL, "NULL argument");
    if (!aligned16(buf_dev)) return fail(FID_EINVAL, "buffer not 16-byte aligned");
    if (probe < FID_PROBE_MFMA_FP4 || probe > FID_PROBE_HBM_COPY) return fail(FID_EINVAL, "probe %d", probe);
    FID_TRY(set_device(ctx));
    const int blocks = ctx->num_cus * kProbeBlocksPerCU;
    const size_t lanes = (size_t)blocks * kProbeThreads;
    const bool compute = probe != FID_PROBE_HBM_COPY;
    if (compute && buf_bytes < lanes * sizeof(int32_t))
        return fail(FID_EINVAL, "buffer of %zu bytes < %zu needed", buf_bytes, lanes * sizeof(int32_t));
    const int64_t n16 = (int64_t)(buf_bytes / 2 / 16);
    if (!compute && n16 < 1) return fail(FID_EINVAL, "copy buffer too small");
    int32_t* out = static_cast<int32_t*>(buf_dev);
    const v4i* src = static_cast<const v4i*>(buf_dev);
    v4i* dst = static_cast<v4i*>(buf_dev) + n16;
    // about 2 ms per launch on 256 CUs
    const int iters = probe == FID_PROBE_VALU ? 8192 : probe == FID_PROBE_MFMA_FP4 ? 4096 : 2048;
    const int reps = 5;
    auto launch = [&]() -> hipError_t {
        switch (probe) {
        case FID_PROBE_MFMA_FP4:
            hipLaunchKernelGGL(probe_fp4_kernel, dim3(blocks), dim3(kProbeThreads), 0, ctx->stream, iters, out);
            break;
        case FID_PROBE_MFMA_I8:
            hipLaunchKernelGGL(probe_i8_kernel, dim3(blocks), dim3(kProbeThreads), 0, ctx->stream, iters, out);
            break;
        case FID_PROBE_VALU:
            hipLaunchKernelGGL(probe_valu_kernel, dim3(blocks), dim3(kProbeThreads), 0, ctx->stream, iters,
                               0x5A5A5A5Au, out);
            break;
        default:
            hipLaunchKernelGGL(probe_copy_kernel, dim3(blocks), dim3(kProbeThreads), 0, ctx->stream, src, dst,
                               n16);
        }
        return hipGetLastError();
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    FID_HIP(hipEventCreate(&e0), "hipEventCreate");
    int st = FID_OK;
    if (hipEventCreate(&e1) != hipSuccess) st = fail(FID_EHIP, "hipEventCreate");
    if (!st && launch() != hipSuccess) st = fail(FID_EHIP, "probe launch");  // warm-up
    if (!st && hipEventRecord(e0, ctx->stream) != hipSuccess) st = fail(FID_EHIP, "hipEventRecord");
    for (int r = 0; r < reps && !st; ++r)
        if (launch() != hipSuccess) st = fail(FID_EHIP, "probe launch");
    if (!st && hipEventRecord(e1, ctx->stream) != hipSuccess) st = fail(FID_EHIP, "hipEventRecord");
    float t = 0.f;
    if (!st && hipEventSynchronize(e1) != hipSuccess) st = fail(FID_EHIP, "hipEventSynchronize");
    if (!st && hipEventElapsedTime(&t, e0, e1) != hipSuccess) st = fail(FID_EHIP, "hipEventElapsedTime");
    hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (st) return st;
    const double per = (double)t / reps;  // ms per launch
    const double waves = (double)blocks * (kProbeThreads / 64);
    double work = 0.0;
    switch (probe) {
    case FID_PROBE_MFMA_FP4: work = waves * iters * kChains * (16.0 * 16.0 * 128.0); break;
    case FID_PROBE_MFMA_I8: work = waves * iters * kChains * (32.0 * 32.0 * 32.0); break;
    case FID_PROBE_VALU: work = waves * 64.0 * iters * kChains * 2.0; break;
    default: work = 2.0 * (double)n16 * 16.0;
    }
    *ms = per;
    *rate = work / (per * 1e-3);
    return FID_OK;
}
