// Seeded synthetic SNP profiles (GPU side).  Part of the shared input
// generator, not of the comparison library: it writes the same reference
// bytes as fg_ref_bytes() in fidgen.c -- the counter-based splitmix64 draw
// u32(seed, 1, r, k) < thr[k] -- straight into device memory, so very large
// databases never cross PCIe as bytes.
#include <hip/hip_runtime.h>
#include <stdint.h>

__device__ __forceinline__ uint64_t fgd_mix(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint8_t fgd_ref_bit(uint64_t seed, uint64_t r, uint32_t k, uint32_t thr)
{
    uint64_t key = seed ^ (1ull << 56) ^ (r << 16) ^ (uint64_t)k;
    return (uint32_t)(fgd_mix(key) >> 32) < thr;
}

// One thread per 4 consecutive loci of one row; rows are ld bytes apart.
__global__ void fgd_ref_bytes_kernel(uint64_t seed, const uint32_t* __restrict__ thr,
                                     int32_t n_loci, int64_t r0, int64_t n,
                                     uint8_t* __restrict__ out, int64_t ld)
{
    const int64_t groups = (n_loci + 3) / 4;
    const int64_t total = n * groups;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / groups;
        const int32_t k0 = (int32_t)(t - i * groups) * 4;
        const uint64_t r = (uint64_t)(r0 + i);
        uint8_t* dst = out + i * ld + k0;
        if (k0 + 4 <= n_loci && (((uintptr_t)dst) & 3) == 0) {
            uint32_t v = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                v |= (uint32_t)fgd_ref_bit(seed, r, (uint32_t)(k0 + j), thr[k0 + j]) << (8 * j);
            *reinterpret_cast<uint32_t*>(dst) = v;
        } else {
            for (int j = 0; j < 4 && k0 + j < n_loci; ++j)
                dst[j] = fgd_ref_bit(seed, r, (uint32_t)(k0 + j), thr[k0 + j]);
        }
    }
}

extern "C" int fg_gpu_ref_bytes(uint64_t seed, const uint32_t* thr_dev, int32_t n_loci,
                                int64_t r0, int64_t n, uint8_t* out_dev, int64_t ld,
                                void* stream)
{
    if (n <= 0) return 0;
    if (!thr_dev || !out_dev || n_loci < 1 || ld < n_loci || r0 < 0) return -1;
    const int64_t total = n * ((n_loci + 3) / 4);
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fgd_ref_bytes_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       (hipStream_t)stream, seed, thr_dev, n_loci, r0, n, out_dev, ld);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}
