// Device-to-device copy at full memory rate: the practical bandwidth ceiling
// of the GPU, and the kernel of known traffic that calibrates the memory
// counters against which the field update is measured.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/fdtd.h"

namespace {

constexpr int BLOCK = 256;
constexpr int UNROLL = 4;   // 16-byte vectors in flight per thread

// Whole chunks of BLOCK * UNROLL vectors: every load of a thread is issued
// before its first store.
__global__ void __launch_bounds__(BLOCK) k_copy(const float4 *__restrict__ src,
                                                float4 *__restrict__ dst, size_t chunks)
{
    for (size_t c = blockIdx.x; c < chunks; c += gridDim.x) {
        const size_t base = c * BLOCK * UNROLL + threadIdx.x;
        float4 v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) v[u] = src[base + (size_t)u * BLOCK];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) dst[base + (size_t)u * BLOCK] = v[u];
    }
}

// The vectors after the last whole chunk.
__global__ void __launch_bounds__(BLOCK) k_copy_tail(const float4 *__restrict__ src,
                                                     float4 *__restrict__ dst, size_t first,
                                                     size_t n)
{
    const size_t q = first + (size_t)blockIdx.x * BLOCK + threadIdx.x;
    if (q < n) dst[q] = src[q];
}

}  // namespace

extern "C" fdtd_status fdtd_device_copy(void *dst, const void *src, size_t bytes, void *stream)
{
    if (bytes == 0) return FDTD_OK;
    if (!dst || !src) return FDTD_E_INVALID_ARG;
    if (((uintptr_t)dst | (uintptr_t)src | bytes) & 15) return FDTD_E_INVALID_ARG;
    const uintptr_t d = (uintptr_t)dst, s = (uintptr_t)src;
    if (d < s + bytes && s < d + bytes) return FDTD_E_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t n = bytes / 16, chunks = n / (BLOCK * UNROLL);
    if (chunks > 0) {
        const unsigned grid = (unsigned)(chunks < 256 * 32 ? chunks : 256 * 32);
        k_copy<<<grid, BLOCK, 0, st>>>(static_cast<const float4 *>(src), static_cast<float4 *>(dst),
                                       chunks);
    }
    const size_t first = chunks * BLOCK * UNROLL;
    if (first < n) {
        const unsigned grid = (unsigned)((n - first + BLOCK - 1) / BLOCK);
        k_copy_tail<<<grid, BLOCK, 0, st>>>(static_cast<const float4 *>(src),
                                            static_cast<float4 *>(dst), first, n);
    }
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_E_HIP;
}
