// A plain streaming copy, used to measure the bandwidth a streaming kernel
// reaches on the device (the practical ceiling of the memory-bound lattice
// sweep, reported beside the vendor's peak).  Not a step of the method.
#include <hip/hip_runtime.h>

#include "../../include/capib.h"

namespace {

constexpr int COPY_THREADS = 256;
constexpr int COPY_UNROLL = 4;   // 16-byte chunks per thread per pass, loads in flight together

__global__ __launch_bounds__(COPY_THREADS) void k_copy(uint4 *__restrict__ dst, const uint4 *__restrict__ src,
                                                        long long n) {
    const long long stride = (long long)gridDim.x * COPY_THREADS;
    long long i = (long long)blockIdx.x * COPY_THREADS * COPY_UNROLL + threadIdx.x;
    for (; i + (COPY_UNROLL - 1) * COPY_THREADS < n; i += stride * COPY_UNROLL) {
        uint4 v[COPY_UNROLL];
#pragma unroll
        for (int k = 0; k < COPY_UNROLL; k++) v[k] = src[i + k * COPY_THREADS];
#pragma unroll
        for (int k = 0; k < COPY_UNROLL; k++) dst[i + k * COPY_THREADS] = v[k];
    }
    // the last partial pass
    for (int k = 0; k < COPY_UNROLL; k++)
        if (i + k * COPY_THREADS < n) dst[i + k * COPY_THREADS] = src[i + k * COPY_THREADS];
}

}  // namespace

extern "C" capib_status capib_copy_bandwidth(void *dst, const void *src, size_t bytes, void *hip_stream) {
    if (!dst || !src || (bytes & 15) || (((uintptr_t)dst | (uintptr_t)src) & 15)) return CAPIB_E_ARG;
    const char *d = (const char *)dst, *s = (const char *)src;
    if (d < s + bytes && s < d + bytes) return CAPIB_E_ARG;
    const long long n = (long long)(bytes / 16);
    if (n == 0) return CAPIB_OK;
    // enough workgroups for several per compute unit, each pass moving
    // COPY_THREADS * COPY_UNROLL chunks
    const long long per = (long long)COPY_THREADS * COPY_UNROLL;
    long long grid = (n + per - 1) / per;
    if (grid > 256 * 64) grid = 256 * 64;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)grid), dim3(COPY_THREADS), 0, (hipStream_t)hip_stream, (uint4 *)dst,
                       (const uint4 *)src, n);
    return hipGetLastError() == hipSuccess ? CAPIB_OK : CAPIB_E_HIP;
}
