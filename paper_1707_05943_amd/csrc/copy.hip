// A plain streaming copy: the HBM bandwidth it attains is the practical
// ceiling for the march's traffic (every byte the march moves is read or
// written once, as in a copy), so it is measured beside the march.

#include "fdtd_common.h"

namespace {

typedef double v2 __attribute__((ext_vector_type(2)));
constexpr int CP_THREADS = 256;
constexpr int CP_BLOCKS = 16384;     // 64 workgroups per compute unit
constexpr int CP_U = 4;              // 16-byte loads in flight per thread

// 16-byte elements 0..n-1; every wave instruction moves 1 KiB of consecutive bytes
__global__ __launch_bounds__(CP_THREADS) void k_stream_copy(const v2* __restrict__ src, v2* __restrict__ dst, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (CP_U - 1) * stride < n; i += CP_U * stride) {
        v2 x[CP_U];
        #pragma unroll
        for (int u = 0; u < CP_U; ++u) x[u] = src[i + u * stride];
        #pragma unroll
        for (int u = 0; u < CP_U; ++u) dst[i + u * stride] = x[u];
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" int fdtd_stream_copy(void* d_dst, const void* d_src, size_t bytes, void* hip_stream)
{
    if (!d_dst || !d_src || (bytes & 15) || (((uintptr_t)d_dst | (uintptr_t)d_src) & 15)) return FDTD_EINVAL;
    if (bytes == 0) return FDTD_OK;
    hipLaunchKernelGGL(k_stream_copy, dim3(CP_BLOCKS), dim3(CP_THREADS), 0, (hipStream_t)hip_stream,
                       (const v2*)d_src, (v2*)d_dst, (int64_t)(bytes / 16));
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}
