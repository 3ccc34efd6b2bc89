// Plain streaming kernels that measure the HBM rate attainable on the device:
// the practical ceiling the bandwidth-bound step is compared with, beside the
// 8 TB/s peak.  Each moves 16-byte (two-double) elements with non-temporal
// loads and stores (the access form the step kernels use for populations), U
// elements per thread per loop trip, in a grid-stride loop over `grid`
// workgroups of 256 threads:
//   copy   dst[i] = src[i]          reads and writes `bytes`
//   read   sum of src per workgroup reads `bytes`, writes one double per workgroup
//   write  dst[i] = 1.0             writes `bytes`
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/lbm.h"
#include "lbm_internal.hpp"

namespace {

using v2d = double __attribute__((ext_vector_type(2)));
constexpr int PT = 256;  // threads per workgroup
constexpr int U = 4;     // 16-byte elements per thread per trip (all loads issued before the stores)

__global__ void __launch_bounds__(PT) k_probe_copy(const v2d* __restrict__ src, v2d* __restrict__ dst, long n) {
    const long stride = (long)gridDim.x * PT * U;
    for (long i = (long)blockIdx.x * PT * U + threadIdx.x; i < n; i += stride) {
        v2d v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long j = i + (long)u * PT;
            v[u] = __builtin_nontemporal_load(src + (j < n ? j : n - 1));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long j = i + (long)u * PT;
            if (j < n) __builtin_nontemporal_store(v[u], dst + j);
        }
    }
}

__global__ void __launch_bounds__(PT) k_probe_read(const v2d* __restrict__ src, double* __restrict__ out, long n) {
    const long stride = (long)gridDim.x * PT * U;
    double acc = 0.0;
    for (long i = (long)blockIdx.x * PT * U + threadIdx.x; i < n; i += stride) {
        v2d v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long j = i + (long)u * PT;
            v[u] = __builtin_nontemporal_load(src + (j < n ? j : n - 1));
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i + (long)u * PT < n) acc += v[u].x + v[u].y;
    }
    __shared__ double red[PT / 64];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void __launch_bounds__(PT) k_probe_write(v2d* __restrict__ dst, long n) {
    const long stride = (long)gridDim.x * PT * U;
    v2d one;
    one.x = 1.0;
    one.y = 1.0;
    for (long i = (long)blockIdx.x * PT * U + threadIdx.x; i < n; i += stride) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long j = i + (long)u * PT;
            if (j < n) __builtin_nontemporal_store(one, dst + j);
        }
    }
}

}  // namespace

extern "C" lbm_status lbm_stream_probe(int32_t kind, const void* src, void* dst, size_t bytes, int32_t grid,
                                       hipStream_t stream) {
    using lbm_internal::fail;
    if (kind < 0 || kind > 2) return fail(LBM_EINVAL, "unknown probe kind %d", kind);
    if (grid < 1 || grid > (1 << 24)) return fail(LBM_EINVAL, "probe grid %d out of range", grid);
    if (bytes < 16 || bytes % 16 != 0) return fail(LBM_EINVAL, "probe size %zu must be a positive multiple of 16", bytes);
    if ((kind != 2 && !src) || !dst) return fail(LBM_EINVAL, "NULL buffer");
    if (((uintptr_t)src & 15) != 0 || ((uintptr_t)dst & 15) != 0) return fail(LBM_EINVAL, "buffers must be 16-byte aligned");
    const long n = (long)(bytes / 16);
    const v2d* s = static_cast<const v2d*>(src);
    if (kind == 0)
        hipLaunchKernelGGL(k_probe_copy, dim3(grid), dim3(PT), 0, stream, s, static_cast<v2d*>(dst), n);
    else if (kind == 1)
        hipLaunchKernelGGL(k_probe_read, dim3(grid), dim3(PT), 0, stream, s, static_cast<double*>(dst), n);
    else
        hipLaunchKernelGGL(k_probe_write, dim3(grid), dim3(PT), 0, stream, static_cast<v2d*>(dst), n);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}
