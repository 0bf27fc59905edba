// Streaming copy in 16-byte vectors with non-temporal loads and stores: the
// attainable-bandwidth reference the sweep kernels are compared with (one
// read and one write per byte, nothing else).
#include "lope_internal.h"

namespace lope {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kCopyThreads = 256;
constexpr int kCopyUnroll = 4;   // vectors in flight per thread

__global__ void __launch_bounds__(kCopyThreads)
k_copy16(const u32x4* __restrict__ src, u32x4* __restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kCopyThreads * kCopyUnroll;
    for (int64_t base = (int64_t)blockIdx.x * kCopyThreads * kCopyUnroll + threadIdx.x; base < n; base += stride) {
        u32x4 v[kCopyUnroll];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) {
            const int64_t i = base + (int64_t)u * kCopyThreads;
            if (i < n) v[u] = __builtin_nontemporal_load(src + i);
        }
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) {
            const int64_t i = base + (int64_t)u * kCopyThreads;
            if (i < n) __builtin_nontemporal_store(v[u], dst + i);
        }
    }
}

}  // namespace

hipError_t launch_copy16(const void* src, void* dst, int64_t bytes, hipStream_t s) {
    const int64_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    const int64_t per_block = (int64_t)kCopyThreads * kCopyUnroll;
    int64_t blocks = (n + per_block - 1) / per_block;
    const int64_t cap = (int64_t)device_cu_count() * 16;   // a few resident rounds; the rest by grid stride
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(kCopyThreads), 0, s, (const u32x4*)src, (u32x4*)dst, n);
    return hipGetLastError();
}

}  // namespace lope
