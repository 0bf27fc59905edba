// Convergence residual: max over the interior of |y[x] - x[x]|, in float64.
//
// The difference of the two stored values is taken in float64, then its
// magnitude; the maximum does not depend on the order of evaluation, so the
// result is exact and reproducible.  A NaN difference wins over every number
// (and stays NaN), matching a maximum that propagates NaN.  Workgroups stride
// over interior rows; each reduces its rows within the wave (cross-lane
// shuffles), then across waves in LDS, and merges its maximum into the output
// with one 64-bit unsigned atomic max: non-negative doubles (and the positive
// NaN) order like their bit patterns.
#include "lope_internal.h"

namespace lope {
namespace {

constexpr int kResThreads = 256;

template <typename T>
__global__ void __launch_bounds__(kResThreads)
k_residual_max(DevGrid x, DevGrid y, unsigned long long* out) {
    __shared__ double part[kResThreads / 64];
    const T* __restrict__ xp = (const T*)x.origin;
    const T* __restrict__ yp = (const T*)y.origin;
    const int64_t rows = (int64_t)x.ny * x.nz;
    double m = 0.0;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int64_t iy = r % x.ny, iz = r / x.ny;
        const T* xr = xp + iy * x.sy + iz * x.sz;
        const T* yr = yp + iy * y.sy + iz * y.sz;
        for (int i = threadIdx.x; i < x.nx; i += kResThreads) {
            const double d = fabs((double)yr[i] - (double)xr[i]);
            m = nan_max(m, d);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = nan_max(m, __shfl_xor(m, off, 64));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) part[wave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = part[0];
#pragma unroll
        for (int w = 1; w < kResThreads / 64; ++w) b = nan_max(b, part[w]);
        atomicMax(out, (unsigned long long)__double_as_longlong(b));
    }
}

__global__ void k_zero_u64(unsigned long long* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = 0ull;
}

}  // namespace

hipError_t launch_residual_zero(double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned long long*>(out));
    return hipGetLastError();
}

hipError_t launch_residual_max(const DevGrid& x, const DevGrid& y, int dtype, double* out, hipStream_t s) {
    unsigned long long* o = reinterpret_cast<unsigned long long*>(out);
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, o);
    const int64_t rows = (int64_t)x.ny * x.nz;
    if (rows == 0 || x.nx == 0) return hipGetLastError();
    const int blocks = (int)(rows < 8192 ? rows : 8192);
    if (dtype == LOPE_F32)
        hipLaunchKernelGGL(k_residual_max<float>, dim3(blocks), dim3(kResThreads), 0, s, x, y, o);
    else
        hipLaunchKernelGGL(k_residual_max<double>, dim3(blocks), dim3(kResThreads), 0, s, x, y, o);
    return hipGetLastError();
}

}  // namespace lope
