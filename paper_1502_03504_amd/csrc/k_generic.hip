// Generic kernels: one-thread-per-point sweep for any stencil the tuned
// families do not cover, the stored-halo fill, gradient folding and the
// Dirichlet-value gradient reduction.
#include <atomic>

#include "lope_internal.h"

namespace lope {
namespace {

constexpr int kThreads = 256;

// Value of the halo-extended field at interior-relative (gx, gy, gz): the
// boundary rule of the halo transfer (Dirichlet value if outside along any
// Dirichlet axis, else the periodically wrapped interior value).
template <typename T>
__device__ __forceinline__ T rule_load(const T* __restrict__ p, const DevGrid& g, const DevRule& r,
                                       int gx, int gy, int gz) {
    const bool ox = gx < 0 || gx >= g.nx;
    const bool oy = gy < 0 || gy >= g.ny;
    const bool oz = gz < 0 || gz >= g.nz;
    if ((ox && !r.per[0]) || (oy && !r.per[1]) || (oz && !r.per[2])) return (T)r.g;
    const int wx = wrap_index(gx, g.nx), wy = wrap_index(gy, g.ny), wz = wrap_index(gz, g.nz);
    return p[(int64_t)wx + (int64_t)wy * g.sy + (int64_t)wz * g.sz];
}

// y[x] = sum of the non-zero taps, as c0*v0 followed by a chain of fmas in
// lexicographic offset order.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_generic(DevGrid src, DevGrid dst, DevRule rule, TapList<T> taps) {
    const T* __restrict__ sp = (const T*)src.origin;
    T* __restrict__ dp = (T*)dst.origin;
    const int64_t total = (int64_t)src.nx * src.ny * src.nz;
    const int64_t step = (int64_t)gridDim.x * kThreads;
    for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < total; idx += step) {
        const int x = (int)(idx % src.nx);
        const int64_t rest = idx / src.nx;
        const int y = (int)(rest % src.ny);
        const int z = (int)(rest / src.ny);
        T acc = (T)0;
        for (int t = 0; t < taps.n; ++t) {
            const T v = rule_load(sp, src, rule, x + taps.off[t][0], y + taps.off[t][1],
                                  z + taps.off[t][2]);
            acc = (t == 0) ? taps.c[t] * v : fma(taps.c[t], v, acc);
        }
        dp[(int64_t)x + (int64_t)y * dst.sy + (int64_t)z * dst.sz] = acc;
    }
}

// One workgroup per padded row (y, z); writes only the halo cells of the row.
// One workgroup per padded row (y, z), halo widths lo/hi per axis: rows
// inside the interior fill their left and right halo cells, the others the
// whole padded row.
struct HaloWidths {
    int lo[3], hi[3];
};

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_halo_fill(DevGrid g, DevRule rule, HaloWidths w) {
    T* __restrict__ p = (T*)g.origin;
    const int wy = g.ny + w.lo[1] + w.hi[1];
    const int row = blockIdx.x;
    const int py = row % wy - w.lo[1];
    const int pz = row / wy - w.lo[2];
    const bool interior_row = py >= 0 && py < g.ny && pz >= 0 && pz < g.nz;
    const int64_t base = (int64_t)py * g.sy + (int64_t)pz * g.sz;
    const int hx = w.lo[0] + w.hi[0];
    if (interior_row) {
        for (int t = threadIdx.x; t < hx; t += kThreads) {
            const int px = t < w.lo[0] ? t - w.lo[0] : g.nx + (t - w.lo[0]);
            p[base + px] = rule_load(p, g, rule, px, py, pz);
        }
    } else {
        for (int t = threadIdx.x; t < g.nx + hx; t += kThreads) {
            const int px = t - w.lo[0];
            p[base + px] = rule_load(p, g, rule, px, py, pz);
        }
    }
}

// total += partial; partial = 0  (interiors of equal extents)
template <typename TP>
__global__ void __launch_bounds__(kThreads)
k_accumulate(DevGrid part, DevGrid total) {
    TP* __restrict__ pp = (TP*)part.origin;
    double* __restrict__ tp = (double*)total.origin;
    const int64_t n = (int64_t)part.nx * part.ny * part.nz;
    const int64_t step = (int64_t)gridDim.x * kThreads;
    for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < n; idx += step) {
        const int x = (int)(idx % part.nx);
        const int64_t rest = idx / part.nx;
        const int64_t y = rest % part.ny, z = rest / part.ny;
        const int64_t po = x + y * part.sy + z * part.sz;
        const int64_t to = x + y * total.sy + z * total.sz;
        tp[to] += (double)pp[po];
        pp[po] = (TP)0;
    }
}

// gbar = sum_x ybar[x] * sum_{taps o with x+o in a Dirichlet halo} c_o, in
// two passes with a fixed summation order (the same value on every run):
// workgroup b sums its grid-stride share of the points per thread, then a
// tree over its threads, into partials[b]; one workgroup then sums the
// partials the same way.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_gbar_partial(DevGrid y, DevRule rule, TapList<T> taps, double* __restrict__ partials) {
    __shared__ double red[kThreads];
    const T* __restrict__ yp = (const T*)y.origin;
    const int64_t total = (int64_t)y.nx * y.ny * y.nz;
    const int64_t step = (int64_t)gridDim.x * kThreads;
    double acc = 0.0;
    for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < total; idx += step) {
        const int x = (int)(idx % y.nx);
        const int64_t rest = idx / y.nx;
        const int yy = (int)(rest % y.ny);
        const int z = (int)(rest / y.ny);
        double w = 0.0;
        for (int t = 0; t < taps.n; ++t) {
            const int gx = x + taps.off[t][0], gy = yy + taps.off[t][1], gz = z + taps.off[t][2];
            const bool dout = (!rule.per[0] && (gx < 0 || gx >= y.nx)) ||
                              (!rule.per[1] && (gy < 0 || gy >= y.ny)) ||
                              (!rule.per[2] && (gz < 0 || gz >= y.nz));
            if (dout) w += (double)taps.c[t];
        }
        if (w != 0.0) acc += w * (double)yp[(int64_t)x + (int64_t)yy * y.sy + (int64_t)z * y.sz];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// *out = sum of partials[0 .. n), one workgroup.  Every read happens before
// the first barrier and the one write after the last, so out may be
// partials itself.
__global__ void __launch_bounds__(kThreads) k_gbar_final(const double* partials, int n, double* out) {
    __shared__ double red[kThreads];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += kThreads) acc += partials[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

template <typename T>
TapList<T> make_taps(const SweepJob& j) {
    TapList<T> t{};
    t.n = j.ntaps;
    for (int i = 0; i < j.ntaps; ++i) {
        t.off[i][0] = j.off[i][0];
        t.off[i][1] = j.off[i][1];
        t.off[i][2] = j.off[i][2];
        t.c[i] = (T)j.c[i];
    }
    return t;
}

int grid_blocks(int64_t total) {
    int64_t b = (total + kThreads - 1) / kThreads;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (int)b;
}

}  // namespace

int device_cu_count() {
    constexpr int kMaxDevices = 64;
    static std::atomic<int> cached[kMaxDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
        (void)hipGetLastError();
        return 256;
    }
    if (dev < kMaxDevices) {
        const int c = cached[dev].load(std::memory_order_relaxed);
        if (c > 0) return c;
    }
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        n = 256;
    }
    if (dev < kMaxDevices) cached[dev].store(n, std::memory_order_relaxed);
    return n;
}

hipError_t launch_generic(const SweepJob& j, hipStream_t s) {
    const int64_t total = (int64_t)j.src.nx * j.src.ny * j.src.nz;
    const int blocks = grid_blocks(total);
    if (j.dtype == LOPE_F32)
        hipLaunchKernelGGL(k_generic<float>, dim3(blocks), dim3(kThreads), 0, s, j.src, j.dst,
                           j.rule, make_taps<float>(j));
    else
        hipLaunchKernelGGL(k_generic<double>, dim3(blocks), dim3(kThreads), 0, s, j.src, j.dst,
                           j.rule, make_taps<double>(j));
    return hipGetLastError();
}

hipError_t launch_halo_fill(const DevGrid& g, const int lo[3], const int hi[3], int dtype, const DevRule& rule,
                            hipStream_t s) {
    HaloWidths w;
    int any = 0;
    for (int a = 0; a < 3; ++a) {
        w.lo[a] = lo[a];
        w.hi[a] = hi[a];
        any |= lo[a] | hi[a];
    }
    const int64_t rows = (int64_t)(g.ny + lo[1] + hi[1]) * (g.nz + lo[2] + hi[2]);
    if (rows <= 0 || !any) return hipSuccess;
    if (dtype == LOPE_F32)
        hipLaunchKernelGGL(k_halo_fill<float>, dim3((unsigned)rows), dim3(kThreads), 0, s, g, rule, w);
    else
        hipLaunchKernelGGL(k_halo_fill<double>, dim3((unsigned)rows), dim3(kThreads), 0, s, g, rule, w);
    return hipGetLastError();
}

hipError_t launch_accumulate(const DevGrid& part, int part_dtype, const DevGrid& total,
                             hipStream_t s) {
    const int blocks = grid_blocks((int64_t)part.nx * part.ny * part.nz);
    if (part_dtype == LOPE_F32)
        hipLaunchKernelGGL(k_accumulate<float>, dim3(blocks), dim3(kThreads), 0, s, part, total);
    else
        hipLaunchKernelGGL(k_accumulate<double>, dim3(blocks), dim3(kThreads), 0, s, part, total);
    return hipGetLastError();
}

hipError_t launch_gbar(const SweepJob& j, double* partials, double* out, hipStream_t s) {
    const int blocks = grid_blocks((int64_t)j.src.nx * j.src.ny * j.src.nz);
    const int b = blocks > kGbarPartials ? kGbarPartials : blocks;
    if (j.dtype == LOPE_F32)
        hipLaunchKernelGGL(k_gbar_partial<float>, dim3(b), dim3(kThreads), 0, s, j.src, j.rule, make_taps<float>(j),
                           partials);
    else
        hipLaunchKernelGGL(k_gbar_partial<double>, dim3(b), dim3(kThreads), 0, s, j.src, j.rule,
                           make_taps<double>(j), partials);
    hipLaunchKernelGGL(k_gbar_final, dim3(1), dim3(kThreads), 0, s, partials, b, out);
    return hipGetLastError();
}

}  // namespace lope
