// Two local-element functions per step, one thread per point (the path for
// every shape the fused two-level kernels do not cover).
//
// For an output point x the thread evaluates the intermediate v = S1(B(u)) at
// each point x + o2 the second stencil reads (B(v): a Dirichlet cell outside
// the interior is g, a periodic one is the value at the wrapped index), with
// the same per-point arithmetic as a sweep (c0*v0 then fmas over S1's taps in
// lexicographic order), then forms alpha*u[x] (if alpha != 0) followed by fmas
// over S2's taps.  Nothing intermediate is stored.  Cost per point: the product
// of the two tap counts.
#include "lope_internal.h"

namespace lope {
namespace {

constexpr int kStageThreads = 256;

template <typename T>
struct StageTaps {
    int32_t n, pad;
    int8_t off[kStageTaps][3];
    T c[kStageTaps];
};

template <typename T>
StageTaps<T> stage_taps(const SweepJob& j) {
    StageTaps<T> t{};
    t.n = j.ntaps;
    for (int i = 0; i < j.ntaps; ++i) {
        for (int a = 0; a < 3; ++a) t.off[i][a] = j.off[i][a];
        t.c[i] = (T)j.c[i];
    }
    return t;
}

// The value the boundary rule gives at (gx, gy, gz) for the array p: g outside
// along a Dirichlet axis, else the element at the wrapped index.
template <typename T>
__device__ __forceinline__ bool rule_index(const DevGrid& g, const DevRule& r, int& gx, int& gy, int& gz) {
    const bool ox = gx < 0 || gx >= g.nx, oy = gy < 0 || gy >= g.ny, oz = gz < 0 || gz >= g.nz;
    if ((ox && !r.per[0]) || (oy && !r.per[1]) || (oz && !r.per[2])) return false;
    gx = wrap_index(gx, g.nx);
    gy = wrap_index(gy, g.ny);
    gz = wrap_index(gz, g.nz);
    return true;
}

template <typename T, bool ALPHA>
__global__ void __launch_bounds__(kStageThreads)
k_stages(DevGrid src, DevGrid dst, DevRule rule, StageTaps<T> t1, StageTaps<T> t2, T alpha) {
    const T* __restrict__ sp = (const T*)src.origin;
    T* __restrict__ dp = (T*)dst.origin;
    const T g = (T)rule.g;
    const int64_t total = (int64_t)src.nx * src.ny * src.nz;
    const int64_t step = (int64_t)gridDim.x * kStageThreads;
    for (int64_t idx = (int64_t)blockIdx.x * kStageThreads + threadIdx.x; idx < total; idx += step) {
        const int x = (int)(idx % src.nx);
        const int64_t rest = idx / src.nx;
        const int y = (int)(rest % src.ny), z = (int)(rest / src.ny);
        T acc = ALPHA ? alpha * sp[(int64_t)x + (int64_t)y * src.sy + (int64_t)z * src.sz] : (T)0;
        for (int b = 0; b < t2.n; ++b) {
            int vx = x + t2.off[b][0], vy = y + t2.off[b][1], vz = z + t2.off[b][2];
            T v = g;   // v = S1(B(u)) at the wrapped point, or g outside along a Dirichlet axis
            if (rule_index<T>(src, rule, vx, vy, vz)) {
                v = (T)0;
                for (int a = 0; a < t1.n; ++a) {
                    int ux = vx + t1.off[a][0], uy = vy + t1.off[a][1], uz = vz + t1.off[a][2];
                    const T u = rule_index<T>(src, rule, ux, uy, uz)
                                    ? sp[(int64_t)ux + (int64_t)uy * src.sy + (int64_t)uz * src.sz]
                                    : g;
                    v = (a == 0) ? t1.c[a] * u : fma(t1.c[a], u, v);
                }
            }
            acc = (!ALPHA && b == 0) ? t2.c[b] * v : fma(t2.c[b], v, acc);
        }
        dp[(int64_t)x + (int64_t)y * dst.sy + (int64_t)z * dst.sz] = acc;
    }
}

template <typename T>
hipError_t launch_t(const StageJob& j, hipStream_t s) {
    const int64_t total = (int64_t)j.s1.src.nx * j.s1.src.ny * j.s1.src.nz;
    int64_t blocks = (total + kStageThreads - 1) / kStageThreads;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) return hipSuccess;
    const StageTaps<T> t1 = stage_taps<T>(j.s1), t2 = stage_taps<T>(j.s2);
    if (j.alpha != 0.0)
        hipLaunchKernelGGL((k_stages<T, true>), dim3((unsigned)blocks), dim3(kStageThreads), 0, s, j.s1.src, j.s1.dst,
                           j.s1.rule, t1, t2, (T)j.alpha);
    else
        hipLaunchKernelGGL((k_stages<T, false>), dim3((unsigned)blocks), dim3(kStageThreads), 0, s, j.s1.src,
                           j.s1.dst, j.s1.rule, t1, t2, (T)0);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stages_generic(const StageJob& j, hipStream_t s) {
    if (j.s1.ntaps > kStageTaps || j.s2.ntaps > kStageTaps) return hipErrorInvalidValue;
    return j.s1.dtype == LOPE_F32 ? launch_t<float>(j, s) : launch_t<double>(j, s);
}

}  // namespace lope
