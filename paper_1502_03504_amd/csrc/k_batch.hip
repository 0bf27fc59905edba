// Batched sweeps: many independent 2D grids (radius-1 star or box
// stencils, each with its own boundary rule) advanced n_steps sweeps each in
// ONE persistent launch.
//
// Work decomposition.  Every grid is cut into full-width row slabs of about
// kSlabPoints points.  A work item is (step s, slab); the items of each
// queue are numbered step-major, so every item depends only on items with a
// smaller number: slab (s, k) needs slabs k-1, k, k+1 of the same grid
// (wrapped when y is periodic) to have finished step s-1, both because it
// reads their rows and because it overwrites the buffer they read at step
// s-1.  Workgroups take the next item with an atomic counter and wait for
// its dependencies on per-slab step counters.  Whenever a workgroup waits,
// the earliest unfinished item it waits for was taken earlier by a running
// workgroup whose own dependencies are older still, so the earliest
// unfinished item always progresses and the queue drains.  A bounded spin
// turns a broken invariant into an error flag instead of a hang.
//
// Grids are dealt to 8 queues (one per XCD: workgroup b serves queue b % 8,
// matching the round-robin dispatch of workgroups to XCDs) balancing points,
// so the slabs of one grid, and their shared boundary rows, stay in one
// XCD's L2.  Release/acquire at agent scope on the counters makes the rows
// written by one slab visible to the slabs that read them, whichever XCD
// they run on.
//
// A slab is swept like the 2D marching kernel: rows enter an LDS ring of 4
// rows, each output row is the fma chain over the grid's taps in
// lexicographic order (5 taps for a star, 9 for a box), so the result equals
// lope_iterate with one sweep per pass, value for value.
#include "lope_internal.h"

namespace lope {

constexpr int kBatchThreads = 256;

// Widest padded row held in LDS: nx <= 2048 (float) or 1024 (double).
template <typename T>
struct BatchWidth {
    static constexpr int value = sizeof(T) == 4 ? 2048 + 2 : 1024 + 2;
};

namespace {

__device__ __forceinline__ int ld_relaxed(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__global__ void __launch_bounds__(kBatchThreads)
k_batch(const BatchGrid* __restrict__ grids, const BatchSlab* __restrict__ slabs,
        const BatchQueue* __restrict__ queues, int* done, unsigned long long* heads, int* err, int n_steps,
        unsigned long long wait_ticks) {
    __shared__ T ring[4][BatchWidth<T>::value];
    __shared__ long long item_sh;
    __shared__ int ok_sh;
    const int q = blockIdx.x % kNumXcd;
    const BatchQueue Q = queues[q];
    const int tid = threadIdx.x;

    for (;;) {
        if (tid == 0) {
            item_sh = (long long)atomicAdd(&heads[q], 1ull);
            ok_sh = 1;
        }
        __syncthreads();
        const long long item = item_sh;
        if (item >= Q.nitems) break;
        const int s = (int)(item / Q.nslabs);
        const int sid = Q.first_slab + (int)(item % Q.nslabs);
        const BatchSlab S = slabs[sid];
        const BatchGrid& Gr = grids[S.grid];

        // Wait until this slab and its neighbours finished step s-1.  The poll
        // is a relaxed atomic load (no cache invalidation per poll); one
        // acquire fence follows once every dependency is met.  The wait is
        // bounded by the real-time counter, so a broken invariant ends in the
        // error flag, never in a hang.
        if (tid == 0 && s > 0) {
            const int deps[3] = {sid, S.up, S.down};
            const unsigned long long t0 = wall_clock64();
            for (int d = 0; d < 3 && ok_sh; ++d) {
                if (deps[d] < 0) continue;
                while (ld_relaxed(&done[deps[d]]) < s) {
                    if (wall_clock64() - t0 > wait_ticks || ld_relaxed(err)) {
                        ok_sh = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(8);
                }
            }
            if (ok_sh) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            else atomicExch(err, 1);
        }
        __syncthreads();
        if (!ok_sh) break;

        const DevGrid in = (s & 1) ? Gr.dst : Gr.src;
        const DevGrid out = (s & 1) ? Gr.src : Gr.dst;
        const T* __restrict__ ip = (const T*)in.origin;
        T* __restrict__ op = (T*)out.origin;
        const int nx = in.nx, ny = in.ny;
        const int W = nx + 2;
        const bool perx = Gr.rule.per[0] != 0, pery = Gr.rule.per[1] != 0;
        const T g = (T)Gr.rule.g;
        T c[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) c[t] = (T)Gr.c[t];
        const bool box = Gr.box != 0;

        // Row j enters ring slot j mod 4 at march step j; after the barrier the
        // step computes output row j-1 from rows j-2, j-1, j.  The next step
        // overwrites slot (j+1) mod 4 = (j-3) mod 4, which no thread reads now.
        for (int j = S.y0 - 1; j <= S.y1; ++j) {
            {
                T* dstrow = ring[(j + 4) & 3];
                const bool oy = j < 0 || j >= ny;
                if (oy && !pery) {
                    for (int px = tid; px < W; px += kBatchThreads) dstrow[px] = g;
                } else {
                    const int wy = pery ? wrap_index(j, ny) : j;
                    const T* row = ip + (int64_t)wy * in.sy;
                    for (int px = tid; px < W; px += kBatchThreads) {
                        const int gx = px - 1;
                        T v;
                        if (gx < 0 || gx >= nx) v = perx ? row[wrap_index(gx, nx)] : g;
                        else v = row[gx];
                        dstrow[px] = v;
                    }
                }
            }
            lds_barrier();
            const int yo = j - 1;
            if (yo >= S.y0) {
                const T* r0 = ring[(yo - 1 + 4) & 3];
                const T* r1 = ring[(yo + 4) & 3];
                const T* r2 = ring[(yo + 1 + 4) & 3];
                for (int px = tid + 1; px <= nx; px += kBatchThreads) {
                    T v;
                    if (box) {
                        v = c[0] * r0[px - 1];
                        v = fma(c[1], r0[px], v);
                        v = fma(c[2], r0[px + 1], v);
                        v = fma(c[3], r1[px - 1], v);
                        v = fma(c[4], r1[px], v);
                        v = fma(c[5], r1[px + 1], v);
                        v = fma(c[6], r2[px - 1], v);
                        v = fma(c[7], r2[px], v);
                        v = fma(c[8], r2[px + 1], v);
                    } else {
                        v = c[1] * r0[px];
                        v = fma(c[3], r1[px - 1], v);
                        v = fma(c[4], r1[px], v);
                        v = fma(c[5], r1[px + 1], v);
                        v = fma(c[7], r2[px], v);
                    }
                    __builtin_nontemporal_store(v, op + (int64_t)yo * out.sy + (px - 1));
                }
            }
        }
        // publish: every wave makes its stores visible at agent scope, then one
        // thread releases the counter
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (tid == 0) __hip_atomic_store(&done[sid], s + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void k_batch_reset(int* done, int nslabs, unsigned long long* heads, int* err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nslabs) done[i] = 0;
    if (i < kNumXcd) heads[i] = 0ull;
    if (i == 0) *err = 0;
}

}  // namespace

hipError_t launch_batch(const BatchGrid* grids, const BatchSlab* slabs, const BatchQueue* queues, int* done,
                        int nslabs, unsigned long long* heads, int* err, int n_steps, int dtype, int nwg,
                        unsigned long long wait_ticks, hipStream_t s) {
    const int rb = (nslabs > kNumXcd ? nslabs : kNumXcd);
    hipLaunchKernelGGL(k_batch_reset, dim3((rb + 255) / 256), dim3(256), 0, s, done, nslabs, heads, err);
    if (dtype == LOPE_F32)
        hipLaunchKernelGGL(k_batch<float>, dim3(nwg), dim3(kBatchThreads), 0, s, grids, slabs, queues, done, heads,
                           err, n_steps, wait_ticks);
    else
        hipLaunchKernelGGL(k_batch<double>, dim3(nwg), dim3(kBatchThreads), 0, s, grids, slabs, queues, done, heads,
                           err, n_steps, wait_ticks);
    return hipGetLastError();
}

int batch_occupancy(int dtype) {
    int blocks = 0;
    hipError_t e;
    if (dtype == LOPE_F32)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch<float>, kBatchThreads, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch<double>, kBatchThreads, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return blocks > 0 ? blocks : 1;
}

}  // namespace lope
