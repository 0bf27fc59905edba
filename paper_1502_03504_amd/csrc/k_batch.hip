// Batched sweeps: many independent 2D grids (radius-1 star or box
// stencils, each with its own boundary rule), all advanced by one sweep per
// launch.
//
// Every grid is cut into full-width row slabs of about 16K points.  One launch
// covers every slab of every grid for one sweep (one workgroup per slab), so
// a batch of G grids advances n sweeps in n launches instead of G*n.  Slabs of
// one launch are independent: each reads the previous state (the grid's
// source buffer on even sweeps, its destination on odd ones) and writes only
// its own rows of the other buffer.  Workgroup ids are laid out so that the
// slabs of one grid go to one XCD (workgroup b runs on XCD b mod 8), keeping a
// grid's shared boundary rows in one L2.
//
// A slab is swept like the 2D marching kernel: rows enter an LDS ring of 4
// rows; each output row is the fma chain over the grid's taps in
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

template <typename T>
__global__ void __launch_bounds__(kBatchThreads)
k_batch_step(const BatchGrid* __restrict__ grids, const BatchSlab* __restrict__ slabs,
             const int* __restrict__ order, int nslabs, int nslabs_padded, int parity) {
    __shared__ T ring[4][BatchWidth<T>::value];
    const int logical = xcd_logical_block(nslabs_padded);
    if (logical >= nslabs) return;
    const int sid = order[logical];
    const BatchSlab S = slabs[sid];
    const BatchGrid& Gr = grids[S.grid];
    const int tid = threadIdx.x;

    const DevGrid in = parity ? Gr.dst : Gr.src;
    const DevGrid out = parity ? Gr.src : Gr.dst;
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
}

}  // namespace

hipError_t launch_batch_step(const BatchGrid* grids, const BatchSlab* slabs, const int* order, int nslabs,
                             int parity, int dtype, hipStream_t s) {
    if (nslabs <= 0) return hipSuccess;
    const int nbp = padded_block_count(nslabs);
    if (dtype == LOPE_F32)
        hipLaunchKernelGGL(k_batch_step<float>, dim3(nbp), dim3(kBatchThreads), 0, s, grids, slabs, order, nslabs,
                           nbp, parity);
    else
        hipLaunchKernelGGL(k_batch_step<double>, dim3(nbp), dim3(kBatchThreads), 0, s, grids, slabs, order, nslabs,
                           nbp, parity);
    return hipGetLastError();
}

}  // namespace lope
