// Batched sweeps: many independent 2D grids (radius-1 star or box
// stencils, each with its own boundary rule), advanced together.
//
// The plan cuts every grid into tiles of the 2D marching kernel (BX output
// columns by a chunk of rows; a narrow 256-wide tile for grids that fit one,
// else 512-wide tiles) and lists them in a work table.  One launch sweeps
// every tile of every grid TD times (temporal blocking, plane2d_tile), so a
// batch of G grids advances n sweeps in about n/TD launches instead of G*n.
// Tiles of one launch are independent: each reads the state before the pass
// and writes only its own output cells of the other buffer.  Work-table
// entries of one grid are consecutive, and workgroup ids are laid out so that
// consecutive entries run on one XCD (workgroup b runs on XCD b mod 8),
// keeping a grid's shared boundary rows in one L2.  Per point the result
// equals lope_iterate's, value for value.
#include "plane2d_tile.h"

namespace lope {
namespace {

constexpr int kBatchThreads = 256;

template <typename T, int TD>
__global__ void __launch_bounds__(kBatchThreads)
k_batch_td(const BatchGrid* __restrict__ grids, const BatchItem* __restrict__ items, int nitems, int nitems_padded,
           int parity) {
    constexpr int NT = kBatchThreads;
    constexpr int BXW = 2 * NT - 2 * TD;   // wide tile: 512 columns with halo
    constexpr int BXN = NT - 2 * TD;       // narrow tile: 256 columns with halo
    __shared__ T lds[Plane2dShape<T, 1, TD, BXW, NT>::LDS_ELEMS];
    const int logical = xcd_logical_block(nitems_padded);
    if (logical >= nitems) return;
    const BatchItem it = items[logical];
    const BatchGrid& gr = grids[it.grid];
    const DevGrid in = parity ? gr.dst : gr.src;
    const DevGrid out = parity ? gr.src : gr.dst;
    T cf[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) cf[t] = (T)gr.c[t];
    if (it.wide) {
        if (gr.box)
            plane2d_tile<T, 1, TD, BXW, NT, true>(in, out, gr.rule, cf, it.x0, it.y0, it.y1, lds);
        else
            plane2d_tile<T, 1, TD, BXW, NT, false>(in, out, gr.rule, cf, it.x0, it.y0, it.y1, lds);
    } else {
        if (gr.box)
            plane2d_tile<T, 1, TD, BXN, NT, true>(in, out, gr.rule, cf, it.x0, it.y0, it.y1, lds);
        else
            plane2d_tile<T, 1, TD, BXN, NT, false>(in, out, gr.rule, cf, it.x0, it.y0, it.y1, lds);
    }
}

template <typename T, int TD>
void launch_td(const BatchGrid* grids, const BatchItem* items, int nitems, int nbp, int parity, hipStream_t s) {
    hipLaunchKernelGGL((k_batch_td<T, TD>), dim3(nbp), dim3(kBatchThreads), 0, s, grids, items, nitems, nbp, parity);
}

}  // namespace

int batch_tile_width(int tdepth, bool wide) { return (wide ? 2 * kBatchThreads : kBatchThreads) - 2 * tdepth; }

hipError_t launch_batch_pass(const BatchGrid* grids, const BatchItem* items, int nitems, int tdepth, int parity,
                             int dtype, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    const int nbp = padded_block_count(nitems);
    if (dtype == LOPE_F32) {
        switch (tdepth) {
            case 1: launch_td<float, 1>(grids, items, nitems, nbp, parity, s); break;
            case 2: launch_td<float, 2>(grids, items, nitems, nbp, parity, s); break;
            case 3: launch_td<float, 3>(grids, items, nitems, nbp, parity, s); break;
            case 4: launch_td<float, 4>(grids, items, nitems, nbp, parity, s); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (tdepth) {
            case 1: launch_td<double, 1>(grids, items, nitems, nbp, parity, s); break;
            case 2: launch_td<double, 2>(grids, items, nitems, nbp, parity, s); break;
            case 3: launch_td<double, 3>(grids, items, nitems, nbp, parity, s); break;
            case 4: launch_td<double, 4>(grids, items, nitems, nbp, parity, s); break;
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

}  // namespace lope
