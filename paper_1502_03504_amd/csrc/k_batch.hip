// Batched sweeps: many independent 2D grids (radius-1 star or box stencils,
// each with its own coefficients and boundary rule), advanced together.
//
// The plan cuts every grid into strips of 64 - 2*TD output columns by chunks
// of rows and lists them in a work table, one entry per wavefront.  One
// launch sweeps every strip of every grid TD times (plane2d_wave_strip: a
// wave marches its strip with the x neighbours moved across lanes and the
// rows in registers), so a batch of G grids advances n sweeps in about n/TD
// launches instead of G*n.  Entries of one launch are independent: each reads
// the state before the pass and writes only its own output cells of the other
// buffer.  Entries of one grid are consecutive, and workgroup ids are laid
// out so that consecutive entries run on one XCD (workgroup b runs on XCD
// b mod 8), keeping a grid's shared halo rows and columns in one L2.  Per
// point the result equals lope_iterate's, value for value.
#include "batch_strip.h"

namespace lope {
namespace {

constexpr int kBatchWaves = 4;   // waves per workgroup

template <typename T, int TD>
__global__ void __launch_bounds__(kBatchWaves * 64)
k_batch_wave(const BatchGrid* __restrict__ grids, const BatchItem* __restrict__ items, int nitems,
             int nblocks_padded, int parity) {
    // one work-table entry per wave; the index is uniform across the wave
    const int w = xcd_logical_block(nblocks_padded) * kBatchWaves +
                  __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (w >= nitems) return;   // whole waves leave; the kernel has no barrier
    const BatchItem it = items[w];
    batch_strip<T, TD>(grids[it.grid], parity, it);
}

template <typename T, int TD>
void launch_td(const BatchGrid* grids, const BatchItem* items, int nitems, int parity, hipStream_t s) {
    const int nb = (nitems + kBatchWaves - 1) / kBatchWaves;
    const int nbp = padded_block_count(nb);
    hipLaunchKernelGGL((k_batch_wave<T, TD>), dim3(nbp), dim3(kBatchWaves * 64), 0, s, grids, items, nitems, nbp,
                       parity);
}

}  // namespace

int batch_strip_width(int tdepth) { return 64 - 2 * tdepth; }

hipError_t launch_batch_pass(const BatchGrid* grids, const BatchItem* items, int nitems, int tdepth, int parity,
                             int dtype, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    if (dtype == LOPE_F32) {
        switch (tdepth) {
            case 1: launch_td<float, 1>(grids, items, nitems, parity, s); break;
            case 2: launch_td<float, 2>(grids, items, nitems, parity, s); break;
            case 3: launch_td<float, 3>(grids, items, nitems, parity, s); break;
            case 4: launch_td<float, 4>(grids, items, nitems, parity, s); break;
            case 5: launch_td<float, 5>(grids, items, nitems, parity, s); break;
            case 6: launch_td<float, 6>(grids, items, nitems, parity, s); break;
            case 7: launch_td<float, 7>(grids, items, nitems, parity, s); break;
            case 8: launch_td<float, 8>(grids, items, nitems, parity, s); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (tdepth) {
            case 1: launch_td<double, 1>(grids, items, nitems, parity, s); break;
            case 2: launch_td<double, 2>(grids, items, nitems, parity, s); break;
            case 3: launch_td<double, 3>(grids, items, nitems, parity, s); break;
            case 4: launch_td<double, 4>(grids, items, nitems, parity, s); break;
            case 5: launch_td<double, 5>(grids, items, nitems, parity, s); break;
            case 6: launch_td<double, 6>(grids, items, nitems, parity, s); break;
            case 7: launch_td<double, 7>(grids, items, nitems, parity, s); break;
            case 8: launch_td<double, 8>(grids, items, nitems, parity, s); break;
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

}  // namespace lope
