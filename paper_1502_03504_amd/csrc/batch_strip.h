// One strip of one grid of a batch, swept TD times by one wave: the body
// shared by the per-pass batched kernel and the persistent one.  The grid's
// rule selects the compiled Dirichlet-axis variant at run time (a
// wave-uniform choice).
#pragma once

#include "plane2d_wave.h"

namespace lope {

template <typename T, int TD, bool BOX, bool DEV>
__device__ __forceinline__ void batch_strip_rule(const BatchGrid& gr, const DevGrid& in, const DevGrid& out,
                                                 const T (&c9)[9], const BatchItem& it) {
    const T g = (T)gr.rule.g;
    const bool dx = gr.rule.per[0] == 0, dy = gr.rule.per[1] == 0;
    if (dx && dy)
        plane2d_wave_strip<T, TD, BOX, true, true, false, 0, DEV>(in, out, g, c9, it.x0, it.y0, it.y1);
    else if (dx)
        plane2d_wave_strip<T, TD, BOX, true, false, false, 0, DEV>(in, out, g, c9, it.x0, it.y0, it.y1);
    else if (dy)
        plane2d_wave_strip<T, TD, BOX, false, true, false, 0, DEV>(in, out, g, c9, it.x0, it.y0, it.y1);
    else
        plane2d_wave_strip<T, TD, BOX, false, false, false, 0, DEV>(in, out, g, c9, it.x0, it.y0, it.y1);
}

// The strip's pass: reads the buffer `parity` selects (0: src) and writes the
// other (DEV: with device-scope accesses).
template <typename T, int TD, bool DEV = false>
__device__ __forceinline__ void batch_strip(const BatchGrid& gr, int parity, const BatchItem& it) {
    const DevGrid in = parity ? gr.dst : gr.src;
    const DevGrid out = parity ? gr.src : gr.dst;
    T c9[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) c9[t] = (T)gr.c[t];
    if (gr.box)
        batch_strip_rule<T, TD, true, DEV>(gr, in, out, c9, it);
    else
        batch_strip_rule<T, TD, false, DEV>(gr, in, out, c9, it);
}

}  // namespace lope
