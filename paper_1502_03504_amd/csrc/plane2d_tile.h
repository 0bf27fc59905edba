// One tile of the 2D y-marching sweep with TD sweeps fused (shared by the
// single-grid kernel and the batched kernel).
//
// The tile covers output columns [x0, x0+BX) and rows [y0, yend).  It loads
// rows of the input widened by G = R*TD cells on each side, one row per march
// step.  Level k (state after k sweeps) is a ring of 2R+2 rows in LDS; at step
// j level 0 receives row j and level k computes row j - k(R+1) from the 2R+1
// level k-1 rows published at step j-1, writing into a ring slot that no
// thread reads in the same step (one barrier per row).  Level TD goes to dst.
// The next input row is loaded into registers before the barrier, so its
// latency overlaps the step.  Each point is c0*v0 followed by fmas in
// lexicographic offset order (x fastest) over the star (4R+1) or box
// ((2R+1)^2) taps, the same at every level.  Boundary rule applied while
// loading: along a Dirichlet axis a cell outside the interior is g at every
// level; along a periodic axis it is loaded from the wrapped index.
#pragma once

#include "lope_internal.h"

namespace lope {

template <typename T, int R, int TD, int BX, int NT>
struct Plane2dShape {
    static constexpr int G = R * TD;
    static constexpr int W = BX + 2 * G;
    static constexpr int NP = (W + NT - 1) / NT;
    static constexpr int NS = 2 * R + 2;
    static constexpr int K = 2 * R + 1;
    static constexpr int LDS_ELEMS = TD * NS * W;
};

template <typename T, int R, int TD, int BX, int NT, bool BOX>
__device__ __forceinline__ void plane2d_tile(const DevGrid& src, const DevGrid& dst, const DevRule& rule,
                                             const T (&cf)[(2 * R + 1) * (2 * R + 1)], int x0, int y0, int yend,
                                             T* lds_raw) {
    typedef Plane2dShape<T, R, TD, BX, NT> S;
    constexpr int G = S::G, W = S::W, NP = S::NP, NS = S::NS, K = S::K;
    T (*ring)[NS][W] = reinterpret_cast<T (*)[NS][W]>(lds_raw);

    const int nx = src.nx, ny = src.ny;
    const bool perx = rule.per[0] != 0, pery = rule.per[1] != 0;
    const T g = (T)rule.g;
    const T* __restrict__ sp = (const T*)src.origin;
    T* __restrict__ dp = (T*)dst.origin;
    const int tid = threadIdx.x;

    int soff[NP];
    int lev[NP];
    bool dx[NP];
    bool keep[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const int px = tid + i * NT;
        const int gx = x0 - G + px;
        const bool used = px < W;
        const int l = min(px, W - 1 - px) / R;
        lev[i] = used ? min(l, TD) : -1;
        const bool ox = gx < 0 || gx >= nx;
        dx[i] = !perx && ox;
        soff[i] = perx ? wrap_index(gx, nx) : min(max(gx, 0), nx - 1);
        keep[i] = used && l >= TD && !ox;
    }

    T pre[NP];
    auto load_row = [&](int j) {
        const bool oy = j < 0 || j >= ny;
        if (!pery && oy) {
#pragma unroll
            for (int i = 0; i < NP; ++i) pre[i] = g;
            return;
        }
        const int64_t yo = (int64_t)(pery ? wrap_index(j, ny) : j) * src.sy;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            if (lev[i] < 0 || dx[i]) pre[i] = g;
            else pre[i] = sp[yo + soff[i]];
        }
    };
    auto slot = [](int row) { return ((row % NS) + NS) % NS; };

    const int jstart = y0 - G;
    const int jlast_load = yend - 1 + G;
    const int jend = yend - 1 + TD * (R + 1);
    load_row(jstart);

    for (int j = jstart; j <= jend; ++j) {
#pragma unroll
        for (int k = 1; k <= TD; ++k) {
            const int yk = j - k * (R + 1);
            const bool yd = !pery && (yk < 0 || yk >= ny);
            int rows[K];
#pragma unroll
            for (int o = 0; o < K; ++o) rows[o] = slot(yk - R + o);
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                if (lev[i] < k) continue;
                const int px = tid + i * NT;
                T v;
                if (yd || dx[i]) {
                    v = g;
                } else {
                    bool first = true;
#pragma unroll
                    for (int oy = -R; oy <= R; ++oy) {
                        const T* row = ring[k - 1][rows[oy + R]];
#pragma unroll
                        for (int ox = -R; ox <= R; ++ox) {
                            if (!BOX && ox != 0 && oy != 0) continue;
                            const T c = cf[(ox + R) + (oy + R) * K];
                            const T val = row[px + ox];
                            v = first ? c * val : fma(c, val, v);
                            first = false;
                        }
                    }
                }
                if (k == TD) {
                    if (keep[i] && yk >= y0 && yk < yend)
                        __builtin_nontemporal_store(v, dp + (int64_t)yk * dst.sy + (x0 - G + px));
                } else {
                    ring[k][slot(yk)][px] = v;
                }
            }
        }
        {
            const int sj = slot(j);
#pragma unroll
            for (int i = 0; i < NP; ++i)
                if (lev[i] >= 0) ring[0][sj][tid + i * NT] = pre[i];
        }
        if (j + 1 <= jlast_load) load_row(j + 1);
        lds_barrier();
    }
}

}  // namespace lope
