// 2D stencils of radius R (box: (2R+1)^2 taps; star: 4R+1 taps):
// y-marching workgroups with a ring of rows in LDS and TD sweeps fused per
// pass (temporal blocking).
//
// A workgroup owns BX output columns and a chunk of rows.  It loads rows of
// the input widened by G = R*TD cells on each side, one row per march step.
// Level k (state after k sweeps) is kept as a ring of 2R+2 rows in LDS; at
// step j level 0 receives row j and level k computes row j - k(R+1) from the
// 2R+1 level k-1 rows published at step j-1, writing into a ring slot that
// no thread reads during the same step (hence one barrier per row).  Level
// TD goes to the destination.  The per-point sum is c0*v0 followed by a chain
// of fmas in lexicographic offset order (x fastest), at every level.
// Boundary rule applied while loading (see the 3D kernel).
#include "lope_internal.h"

namespace lope {
namespace {

template <typename T, int R>
struct Coef2 {
    T c[(2 * R + 1) * (2 * R + 1)];
};

template <typename T, int R, int TD, int BX, int NT, bool BOX>
__global__ void __launch_bounds__(NT)
k_plane2d(DevGrid src, DevGrid dst, DevRule rule, Coef2<T, R> cf, int chunk, int tiles_x,
          int nblocks, int nblocks_padded) {
    constexpr int G = R * TD;
    constexpr int W = BX + 2 * G;
    constexpr int NP = (W + NT - 1) / NT;
    constexpr int NS = 2 * R + 2;
    constexpr int K = 2 * R + 1;

    __shared__ T ring[TD][NS][W];

    const int logical = xcd_logical_block(nblocks_padded);
    if (logical >= nblocks) return;
    const int tx = logical % tiles_x;
    const int ty = logical / tiles_x;

    const int nx = src.nx, ny = src.ny;
    const int x0 = tx * BX, y0 = ty * chunk;
    const int yend = min(y0 + chunk, ny);
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
                            const T c = cf.c[(ox + R) + (oy + R) * K];
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

template <typename T, int R, int TD, int BX, int NT, bool BOX>
hipError_t run_plane2d(const SweepJob& j, int chunk, hipStream_t s) {
    Coef2<T, R> cf;
    const int r = j.radius;
    const int w = 2 * r + 1;
    for (int oy = -R; oy <= R; ++oy)
        for (int ox = -R; ox <= R; ++ox) {
            T c = (T)0;
            if (ox >= -r && ox <= r && oy >= -r && oy <= r) c = (T)j.dense[(ox + r) + (oy + r) * w];
            cf.c[(ox + R) + (oy + R) * (2 * R + 1)] = c;
        }
    if (chunk <= 0) chunk = 64;
    const int tiles_x = (j.src.nx + BX - 1) / BX;
    const int tiles_y = (j.src.ny + chunk - 1) / chunk;
    const int64_t nb64 = (int64_t)tiles_x * tiles_y;
    if (nb64 > (1ll << 30)) return hipErrorInvalidConfiguration;
    const int nb = (int)nb64;
    const int nbp = padded_block_count(nb);
    hipLaunchKernelGGL((k_plane2d<T, R, TD, BX, NT, BOX>), dim3(nbp), dim3(NT), 0, s, j.src, j.dst,
                       j.rule, cf, chunk, tiles_x, nb, nbp);
    return hipGetLastError();
}

#define PLANE2D(T, DT, R, TD, W, NT, BOX, CH)                                                   \
    {"plane2d_" #T "_r" #R "_t" #TD "_w" #W "_nt" #NT "_" #BOX, FAM_PLANE2D, 2, R, TD, DT, BOX, \
     (W) - 2 * (R) * (TD), 0, NT, CH, &run_plane2d<T, R, TD, (W) - 2 * (R) * (TD), NT, BOX>}

const Variant kPlane2d[] = {
    PLANE2D(float, LOPE_F32, 1, 1, 512, 256, true, 64),
    PLANE2D(float, LOPE_F32, 1, 2, 512, 256, true, 64),
    PLANE2D(float, LOPE_F32, 1, 3, 512, 256, true, 64),
    PLANE2D(float, LOPE_F32, 1, 4, 512, 256, true, 64),
    PLANE2D(float, LOPE_F32, 1, 1, 256, 256, true, 64),
    PLANE2D(float, LOPE_F32, 1, 1, 512, 256, false, 64),
    PLANE2D(float, LOPE_F32, 1, 2, 512, 256, false, 64),
    PLANE2D(float, LOPE_F32, 2, 1, 512, 256, true, 64),
    PLANE2D(float, LOPE_F32, 2, 1, 512, 256, false, 64),
    PLANE2D(double, LOPE_F64, 1, 1, 256, 256, true, 32),
    PLANE2D(double, LOPE_F64, 1, 1, 256, 256, false, 32),
    PLANE2D(double, LOPE_F64, 1, 2, 256, 256, false, 32),
    PLANE2D(double, LOPE_F64, 1, 4, 256, 256, false, 32),
    PLANE2D(double, LOPE_F64, 2, 1, 256, 256, true, 32),
};

}  // namespace

int plane2d_variants(const Variant** out) {
    *out = kPlane2d;
    return (int)(sizeof(kPlane2d) / sizeof(kPlane2d[0]));
}

}  // namespace lope
