// 2D stencils of radius R (box: (2R+1)^2 taps; star: 4R+1 taps): y-marching
// workgroups, TD sweeps fused per pass.  Each workgroup sweeps one tile (BX
// output columns, a chunk of rows) with plane2d_tile.
#include "plane2d_tile.h"

namespace lope {
namespace {

template <typename T, int R>
struct Coef2 {
    T c[(2 * R + 1) * (2 * R + 1)];
};

template <typename T, int R, int TD, int BX, int NT, bool BOX>
__global__ void __launch_bounds__(NT)
k_plane2d(DevGrid src, DevGrid dst, DevRule rule, Coef2<T, R> cf, int chunk, int tiles_x, int nblocks,
          int nblocks_padded) {
    __shared__ T lds[Plane2dShape<T, R, TD, BX, NT>::LDS_ELEMS];
    const int logical = xcd_logical_block(nblocks_padded);
    if (logical >= nblocks) return;
    const int tx = logical % tiles_x;
    const int ty = logical / tiles_x;
    const int y0 = ty * chunk;
    plane2d_tile<T, R, TD, BX, NT, BOX>(src, dst, rule, cf.c, tx * BX, y0, min(y0 + chunk, src.ny), lds);
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
    hipLaunchKernelGGL((k_plane2d<T, R, TD, BX, NT, BOX>), dim3(nbp), dim3(NT), 0, s, j.src, j.dst, j.rule, cf, chunk,
                       tiles_x, nb, nbp);
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
