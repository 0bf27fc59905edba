// 2D radius-1 stencils (box or star), TD sweeps per pass, one wavefront per
// strip of 64 - 2*TD output columns and a chunk of rows (plane2d_wave_strip):
// no LDS and no barriers.  Workgroups of NW waves; consecutive waves take
// neighbouring strips of the same rows.
#include "plane2d_wave.h"

namespace lope {
namespace {

template <typename T, int TD, bool BOX, int NW, bool DX, bool DY, bool RES, int STG>
__global__ void __launch_bounds__(NW * 64)
k_plane2d_wave(DevGrid src, DevGrid dst, DevRule rule, Coef9<T> cf, Coef9<T> cf2, T alpha, int chunk, int strips,
               int nwaves, int nblocks_padded, double* residual) {
    // the wave index is uniform across the wave: say so, so that rows, loop
    // bounds and the row rule stay scalar
    const int wave = xcd_logical_block(nblocks_padded) * NW + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (wave >= nwaves) return;   // whole waves leave; the kernel has no barrier
    const int tx = wave % strips, ty = wave / strips;
    const int y0 = ty * chunk;
    plane2d_wave_strip<T, TD, BOX, DX, DY, RES, STG>(src, dst, (T)rule.g, cf.c, tx * (64 - 2 * TD), y0,
                                                     min(y0 + chunk, src.ny), residual, cf2.c, alpha);
}

template <typename T>
Coef9<T> coef9(const SweepJob& j) {
    Coef9<T> cf;
    for (int t = 0; t < 9; ++t) cf.c[t] = (T)j.dense[t];   // (ox + 1) + 3 * (oy + 1)
    return cf;
}

// One pass with the kernel built for rule case (DX, DY) and residual flag
// RES.  The automatic row chunk: as long as the resident waves (at the
// register use of this very build) still cover every chunk in few rounds.
template <typename T, int TD, bool BOX, int NW, int STG, bool DX, bool DY, bool RES>
hipError_t launch_wave_case(const SweepJob& j, const Coef9<T>& cf, const Coef9<T>& cf2, T alpha, int chunk,
                            hipStream_t s) {
    constexpr auto kernel = k_plane2d_wave<T, TD, BOX, NW, DX, DY, RES, STG>;
    const int out_cols = 64 - 2 * TD;
    const int strips = (j.src.nx + out_cols - 1) / out_cols;
    if (chunk <= 0) {
        static const int bpc = blocks_per_cu(kernel, NW * 64);
        chunk = balanced_chunk(strips, j.src.ny, (int64_t)device_cu_count() * bpc * NW, 2 * TD + 2, 2 * TD);
    }
    const int chunks = (j.src.ny + chunk - 1) / chunk;
    const int64_t nw64 = (int64_t)strips * chunks;
    if (nw64 > (1ll << 30)) return hipErrorInvalidConfiguration;
    const int nw = (int)nw64;
    const int nbp = padded_block_count((nw + NW - 1) / NW);
    hipLaunchKernelGGL(kernel, dim3(nbp), dim3(NW * 64), 0, s, j.src, j.dst, j.rule, cf, cf2, alpha, chunk, strips,
                       nw, nbp, j.residual);
    return hipGetLastError();
}

template <typename T, int TD, bool BOX, int NW, int STG>
hipError_t launch_wave(const SweepJob& j, const Coef9<T>& cf, const Coef9<T>& cf2, T alpha, int chunk,
                       hipStream_t s) {
    const bool dx = !j.rule.per[0], dy = !j.rule.per[1];
#define LOPE_WAVE_RULE(C)                                                                          \
    if (dx && dy)                                                                                  \
        return launch_wave_case<T, TD, BOX, NW, STG, true, true, C>(j, cf, cf2, alpha, chunk, s);   \
    else if (dx)                                                                                   \
        return launch_wave_case<T, TD, BOX, NW, STG, true, false, C>(j, cf, cf2, alpha, chunk, s);  \
    else if (dy)                                                                                   \
        return launch_wave_case<T, TD, BOX, NW, STG, false, true, C>(j, cf, cf2, alpha, chunk, s);  \
    else                                                                                           \
        return launch_wave_case<T, TD, BOX, NW, STG, false, false, C>(j, cf, cf2, alpha, chunk, s)
    if (STG == 0 && j.residual) {
        LOPE_WAVE_RULE(STG == 0);
    } else {
        LOPE_WAVE_RULE(false);
    }
#undef LOPE_WAVE_RULE
}

template <typename T, int TD, bool BOX, int NW>
hipError_t run_plane2d_wave(const SweepJob& j, int chunk, hipStream_t s) {
    const Coef9<T> cf = coef9<T>(j);
    return launch_wave<T, TD, BOX, NW, 0>(j, cf, cf, (T)0, chunk, s);
}

// One two-stage step per pass (levels 1 and 2 with the two stencils).
template <typename T, int TD, bool BOX, int NW>
hipError_t run_plane2d_wave_stages(const StageJob& sj, int chunk, hipStream_t s) {
    if constexpr (TD != 2) {
        return hipErrorInvalidValue;
    } else {
        const Coef9<T> cf = coef9<T>(sj.s1), cf2 = coef9<T>(sj.s2);
        if (sj.alpha != 0.0) return launch_wave<T, TD, BOX, NW, 2>(sj.s1, cf, cf2, (T)sj.alpha, chunk, s);
        return launch_wave<T, TD, BOX, NW, 1>(sj.s1, cf, cf2, (T)0, chunk, s);
    }
}

#define PWAVE(T, DT, TD, BOX, NW, CH)                                                                  \
    {"plane2dw_" #T "_r1_t" #TD "_nw" #NW "_" #BOX, FAM_PLANE2D, 2, 1, TD, DT, BOX, 64 - 2 * (TD), 0, \
     (NW) * 64, CH, &run_plane2d_wave<T, TD, BOX, NW>, 1,                                          \
     (TD) == 2 ? &run_plane2d_wave_stages<T, TD, BOX, NW> : nullptr}

const Variant kPlane2dWave[] = {
    PWAVE(float, LOPE_F32, 1, true, 4, 0),
    PWAVE(float, LOPE_F32, 2, true, 4, 0),
    PWAVE(float, LOPE_F32, 3, true, 4, 0),
    PWAVE(float, LOPE_F32, 4, true, 4, 0),
    PWAVE(float, LOPE_F32, 5, true, 4, 0),
    PWAVE(float, LOPE_F32, 6, true, 4, 0),
    PWAVE(float, LOPE_F32, 8, true, 4, 0),
    PWAVE(float, LOPE_F32, 1, false, 4, 0),
    PWAVE(float, LOPE_F32, 2, false, 4, 0),
    PWAVE(float, LOPE_F32, 3, false, 4, 0),
    PWAVE(float, LOPE_F32, 4, false, 4, 0),
    PWAVE(double, LOPE_F64, 1, false, 4, 0),
    PWAVE(double, LOPE_F64, 2, false, 4, 0),
    PWAVE(double, LOPE_F64, 4, false, 4, 0),
    PWAVE(double, LOPE_F64, 6, false, 4, 0),
    PWAVE(double, LOPE_F64, 8, false, 4, 0),
    PWAVE(double, LOPE_F64, 2, true, 4, 0),
};

}  // namespace

int plane2d_wave_variants(const Variant** out) {
    *out = kPlane2dWave;
    return (int)(sizeof(kPlane2dWave) / sizeof(kPlane2dWave[0]));
}

}  // namespace lope
