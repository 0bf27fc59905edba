// Two reverse steps of the variable-coefficient diffusion fused in one pass.
//
// Given lam_{t+1}, u_t, u_{t-1} and kappa it produces
//   lam_t     = A(kappa) lam_{t+1}                       (kept on chip)
//   lam_{t-1} = A(kappa) lam_t                           (written)
//   gk       += G(u_t, lam_{t+1}) + G(u_{t-1}, lam_t)    (one read-modify-write)
// with (A v)_x = v_x + dt sum_q K_q (v_q - v_x), K_q = (kappa_x + kappa_q)/2,
// and G(u, l)_x = dt/2 sum_q (u_q - u_x)(l_x - l_q), q over the six face
// neighbours in the order x-, x+, y-, y+, z-, z+ (periodic grid).  The
// arithmetic per cell is the same as two calls of the one-step reverse
// kernel; only the kappa-gradient accumulator differs in rounding (one add of
// the two terms' sum instead of two adds).
//
// A workgroup marches a z-chunk of a BX x BY output tile widened by 2 cells in
// x and y (one per fused step).  Every thread owns fixed positions of the
// widened tile.  Per position it keeps z-windows in registers: lam_{t+1} and
// u_t (3 planes), kappa (5 planes: both steps read it, two planes apart),
// u_{t-1} (3 planes, loaded two planes behind the others) and lam_t (3 planes
// of computed values).  The centre planes needed for x/y neighbours sit in
// LDS (lam_{t+1}, kappa, u_t at the first step's plane; lam_t, kappa,
// u_{t-1} at the second step's plane), double-buffered, one barrier per
// plane.  At march step j the first step computes plane j-2 and the second
// plane j-4; the first step's kappa-gradient term of a core cell waits in a
// register window until the second step reaches the same plane.
#include "lope_internal.h"

namespace lope {
namespace {

constexpr int A2_BX = 64, A2_BY = 16, A2_NT = 512;
constexpr int A2_W = A2_BX + 4, A2_H = A2_BY + 4, A2_NPOS = A2_W * A2_H;
constexpr int A2_NP = (A2_NPOS + A2_NT - 1) / A2_NT;

template <typename T, typename TG>
__global__ void __launch_bounds__(A2_NT)
k_var_adjoint2(DevGrid lnext, DevGrid lout, DevGrid ut, DevGrid utm1, DevGrid kap, DevGrid gk, T dt, int chunk,
               int tiles_x, int tiles_y, int nblocks, int nblocks_padded) {
    constexpr int W = A2_W, NP = A2_NP, NPOS = A2_NPOS, NT = A2_NT;
    // LDS planes: 0 lam_{t+1}, 1 kappa(first), 2 u_t, 3 lam_t, 4 kappa(second), 5 u_{t-1}
    __shared__ T lds[2][6][NPOS];

    const int logical = xcd_logical_block(nblocks_padded);
    if (logical >= nblocks) return;
    const int tix = logical % tiles_x;
    const int rest = logical / tiles_x;
    const int x0 = tix * A2_BX, y0 = (rest % tiles_y) * A2_BY, z0 = (rest / tiles_y) * chunk;
    const int nx = lout.nx, ny = lout.ny, nz = lout.nz;
    const int zend = min(z0 + chunk, nz);
    const int tid = threadIdx.x;

    int64_t off[NP][4];   // wrapped column offsets in lnext, ut, utm1, kap
    int depth[NP];        // distance to the widened tile's edge (-1: unused)
    bool keep[NP];        // core cell inside the interior
    int64_t oo[NP], og[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const int p = tid + i * NT;
        const int px = p % W, py = p / W;
        const int gx = x0 - 2 + px, gy = y0 - 2 + py;
        depth[i] = p < NPOS ? min(min(px, W - 1 - px), min(py, A2_H - 1 - py)) : -1;
        const int wx = wrap_index(gx, nx), wy = wrap_index(gy, ny);
        off[i][0] = (int64_t)wx + (int64_t)wy * lnext.sy;
        off[i][1] = (int64_t)wx + (int64_t)wy * ut.sy;
        off[i][2] = (int64_t)wx + (int64_t)wy * utm1.sy;
        off[i][3] = (int64_t)wx + (int64_t)wy * kap.sy;
        keep[i] = depth[i] >= 2 && gx < nx && gy < ny;
        oo[i] = (int64_t)gx + (int64_t)gy * lout.sy;
        og[i] = (int64_t)gx + (int64_t)gy * gk.sy;
    }
    const T* __restrict__ pl = (const T*)lnext.origin;
    const T* __restrict__ pu = (const T*)ut.origin;
    const T* __restrict__ pv = (const T*)utm1.origin;
    const T* __restrict__ pk = (const T*)kap.origin;
    T* __restrict__ po = (T*)lout.origin;
    TG* __restrict__ pg = (TG*)gk.origin;

    T rA[NP][3], rU[NP][3], rK[NP][5], rV[NP][3], rL[NP][3], gterm[NP][3];
    T nA[NP], nU[NP], nK[NP], nV[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
#pragma unroll
        for (int s = 0; s < 3; ++s) rA[i][s] = rU[i][s] = rV[i][s] = rL[i][s] = gterm[i][s] = (T)0;
#pragma unroll
        for (int s = 0; s < 5; ++s) rK[i][s] = (T)0;
    }
    // loads of march step j: lam_{t+1}, u_t, kappa at plane j; u_{t-1} at plane j-2
    auto load = [&](int j) {
        const int z = wrap_index(j, nz), zv = wrap_index(j - 2, nz);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            if (depth[i] < 0) continue;
            nA[i] = pl[off[i][0] + (int64_t)z * lnext.sz];
            nU[i] = pu[off[i][1] + (int64_t)z * ut.sz];
            nK[i] = pk[off[i][3] + (int64_t)z * kap.sz];
            nV[i] = pv[off[i][2] + (int64_t)zv * utm1.sz];
        }
    };
    const T half = (T)0.5;
    const T hdt = (T)0.5 * dt;
    const int jstart = z0 - 2;
    const int jend = zend + 3;
    load(jstart);
    for (int j = jstart; j <= jend; ++j) {
        const int rb = (j & 1) ^ 1, wb = j & 1;
        const T* LA = lds[rb][0];
        const T* LK1 = lds[rb][1];
        const T* LU = lds[rb][2];
        const T* LL = lds[rb][3];
        const T* LK2 = lds[rb][4];
        const T* LV = lds[rb][5];
        T newL[NP], newG[NP];
        const int z2 = j - 4;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            newL[i] = (T)0;
            newG[i] = (T)0;
            if (depth[i] < 1) continue;
            const int p = tid + i * NT;
            // first step at plane j-2: lam_t (depth >= 1) and its kappa term (core)
            {
                const T ac = rA[i][1], kc = rK[i][3];
                const T an[6] = {LA[p - 1], LA[p + 1], LA[p - W], LA[p + W], rA[i][0], rA[i][2]};
                const T kn[6] = {LK1[p - 1], LK1[p + 1], LK1[p - W], LK1[p + W], rK[i][2], rK[i][4]};
                T acc = (T)0;
#pragma unroll
                for (int q = 0; q < 6; ++q) acc = fma(half * (kc + kn[q]), an[q] - ac, acc);
                newL[i] = fma(dt, acc, ac);
                if (depth[i] >= 2) {
                    const T uc = rU[i][1];
                    const T un[6] = {LU[p - 1], LU[p + 1], LU[p - W], LU[p + W], rU[i][0], rU[i][2]};
                    T g = (T)0;
#pragma unroll
                    for (int q = 0; q < 6; ++q) g = fma(un[q] - uc, ac - an[q], g);
                    newG[i] = hdt * g;
                }
            }
            // second step at plane j-4: lam_{t-1} and the total kappa term (core)
            if (depth[i] >= 2 && keep[i] && z2 >= z0 && z2 < zend) {
                const T lc = rL[i][1], kc = rK[i][1], vc = rV[i][1];
                const T ln[6] = {LL[p - 1], LL[p + 1], LL[p - W], LL[p + W], rL[i][0], rL[i][2]};
                const T kn[6] = {LK2[p - 1], LK2[p + 1], LK2[p - W], LK2[p + W], rK[i][0], rK[i][2]};
                const T vn[6] = {LV[p - 1], LV[p + 1], LV[p - W], LV[p + W], rV[i][0], rV[i][2]};
                T acc = (T)0, g = (T)0;
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    acc = fma(half * (kc + kn[q]), ln[q] - lc, acc);
                    g = fma(vn[q] - vc, lc - ln[q], g);
                }
                __builtin_nontemporal_store(fma(dt, acc, lc), po + oo[i] + (int64_t)z2 * lout.sz);
                TG* gp = pg + og[i] + (int64_t)z2 * gk.sz;
                *gp = *gp + (TG)(gterm[i][1] + hdt * g);
            }
        }
        // advance every window by one plane
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            rA[i][0] = rA[i][1]; rA[i][1] = rA[i][2]; rA[i][2] = nA[i];
            rU[i][0] = rU[i][1]; rU[i][1] = rU[i][2]; rU[i][2] = nU[i];
            rV[i][0] = rV[i][1]; rV[i][1] = rV[i][2]; rV[i][2] = nV[i];
#pragma unroll
            for (int s = 0; s < 4; ++s) rK[i][s] = rK[i][s + 1];
            rK[i][4] = nK[i];
            rL[i][0] = rL[i][1]; rL[i][1] = rL[i][2]; rL[i][2] = newL[i];
            gterm[i][0] = gterm[i][1]; gterm[i][1] = gterm[i][2]; gterm[i][2] = newG[i];
        }
        // publish the centre planes of the next step
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            if (depth[i] < 0) continue;
            const int p = tid + i * NT;
            lds[wb][0][p] = rA[i][1];
            lds[wb][1][p] = rK[i][3];
            lds[wb][2][p] = rU[i][1];
            lds[wb][3][p] = rL[i][1];
            lds[wb][4][p] = rK[i][1];
            lds[wb][5][p] = rV[i][1];
        }
        if (j + 1 <= jend) load(j + 1);
        lds_barrier();
    }
}

}  // namespace

hipError_t launch_var_adjoint2(const DevGrid& lam_next, const DevGrid& lam_out, const DevGrid& u_t,
                               const DevGrid& u_tm1, const DevGrid& kappa, const DevGrid& gk, int dtype,
                               int gk_dtype, double dt, hipStream_t s) {
    const int tiles_x = (lam_out.nx + A2_BX - 1) / A2_BX;
    const int tiles_y = (lam_out.ny + A2_BY - 1) / A2_BY;
    const int txy = tiles_x * tiles_y;
    const int want = (1024 + txy - 1) / txy;
    int chunk = (lam_out.nz + want - 1) / want;
    if (chunk < 32) chunk = 32;
    const int tiles_z = (lam_out.nz + chunk - 1) / chunk;
    const int nb = txy * tiles_z;
    const int nbp = padded_block_count(nb);
    if (dtype == LOPE_F32 && gk_dtype == LOPE_F32)
        hipLaunchKernelGGL((k_var_adjoint2<float, float>), dim3(nbp), dim3(A2_NT), 0, s, lam_next, lam_out, u_t, u_tm1,
                           kappa, gk, (float)dt, chunk, tiles_x, tiles_y, nb, nbp);
    else if (dtype == LOPE_F32)
        hipLaunchKernelGGL((k_var_adjoint2<float, double>), dim3(nbp), dim3(A2_NT), 0, s, lam_next, lam_out, u_t,
                           u_tm1, kappa, gk, (float)dt, chunk, tiles_x, tiles_y, nb, nbp);
    else if (gk_dtype == LOPE_F64)
        hipLaunchKernelGGL((k_var_adjoint2<double, double>), dim3(nbp), dim3(A2_NT), 0, s, lam_next, lam_out, u_t,
                           u_tm1, kappa, gk, dt, chunk, tiles_x, tiles_y, nb, nbp);
    else
        hipLaunchKernelGGL((k_var_adjoint2<double, float>), dim3(nbp), dim3(A2_NT), 0, s, lam_next, lam_out, u_t,
                           u_tm1, kappa, gk, dt, chunk, tiles_x, tiles_y, nb, nbp);
    return hipGetLastError();
}

}  // namespace lope
