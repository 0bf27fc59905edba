// Variable-coefficient diffusion on a periodic 3D grid and its reverse step.
//
//   forward:  u'_x = u_x + dt * sum_{a,s} K^s_a(x) (u_{x+s e_a} - u_x),
//             K^s_a(x) = (kappa_x + kappa_{x+s e_a}) / 2
//   reverse:  lam_x  = lam'_x + dt * sum_{a,s} K^s_a(x) (lam'_{x+s e_a} - lam'_x)
//             gk_x  += dt/2 * sum_{a,s} (u_{x+s e_a} - u_x) (lam'_x - lam'_{x+s e_a})
//
// The reverse step uses that the step matrix is symmetric (it equals its
// transpose), and the kappa term collects, for every face touching x, the
// derivative of that face's flux with respect to kappa_x.
//
// Both kernels march along z with the 3-plane z window in registers and the
// centre planes of every input staged in LDS for the x/y neighbours, like the
// constant-coefficient star kernel (radius 1, one sweep per pass).
#include "lope_internal.h"

namespace lope {
namespace {

constexpr int BX = 64, BY = 16, NT = 256;
constexpr int W = BX + 2, H = BY + 2, NPOS = W * H;
constexpr int NP = (NPOS + NT - 1) / NT;

struct Tile {
    int x0, y0, z0, zend;
};

__device__ __forceinline__ bool tile_of(const DevGrid& g, int chunk, int tiles_x, int tiles_y, int nblocks,
                                        int nbp, Tile& t) {
    const int logical = xcd_logical_block(nbp);
    if (logical >= nblocks) return false;
    const int tx = logical % tiles_x;
    const int rest = logical / tiles_x;
    t.x0 = tx * BX;
    t.y0 = (rest % tiles_y) * BY;
    t.z0 = (rest / tiles_y) * chunk;
    t.zend = min(t.z0 + chunk, g.nz);
    return true;
}

// Column offsets of the owned positions (wrapped, periodic) and output flags.
__device__ __forceinline__ void positions(const DevGrid& g, const Tile& t, int64_t (&off)[NP], bool (&used)[NP],
                                          bool (&core)[NP], int (&gxy)[NP][2]) {
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const int p = threadIdx.x + i * NT;
        const int px = p % W, py = p / W;
        const int gx = t.x0 - 1 + px, gy = t.y0 - 1 + py;
        used[i] = p < NPOS;
        core[i] = used[i] && px >= 1 && px <= BX && py >= 1 && py <= BY && gx < g.nx && gy < g.ny;
        off[i] = (int64_t)wrap_index(gx, g.nx) + (int64_t)wrap_index(gy, g.ny) * g.sy;
        gxy[i][0] = gx;
        gxy[i][1] = gy;
    }
}

template <typename T>
__global__ void __launch_bounds__(NT)
k_var_forward(DevGrid src, DevGrid dst, DevGrid kap, T dt, int chunk, int tiles_x, int tiles_y, int nblocks,
              int nbp) {
    __shared__ T lu[2][NPOS];
    __shared__ T lk[2][NPOS];
    Tile t;
    if (!tile_of(src, chunk, tiles_x, tiles_y, nblocks, nbp, t)) return;
    const T* __restrict__ up = (const T*)src.origin;
    const T* __restrict__ kp = (const T*)kap.origin;
    T* __restrict__ dp = (T*)dst.origin;
    int64_t offu[NP];
    bool used[NP], core[NP];
    int gxy[NP][2];
    positions(src, t, offu, used, core, gxy);
    int64_t offk[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) offk[i] = (int64_t)wrap_index(gxy[i][0], kap.nx) + (int64_t)wrap_index(gxy[i][1], kap.ny) * kap.sy;

    T ru[NP][3], rk[NP][3], pu[NP], pk[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int s = 0; s < 3; ++s) ru[i][s] = rk[i][s] = (T)0;
    auto load = [&](int j) {
        const int z = wrap_index(j, src.nz);
        const int64_t zu = (int64_t)z * src.sz, zk = (int64_t)z * kap.sz;
#pragma unroll
        for (int i = 0; i < NP; ++i)
            if (used[i]) {
                pu[i] = up[offu[i] + zu];
                pk[i] = kp[offk[i] + zk];
            }
    };
    const T half = (T)0.5;
    const int jstart = t.z0 - 1, jlast = t.zend, jend = t.zend + 1;
    load(jstart);
    for (int j = jstart; j <= jend; ++j) {
        const int rb = (j & 1) ^ 1, wb = j & 1;
        const int z = j - 2;
        if (z >= t.z0) {
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                if (!core[i]) continue;
                const int p = threadIdx.x + i * NT;
                const T uc = ru[i][1], kc = rk[i][1];
                const T un[6] = {lu[rb][p - 1], lu[rb][p + 1], lu[rb][p - W], lu[rb][p + W], ru[i][0], ru[i][2]};
                const T kn[6] = {lk[rb][p - 1], lk[rb][p + 1], lk[rb][p - W], lk[rb][p + W], rk[i][0], rk[i][2]};
                T acc = (T)0;
#pragma unroll
                for (int q = 0; q < 6; ++q) acc = fma(half * (kc + kn[q]), un[q] - uc, acc);
                __builtin_nontemporal_store(fma(dt, acc, uc),
                                            dp + (int64_t)gxy[i][0] + (int64_t)gxy[i][1] * dst.sy + (int64_t)z * dst.sz);
            }
        }
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            ru[i][0] = ru[i][1];
            ru[i][1] = ru[i][2];
            ru[i][2] = pu[i];
            rk[i][0] = rk[i][1];
            rk[i][1] = rk[i][2];
            rk[i][2] = pk[i];
            if (used[i]) {
                lu[wb][threadIdx.x + i * NT] = ru[i][1];
                lk[wb][threadIdx.x + i * NT] = rk[i][1];
            }
        }
        if (j + 1 <= jlast) load(j + 1);
        lds_barrier();
    }
}

template <typename T, typename TG>
__global__ void __launch_bounds__(NT)
k_var_adjoint(DevGrid lnext, DevGrid lam, DevGrid ug, DevGrid kap, DevGrid gk, T dt, int chunk, int tiles_x,
              int tiles_y, int nblocks, int nbp) {
    __shared__ T ll[2][NPOS];
    __shared__ T lu[2][NPOS];
    __shared__ T lk[2][NPOS];
    Tile t;
    if (!tile_of(lnext, chunk, tiles_x, tiles_y, nblocks, nbp, t)) return;
    const T* __restrict__ lp = (const T*)lnext.origin;
    const T* __restrict__ up = (const T*)ug.origin;
    const T* __restrict__ kp = (const T*)kap.origin;
    T* __restrict__ op = (T*)lam.origin;
    TG* __restrict__ gp = (TG*)gk.origin;
    int64_t offl[NP];
    bool used[NP], core[NP];
    int gxy[NP][2];
    positions(lnext, t, offl, used, core, gxy);
    int64_t offu[NP], offk[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const int wx = wrap_index(gxy[i][0], lnext.nx), wy = wrap_index(gxy[i][1], lnext.ny);
        offu[i] = (int64_t)wx + (int64_t)wy * ug.sy;
        offk[i] = (int64_t)wx + (int64_t)wy * kap.sy;
    }
    T rl[NP][3], ru[NP][3], rk[NP][3], pl[NP], pu[NP], pk[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int s = 0; s < 3; ++s) rl[i][s] = ru[i][s] = rk[i][s] = (T)0;
    auto load = [&](int j) {
        const int z = wrap_index(j, lnext.nz);
#pragma unroll
        for (int i = 0; i < NP; ++i)
            if (used[i]) {
                pl[i] = lp[offl[i] + (int64_t)z * lnext.sz];
                pu[i] = up[offu[i] + (int64_t)z * ug.sz];
                pk[i] = kp[offk[i] + (int64_t)z * kap.sz];
            }
    };
    const T half = (T)0.5;
    const T hdt = (T)0.5 * dt;
    const int jstart = t.z0 - 1, jlast = t.zend, jend = t.zend + 1;
    load(jstart);
    for (int j = jstart; j <= jend; ++j) {
        const int rb = (j & 1) ^ 1, wb = j & 1;
        const int z = j - 2;
        if (z >= t.z0) {
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                if (!core[i]) continue;
                const int p = threadIdx.x + i * NT;
                const T lc = rl[i][1], uc = ru[i][1], kc = rk[i][1];
                const T ln[6] = {ll[rb][p - 1], ll[rb][p + 1], ll[rb][p - W], ll[rb][p + W], rl[i][0], rl[i][2]};
                const T un[6] = {lu[rb][p - 1], lu[rb][p + 1], lu[rb][p - W], lu[rb][p + W], ru[i][0], ru[i][2]};
                const T kn[6] = {lk[rb][p - 1], lk[rb][p + 1], lk[rb][p - W], lk[rb][p + W], rk[i][0], rk[i][2]};
                T accl = (T)0, accg = (T)0;
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    accl = fma(half * (kc + kn[q]), ln[q] - lc, accl);
                    accg = fma(un[q] - uc, lc - ln[q], accg);
                }
                const int64_t ob = (int64_t)gxy[i][0] + (int64_t)gxy[i][1] * lam.sy + (int64_t)z * lam.sz;
                __builtin_nontemporal_store(fma(dt, accl, lc), op + ob);
                const int64_t gb = (int64_t)gxy[i][0] + (int64_t)gxy[i][1] * gk.sy + (int64_t)z * gk.sz;
                gp[gb] = gp[gb] + (TG)(hdt * accg);
            }
        }
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            rl[i][0] = rl[i][1]; rl[i][1] = rl[i][2]; rl[i][2] = pl[i];
            ru[i][0] = ru[i][1]; ru[i][1] = ru[i][2]; ru[i][2] = pu[i];
            rk[i][0] = rk[i][1]; rk[i][1] = rk[i][2]; rk[i][2] = pk[i];
            if (used[i]) {
                const int p = threadIdx.x + i * NT;
                ll[wb][p] = rl[i][1];
                lu[wb][p] = ru[i][1];
                lk[wb][p] = rk[i][1];
            }
        }
        if (j + 1 <= jlast) load(j + 1);
        lds_barrier();
    }
}

void geometry(const DevGrid& g, int& chunk, int& tiles_x, int& tiles_y, int& nb, int& nbp) {
    tiles_x = (g.nx + BX - 1) / BX;
    tiles_y = (g.ny + BY - 1) / BY;
    const int txy = tiles_x * tiles_y;
    int want = (2048 + txy - 1) / txy;
    chunk = (g.nz + want - 1) / want;
    if (chunk < 16) chunk = 16;
    const int tiles_z = (g.nz + chunk - 1) / chunk;
    nb = txy * tiles_z;
    nbp = padded_block_count(nb);
}

}  // namespace

hipError_t launch_var_forward(const DevGrid& src, const DevGrid& dst, const DevGrid& kappa, int dtype, double dt,
                              hipStream_t s) {
    int chunk, tx, ty, nb, nbp;
    geometry(src, chunk, tx, ty, nb, nbp);
    if (dtype == LOPE_F32)
        hipLaunchKernelGGL(k_var_forward<float>, dim3(nbp), dim3(NT), 0, s, src, dst, kappa, (float)dt, chunk, tx,
                           ty, nb, nbp);
    else
        hipLaunchKernelGGL(k_var_forward<double>, dim3(nbp), dim3(NT), 0, s, src, dst, kappa, dt, chunk, tx, ty, nb,
                           nbp);
    return hipGetLastError();
}

hipError_t launch_var_adjoint(const DevGrid& lam_next, const DevGrid& lam, const DevGrid& u, const DevGrid& kappa,
                              const DevGrid& gk, int dtype, int gk_dtype, double dt, hipStream_t s) {
    int chunk, tx, ty, nb, nbp;
    geometry(lam_next, chunk, tx, ty, nb, nbp);
    if (dtype == LOPE_F32 && gk_dtype == LOPE_F32)
        hipLaunchKernelGGL((k_var_adjoint<float, float>), dim3(nbp), dim3(NT), 0, s, lam_next, lam, u, kappa, gk,
                           (float)dt, chunk, tx, ty, nb, nbp);
    else if (dtype == LOPE_F32)
        hipLaunchKernelGGL((k_var_adjoint<float, double>), dim3(nbp), dim3(NT), 0, s, lam_next, lam, u, kappa, gk,
                           (float)dt, chunk, tx, ty, nb, nbp);
    else if (gk_dtype == LOPE_F64)
        hipLaunchKernelGGL((k_var_adjoint<double, double>), dim3(nbp), dim3(NT), 0, s, lam_next, lam, u, kappa, gk,
                           dt, chunk, tx, ty, nb, nbp);
    else
        hipLaunchKernelGGL((k_var_adjoint<double, float>), dim3(nbp), dim3(NT), 0, s, lam_next, lam, u, kappa, gk,
                           dt, chunk, tx, ty, nb, nbp);
    return hipGetLastError();
}

}  // namespace lope
