// Variable-coefficient diffusion (periodic 3D) with 16-byte vector memory
// access: forward step and reverse step.
//
// Same update as the scalar kernels:
//   forward:  u'_x = u_x + dt * sum_q K_q (u_q - u_x),          K_q = (kappa_x + kappa_q)/2
//   reverse:  lam_x = lam'_x + dt * sum_q K_q (lam'_q - lam'_x)
//             gk_x += dt/2 * sum_q (u_q - u_x) (lam'_x - lam'_q)
// with q running over the six face neighbours in the order x-, x+, y-, y+,
// z-, z+.
//
// Layout of the work as in the vector star kernel: a workgroup marches a
// z-chunk of a BX x BY tile; each thread owns VEC consecutive x positions on
// RPT rows and keeps the last 3 planes of every input field for them in
// registers (z neighbours); the centre plane of every field with a one-cell
// x/y halo is published in LDS, double-buffered, one barrier per plane.
// Inputs are fetched two planes ahead of the plane being computed, halos one
// plane ahead.  All fields are periodic on every axis.
//
// Requirements (checked by the caller): every origin 16-byte aligned, y and
// z strides multiples of VEC elements.
#include "lope_internal.h"

namespace lope {
namespace {

template <typename T>
struct DVec;
template <>
struct DVec<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int n = 4;
};
template <>
struct DVec<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int n = 2;
};

constexpr int kBX = 64, kBY = 16, kNT = 256;

// NF input fields: forward (u, kappa); reverse (lam', u, kappa).
template <typename T, bool ADJ, typename TG>
__global__ void __launch_bounds__(kNT)
k_var_vec(DevGrid f0, DevGrid f1, DevGrid f2, DevGrid out, DevGrid gk, T dt, int chunk, int tiles_x, int tiles_y,
          int nblocks, int nblocks_padded) {
    typedef typename DVec<T>::type VT;
    constexpr int NF = ADJ ? 3 : 2;
    constexpr int VEC = DVec<T>::n;
    constexpr int BX = kBX, BY = kBY, NT = kNT;
    constexpr int TX = BX / VEC;
    constexpr int TYT = NT / TX;
    constexpr int RPT = BY / TYT;
    constexpr int kLead = VEC;                 // >= 1 halo column, keeps the core 16-byte aligned
    constexpr int LW = kLead + BX + kLead;
    constexpr int LH = BY + 2;
    constexpr int NHROW = 2 * TX;
    constexpr int NHCOL = 2 * BY;
    constexpr int NHALO = NHROW + NHCOL;
    constexpr int HPT = (NHALO + NT - 1) / NT;
    static_assert(BX % VEC == 0 && NT % TX == 0 && BY % TYT == 0, "tile shape");

    __shared__ __attribute__((aligned(16))) T lds[2][NF][LH][LW];

    const int logical = xcd_logical_block(nblocks_padded);
    if (logical >= nblocks) return;
    const int tix = logical % tiles_x;
    const int rest = logical / tiles_x;
    const int x0 = tix * BX, y0 = (rest % tiles_y) * BY, z0 = (rest / tiles_y) * chunk;
    const int nx = out.nx, ny = out.ny, nz = out.nz;
    const int zend = min(z0 + chunk, nz);
    const DevGrid F[3] = {f0, f1, f2};

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int cx = x0 + tx * VEC;
    const bool xfull = cx + VEC <= nx;
    int cy[RPT];
    bool yin[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        cy[k] = y0 + ty + k * TYT;
        yin[k] = cy[k] < ny;
    }
    auto elem = [&](int f, int gx, int gy, int z) -> T {
        const T* p = (const T*)F[f].origin;
        return p[(int64_t)z * F[f].sz + (int64_t)wrap_index(gy, ny) * F[f].sy + wrap_index(gx, nx)];
    };
    auto load_core = [&](int j, T (&v)[NF][RPT][VEC]) {
        const int z = wrap_index(j, nz);
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                if (xfull) {
                    const T* p = (const T*)F[f].origin;
                    const VT q = *(const VT*)(p + (int64_t)z * F[f].sz + (int64_t)wrap_index(cy[k], ny) * F[f].sy + cx);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) v[f][k][e] = ((const T*)&q)[e];
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) v[f][k][e] = elem(f, cx + e, cy[k], z);
                }
            }
    };
    auto load_halo = [&](int j, T (&hv)[NF][HPT][VEC]) {
        const int z = wrap_index(j, nz);
#pragma unroll
        for (int m = 0; m < HPT; ++m) {
            const int h = tid + m * NT;
            if (h >= NHALO) continue;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                if (h < NHROW) {
                    const int r = h / TX, hx = h % TX;
                    const int gy = r == 0 ? y0 - 1 : y0 + BY;
                    const int gx = x0 + hx * VEC;
                    if (gx + VEC <= nx) {
                        const T* p = (const T*)F[f].origin;
                        const VT q = *(const VT*)(p + (int64_t)z * F[f].sz + (int64_t)wrap_index(gy, ny) * F[f].sy + gx);
#pragma unroll
                        for (int e = 0; e < VEC; ++e) hv[f][m][e] = ((const T*)&q)[e];
                    } else {
#pragma unroll
                        for (int e = 0; e < VEC; ++e) hv[f][m][e] = elem(f, gx + e, gy, z);
                    }
                } else {
                    const int c = h - NHROW;
                    const int side = c / BY, row = c % BY;
                    hv[f][m][0] = elem(f, side == 0 ? x0 - 1 : x0 + BX, y0 + row, z);
                }
            }
        }
    };
    auto store_halo = [&](int b, const T (&hv)[NF][HPT][VEC]) {
#pragma unroll
        for (int m = 0; m < HPT; ++m) {
            const int h = tid + m * NT;
            if (h >= NHALO) continue;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                if (h < NHROW) {
                    const int r = h / TX, hx = h % TX;
                    const int ly = r == 0 ? 0 : BY + 1;
#pragma unroll
                    for (int e = 0; e < VEC; ++e) lds[b][f][ly][kLead + hx * VEC + e] = hv[f][m][e];
                } else {
                    const int c = h - NHROW;
                    const int side = c / BY, row = c % BY;
                    lds[b][f][1 + row][side == 0 ? kLead - 1 : kLead + BX] = hv[f][m][0];
                }
            }
        }
    };
    auto store_core = [&](int b, const T (&ring)[NF][RPT][3][VEC]) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int k = 0; k < RPT; ++k)
#pragma unroll
                for (int e = 0; e < VEC; ++e) lds[b][f][1 + ty + k * TYT][kLead + tx * VEC + e] = ring[f][k][1][e];
    };

    T ring[NF][RPT][3][VEC];
    T pre[NF][RPT][VEC];
    T hpre[NF][HPT][VEC];
    {
        T tmp[NF][RPT][VEC];
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            load_core(z0 - 1 + s, tmp);
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int k = 0; k < RPT; ++k)
#pragma unroll
                    for (int e = 0; e < VEC; ++e) ring[f][k][s][e] = tmp[f][k][e];
        }
    }
    load_halo(z0, hpre);
    store_halo(0, hpre);
    store_core(0, ring);
    load_core(z0 + 2, pre);
    load_halo(z0 + 1, hpre);
    lds_barrier();

    const T half = (T)0.5;
    const T hdt = (T)0.5 * dt;
    for (int zc = z0; zc < zend; ++zc) {
        const int b = (zc - z0) & 1;
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int ly = 1 + ty + k * TYT;
            const int lx = kLead + tx * VEC;
            T o1[VEC], o2[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                // neighbour values of field f in the order x-, x+, y-, y+, z-, z+
                auto nb = [&](int f, int q) -> T {
                    switch (q) {
                        case 0: return lds[b][f][ly][lx + e - 1];
                        case 1: return lds[b][f][ly][lx + e + 1];
                        case 2: return lds[b][f][ly - 1][lx + e];
                        case 3: return lds[b][f][ly + 1][lx + e];
                        case 4: return ring[f][k][0][e];
                        default: return ring[f][k][2][e];
                    }
                };
                if (!ADJ) {
                    const T uc = ring[0][k][1][e], kc = ring[1][k][1][e];
                    T acc = (T)0;
#pragma unroll
                    for (int q = 0; q < 6; ++q) acc = fma(half * (kc + nb(1, q)), nb(0, q) - uc, acc);
                    o1[e] = fma(dt, acc, uc);
                } else {
                    const T lc = ring[0][k][1][e], uc = ring[1][k][1][e], kc = ring[2][k][1][e];
                    T accl = (T)0, accg = (T)0;
#pragma unroll
                    for (int q = 0; q < 6; ++q) {
                        const T ln = nb(0, q);
                        accl = fma(half * (kc + nb(2, q)), ln - lc, accl);
                        accg = fma(nb(1, q) - uc, lc - ln, accg);
                    }
                    o1[e] = fma(dt, accl, lc);
                    o2[e] = hdt * accg;
                }
            }
            if (yin[k]) {
                const int64_t ro = (int64_t)zc * out.sz + (int64_t)cy[k] * out.sy + cx;
                T* op = (T*)out.origin + ro;
                if (xfull) {
                    VT q;
#pragma unroll
                    for (int e = 0; e < VEC; ++e) ((T*)&q)[e] = o1[e];
                    __builtin_nontemporal_store(q, (VT*)op);
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        if (cx + e < nx) __builtin_nontemporal_store(o1[e], op + e);
                }
                if (ADJ) {
                    TG* gp = (TG*)gk.origin + (int64_t)zc * gk.sz + (int64_t)cy[k] * gk.sy + cx;
                    if constexpr (sizeof(TG) == sizeof(T)) {
                        if (xfull) {
                            VT q = *(const VT*)gp;
#pragma unroll
                            for (int e = 0; e < VEC; ++e) ((T*)&q)[e] = ((T*)&q)[e] + o2[e];
                            *(VT*)gp = q;
                            continue;
                        }
                    }
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        if (cx + e < nx) gp[e] = gp[e] + (TG)o2[e];
                }
            }
        }
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int k = 0; k < RPT; ++k)
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    ring[f][k][0][e] = ring[f][k][1][e];
                    ring[f][k][1][e] = ring[f][k][2][e];
                    ring[f][k][2][e] = pre[f][k][e];
                }
        if (zc + 1 < zend) {
            store_halo(b ^ 1, hpre);
            store_core(b ^ 1, ring);
            if (zc + 2 < zend) {
                load_core(zc + 3, pre);
                load_halo(zc + 2, hpre);
            }
        }
        lds_barrier();
    }
}

int chunk_for(const DevGrid& g, int& tiles_x, int& tiles_y, int& nb, int& nbp) {
    tiles_x = (g.nx + kBX - 1) / kBX;
    tiles_y = (g.ny + kBY - 1) / kBY;
    const int txy = tiles_x * tiles_y;
    const int want = (2048 + txy - 1) / txy;
    int chunk = (g.nz + want - 1) / want;
    if (chunk < 16) chunk = 16;
    const int tiles_z = (g.nz + chunk - 1) / chunk;
    nb = txy * tiles_z;
    nbp = padded_block_count(nb);
    return chunk;
}

}  // namespace

bool var_vec_fits(const DevGrid* gs, int count, int dtype) {
    const int64_t vec = dtype == LOPE_F64 ? 2 : 4;
    for (int i = 0; i < count; ++i)
        if (((uintptr_t)gs[i].origin % 16) != 0 || gs[i].sy % vec != 0 || gs[i].sz % vec != 0) return false;
    return true;
}

hipError_t launch_var_forward_vec(const DevGrid& src, const DevGrid& dst, const DevGrid& kappa, int dtype, double dt,
                                  hipStream_t s) {
    int tx, ty, nb, nbp;
    const int chunk = chunk_for(dst, tx, ty, nb, nbp);
    if (dtype == LOPE_F32)
        hipLaunchKernelGGL((k_var_vec<float, false, float>), dim3(nbp), dim3(kNT), 0, s, src, kappa, kappa, dst, dst,
                           (float)dt, chunk, tx, ty, nb, nbp);
    else
        hipLaunchKernelGGL((k_var_vec<double, false, double>), dim3(nbp), dim3(kNT), 0, s, src, kappa, kappa, dst, dst,
                           dt, chunk, tx, ty, nb, nbp);
    return hipGetLastError();
}

hipError_t launch_var_adjoint_vec(const DevGrid& lam_next, const DevGrid& lam, const DevGrid& u, const DevGrid& kappa,
                                  const DevGrid& gk, int dtype, int gk_dtype, double dt, hipStream_t s) {
    int tx, ty, nb, nbp;
    const int chunk = chunk_for(lam, tx, ty, nb, nbp);
    if (dtype == LOPE_F32 && gk_dtype == LOPE_F32)
        hipLaunchKernelGGL((k_var_vec<float, true, float>), dim3(nbp), dim3(kNT), 0, s, lam_next, u, kappa, lam, gk,
                           (float)dt, chunk, tx, ty, nb, nbp);
    else if (dtype == LOPE_F32)
        hipLaunchKernelGGL((k_var_vec<float, true, double>), dim3(nbp), dim3(kNT), 0, s, lam_next, u, kappa, lam, gk,
                           (float)dt, chunk, tx, ty, nb, nbp);
    else if (gk_dtype == LOPE_F64)
        hipLaunchKernelGGL((k_var_vec<double, true, double>), dim3(nbp), dim3(kNT), 0, s, lam_next, u, kappa, lam, gk,
                           dt, chunk, tx, ty, nb, nbp);
    else
        hipLaunchKernelGGL((k_var_vec<double, true, float>), dim3(nbp), dim3(kNT), 0, s, lam_next, u, kappa, lam, gk,
                           dt, chunk, tx, ty, nb, nbp);
    return hipGetLastError();
}

}  // namespace lope
