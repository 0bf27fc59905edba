// 3D star stencils with TD sweeps fused per pass (temporal blocking) and
// 16-byte vector access, for radius R <= VEC (4 floats or 2 doubles).
//
// A workgroup marches a z-chunk of a BX x BY output tile.  Level k (state
// after k sweeps, k = 0..TD) lives on the tile widened by G = R*TD cells in y
// and by GA = G rounded up to whole vectors in x, so every position is one
// aligned vector.  Each thread owns fixed vector positions of the widened
// tile at all levels and keeps, per level, the last 2R+1 planes of its
// positions in registers (z neighbours); each level's centre plane is
// published in LDS (double-buffered, one barrier per plane) for the x/y
// neighbours.  At march step j level 0 receives plane j and level k computes
// plane j - k(R+1) from level k-1.  Every element of every position is
// computed at every level; the valid region shrinks by R per level, and an
// element whose inputs fall outside it is never used by a valid element (the
// LDS rows carry VEC padding columns so such reads stay in bounds).  Level
// TD is stored for the core tile only.
//
// Per point: c0*v0 then fmas in lexicographic offset order (z-R .. z-1,
// y-R .. y-1, x-R .. x+R, y+1 .. y+R, z+1 .. z+R), the same as every other
// kernel, so TD fused sweeps equal TD single sweeps exactly.  The boundary
// rule is applied at load for level 0; at every level an element outside the
// interior along a Dirichlet axis holds g.
//
// Requirements (checked by the caller): origin 16-byte aligned, y and z
// strides multiples of VEC elements.
#include "lope_internal.h"

namespace lope {
namespace {

template <typename T, int R>
struct TStarCoef {
    T c[6 * R + 1];
};

template <typename T>
struct TVec;
template <>
struct TVec<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int n = 4;
};
template <>
struct TVec<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int n = 2;
};

template <typename T, int R, int TD, int BX, int BY, int NT>
__global__ void __launch_bounds__(NT)
k_star3d_vtb(DevGrid src, DevGrid dst, DevRule rule, TStarCoef<T, R> cf, int chunk, int tiles_x, int tiles_y,
             int nblocks, int nblocks_padded) {
    typedef typename TVec<T>::type VT;
    constexpr int VEC = TVec<T>::n;
    static_assert(R <= VEC, "radius up to one vector");
    constexpr int G = R * TD;
    constexpr int GA = ((G + VEC - 1) / VEC) * VEC;
    constexpr int W0 = BX + 2 * GA;          // widened tile width (elements)
    constexpr int VW = W0 / VEC;             // vectors per row
    constexpr int H0 = BY + 2 * G;           // widened tile rows
    constexpr int NV = VW * H0;              // vector positions
    constexpr int NPV = (NV + NT - 1) / NT;  // positions per thread
    constexpr int PAD = VEC;                 // LDS padding columns each side
    constexpr int LW = PAD + W0 + PAD;
    constexpr int RING = 2 * R + 1;
    static_assert(BX % VEC == 0, "tile width in whole vectors");

    __shared__ __attribute__((aligned(16))) T lds[TD][2][H0][LW];

    const int logical = xcd_logical_block(nblocks_padded);
    if (logical >= nblocks) return;
    const int tix = logical % tiles_x;
    const int rest = logical / tiles_x;
    const int tiy = rest % tiles_y;
    const int tiz = rest / tiles_y;
    const int nx = src.nx, ny = src.ny, nz = src.nz;
    const int x0 = tix * BX, y0 = tiy * BY, z0 = tiz * chunk;
    const int zend = min(z0 + chunk, nz);
    const bool perx = rule.per[0] != 0, pery = rule.per[1] != 0, perz = rule.per[2] != 0;
    const T g = (T)rule.g;
    const T* __restrict__ sp = (const T*)src.origin;
    T* __restrict__ dp = (T*)dst.origin;
    const int tid = threadIdx.x;

    // per owned position: tile coordinates, global coordinates, flags
    int pvx[NPV], ppy[NPV];
    bool used[NPV];
    bool core[NPV];          // level-TD output vector inside the core tile
    bool yd[NPV];            // row outside the interior along a Dirichlet y axis
    unsigned xd[NPV];        // bit e: element e outside along a Dirichlet x axis
    bool vfast[NPV];         // whole vector interior in x and row loadable
    int64_t roff[NPV];       // src offset of the (wrapped) row start
#pragma unroll
    for (int i = 0; i < NPV; ++i) {
        const int p = tid + i * NT;
        used[i] = p < NV;
        const int vx = used[i] ? p % VW : 0, py = used[i] ? p / VW : 0;
        pvx[i] = vx;
        ppy[i] = py;
        const int gx = x0 - GA + vx * VEC, gy = y0 - G + py;
        const bool oy = gy < 0 || gy >= ny;
        yd[i] = oy && !pery;
        unsigned m = 0;
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            if (!perx && (gx + e < 0 || gx + e >= nx)) m |= 1u << e;
        xd[i] = m;
        vfast[i] = gx >= 0 && gx + VEC <= nx && !yd[i];
        const int wy = oy ? (pery ? wrap_index(gy, ny) : 0) : gy;
        roff[i] = (int64_t)wy * src.sy;
        core[i] = used[i] && py >= G && py < G + BY && vx >= GA / VEC && vx < (GA + BX) / VEC && gy < ny && gx < nx;
    }

    T ring[TD][NPV][RING][VEC];
    T pre[NPV][VEC];
#pragma unroll
    for (int k = 0; k < TD; ++k)
#pragma unroll
        for (int i = 0; i < NPV; ++i)
#pragma unroll
            for (int s = 0; s < RING; ++s)
#pragma unroll
                for (int e = 0; e < VEC; ++e) ring[k][i][s][e] = (T)0;

    auto load_plane = [&](int j) {
        const bool oz = j < 0 || j >= nz;
        if (oz && !perz) {
#pragma unroll
            for (int i = 0; i < NPV; ++i)
#pragma unroll
                for (int e = 0; e < VEC; ++e) pre[i][e] = g;
            return;
        }
        const int64_t zo = (int64_t)(perz ? wrap_index(j, nz) : j) * src.sz;
#pragma unroll
        for (int i = 0; i < NPV; ++i) {
            if (!used[i]) continue;
            const int gx = x0 - GA + pvx[i] * VEC;
            if (vfast[i]) {
                const VT q = *(const VT*)(sp + zo + roff[i] + gx);
#pragma unroll
                for (int e = 0; e < VEC; ++e) pre[i][e] = ((const T*)&q)[e];
            } else if (yd[i]) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) pre[i][e] = g;
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    pre[i][e] = ((xd[i] >> e) & 1u) ? g : sp[zo + roff[i] + wrap_index(gx + e, nx)];
            }
        }
    };

    const int jstart = z0 - G;
    const int jlast_load = zend - 1 + G;
    const int jend = zend - 1 + TD * (R + 1);
    load_plane(jstart);

    for (int j = jstart; j <= jend; ++j) {
        const int rb = (j & 1) ^ 1;
        const int wb = j & 1;
        T nv[TD][NPV][VEC];
#pragma unroll
        for (int k = 1; k <= TD; ++k) {
            const int zk = j - k * (R + 1);
            const bool zdir = !perz && (zk < 0 || zk >= nz);
#pragma unroll
            for (int i = 0; i < NPV; ++i) {
                if (!used[i]) continue;
                if (k == TD && !core[i]) continue;
                const int ly = ppy[i];
                const int lx = PAD + pvx[i] * VEC;
                T (*L)[LW] = lds[k - 1][rb];
                // x neighbours beyond the vector come from the adjacent vectors in LDS
                T left[R], right[R];
#pragma unroll
                for (int o = 0; o < R; ++o) {
                    left[o] = L[ly][lx - R + o];
                    right[o] = L[ly][lx + VEC + o];
                }
                T yv[2 * R][VEC];
#pragma unroll
                for (int o = 0; o < 2 * R; ++o) {
                    const int row = ly + (o < R ? o - R : o - R + 1);
                    const int rr = row < 0 ? 0 : (row >= H0 ? H0 - 1 : row);
                    const VT q = *(const VT*)&L[rr][lx];
#pragma unroll
                    for (int e = 0; e < VEC; ++e) yv[o][e] = ((const T*)&q)[e];
                }
                T out[VEC];
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    auto xval = [&](int o) -> T {   // element e+o of the centre row
                        const int q = e + o;
                        if (q < 0) return left[q + R];
                        if (q >= VEC) return right[q - VEC];
                        return ring[k - 1][i][R][q];
                    };
                    T v = cf.c[0] * ring[k - 1][i][0][e];
#pragma unroll
                    for (int s = 1; s < R; ++s) v = fma(cf.c[s], ring[k - 1][i][s][e], v);
#pragma unroll
                    for (int o = 0; o < R; ++o) v = fma(cf.c[R + o], yv[o][e], v);
#pragma unroll
                    for (int o = -R; o <= R; ++o) v = fma(cf.c[3 * R + o], xval(o), v);
#pragma unroll
                    for (int o = 0; o < R; ++o) v = fma(cf.c[4 * R + 1 + o], yv[R + o][e], v);
#pragma unroll
                    for (int o = 1; o <= R; ++o) v = fma(cf.c[5 * R + o], ring[k - 1][i][R + o][e], v);
                    out[e] = (zdir || yd[i] || ((xd[i] >> e) & 1u)) ? g : v;
                }
                if (k == TD) {
                    if (zk >= z0 && zk < zend) {
                        const int gx = x0 - GA + pvx[i] * VEC;
                        const int gy = y0 - G + ppy[i];
                        T* o = dp + (int64_t)zk * dst.sz + (int64_t)gy * dst.sy + gx;
                        if (gx + VEC <= nx) {
                            VT q;
#pragma unroll
                            for (int e = 0; e < VEC; ++e) ((T*)&q)[e] = out[e];
                            __builtin_nontemporal_store(q, (VT*)o);
                        } else {
#pragma unroll
                            for (int e = 0; e < VEC; ++e)
                                if (gx + e < nx) __builtin_nontemporal_store(out[e], o + e);
                        }
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) nv[k][i][e] = out[e];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < TD; ++k)
#pragma unroll
            for (int i = 0; i < NPV; ++i)
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
#pragma unroll
                    for (int s = 0; s < RING - 1; ++s) ring[k][i][s][e] = ring[k][i][s + 1][e];
                    ring[k][i][RING - 1][e] = (k == 0) ? pre[i][e] : nv[k][i][e];
                }
#pragma unroll
        for (int k = 0; k < TD; ++k)
#pragma unroll
            for (int i = 0; i < NPV; ++i) {
                if (!used[i]) continue;
                VT q;
#pragma unroll
                for (int e = 0; e < VEC; ++e) ((T*)&q)[e] = ring[k][i][R][e];
                *(VT*)&lds[k][wb][ppy[i]][PAD + pvx[i] * VEC] = q;
            }
        if (j + 1 <= jlast_load) load_plane(j + 1);
        lds_barrier();
    }
}

template <typename T, int R, int TD, int BX, int BY, int NT>
hipError_t run_star3d_vtb(const SweepJob& j, int chunk, hipStream_t s) {
    TStarCoef<T, R> cf;
    const int r = j.radius;
    const int w = 2 * r + 1;
    auto dense = [&](int ox, int oy, int oz) { return (T)j.dense[(ox + r) + (oy + r) * w + (oz + r) * w * w]; };
    for (int o = -R; o < 0; ++o) cf.c[o + R] = dense(0, 0, o);
    for (int o = -R; o < 0; ++o) cf.c[2 * R + o] = dense(0, o, 0);
    for (int o = -R; o <= R; ++o) cf.c[3 * R + o] = dense(o, 0, 0);
    for (int o = 1; o <= R; ++o) cf.c[4 * R + o] = dense(0, o, 0);
    for (int o = 1; o <= R; ++o) cf.c[5 * R + o] = dense(0, 0, o);
    if (chunk <= 0) chunk = 64;
    const int tiles_x = (j.src.nx + BX - 1) / BX;
    const int tiles_y = (j.src.ny + BY - 1) / BY;
    const int tiles_z = (j.src.nz + chunk - 1) / chunk;
    const int64_t nb64 = (int64_t)tiles_x * tiles_y * tiles_z;
    if (nb64 > (1ll << 30)) return hipErrorInvalidConfiguration;
    const int nb = (int)nb64;
    const int nbp = padded_block_count(nb);
    hipLaunchKernelGGL((k_star3d_vtb<T, R, TD, BX, BY, NT>), dim3(nbp), dim3(NT), 0, s, j.src, j.dst, j.rule, cf,
                       chunk, tiles_x, tiles_y, nb, nbp);
    return hipGetLastError();
}

#define VTB(T, DT, R, TD, BX, BY, NT, CH)                                                                       \
    {"star3dvt_" #T "_r" #R "_t" #TD "_" #BX "x" #BY "_nt" #NT, FAM_STAR3D_VEC, 3, R, TD, DT, 0, BX, BY, NT, CH, \
     &run_star3d_vtb<T, R, TD, BX, BY, NT>}

const Variant kStar3dVtb[] = {
    VTB(float, LOPE_F32, 1, 2, 64, 16, 256, 128),
    VTB(float, LOPE_F32, 1, 2, 64, 32, 512, 128),
    VTB(float, LOPE_F32, 1, 3, 64, 16, 256, 128),
    VTB(float, LOPE_F32, 1, 3, 64, 32, 512, 128),
    VTB(float, LOPE_F32, 1, 4, 64, 16, 256, 128),
    VTB(float, LOPE_F32, 1, 4, 64, 32, 512, 128),
    VTB(float, LOPE_F32, 2, 2, 64, 16, 256, 128),
    VTB(double, LOPE_F64, 1, 2, 32, 16, 256, 32),
    VTB(double, LOPE_F64, 1, 3, 32, 16, 256, 32),
    VTB(double, LOPE_F64, 2, 2, 32, 16, 256, 32),
};

}  // namespace

int star3d_vtb_variants(const Variant** out) {
    *out = kStar3dVtb;
    return (int)(sizeof(kStar3dVtb) / sizeof(kStar3dVtb[0]));
}

}  // namespace lope
