// 3D star stencils (radius R, 6R+1 taps): z-marching workgroups with
// register rings along z, the centre plane staged in LDS for the x/y
// neighbours, and TD sweeps fused per pass (temporal blocking).
//
// A workgroup owns an output tile of BX x BY columns and a chunk of z planes.
// It loads the input tile widened by G = R*TD cells on each side (the halo
// that TD sweeps need) one z plane at a time.  Level k (k = 0..TD) is the
// state after k sweeps; level k is valid on the tile shrunk by R*k cells.
// Every thread owns a fixed set of (x, y) positions of the widened tile at
// all levels, so the z neighbours of a position are always in that thread's
// registers: ring[k][i][0..2R] holds the last 2R+1 planes of level k at
// position i.  The x/y neighbours come from the centre plane of each level,
// published in LDS (two buffers, one barrier per plane).
//
// Pipeline: at march step j, level 0 receives plane j and level k computes
// plane j - k(R+1) from the level k-1 planes published at step j-1.  Level TD
// is written to the destination.  The per-point sum is c0*v0 followed by a
// chain of fmas in lexicographic offset order (z-R .. z-1, y-R .. y-1,
// x-R .. x+R, y+1 .. y+R, z+1 .. z+R), identical at every level, so a fused
// pass gives exactly the values of TD separate sweeps.
//
// Boundary rule applied while loading: along a Dirichlet axis a cell outside
// the interior is g at every level; along a periodic axis the cell is loaded
// from the wrapped index and evolves like the cell it copies.
#include "lope_internal.h"

namespace lope {
namespace {

template <typename T, int R>
struct StarCoef {
    T c[6 * R + 1];
};

template <typename T, int R, int TD, int BX, int BY, int NT>
__global__ void __launch_bounds__(NT)
k_star3d(DevGrid src, DevGrid dst, DevRule rule, StarCoef<T, R> cf, int chunk, int tiles_x,
         int tiles_y, int nblocks, int nblocks_padded) {
    constexpr int G = R * TD;
    constexpr int W = BX + 2 * G;
    constexpr int H = BY + 2 * G;
    constexpr int NPOS = W * H;
    constexpr int NP = (NPOS + NT - 1) / NT;
    constexpr int RING = 2 * R + 1;

    __shared__ T lds[TD][2][NPOS];

    const int logical = xcd_logical_block(nblocks_padded);
    if (logical >= nblocks) return;
    const int tx = logical % tiles_x;
    const int rest = logical / tiles_x;
    const int ty = rest % tiles_y;
    const int tz = rest / tiles_y;

    const int nx = src.nx, ny = src.ny, nz = src.nz;
    const int x0 = tx * BX, y0 = ty * BY, z0 = tz * chunk;
    const int zend = min(z0 + chunk, nz);
    const bool perx = rule.per[0] != 0, pery = rule.per[1] != 0, perz = rule.per[2] != 0;
    const T g = (T)rule.g;
    const T* __restrict__ sp = (const T*)src.origin;
    T* __restrict__ dp = (T*)dst.origin;
    const int tid = threadIdx.x;

    int64_t soff[NP];   // offset of the (wrapped) column in src
    int64_t doff[NP];   // offset of the column in dst
    int lev[NP];        // highest level the position belongs to, -1 if unused
    bool dxy[NP];       // outside the interior along a Dirichlet x or y axis
    bool keep[NP];      // an output position inside the interior
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const int p = tid + i * NT;
        const int px = p % W, py = p / W;
        const int gx = x0 - G + px, gy = y0 - G + py;
        const bool used = p < NPOS;
        const int l = min(min(px, W - 1 - px), min(py, H - 1 - py)) / R;
        lev[i] = used ? min(l, TD) : -1;
        const bool ox = gx < 0 || gx >= nx, oy = gy < 0 || gy >= ny;
        dxy[i] = (!perx && ox) || (!pery && oy);
        const int wx = perx ? wrap_index(gx, nx) : min(max(gx, 0), nx - 1);
        const int wy = pery ? wrap_index(gy, ny) : min(max(gy, 0), ny - 1);
        soff[i] = (int64_t)wx + (int64_t)wy * src.sy;
        doff[i] = (int64_t)gx + (int64_t)gy * dst.sy;
        keep[i] = used && l >= TD && !ox && !oy;
    }

    T ring[TD][NP][RING];
    T pre[NP];
#pragma unroll
    for (int k = 0; k < TD; ++k)
#pragma unroll
        for (int i = 0; i < NP; ++i)
#pragma unroll
            for (int s = 0; s < RING; ++s) ring[k][i][s] = (T)0;

    auto load_plane = [&](int j) {
        const bool oz = j < 0 || j >= nz;
        if (!perz && oz) {
#pragma unroll
            for (int i = 0; i < NP; ++i) pre[i] = g;
            return;
        }
        const int64_t zo = (int64_t)(perz ? wrap_index(j, nz) : j) * src.sz;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            if (lev[i] < 0 || dxy[i]) pre[i] = g;
            else pre[i] = sp[soff[i] + zo];
        }
    };

    const int jstart = z0 - G;
    const int jlast_load = zend - 1 + G;
    const int jend = zend - 1 + TD * (R + 1);
    load_plane(jstart);

    for (int j = jstart; j <= jend; ++j) {
        const int rb = (j & 1) ^ 1;
        const int wb = j & 1;
        T nv[TD][NP];
#pragma unroll
        for (int k = 1; k <= TD; ++k) {
            const int zk = j - k * (R + 1);
            const bool zd = !perz && (zk < 0 || zk >= nz);
            const T* L = lds[k - 1][rb];
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                if (lev[i] < k) continue;
                const int p = tid + i * NT;
                T v;
                if (zd || dxy[i]) {
                    v = g;
                } else {
                    v = cf.c[0] * ring[k - 1][i][0];
#pragma unroll
                    for (int s = 1; s < R; ++s) v = fma(cf.c[s], ring[k - 1][i][s], v);
#pragma unroll
                    for (int o = -R; o < 0; ++o) v = fma(cf.c[2 * R + o], L[p + o * W], v);
#pragma unroll
                    for (int o = -R; o <= R; ++o)
                        v = fma(cf.c[3 * R + o], o == 0 ? ring[k - 1][i][R] : L[p + o], v);
#pragma unroll
                    for (int o = 1; o <= R; ++o) v = fma(cf.c[4 * R + o], L[p + o * W], v);
#pragma unroll
                    for (int o = 1; o <= R; ++o) v = fma(cf.c[5 * R + o], ring[k - 1][i][R + o], v);
                }
                if (k == TD) {
                    if (keep[i] && zk >= z0 && zk < zend)
                        __builtin_nontemporal_store(v, dp + doff[i] + (int64_t)zk * dst.sz);
                } else {
                    nv[k][i] = v;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < TD; ++k)
#pragma unroll
            for (int i = 0; i < NP; ++i) {
#pragma unroll
                for (int s = 0; s < RING - 1; ++s) ring[k][i][s] = ring[k][i][s + 1];
                ring[k][i][RING - 1] = (k == 0) ? pre[i] : nv[k][i];
            }
#pragma unroll
        for (int k = 0; k < TD; ++k)
#pragma unroll
            for (int i = 0; i < NP; ++i)
                if (lev[i] >= k) lds[k][wb][tid + i * NT] = ring[k][i][R];
        if (j + 1 <= jlast_load) load_plane(j + 1);
        lds_barrier();
    }
}

template <typename T, int R, int TD, int BX, int BY, int NT>
hipError_t run_star3d(const SweepJob& j, int chunk, hipStream_t s) {
    StarCoef<T, R> cf;
    const int r = j.radius;
    const int w = 2 * r + 1;
    auto dense = [&](int ox, int oy, int oz) {
        return (T)j.dense[(ox + r) + (oy + r) * w + (oz + r) * w * w];
    };
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
    hipLaunchKernelGGL((k_star3d<T, R, TD, BX, BY, NT>), dim3(nbp), dim3(NT), 0, s, j.src, j.dst,
                       j.rule, cf, chunk, tiles_x, tiles_y, nb, nbp);
    return hipGetLastError();
}

#define STAR3D(T, DT, R, TD, BX, BY, NT, CH)                                              \
    {"star3d_" #T "_r" #R "_t" #TD "_" #BX "x" #BY "_nt" #NT, FAM_STAR3D, 3, R, TD, DT, 0, \
     BX, BY, NT, CH, &run_star3d<T, R, TD, BX, BY, NT>}

// One sweep per pass for every radius: the scalar march the vector kernels
// fall back to on grids whose origins or strides are not 16-byte multiples.
// (Fused passes run on the straight-line and wave-brick families.)
const Variant kStar3d[] = {
    STAR3D(float, LOPE_F32, 1, 1, 64, 32, 256, 64),
    STAR3D(float, LOPE_F32, 1, 1, 128, 16, 256, 64),
    STAR3D(float, LOPE_F32, 2, 1, 64, 32, 256, 64),
    STAR3D(float, LOPE_F32, 3, 1, 64, 32, 256, 64),
    STAR3D(float, LOPE_F32, 4, 1, 64, 32, 256, 64),
    STAR3D(double, LOPE_F64, 1, 1, 64, 32, 256, 64),
    STAR3D(double, LOPE_F64, 2, 1, 64, 32, 256, 64),
    STAR3D(double, LOPE_F64, 3, 1, 64, 32, 256, 64),
    STAR3D(double, LOPE_F64, 4, 1, 64, 32, 256, 64),
};

}  // namespace

int star3d_variants(const Variant** out) {
    *out = kStar3d;
    return (int)(sizeof(kStar3d) / sizeof(kStar3d[0]));
}

}  // namespace lope
