// 3D star stencils, one sweep per pass, with 16-byte vector memory access.
//
// A workgroup marches a z-chunk of a BX x BY output tile.  Each thread owns
// VEC consecutive x positions (one 16-byte vector) on RPT rows of the core
// tile and keeps, for those points only, the last 2R+1 planes in registers
// (the z neighbours).  The centre plane of the tile plus its x/y halo
// (R rows above and below, R columns left and right; the star needs no
// corners) is published in LDS, double-buffered, one barrier per plane.
// Core planes are fetched R+1+PF planes ahead of the plane being computed
// and halos HPF planes ahead (PF, HPF = 1 or 2 alternating prefetch
// buffers), so the loads of the next steps are in flight while this one
// computes; the deeper prefetch costs registers, which the wider stencils
// can spare for the halo (one vector per thread) but not for the core.  The
// x halo is loaded as whole aligned vectors once at least half of each
// vector is used.  WPE (waves per SIMD asked of the register allocator;
// 1 = no request) holds the allocation to the occupancy the tile needs.
//
// The LDS row holds the core at a 16-byte aligned column (kLead) so the
// centre and y-neighbour rows are read as vectors.  Every point is summed as
// c0*v0 followed by fmas in lexicographic offset order (z-R .. z-1,
// y-R .. y-1, x-R .. x+R, y+1 .. y+R, z+1 .. z+R), identical to the other
// kernels.  The boundary rule is applied while loading; positions of a
// ragged tile beyond the interior hold rule values (wrapped or g).
//
// Requirements (checked by the caller): origin 16-byte aligned, y and z
// strides multiples of VEC elements.
#include "lope_internal.h"

namespace lope {
namespace {

template <typename T, int R>
struct VStarCoef {
    T c[6 * R + 1];
};

template <typename T>
struct Vec;
template <>
struct Vec<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int n = 4;
};
template <>
struct Vec<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int n = 2;
};

template <typename T, int R, int BX, int BY, int NT, int PF, int HPF, int WPE>
__global__ void __launch_bounds__(NT, WPE)
k_star3d_vec(DevGrid src, DevGrid dst, DevRule rule, VStarCoef<T, R> cf, int chunk, int tiles_x, int tiles_y,
             int nblocks, int nblocks_padded) {
    typedef typename Vec<T>::type VT;
    constexpr int VEC = Vec<T>::n;
    constexpr int TX = BX / VEC;            // threads across a core row
    constexpr int TYT = NT / TX;            // core rows per thread pass
    constexpr int RPT = BY / TYT;           // core rows per thread
    constexpr int kLead = 16 / sizeof(T) > R ? 16 / sizeof(T) : ((R + VEC - 1) / VEC) * VEC;
    constexpr int LW = kLead + BX + kLead;  // LDS row length (core at column kLead)
    constexpr int LH = BY + 2 * R;          // LDS rows (core at row R)
    constexpr int RING = 2 * R + 1;
    constexpr int NHROW = 2 * R * TX;       // halo row vectors (R rows above, R below)
    // x halo: whole aligned vectors (the kLead columns left and right of each
    // core row) once a vector holds at least half useful values, else the R
    // columns as scalars
    constexpr bool kVecCols = 2 * R >= VEC;
    constexpr int NCV = kLead / VEC;        // x-halo vectors per side per row
    constexpr int NHCOL = kVecCols ? 2 * NCV * BY : 2 * R * BY;
    constexpr int NHALO = NHROW + NHCOL;
    constexpr int HPT = (NHALO + NT - 1) / NT;   // halo items per thread
    static_assert(BX % VEC == 0 && NT % TX == 0 && BY % TYT == 0, "tile shape");
    static_assert((PF == 1 || PF == 2) && (HPF == 1 || HPF == 2), "the march is unrolled by two");

    __shared__ __attribute__((aligned(16))) T lds[2][LH][LW];

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
    const int tx = tid % TX, ty = tid / TX;
    const int cx = x0 + tx * VEC;                     // first x of this thread's vector
    const bool xfull = cx + VEC <= nx;                // the whole vector is interior
    // core rows of this thread
    int cy[RPT];
    bool yin[RPT];
    int64_t soff[RPT];                                // offset of (cx, wrapped row) in src
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        cy[k] = y0 + ty + k * TYT;
        yin[k] = cy[k] < ny;
        const int wy = yin[k] ? cy[k] : (pery ? wrap_index(cy[k], ny) : ny - 1);
        soff[k] = (int64_t)wy * src.sy;
    }
    // rule value of a single element at (gx, gy) in plane z (z already valid)
    auto elem = [&](int gx, int gy, int64_t zo) -> T {
        const bool ox = gx < 0 || gx >= nx, oy = gy < 0 || gy >= ny;
        if ((ox && !perx) || (oy && !pery)) return g;
        return sp[zo + (int64_t)wrap_index(gy, ny) * src.sy + wrap_index(gx, nx)];
    };
    auto load_core = [&](int j, T (&v)[RPT][VEC]) {
        const bool oz = j < 0 || j >= nz;
        if (oz && !perz) {
#pragma unroll
            for (int k = 0; k < RPT; ++k)
#pragma unroll
                for (int e = 0; e < VEC; ++e) v[k][e] = g;
            return;
        }
        const int64_t zo = (int64_t)(perz ? wrap_index(j, nz) : j) * src.sz;
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            if (xfull && (yin[k] || pery)) {
                const VT q = *(const VT*)(sp + zo + soff[k] + cx);
#pragma unroll
                for (int e = 0; e < VEC; ++e) v[k][e] = ((const T*)&q)[e];
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e) v[k][e] = elem(cx + e, cy[k], zo);
            }
        }
    };
    // halo items: vectors of the R rows above/below the core, scalars of the R
    // columns left/right
    auto load_halo = [&](int j, T (&hv)[HPT][VEC]) {
        const bool oz = j < 0 || j >= nz;
        const bool zd = oz && !perz;
        const int64_t zo = zd ? 0 : (int64_t)(perz ? wrap_index(j, nz) : j) * src.sz;
#pragma unroll
        for (int m = 0; m < HPT; ++m) {
            const int h = tid + m * NT;
            if (h >= NHALO) continue;
            if (zd) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) hv[m][e] = g;
                continue;
            }
            if (h < NHROW) {
                const int r = h / TX, hx = h % TX;
                const int gy = r < R ? y0 - R + r : y0 + BY + (r - R);
                const int gx = x0 + hx * VEC;
                const bool oy = gy < 0 || gy >= ny;
                if (gx + VEC <= nx && !(oy && !pery)) {
                    const int64_t o = zo + (int64_t)wrap_index(gy, ny) * src.sy + gx;
                    const VT q = *(const VT*)(sp + o);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) hv[m][e] = ((const T*)&q)[e];
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) hv[m][e] = elem(gx + e, gy, zo);
                }
            } else if constexpr (kVecCols) {
                const int c = h - NHROW;
                const int side = c / (NCV * BY), rem = c % (NCV * BY);
                const int cv = rem / BY, gy = y0 + rem % BY;
                const int gx = side == 0 ? x0 - kLead + cv * VEC : x0 + BX + cv * VEC;
                if (gx >= 0 && gx + VEC <= nx && (gy < ny || pery)) {
                    const int64_t o = zo + (int64_t)wrap_index(gy, ny) * src.sy + gx;
                    const VT q = *(const VT*)(sp + o);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) hv[m][e] = ((const T*)&q)[e];
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) hv[m][e] = elem(gx + e, gy, zo);
                }
            } else {
                const int c = h - NHROW;
                const int side = c / (R * BY), rem = c % (R * BY);
                const int col = rem / BY, row = rem % BY;
                const int gx = side == 0 ? x0 - R + col : x0 + BX + col;
                hv[m][0] = elem(gx, y0 + row, zo);
            }
        }
    };
    auto store_halo = [&](T (*L)[LW], const T (&hv)[HPT][VEC]) {
#pragma unroll
        for (int m = 0; m < HPT; ++m) {
            const int h = tid + m * NT;
            if (h >= NHALO) continue;
            if (h < NHROW) {
                const int r = h / TX, hx = h % TX;
                const int ly = r < R ? r : BY + r;
#pragma unroll
                for (int e = 0; e < VEC; ++e) L[ly][kLead + hx * VEC + e] = hv[m][e];
            } else if constexpr (kVecCols) {
                const int c = h - NHROW;
                const int side = c / (NCV * BY), rem = c % (NCV * BY);
                const int cv = rem / BY, row = rem % BY;
                const int lx = side == 0 ? cv * VEC : kLead + BX + cv * VEC;
#pragma unroll
                for (int e = 0; e < VEC; ++e) L[R + row][lx + e] = hv[m][e];
            } else {
                const int c = h - NHROW;
                const int side = c / (R * BY), rem = c % (R * BY);
                const int col = rem / BY, row = rem % BY;
                const int lx = side == 0 ? kLead - R + col : kLead + BX + col;
                L[R + row][lx] = hv[m][0];
            }
        }
    };

    T ring[RPT][RING][VEC];
    T pre[PF][RPT][VEC];
    T hal[HPF][HPT][VEC];
    // prologue: planes z0-R .. z0+R into the ring, centre plane z0 into LDS[0],
    // then the next PF core planes and HPF halos in flight
#pragma unroll
    for (int s = 0; s < RING; ++s) {
        T tmp[RPT][VEC];
        load_core(z0 - R + s, tmp);
#pragma unroll
        for (int k = 0; k < RPT; ++k)
#pragma unroll
            for (int e = 0; e < VEC; ++e) ring[k][s][e] = tmp[k][e];
    }
    load_halo(z0, hal[0]);
    store_halo(lds[0], hal[0]);
#pragma unroll
    for (int k = 0; k < RPT; ++k)
#pragma unroll
        for (int e = 0; e < VEC; ++e) lds[0][R + ty + k * TYT][kLead + tx * VEC + e] = ring[k][R][e];
#pragma unroll
    for (int p = 0; p < PF; ++p) load_core(z0 + R + 1 + p, pre[p]);
#pragma unroll
    for (int q = 0; q < HPF; ++q) load_halo(z0 + 1 + q, hal[q]);
    lds_barrier();

    // One march step: compute plane zc, shift in core plane zc+R+1 (held in
    // pre[U % PF]), publish plane zc+1 (its halo in hal[U % HPF]), then
    // refill those buffers with the planes PF and HPF steps ahead.  U is the
    // step's position in the two-step unrolled loop, so buffer indices are
    // compile-time constants.
    auto step = [&](int zc, auto U) {
        constexpr int u = decltype(U)::value;
        T (&cur)[RPT][VEC] = pre[u % PF];
        T (&hp)[HPT][VEC] = hal[u % HPF];
        constexpr int buf = u;
        T (*L)[LW] = lds[buf];
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int ly = R + ty + k * TYT;
            const int lx = kLead + tx * VEC;
            T out[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                T v = cf.c[0] * ring[k][0][e];
#pragma unroll
                for (int s = 1; s < R; ++s) v = fma(cf.c[s], ring[k][s][e], v);
#pragma unroll
                for (int o = -R; o < 0; ++o) v = fma(cf.c[2 * R + o], L[ly + o][lx + e], v);
#pragma unroll
                for (int o = -R; o <= R; ++o) v = fma(cf.c[3 * R + o], o == 0 ? ring[k][R][e] : L[ly][lx + e + o], v);
#pragma unroll
                for (int o = 1; o <= R; ++o) v = fma(cf.c[4 * R + o], L[ly + o][lx + e], v);
#pragma unroll
                for (int o = 1; o <= R; ++o) v = fma(cf.c[5 * R + o], ring[k][R + o][e], v);
                out[e] = v;
            }
            if (yin[k]) {
                T* o = dp + (int64_t)zc * dst.sz + (int64_t)cy[k] * dst.sy + cx;
                if (xfull) {
                    VT q;
#pragma unroll
                    for (int e = 0; e < VEC; ++e) ((T*)&q)[e] = out[e];
                    __builtin_nontemporal_store(q, (VT*)o);
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        if (cx + e < nx) __builtin_nontemporal_store(out[e], o + e);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < RPT; ++k)
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
#pragma unroll
                for (int s = 0; s < RING - 1; ++s) ring[k][s][e] = ring[k][s + 1][e];
                ring[k][RING - 1][e] = cur[k][e];
            }
        if (zc + 1 < zend) {
            T (*N)[LW] = lds[buf ^ 1];
            store_halo(N, hp);
#pragma unroll
            for (int k = 0; k < RPT; ++k)
#pragma unroll
                for (int e = 0; e < VEC; ++e) N[R + ty + k * TYT][kLead + tx * VEC + e] = ring[k][R][e];
            if (zc + PF < zend) load_core(zc + R + 1 + PF, cur);
            if (zc + 1 + HPF < zend) load_halo(zc + 1 + HPF, hp);
        }
        lds_barrier();
    };
    for (int zc = z0; zc < zend; zc += 2) {
        step(zc, std::integral_constant<int, 0>{});
        if (zc + 1 < zend) step(zc + 1, std::integral_constant<int, 1>{});
    }
}

template <typename T, int R, int BX, int BY, int NT, int PF, int HPF, int WPE>
hipError_t run_star3d_vec(const SweepJob& j, int chunk, hipStream_t s) {
    VStarCoef<T, R> cf;
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
    hipLaunchKernelGGL((k_star3d_vec<T, R, BX, BY, NT, PF, HPF, WPE>), dim3(nbp), dim3(NT), 0, s, j.src, j.dst, j.rule, cf, chunk,
                       tiles_x, tiles_y, nb, nbp);
    return hipGetLastError();
}

#define VSTARH(T, DT, R, BX, BY, NT, PF, HPF, NAME, CH, WPE)                                              \
    {"star3dv_" #T "_r" #R "_t1_" #BX "x" #BY "_nt" #NT "_pf" NAME, FAM_STAR3D_VEC, 3, R, 1, DT, 0, BX, BY, NT, \
     CH, &run_star3d_vec<T, R, BX, BY, NT, PF, HPF, WPE>}
#define VSTAR(T, DT, R, BX, BY, NT, PF, CH) VSTARH(T, DT, R, BX, BY, NT, PF, PF, #PF, CH, 1)

// PF: core planes fetched ahead (1 or 2 prefetch buffers); halos as many
// planes ahead unless the name says otherwise ("pf1h2": core 1, halo 2)
const Variant kStar3dVec[] = {
    VSTAR(float, LOPE_F32, 1, 128, 16, 256, 2, 32),
    VSTAR(float, LOPE_F32, 1, 128, 32, 512, 2, 32),
    VSTAR(float, LOPE_F32, 1, 64, 32, 256, 2, 64),
    VSTAR(float, LOPE_F32, 1, 64, 16, 256, 2, 64),
    VSTAR(float, LOPE_F32, 1, 128, 16, 256, 1, 64),
    VSTAR(float, LOPE_F32, 1, 128, 32, 512, 1, 32),
    VSTAR(float, LOPE_F32, 1, 256, 16, 512, 2, 32),
    VSTAR(float, LOPE_F32, 1, 256, 32, 1024, 1, 64),
    VSTARH(float, LOPE_F32, 1, 256, 32, 1024, 1, 2, "1h2", 64, 1),
    VSTARH(float, LOPE_F32, 1, 128, 32, 512, 1, 2, "1h2", 64, 1),
    VSTAR(float, LOPE_F32, 2, 64, 32, 256, 1, 64),
    VSTAR(float, LOPE_F32, 3, 64, 32, 256, 1, 64),
    VSTARH(float, LOPE_F32, 4, 64, 64, 1024, 1, 2, "1h2", 128, 4),
    VSTARH(float, LOPE_F32, 4, 128, 32, 1024, 1, 2, "1h2", 128, 4),
    VSTARH(float, LOPE_F32, 4, 64, 32, 512, 1, 2, "1h2", 128, 4),
    VSTARH(float, LOPE_F32, 4, 64, 16, 256, 1, 2, "1h2", 128, 4),
    VSTAR(float, LOPE_F32, 4, 64, 16, 256, 1, 128),
    VSTAR(double, LOPE_F64, 1, 64, 16, 256, 2, 32),
    VSTAR(double, LOPE_F64, 1, 64, 16, 256, 1, 32),
    VSTAR(double, LOPE_F64, 1, 32, 32, 256, 1, 32),
    VSTAR(double, LOPE_F64, 2, 32, 32, 256, 1, 64),
    VSTAR(double, LOPE_F64, 3, 32, 32, 256, 1, 64),
    VSTAR(double, LOPE_F64, 4, 32, 32, 256, 1, 64),
};

}  // namespace

int star3d_vec_variants(const Variant** out) {
    *out = kStar3dVec;
    return (int)(sizeof(kStar3dVec) / sizeof(kStar3dVec[0]));
}

}  // namespace lope
