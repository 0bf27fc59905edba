// 3D star stencils with temporal blocking, straight-line variant: the same
// z-march as k_star3d (register rings along z, each level's centre plane in
// LDS, TD sweeps per pass, level k computes plane j - k(R+1) at step j), with
// the per-step work free of divergent branches and register moves:
//
// * every thread computes every level at all of its positions; positions
//   whose value no valid output depends on (the outer cells of the widened
//   tile at high levels, the unused positions past the tile) compute
//   throw-away values.  The LDS planes carry a guard band of R rows on both
//   sides and one private slot per unused position, so every LDS access of
//   every position is in bounds; the boundary rule is a select;
// * the z loop is unrolled by the ring length 2R+1, so the ring slot holding
//   plane z-R+s is a compile-time register at every step (no rotation);
// * the launch bounds ask for the occupancy the LDS allows (two workgroups
//   per CU), which keeps the register allocation within that budget;
// * levels are computed from the deepest down, so each level's ring is
//   updated in place right after its last reader (the level above) ran;
// * global addresses are a per-plane base (wave-uniform) plus a 32-bit
//   in-plane byte offset (the caller checks that planes fit 31 bits);
// * on grids periodic in x and y no position holds g, and the blend is
//   compiled out (DXY = false);
// * with RES, the pass also merges max |u_TD - u_(TD-1)| over its outputs
//   (the change made by its last sweep, from values it holds anyway) into a
//   device double, for the convergence test.
//
// The per-point sum is c0*v0 followed by fmas in lexicographic offset order
// (z-R .. z-1, y-R .. y-1, x-R .. x+R, y+1 .. y+R, z+1 .. z+R), as in every
// other kernel, so all variants agree value for value.
#include <type_traits>

#include "lope_internal.h"

namespace lope {
namespace {

template <typename T, int R>
struct FlatCoef {
    T c[6 * R + 1];
};

template <typename T, int R, int TD, int BX, int BY, int NT>
struct FlatShape {
    static constexpr int G = R * TD;
    static constexpr int W = BX + 2 * G;
    static constexpr int H = BY + 2 * G;
    static constexpr int NPOS = W * H;
    static constexpr int NP = (NPOS + NT - 1) / NT;
    static constexpr int RING = 2 * R + 1;
    static constexpr int GUARD = R * W;                 // R rows before and after the tile
    static constexpr int PLANE = 2 * GUARD + NP * NT;   // one slot per (thread, position)
    // Workgroups per CU that the LDS (160 KiB) admits, at most 2, and the
    // waves per SIMD that this takes: the register budget the compiler must
    // meet so that LDS, not registers, sets the occupancy.
    static constexpr int LDS_BYTES = TD * 2 * PLANE * (int)sizeof(T);
    static constexpr int WG_PER_CU = (160 * 1024 / LDS_BYTES) >= 2 ? 2 : 1;
    static constexpr int WAVES_PER_EU = (WG_PER_CU * NT / 64 + 3) / 4;
};

// m ? v : g per lane as a bit blend (one VALU op per 32 bits): a select here
// would be turned into a branch around the loads that feed v.
__device__ __forceinline__ float blend(unsigned m, float v, float g) {
    return __uint_as_float((__float_as_uint(v) & m) | (__float_as_uint(g) & ~m));
}
__device__ __forceinline__ double blend(unsigned long long m, double v, double g) {
    const unsigned long long vb = (unsigned long long)__double_as_longlong(v);
    const unsigned long long gb = (unsigned long long)__double_as_longlong(g);
    return __longlong_as_double((long long)((vb & m) | (gb & ~m)));
}
template <typename T>
struct MaskOf {
    typedef unsigned type;
};
template <>
struct MaskOf<double> {
    typedef unsigned long long type;
};

// f(j + P, phase P) for P = 0 .. N-1 while j + P <= jend, each with a
// compile-time phase (the bound is wave-uniform).
template <int P, int N, typename F>
__device__ __forceinline__ void unroll_steps(int j, int jend, F& f) {
    if constexpr (P < N) {
        if (j + P > jend) return;
        f(j + P, std::integral_constant<int, P>{});
        unroll_steps<P + 1, N>(j, jend, f);
    }
}

// STG: 0 = TD sweeps of one stencil; 1, 2 = one two-stage step (TD = 2):
// level 1 applies cf, level 2 applies cf2 (plus alpha times the starting
// state when STG = 2).
template <typename T, int R, int TD, int BX, int BY, int NT, bool DXY, bool RES, int STG>
__global__ void __launch_bounds__(NT, (FlatShape<T, R, TD, BX, BY, NT>::WAVES_PER_EU))
k_star3d_flat(DevGrid src, DevGrid dst, DevRule rule, FlatCoef<T, R> cf, FlatCoef<T, R> cf2, T alpha, int chunk,
              int tiles_x, int tiles_y, int nblocks, int nblocks_padded, double* residual) {
    static_assert(STG == 0 || TD == 2, "a two-stage step is two levels");
    typedef FlatShape<T, R, TD, BX, BY, NT> S;
    constexpr int G = S::G, W = S::W, H = S::H, NPOS = S::NPOS, NP = S::NP, RING = S::RING;
    constexpr int GUARD = S::GUARD, PLANE = S::PLANE;

    __shared__ T lds[TD][2][PLANE];

    const int logical = xcd_logical_block(nblocks_padded);
    if (logical >= nblocks) return;
    const int tx = logical % tiles_x;
    const int rest = logical / tiles_x;
    const int ty = rest % tiles_y;
    const int tz = rest / tiles_y;

    const int nx = src.nx, ny = src.ny, nz = src.nz;
    const int x0 = tx * BX, y0 = ty * BY, z0 = tz * chunk;
    const int zend = min(z0 + chunk, nz);
    // z stays a run-time rule: its wave-uniform plane checks also keep the
    // scheduler from interleaving levels, which holds the register count down
    const bool perx = rule.per[0] != 0, pery = rule.per[1] != 0, perz = rule.per[2] != 0;
    const T g = (T)rule.g;
    const int tid = threadIdx.x;

    typedef typename MaskOf<T>::type M;
    unsigned soff[NP];   // in-plane byte offset of the (wrapped or clamped) source column
    unsigned doff[NP];   // in-plane byte offset of the output column
    M live[NP];          // all ones, or 0 where the position holds g (outside along a Dirichlet x/y axis);
                         // used only when DXY (some x or y axis is Dirichlet)
    bool keep[NP];       // an output position inside the interior
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const int p = tid + i * NT;
        const bool used = p < NPOS;
        const int px = p % W, py = p / W;
        const int gx = x0 - G + px, gy = y0 - G + py;
        const int l = min(min(px, W - 1 - px), min(py, H - 1 - py)) / R;
        const bool ox = gx < 0 || gx >= nx, oy = gy < 0 || gy >= ny;
        live[i] = ((!perx && ox) || (!pery && oy)) ? (M)0 : ~(M)0;
        const int wx = perx ? wrap_index(gx, nx) : min(max(gx, 0), nx - 1);
        const int wy = pery ? wrap_index(gy, ny) : min(max(gy, 0), ny - 1);
        soff[i] = used ? ((unsigned)wx + (unsigned)wy * (unsigned)src.sy) * (unsigned)sizeof(T) : 0u;
        keep[i] = used && l >= TD && !ox && !oy;
        doff[i] = keep[i] ? ((unsigned)gx + (unsigned)gy * (unsigned)dst.sy) * (unsigned)sizeof(T) : 0u;
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
        if (!perz && (j < 0 || j >= nz)) {
#pragma unroll
            for (int i = 0; i < NP; ++i) pre[i] = g;
            return;
        }
        const char* __restrict__ plane =
            (const char*)((const T*)src.origin + (int64_t)(perz ? wrap_index(j, nz) : j) * src.sz);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const T v = *(const T*)(plane + soff[i]);
            pre[i] = DXY ? blend(live[i], v, g) : v;
        }
    };

    const int jstart = z0 - G;
    const int jlast_load = zend - 1 + G;
    const int jend = zend - 1 + TD * (R + 1);

    // One march step at ring phase PH: ring slot (s + PH) % RING holds the
    // plane at logical position s (0 = oldest) of every level's window.
    double rmax = 0.0;   // RES: max |last sweep - the sweep before| over this thread's outputs
    // STG: the starting state at the point level 1 is computing, kept until
    // level 2 reaches the same plane R+1 steps later
    T dly[NP][RING];
    auto step = [&](int j, auto phase) {
        constexpr int PH = decltype(phase)::value;
        const int rb = (j & 1) ^ 1;
        const int wb = j & 1;
#pragma unroll
        for (int k = TD; k >= 1; --k) {
            const int zk = j - k * (R + 1);
            if (!perz && (zk < 0 || zk >= nz)) {
                // a Dirichlet plane outside the interior: g at every position
                // (never stored: the chunk lies inside the interior)
                if (k < TD) {
#pragma unroll
                    for (int i = 0; i < NP; ++i) ring[k][i][PH] = g;
                }
                continue;
            }
            const T* L = &lds[k - 1][rb][GUARD];
            char* out = (char*)((T*)dst.origin + (int64_t)zk * dst.sz);
            const bool zin = zk >= z0 && zk < zend;
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const int p = tid + i * NT;
                const T* rk = ring[k - 1][i];
                const FlatCoef<T, R>& c = (STG && k == 2) ? cf2 : cf;
                T v;
                if (STG == 2 && k == 2)   // alpha * u, then every tap as an fma
                    v = fma(c.c[0], rk[(0 + PH) % RING], alpha * dly[i][(PH + RING - (R + 1)) % RING]);
                else
                    v = c.c[0] * rk[(0 + PH) % RING];
                if (STG && k == 1) dly[i][PH] = rk[(R + PH) % RING];
#pragma unroll
                for (int s = 1; s < R; ++s) v = fma(c.c[s], rk[(s + PH) % RING], v);
#pragma unroll
                for (int o = -R; o < 0; ++o) v = fma(c.c[2 * R + o], L[p + o * W], v);
#pragma unroll
                for (int o = -R; o <= R; ++o)
                    v = fma(c.c[3 * R + o], o == 0 ? rk[(R + PH) % RING] : L[p + o], v);
#pragma unroll
                for (int o = 1; o <= R; ++o) v = fma(c.c[4 * R + o], L[p + o * W], v);
#pragma unroll
                for (int o = 1; o <= R; ++o) v = fma(c.c[5 * R + o], rk[(R + o + PH) % RING], v);
                if (DXY) v = blend(live[i], v, g);
                if (k == TD) {
                    if (keep[i] && zin) {
                        __builtin_nontemporal_store(v, (T*)(out + doff[i]));
                        // level TD-1 at this point is the state before the last sweep
                        if (RES) rmax = nan_max(rmax, fabs((double)v - (double)rk[(R + PH) % RING]));
                    }
                } else {
                    ring[k][i][PH] = v;   // level k's oldest plane is no longer read
                }
            }
        }
#pragma unroll
        for (int i = 0; i < NP; ++i) ring[0][i][PH] = pre[i];
        // publish every level's new centre plane (logical slot R after the shift)
#pragma unroll
        for (int k = 0; k < TD; ++k)
#pragma unroll
            for (int i = 0; i < NP; ++i) lds[k][wb][GUARD + tid + i * NT] = ring[k][i][(R + 1 + PH) % RING];
        if (j + 1 <= jlast_load) load_plane(j + 1);
        lds_barrier();
    };

    load_plane(jstart);
    for (int j = jstart; j <= jend; j += RING) unroll_steps<0, RING>(j, jend, step);
    if (RES) residual_merge(rmax, residual);
}

template <typename T, int R>
FlatCoef<T, R> flat_coef(const SweepJob& j) {
    FlatCoef<T, R> cf;
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
    return cf;
}

template <typename T, int R, int TD, int BX, int BY, int NT, int STG>
hipError_t launch_flat(const SweepJob& j, const FlatCoef<T, R>& cf, const FlatCoef<T, R>& cf2, T alpha, int chunk,
                       hipStream_t s) {
    if (chunk <= 0) chunk = 64;
    const int tiles_x = (j.src.nx + BX - 1) / BX;
    const int tiles_y = (j.src.ny + BY - 1) / BY;
    const int tiles_z = (j.src.nz + chunk - 1) / chunk;
    const int64_t nb64 = (int64_t)tiles_x * tiles_y * tiles_z;
    if (nb64 > (1ll << 30)) return hipErrorInvalidConfiguration;
    const int nb = (int)nb64;
    const int nbp = padded_block_count(nb);
    const bool dxy = !j.rule.per[0] || !j.rule.per[1];
#define LOPE_FLAT_LAUNCH(A, B)                                                                                     \
    hipLaunchKernelGGL((k_star3d_flat<T, R, TD, BX, BY, NT, A, B, STG>), dim3(nbp), dim3(NT), 0, s, j.src, j.dst, \
                       j.rule, cf, cf2, alpha, chunk, tiles_x, tiles_y, nb, nbp, j.residual)
    if (STG == 0 && j.residual) {
        if (dxy)
            LOPE_FLAT_LAUNCH(true, STG == 0);
        else
            LOPE_FLAT_LAUNCH(false, STG == 0);
    } else {
        if (dxy)
            LOPE_FLAT_LAUNCH(true, false);
        else
            LOPE_FLAT_LAUNCH(false, false);
    }
#undef LOPE_FLAT_LAUNCH
    return hipGetLastError();
}

template <typename T, int R, int TD, int BX, int BY, int NT>
hipError_t run_star3d_flat(const SweepJob& j, int chunk, hipStream_t s) {
    const FlatCoef<T, R> cf = flat_coef<T, R>(j);
    return launch_flat<T, R, TD, BX, BY, NT, 0>(j, cf, cf, (T)0, chunk, s);
}

// One two-stage step per pass (the two-level kernel with the second stencil
// and alpha at level 2).
template <typename T, int R, int TD, int BX, int BY, int NT>
hipError_t run_star3d_flat_stages(const StageJob& sj, int chunk, hipStream_t s) {
    if constexpr (TD != 2) {
        return hipErrorInvalidValue;
    } else {
        const FlatCoef<T, R> cf = flat_coef<T, R>(sj.s1), cf2 = flat_coef<T, R>(sj.s2);
        if (sj.alpha != 0.0) return launch_flat<T, R, TD, BX, BY, NT, 2>(sj.s1, cf, cf2, (T)sj.alpha, chunk, s);
        return launch_flat<T, R, TD, BX, BY, NT, 1>(sj.s1, cf, cf2, (T)0, chunk, s);
    }
}

#define FSTAR(T, DT, R, TD, BX, BY, NT, CH)                                                      \
    {"star3df_" #T "_r" #R "_t" #TD "_" #BX "x" #BY "_nt" #NT, FAM_STAR3D_FLAT, 3, R, TD, DT, 0, \
     BX, BY, NT, CH, &run_star3d_flat<T, R, TD, BX, BY, NT>, 1,                                  \
     (TD) == 2 ? &run_star3d_flat_stages<T, R, TD, BX, BY, NT> : nullptr}

const Variant kStar3dFlat[] = {
    FSTAR(float, LOPE_F32, 1, 3, 64, 32, 512, 128),
    FSTAR(float, LOPE_F32, 1, 3, 64, 32, 768, 128),
    FSTAR(float, LOPE_F32, 1, 3, 64, 32, 1024, 128),
    FSTAR(float, LOPE_F32, 1, 3, 128, 16, 512, 128),
    FSTAR(float, LOPE_F32, 1, 3, 64, 16, 256, 128),
    FSTAR(float, LOPE_F32, 1, 2, 64, 32, 512, 128),
    FSTAR(float, LOPE_F32, 1, 2, 64, 32, 1024, 128),
    FSTAR(float, LOPE_F32, 1, 4, 64, 32, 512, 256),
    FSTAR(float, LOPE_F32, 1, 4, 64, 32, 1024, 256),
    FSTAR(float, LOPE_F32, 1, 4, 64, 16, 256, 256),
    FSTAR(float, LOPE_F32, 4, 1, 64, 32, 512, 128),
    FSTAR(double, LOPE_F64, 1, 3, 32, 32, 256, 32),
    FSTAR(double, LOPE_F64, 1, 3, 32, 32, 512, 32),
    FSTAR(double, LOPE_F64, 1, 3, 64, 16, 512, 32),
    FSTAR(double, LOPE_F64, 1, 2, 32, 32, 256, 32),
    FSTAR(double, LOPE_F64, 1, 4, 32, 32, 512, 32),
};

}  // namespace

int star3d_flat_variants(const Variant** out) {
    *out = kStar3dFlat;
    return (int)(sizeof(kStar3dFlat) / sizeof(kStar3dFlat[0]));
}

}  // namespace lope
