// Variable-coefficient diffusion on a periodic 3D grid, one wavefront per
// brick: the forward step, the one-step reverse and two reverse steps fused.
//
//   forward:  u'_x = u_x + dt * sum_q K_q (u_q - u_x),   K_q = (kappa_x + kappa_q) / 2
//   reverse:  lam_x = lam'_x + dt * sum_q K_q (lam'_q - lam'_x)
//             gk_x += dt/2 * sum_q (u_q - u_x) (lam'_x - lam'_q)
// with q over the six face neighbours in the order x-, x+, y-, y+, z-, z+.
//
// A wave owns 64 consecutive x columns (one per lane, all 64 are outputs) by
// P rows and marches a z-chunk.  Each lane keeps its column's P + 2 rows of
// the current plane in registers (the y neighbours are the rows above and
// below).  The x neighbours come from lanes l-1 and l+1 by DPP lane shifts;
// the two columns just outside the wave (x0 - 1 for lane 0, x0 + 64 for lane
// 63) arrive in one extra load per plane and array that packs them into
// lanes, laid out so that one DPP row rotation brings a row's two outside
// values to lanes 0 and 63, where the shifts keep them.  Every index is
// wrapped (the grids are periodic), so lanes past a ragged x end hold
// wrapped columns that are never stored.
//
// The z direction is the march: when plane j arrives its in-plane terms
// (x-, x+, y-, y+) start its sums; then the face between planes j-1 and j is
// evaluated once and added to both sides (plane j's z- term and plane j-1's
// z+ term are the same products with opposite signs, exactly), which
// completes plane j-1.  Per point the terms are therefore summed in the
// order x-, x+, y-, y+, z-, z+ with one fma each, the same chain as the
// one-thread-per-point LDS kernels.
//
// Loads and stores go through a buffer resource per plane: the plane base in
// scalar registers, the column offset in one VGPR, the row offset as the
// scalar offset (the caller checks plane sizes below 2^31 bytes).
#include "lope_internal.h"

namespace lope {
namespace {

typedef __amdgpu_buffer_rsrc_t Rsrc;

__device__ __forceinline__ Rsrc plane_rsrc(const void* base, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

// Raw-bit loads and stores through a plane's buffer resource.
// AUX: the cache-policy bits of the access (0: default; 2: streaming).
template <typename T, int AUX = 0>
__device__ __forceinline__ T bload(Rsrc r, unsigned voff, int soff) {
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, soff, AUX));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, soff, AUX));
}
template <int AUX = 0>
__device__ __forceinline__ void bstore(float v, Rsrc r, unsigned voff, int soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, soff, AUX);
}
template <int AUX = 0>
__device__ __forceinline__ void bstore(double v, Rsrc r, unsigned voff, int soff) {
    typedef decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)) B64;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(B64, v), r, (int)voff, soff, AUX);
}
// f(integral_constant<S>) ... f(integral_constant<E-1>), unrolled at compile time
template <int S, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (S < E) {
        f(std::integral_constant<int, S>{});
        static_for<S + 1, E>(f);
    }
}

constexpr int kStreamStore = 2;   // cache-policy bits of a streaming store

// DPP lane shifts over the whole wave (bound_ctrl off: a lane whose source
// lies past the wave's end keeps `old`): from_left gives lane l the value of
// lane l-1 (lane 0: old), from_right the value of lane l+1 (lane 63: old).
constexpr int kWaveShr1 = 0x138, kWaveShl1 = 0x130;
template <int CTRL>
__device__ __forceinline__ float lane_shift(float v, float old) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old), __builtin_bit_cast(int, v),
                                                                 CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v, double old) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned long long o = __builtin_bit_cast(unsigned long long, old);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)o, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
    const unsigned hi =
        (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)(o >> 32), (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
// Rotation within every row of 16 lanes: lane i of a row receives lane
// (i + a) mod 16 of the same row (a = 0..15; DPP row_ror by 16 - a).
template <int A>
__device__ __forceinline__ int row_rotate_bits(int v) {
    if constexpr (A % 16 == 0)
        return v;
    else
        return __builtin_amdgcn_update_dpp(v, v, 0x120 + (16 - A % 16), 0xf, 0xf, false);
}
template <int A>
__device__ __forceinline__ float row_rotate(float v) {
    return __builtin_bit_cast(float, row_rotate_bits<A>(__builtin_bit_cast(int, v)));
}
template <int A>
__device__ __forceinline__ double row_rotate(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)row_rotate_bits<A>((int)(unsigned)b);
    const unsigned hi = (unsigned)row_rotate_bits<A>((int)(unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Where a wave's brick sits and how this lane addresses one array.
struct Brick {
    int x0, y0, z0, zend;
};

// W: output columns per wave (64, or 62 for the fused pair).
__device__ __forceinline__ bool brick_of(const DevGrid& g, int P, int chunk, int strips, int segs, int nwaves,
                                         int nbp, int nw_per_block, Brick& b, int W = 64) {
    const int wave = xcd_logical_block(nbp) * nw_per_block + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (wave >= nwaves) return false;
    const int tx = wave % strips, rest = wave / strips;
    b.x0 = tx * W;
    b.y0 = (rest % segs) * P;
    b.z0 = (rest / segs) * chunk;
    b.zend = min(b.z0 + chunk, g.nz);
    return true;
}

// One array's addressing: lane l holds column x_first + l and row r is
// y_first + r (both wrapped); the outside columns x_first - 1 and
// x_first + 64 of rows 1 .. n_edge (at most 16) are packed into one load:
// lane i < 16 holds the left one of row i + 1, lane 48 + ((i + 15) mod 16)
// the right one, so that rotating the rows of lanes by r - 1 (x_neighbours)
// brings row r's left outside value to lane 0 and its right one to lane 63
// in one DPP move.  Column byte offset of this lane, byte offset of its
// outside column, wave-uniform row byte offsets, plane bytes.
template <typename T, int NR>
struct Cols {
    const char* base;
    int64_t pbytes;
    unsigned xo, eo;
    int row[NR];
    __device__ __forceinline__ void init(const DevGrid& g, int x_first, int y_first, int n_edge) {
        const int lane = threadIdx.x & 63;
        base = (const char*)g.origin;
        pbytes = g.sz * (int64_t)sizeof(T);
        xo = (unsigned)wrap_index(x_first + lane, g.nx) * (unsigned)sizeof(T);
        const bool right = lane >= 48;
        const int i = right ? (lane - 48 + 1) & 15 : lane & 15;
        const int ecol = wrap_index(right ? x_first + 64 : x_first - 1, g.nx);
        const int erow = wrap_index(y_first + 1 + (i < n_edge ? i : 0), g.ny);
        eo = ((unsigned)erow * (unsigned)g.sy + (unsigned)ecol) * (unsigned)sizeof(T);
#pragma unroll
        for (int r = 0; r < NR; ++r) row[r] = (int)((unsigned)wrap_index(y_first + r, g.ny) * (unsigned)g.sy * (unsigned)sizeof(T));
    }
    // rows 0 .. NR-1 of plane q (wrapped) into v
    __device__ __forceinline__ void load_rows(int q, int nz, T (&v)[NR]) const {
        const Rsrc rs = plane_rsrc(base + (int64_t)wrap_index(q, nz) * pbytes, pbytes);
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = bload<T>(rs, xo, row[r]);
    }
    // rows 0 .. NR-1 of plane q (wrapped) into v, the outside columns into e
    template <int AUX = 0>
    __device__ __forceinline__ void load(int q, int nz, T (&v)[NR], T& e) const {
        const Rsrc rs = plane_rsrc(base + (int64_t)wrap_index(q, nz) * pbytes, pbytes);
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = bload<T, AUX>(rs, xo, row[r]);
        e = bload<T, AUX>(rs, eo, 0);
    }
};

// x- and x+ neighbours of row R (1..16) of a plane held as (v, e)
template <int R, typename T, int NR>
__device__ __forceinline__ void x_neighbours(const T (&v)[NR], T e, T& left, T& right) {
    static_assert(R >= 1 && R <= 16, "outside columns of rows 1..16");
    const T x = row_rotate<R - 1>(e);   // lane 0: row R's left outside value; lane 63: its right one
    left = lane_shift<kWaveShr1>(v[R], x);
    right = lane_shift<kWaveShl1>(v[R], x);
}

// PF: planes loaded ahead of the one being computed (1 or 2); LA / SA: cache
// policy of the loads / stores.
template <typename T, int P, int NW, int PF = 1, int LA = 0, int SA = 0>
__global__ void __launch_bounds__(NW * 64)
k_varw_forward(DevGrid src, DevGrid dst, DevGrid kap, T dt, int chunk, int strips, int segs, int nwaves, int nbp) {
    constexpr int NR = P + 2, NB = PF + 1;
    Brick b;
    if (!brick_of(src, P, chunk, strips, segs, nwaves, nbp, NW, b)) return;
    Cols<T, NR> cu, ck;
    cu.init(src, b.x0, b.y0 - 1, P);
    ck.init(kap, b.x0, b.y0 - 1, P);
    const int lane = threadIdx.x & 63;
    const int nz = src.nz, ny = src.ny;
    const int64_t dpb = dst.sz * (int64_t)sizeof(T);
    const bool xin = b.x0 + lane < src.nx;   // lanes past a ragged x end store nothing
    const unsigned so = (unsigned)(b.x0 + lane) * (unsigned)sizeof(T);
    const T half = (T)0.5;

    T u[NB][NR], k[NB][NR], eu[NB], ek[NB];   // the current plane and PF planes in flight
    T pu[P], pk[P], acc[P];                   // plane j-1: centre values and its partial sums
    const int jstart = b.z0 - 1, jend = b.zend;
    static_for<0, PF>([&](auto q) __attribute__((always_inline)) {
        constexpr int Q = decltype(q)::value;
        if (jstart + Q <= jend) {
            cu.template load<LA>(jstart + Q, nz, u[Q], eu[Q]);
            ck.template load<LA>(jstart + Q, nz, k[Q], ek[Q]);
        }
    });

    // march step j with plane j in buffer C
    auto step = [&](int j, auto cur_c) __attribute__((always_inline)) {
        constexpr int C = decltype(cur_c)::value, N = (C + PF) % NB;
        if (j + PF <= jend) {
            cu.template load<LA>(j + PF, nz, u[N], eu[N]);
            ck.template load<LA>(j + PF, nz, k[N], ek[N]);
        }
        const T(&U)[NR] = u[C];
        const T(&K)[NR] = k[C];
        T a[P];
        const bool own = j >= b.z0 && j < b.zend;   // plane j is one of the brick's outputs
        if (own) {   // its in-plane terms
            static_for<1, P + 1>([&](auto rc) __attribute__((always_inline)) {
                constexpr int r = decltype(rc)::value;
                const T uc = U[r], kc = K[r];
                T ul, ur, kl, kr;
                x_neighbours<r>(U, eu[C], ul, ur);
                x_neighbours<r>(K, ek[C], kl, kr);
                T s = (T)0;
                s = fma(half * (kc + kl), ul - uc, s);
                s = fma(half * (kc + kr), ur - uc, s);
                s = fma(half * (kc + K[r - 1]), U[r - 1] - uc, s);
                s = fma(half * (kc + K[r + 1]), U[r + 1] - uc, s);
                a[r - 1] = s;
            });
        }
        if (j > jstart) {
            // the face between planes j-1 and j: plane j's z- term, and plane
            // j-1's z+ term, which completes it
            const bool done = j - 1 >= b.z0;
            const Rsrc rd = plane_rsrc((const char*)dst.origin + (int64_t)(j - 1) * dpb, dpb);
#pragma unroll
            for (int r = 0; r < P; ++r) {
                const T w = half * (pk[r] + K[r + 1]);
                const T d = U[r + 1] - pu[r];
                const int y = b.y0 + r;
                if (done && y < ny && xin)
                    bstore<SA>(fma(dt, fma(w, d, acc[r]), pu[r]), rd, so,
                               (int)((unsigned)y * (unsigned)dst.sy * (unsigned)sizeof(T)));
                if (own) a[r] = fma(w, -d, a[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < P; ++r) {
            pu[r] = U[r + 1];
            pk[r] = K[r + 1];
            acc[r] = own ? a[r] : (T)0;
        }
    };
    int j = jstart;
    for (; j + NB - 1 <= jend; j += NB)
        static_for<0, NB>([&](auto c) __attribute__((always_inline)) { step(j + decltype(c)::value, c); });
    static_for<0, NB - 1>([&](auto c) __attribute__((always_inline)) {
        if (j + decltype(c)::value <= jend) step(j + decltype(c)::value, c);
    });
}

template <typename T, typename TG, int P, int NW, int PF = 1, int SA = 0>
__global__ void __launch_bounds__(NW * 64)
k_varw_adjoint(DevGrid lnext, DevGrid lam, DevGrid ug, DevGrid kap, DevGrid gk, T dt, int chunk, int strips, int segs,
               int nwaves, int nbp) {
    constexpr int NR = P + 2, NB = PF + 1;
    Brick b;
    if (!brick_of(lnext, P, chunk, strips, segs, nwaves, nbp, NW, b)) return;
    Cols<T, NR> cl, cu, ck;
    cl.init(lnext, b.x0, b.y0 - 1, P);
    cu.init(ug, b.x0, b.y0 - 1, P);
    ck.init(kap, b.x0, b.y0 - 1, P);
    const int lane = threadIdx.x & 63;
    const int nz = lnext.nz, ny = lnext.ny;
    const bool xin = b.x0 + lane < lnext.nx;   // lanes past a ragged x end store nothing
    const unsigned so = (unsigned)(b.x0 + lane) * (unsigned)sizeof(T);
    const unsigned sg = (unsigned)(b.x0 + lane) * (unsigned)sizeof(TG);
    const int64_t lpb = lam.sz * (int64_t)sizeof(T), gpb = gk.sz * (int64_t)sizeof(TG);
    const T half = (T)0.5, hdt = (T)0.5 * dt;

    T l[NB][NR], u[NB][NR], k[NB][NR], el[NB], eu[NB], ek[NB];
    T pl[P], pu[P], pk[P], al[P], ag[P];
    TG gold[P];   // kappa gradient of plane j-1, read one step ahead
    const int jstart = b.z0 - 1, jend = b.zend;
    static_for<0, PF>([&](auto q) __attribute__((always_inline)) {
        constexpr int Q = decltype(q)::value;
        if (jstart + Q <= jend) {
            cl.load(jstart + Q, nz, l[Q], el[Q]);
            cu.load(jstart + Q, nz, u[Q], eu[Q]);
            ck.load(jstart + Q, nz, k[Q], ek[Q]);
        }
    });
#pragma unroll
    for (int r = 0; r < P; ++r) gold[r] = (TG)0;

    auto step = [&](int j, auto cur_c) __attribute__((always_inline)) {
        constexpr int C = decltype(cur_c)::value, N = (C + PF) % NB;
        if (j + PF <= jend) {
            cl.load(j + PF, nz, l[N], el[N]);
            cu.load(j + PF, nz, u[N], eu[N]);
            ck.load(j + PF, nz, k[N], ek[N]);
        }
        const T(&L)[NR] = l[C];
        const T(&U)[NR] = u[C];
        const T(&K)[NR] = k[C];
        T a[P], g[P];
        TG gnew[P];
        const bool own = j >= b.z0 && j < b.zend;   // plane j is one of the brick's outputs
        if (own) {
            // its kappa gradient (read now, updated when the plane completes)
            // and its in-plane terms
            const Rsrc rgj = plane_rsrc((const char*)gk.origin + (int64_t)j * gpb, gpb);
            static_for<1, P + 1>([&](auto rc) __attribute__((always_inline)) {
                constexpr int r = decltype(rc)::value;
                const int y = b.y0 + r - 1;
                gnew[r - 1] = y < ny && xin ? bload<TG>(rgj, sg, (int)((unsigned)y * (unsigned)gk.sy * (unsigned)sizeof(TG))) : (TG)0;
                const T lc = L[r], uc = U[r], kc = K[r];
                T ll, lr, ul, ur, kl, kr;
                x_neighbours<r>(L, el[C], ll, lr);
                x_neighbours<r>(U, eu[C], ul, ur);
                x_neighbours<r>(K, ek[C], kl, kr);
                T s = (T)0, t = (T)0;
                s = fma(half * (kc + kl), ll - lc, s);
                t = fma(ul - uc, lc - ll, t);
                s = fma(half * (kc + kr), lr - lc, s);
                t = fma(ur - uc, lc - lr, t);
                s = fma(half * (kc + K[r - 1]), L[r - 1] - lc, s);
                t = fma(U[r - 1] - uc, lc - L[r - 1], t);
                s = fma(half * (kc + K[r + 1]), L[r + 1] - lc, s);
                t = fma(U[r + 1] - uc, lc - L[r + 1], t);
                a[r - 1] = s;
                g[r - 1] = t;
            });
        }
        if (j > jstart) {
            // the face between planes j-1 and j (both sides' terms are the same
            // products with opposite signs); plane j-1 completes
            const bool done = j - 1 >= b.z0;
            const Rsrc rl = plane_rsrc((const char*)lam.origin + (int64_t)(j - 1) * lpb, lpb);
            const Rsrc rg = plane_rsrc((const char*)gk.origin + (int64_t)(j - 1) * gpb, gpb);
#pragma unroll
            for (int r = 0; r < P; ++r) {
                const T w = half * (pk[r] + K[r + 1]);
                const T dl = L[r + 1] - pl[r];   // lam'_j - lam'_{j-1}
                const T du = U[r + 1] - pu[r];   // u_j - u_{j-1}
                const int y = b.y0 + r;
                if (done && y < ny && xin) {
                    bstore<SA>(fma(dt, fma(w, dl, al[r]), pl[r]), rl, so,
                               (int)((unsigned)y * (unsigned)lam.sy * (unsigned)sizeof(T)));
                    bstore<SA>(gold[r] + (TG)(hdt * fma(du, -dl, ag[r])), rg, sg,
                               (int)((unsigned)y * (unsigned)gk.sy * (unsigned)sizeof(TG)));
                }
                if (own) {
                    a[r] = fma(w, -dl, a[r]);
                    g[r] = fma(-du, dl, g[r]);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < P; ++r) {
            pl[r] = L[r + 1];
            pu[r] = U[r + 1];
            pk[r] = K[r + 1];
            al[r] = own ? a[r] : (T)0;
            ag[r] = own ? g[r] : (T)0;
            gold[r] = own ? gnew[r] : (TG)0;
        }
    };
    int j = jstart;
    for (; j + NB - 1 <= jend; j += NB)
        static_for<0, NB>([&](auto c) __attribute__((always_inline)) { step(j + decltype(c)::value, c); });
    static_for<0, NB - 1>([&](auto c) __attribute__((always_inline)) {
        if (j + decltype(c)::value <= jend) step(j + decltype(c)::value, c);
    });
}

// Two reverse steps in one pass: from lam'' = lam_{t+1}, u_t, u_{t-1} and
// kappa, the first level forms lam_t = A lam'' and G(u_t, lam'') (kept on
// chip), the second lam_{t-1} = A lam_t (written) and G(u_{t-1}, lam_t); the
// kappa gradient gets hdt*G1 + hdt*G2 in one update, as the LDS pair kernel
// does, value for value.  Lanes hold columns x0 - 1 .. x0 + 62: the first
// level covers all 64 (its outside columns x0 - 2 and x0 + 63 come packed in
// one load per plane and array), the second level's outputs are lanes 1..62,
// whose neighbours are plain lane shifts.  Rows: the first level covers the
// brick's P rows plus one on each side, loaded with two more on each side.
// Along z the first level completes raw plane q - 1 when plane q arrives
// (the shared face as in the one-step kernel), and the second level, fed by
// those completed planes, completes plane q - 2.  u_{t-1} is loaded one plane
// behind lam'', u_t and kappa.
template <typename T, typename TG, int P, int NW>
__global__ void __launch_bounds__(NW * 64)
k_varw_adjoint2(DevGrid lnext, DevGrid lam, DevGrid ut, DevGrid utm1, DevGrid kap, DevGrid gk, T dt, int chunk,
                int strips, int segs, int nwaves, int nbp) {
    constexpr int NR = P + 4;      // raw rows y0-2 .. y0+P+1
    constexpr int R1 = 1, E1 = NR - 1;   // first-level rows [R1, E1)
    constexpr int R2 = 2, E2 = NR - 2;   // second-level rows [R2, E2): the outputs
    constexpr int W = 62;
    Brick b;
    if (!brick_of(lnext, P, chunk, strips, segs, nwaves, nbp, NW, b, W)) return;
    Cols<T, NR> cl, cu, ck, cv;
    cl.init(lnext, b.x0 - 1, b.y0 - 2, E1 - R1);
    cu.init(ut, b.x0 - 1, b.y0 - 2, E1 - R1);
    ck.init(kap, b.x0 - 1, b.y0 - 2, E1 - R1);
    cv.init(utm1, b.x0 - 1, b.y0 - 2, E1 - R1);
    const int lane = threadIdx.x & 63;
    const int nz = lnext.nz, ny = lnext.ny;
    const int gx = b.x0 - 1 + lane;
    const bool xin = lane >= 1 && lane <= W && gx < lnext.nx;   // an output lane
    const unsigned so = (unsigned)(xin ? gx : 0) * (unsigned)sizeof(T);
    const unsigned sg = (unsigned)(xin ? gx : 0) * (unsigned)sizeof(TG);
    const int64_t lpb = lam.sz * (int64_t)sizeof(T), gpb = gk.sz * (int64_t)sizeof(TG);
    const T half = (T)0.5, hdt = (T)0.5 * dt;
    const int z0 = b.z0, zend = b.zend;

    // raw planes: current and in flight (lam'', u_t, kappa with outside columns)
    T l[2][NR], u[2][NR], k[2][NR], el[2], eu[2], ek[2];
    T v[2][NR];                    // u_{t-1}: plane q - 1 and the one in flight
    T pl[NR], pu[NR], pk[NR];      // raw plane q - 1 (first-level rows)
    T a1[NR], t1[NR];              // first level, plane q - 1: partial sums
    T m1[NR], k1[NR], v1[NR];      // second level's plane m - 1: lam_t, kappa, u_{t-1}
    T a2[NR], t2[NR], g1[NR];      // second level, plane m - 1: partial sums, hdt*G1
    TG gold[NR];                   // kappa gradient of plane m - 1
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        pl[r] = pu[r] = pk[r] = a1[r] = t1[r] = m1[r] = k1[r] = v1[r] = a2[r] = t2[r] = g1[r] = (T)0;
        gold[r] = (TG)0;
        v[0][r] = v[1][r] = (T)0;
    }
    const int qstart = z0 - 2, qend = zend + 1;
    cl.load(qstart, nz, l[0], el[0]);
    cu.load(qstart, nz, u[0], eu[0]);
    ck.load(qstart, nz, k[0], ek[0]);

    auto rowoff = [&](int r, int64_t sy, int es) { return (int)((unsigned)(b.y0 + r - R2) * (unsigned)sy * (unsigned)es); };
    auto step = [&](int q, auto cur_c) __attribute__((always_inline)) {
        constexpr int C = decltype(cur_c)::value, N = C ^ 1;
        if (q + 1 <= qend) {
            cl.load(q + 1, nz, l[N], el[N]);
            cu.load(q + 1, nz, u[N], eu[N]);
            ck.load(q + 1, nz, k[N], ek[N]);
        }
        if (q <= zend) cv.load_rows(q, nz, v[N]);   // u_{t-1} at plane q, used at step q + 1
        const T(&L)[NR] = l[C];
        const T(&U)[NR] = u[C];
        const T(&K)[NR] = k[C];
        const T(&V)[NR] = v[C];        // u_{t-1} at plane q - 1
        // first level, plane q: in-plane terms
        T an[NR], tn[NR];
        const bool own1 = q >= z0 - 1 && q <= zend;
        if (own1) {
            static_for<R1, E1>([&](auto rc) __attribute__((always_inline)) {
                constexpr int r = decltype(rc)::value;
                const T lc = L[r], uc = U[r], kc = K[r];
                T ll, lr, ul, ur, kl, kr;
                x_neighbours<r>(L, el[C], ll, lr);
                x_neighbours<r>(U, eu[C], ul, ur);
                x_neighbours<r>(K, ek[C], kl, kr);
                T s = (T)0, t = (T)0;
                s = fma(half * (kc + kl), ll - lc, s);
                t = fma(ul - uc, lc - ll, t);
                s = fma(half * (kc + kr), lr - lc, s);
                t = fma(ur - uc, lc - lr, t);
                s = fma(half * (kc + K[r - 1]), L[r - 1] - lc, s);
                t = fma(U[r - 1] - uc, lc - L[r - 1], t);
                s = fma(half * (kc + K[r + 1]), L[r + 1] - lc, s);
                t = fma(U[r + 1] - uc, lc - L[r + 1], t);
                an[r] = s;
                tn[r] = t;
            });
        }
        // first level: the face between raw planes q - 1 and q completes
        // plane m = q - 1 (lam_t and hdt*G1 there)
        T mm[NR], gm[NR];
        const int m = q - 1;
        if (q > qstart) {
#pragma unroll
            for (int r = R1; r < E1; ++r) {
                const T w = half * (pk[r] + K[r]);
                const T dl = L[r] - pl[r];
                const T du = U[r] - pu[r];
                mm[r] = fma(dt, fma(w, dl, a1[r]), pl[r]);
                gm[r] = hdt * fma(du, -dl, t1[r]);
                if (own1) {
                    an[r] = fma(w, -dl, an[r]);
                    tn[r] = fma(-du, dl, tn[r]);
                }
            }
        }
        // second level at plane m: in-plane terms (rows R2..E2, lanes 1..62),
        // then the face between m - 1 and m, which completes m - 1
        T bn[NR], un2[NR];
        TG gnew[NR];
        const bool own2 = m >= z0 && m < zend;
        if (own2) {
            const Rsrc rgj = plane_rsrc((const char*)gk.origin + (int64_t)m * gpb, gpb);
#pragma unroll
            for (int r = R2; r < E2; ++r) {
                gnew[r] = (b.y0 + r - R2 < ny && xin) ? bload<TG>(rgj, sg, rowoff(r, gk.sy, (int)sizeof(TG))) : (TG)0;
                const T lc = mm[r], vc = V[r], kc = pk[r];
                const T ll = lane_shift<kWaveShr1>(lc, lc), lr = lane_shift<kWaveShl1>(lc, lc);
                const T vl = lane_shift<kWaveShr1>(vc, vc), vr = lane_shift<kWaveShl1>(vc, vc);
                const T kl = lane_shift<kWaveShr1>(kc, kc), kr = lane_shift<kWaveShl1>(kc, kc);
                T s = (T)0, t = (T)0;
                s = fma(half * (kc + kl), ll - lc, s);
                t = fma(vl - vc, lc - ll, t);
                s = fma(half * (kc + kr), lr - lc, s);
                t = fma(vr - vc, lc - lr, t);
                s = fma(half * (kc + pk[r - 1]), mm[r - 1] - lc, s);
                t = fma(V[r - 1] - vc, lc - mm[r - 1], t);
                s = fma(half * (kc + pk[r + 1]), mm[r + 1] - lc, s);
                t = fma(V[r + 1] - vc, lc - mm[r + 1], t);
                bn[r] = s;
                un2[r] = t;
            }
        }
        if (m >= z0 && m <= zend) {
            const bool done = m - 1 >= z0;
            const Rsrc rl = plane_rsrc((const char*)lam.origin + (int64_t)(m - 1) * lpb, lpb);
            const Rsrc rg = plane_rsrc((const char*)gk.origin + (int64_t)(m - 1) * gpb, gpb);
#pragma unroll
            for (int r = R2; r < E2; ++r) {
                const T w = half * (k1[r] + pk[r]);
                const T dl = mm[r] - m1[r];
                const T dv = V[r] - v1[r];
                if (done && b.y0 + r - R2 < ny && xin) {
                    bstore<kStreamStore>(fma(dt, fma(w, dl, a2[r]), m1[r]), rl, so, rowoff(r, lam.sy, (int)sizeof(T)));
                    bstore<kStreamStore>(gold[r] + (TG)(g1[r] + hdt * fma(dv, -dl, t2[r])), rg, sg,
                                         rowoff(r, gk.sy, (int)sizeof(TG)));
                }
                if (own2) {
                    bn[r] = fma(w, -dl, bn[r]);
                    un2[r] = fma(-dv, dl, un2[r]);
                }
            }
        }
        // rotate: raw plane q becomes the previous one; the second level's
        // plane m becomes its previous one
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (r >= R1 && r < E1) {
                a1[r] = own1 ? an[r] : (T)0;
                t1[r] = own1 ? tn[r] : (T)0;
            }
            if (r >= R2 && r < E2) {
                m1[r] = q > qstart ? mm[r] : (T)0;
                g1[r] = q > qstart ? gm[r] : (T)0;
                k1[r] = pk[r];
                v1[r] = V[r];
                a2[r] = own2 ? bn[r] : (T)0;
                t2[r] = own2 ? un2[r] : (T)0;
                gold[r] = own2 ? gnew[r] : (TG)0;
            }
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            pl[r] = L[r];
            pu[r] = U[r];
            pk[r] = K[r];
        }
    };
    int q = qstart;
    for (; q + 1 <= qend; q += 2) {
        step(q, std::integral_constant<int, 0>{});
        step(q + 1, std::integral_constant<int, 1>{});
    }
    if (q <= qend) step(q, std::integral_constant<int, 0>{});
}

// Bricks of 64 columns by P rows; the z-chunk balanced against the waves the
// device holds at once for this very build (as the sweep kernels do).
template <typename K>
bool wave_geometry(K kernel, int nw_per_block, int P, const DevGrid& g, int& chunk, int& strips, int& segs, int& nw,
                   int& nbp, int W = 64) {
    strips = (g.nx + W - 1) / W;
    segs = (g.ny + P - 1) / P;
    static const int bpc = blocks_per_cu(kernel, nw_per_block * 64);
    // at least 16 planes per chunk: each chunk re-reads the plane before and
    // after it, and these kernels are bound by memory traffic, not by the
    // march's start-up
    chunk = balanced_chunk((int64_t)strips * segs, g.nz, (int64_t)device_cu_count() * bpc * nw_per_block, 2, 16);
    const int64_t w = (int64_t)strips * segs * ((g.nz + chunk - 1) / chunk);
    if (w > ((int64_t)1 << 30)) return false;
    nw = (int)w;
    nbp = padded_block_count((nw + nw_per_block - 1) / nw_per_block);
    return true;
}

// Measured on MI355X (float32, 256^3 and 512^3): streaming stores, loads with
// the default policy, one plane in flight; 4-row bricks for the reverse step
// and for forward steps up to 2^25 points (their planes fit the last-level
// cache), 8-row bricks for larger forward steps (fewer re-read halo rows).
constexpr int kVarNW = 4;
constexpr int kStream = kStreamStore;

template <typename T, int P>
hipError_t fwd(const DevGrid& src, const DevGrid& dst, const DevGrid& kappa, double dt, hipStream_t s) {
    constexpr auto kernel = k_varw_forward<T, P, kVarNW, 1, 0, kStream>;
    int chunk, strips, segs, nw, nbp;
    if (!wave_geometry(kernel, kVarNW, P, src, chunk, strips, segs, nw, nbp)) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(kernel, dim3(nbp), dim3(kVarNW * 64), 0, s, src, dst, kappa, (T)dt, chunk, strips, segs, nw, nbp);
    return hipGetLastError();
}

template <typename T, typename TG, int P>
hipError_t adj(const DevGrid& lam_next, const DevGrid& lam, const DevGrid& u, const DevGrid& kappa, const DevGrid& gk,
               double dt, hipStream_t s) {
    constexpr auto kernel = k_varw_adjoint<T, TG, P, kVarNW, 1, kStream>;
    int chunk, strips, segs, nw, nbp;
    if (!wave_geometry(kernel, kVarNW, P, lam_next, chunk, strips, segs, nw, nbp)) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(kernel, dim3(nbp), dim3(kVarNW * 64), 0, s, lam_next, lam, u, kappa, gk, (T)dt, chunk, strips,
                       segs, nw, nbp);
    return hipGetLastError();
}

template <typename T, typename TG, int P>
hipError_t adj2(const DevGrid& lam_next, const DevGrid& lam, const DevGrid& ut, const DevGrid& utm1,
                const DevGrid& kappa, const DevGrid& gk, double dt, hipStream_t s) {
    constexpr auto kernel = k_varw_adjoint2<T, TG, P, kVarNW>;
    int chunk, strips, segs, nw, nbp;
    if (!wave_geometry(kernel, kVarNW, P, lam_next, chunk, strips, segs, nw, nbp, 62))
        return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(kernel, dim3(nbp), dim3(kVarNW * 64), 0, s, lam_next, lam, ut, utm1, kappa, gk, (T)dt, chunk,
                       strips, segs, nw, nbp);
    return hipGetLastError();
}

}  // namespace

bool var_wave_fits(const DevGrid& g, int esize) { return g.sz * (int64_t)esize < ((int64_t)1 << 31); }

hipError_t launch_var_forward_wave(const DevGrid& src, const DevGrid& dst, const DevGrid& kappa, int dtype, double dt,
                                   hipStream_t s) {
    if (dtype == LOPE_F64) return fwd<double, 4>(src, dst, kappa, dt, s);
    if ((int64_t)src.nx * src.ny * src.nz <= ((int64_t)1 << 25)) return fwd<float, 4>(src, dst, kappa, dt, s);
    return fwd<float, 8>(src, dst, kappa, dt, s);
}

hipError_t launch_var_adjoint_wave(const DevGrid& lam_next, const DevGrid& lam, const DevGrid& u, const DevGrid& kappa,
                                   const DevGrid& gk, int dtype, int gk_dtype, double dt, hipStream_t s) {
    if (dtype == LOPE_F32 && gk_dtype == LOPE_F32) return adj<float, float, 4>(lam_next, lam, u, kappa, gk, dt, s);
    if (dtype == LOPE_F32) return adj<float, double, 4>(lam_next, lam, u, kappa, gk, dt, s);
    if (gk_dtype == LOPE_F64) return adj<double, double, 4>(lam_next, lam, u, kappa, gk, dt, s);
    return adj<double, float, 4>(lam_next, lam, u, kappa, gk, dt, s);
}

hipError_t launch_var_adjoint2_wave(const DevGrid& lam_next, const DevGrid& lam, const DevGrid& ut,
                                    const DevGrid& utm1, const DevGrid& kappa, const DevGrid& gk, int dtype,
                                    int gk_dtype, double dt, hipStream_t s) {
    if (dtype == LOPE_F32 && gk_dtype == LOPE_F32) return adj2<float, float, 4>(lam_next, lam, ut, utm1, kappa, gk, dt, s);
    if (dtype == LOPE_F32) return adj2<float, double, 4>(lam_next, lam, ut, utm1, kappa, gk, dt, s);
    if (gk_dtype == LOPE_F64) return adj2<double, double, 4>(lam_next, lam, ut, utm1, kappa, gk, dt, s);
    return adj2<double, float, 4>(lam_next, lam, ut, utm1, kappa, gk, dt, s);
}

}  // namespace lope
