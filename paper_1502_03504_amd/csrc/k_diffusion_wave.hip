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
// The same shifts where the lane past the wave's end is not used: that lane
// reads 0, and the compiler may fold the move into the instruction using it.
template <int CTRL>
__device__ __forceinline__ float lane_shift_free(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double lane_shift_free(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xf, 0xf, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
// Plane index i wrapped into [0, n) (periodic z; i is wave-uniform and at
// most a few planes outside).
__device__ __forceinline__ int plane_wrap(int i, int n) {
    while (i < 0) i += n;
    while (i >= n) i -= n;
    return i;
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
    // (live = false: the same loads through a resource of no bytes, which
    // return 0 and move nothing)
    template <int AUX = 0>
    __device__ __forceinline__ void load(int q, int nz, T (&v)[NR], T& e, bool live = true) const {
        const Rsrc rs = plane_rsrc(base + (int64_t)wrap_index(q, nz) * pbytes, live ? pbytes : 0);
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = bload<T, AUX>(rs, xo, row[r]);
        e = bload<T, AUX>(rs, eo, 0);
    }
    // the same for another array of this very layout, based at `other`, plane
    // qw (already wrapped)
    __device__ __forceinline__ void load_at(const char* other, int qw, T (&v)[NR], T& e, bool live = true) const {
        const Rsrc rs = plane_rsrc(other + (int64_t)qw * pbytes, live ? pbytes : 0);
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = bload<T>(rs, xo, row[r]);
        e = bload<T>(rs, eo, 0);
    }
    __device__ __forceinline__ void load_rows_at(const char* other, int qw, T (&v)[NR], bool live = true) const {
        const Rsrc rs = plane_rsrc(other + (int64_t)qw * pbytes, live ? pbytes : 0);
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = bload<T>(rs, xo, row[r]);
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
// policy of the loads / stores.  The planes and their partial sums live in a
// ring of PF + 2 slots indexed by the step's phase (the march is unrolled by
// the ring's length), so nothing is copied between registers; every step is
// the same code, with the loads of planes the march does not need and the
// stores of planes outside the chunk going through a resource of no bytes
// (a lane or row without an output through the offset 2^31), which the
// range check drops: every wait for a plane's loads counts exactly.
template <typename T, int P, int NW, int PF = 1, int LA = 0, int SA = 0>
__global__ void __launch_bounds__(NW * 64)
k_varw_forward(DevGrid src, DevGrid dst, DevGrid kap, T dt, int chunk, int strips, int segs, int nwaves, int nbp) {
    constexpr int NR = P + 2, NB = PF + 2;
    constexpr unsigned kDrop = 0x80000000u;   // past every plane (planes are below 2^31 bytes)
    Brick b;
    if (!brick_of(src, P, chunk, strips, segs, nwaves, nbp, NW, b)) return;
    Cols<T, NR> cu, ck;
    cu.init(src, b.x0, b.y0 - 1, P);
    ck.init(kap, b.x0, b.y0 - 1, P);
    const int lane = threadIdx.x & 63;
    const int nz = src.nz, ny = src.ny;
    const int64_t dpb = dst.sz * (int64_t)sizeof(T);
    const bool xin = b.x0 + lane < src.nx;   // lanes past a ragged x end store nothing
    const T half = (T)0.5;
    unsigned vo[P];
    int sro[P];
#pragma unroll
    for (int r = 0; r < P; ++r) {
        const int y = b.y0 + r;
        vo[r] = xin && y < ny ? (unsigned)(b.x0 + lane) * (unsigned)sizeof(T) : kDrop;
        sro[r] = (int)((unsigned)(y < ny ? y : 0) * (unsigned)dst.sy * (unsigned)sizeof(T));
    }

    T u[NB][NR], k[NB][NR], eu[NB], ek[NB];   // planes j - 1, j and PF in flight
    T acc[NB][P];                             // partial sums of the plane in the same slot
#pragma unroll
    for (int s = 0; s < NB; ++s) {
#pragma unroll
        for (int r = 0; r < NR; ++r) u[s][r] = k[s][r] = (T)0;
#pragma unroll
        for (int r = 0; r < P; ++r) acc[s][r] = (T)0;
        eu[s] = ek[s] = (T)0;
    }
    const int jstart = b.z0 - 1, jend = b.zend;
    static_for<0, PF>([&](auto q) __attribute__((always_inline)) {
        constexpr int Q = decltype(q)::value;
        cu.template load<LA>(jstart + Q, nz, u[Q], eu[Q], jstart + Q <= jend);
        ck.template load<LA>(jstart + Q, nz, k[Q], ek[Q], jstart + Q <= jend);
    });

    // march step j with plane j in slot C, j - 1 in slot PV
    auto step = [&](int j, auto cur_c) __attribute__((always_inline)) {
        constexpr int C = decltype(cur_c)::value, PV = (C + NB - 1) % NB, N = (C + PF) % NB;
        cu.template load<LA>(j + PF, nz, u[N], eu[N], j + PF <= jend);
        ck.template load<LA>(j + PF, nz, k[N], ek[N], j + PF <= jend);
        const T(&U)[NR] = u[C];
        const T(&K)[NR] = k[C];
        const T(&pU)[NR] = u[PV];
        const T(&pK)[NR] = k[PV];
        // plane j's in-plane terms
        T a[P];
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
        // the face between planes j-1 and j: plane j's z- term, and plane j-1's
        // z+ term, which completes it
        const bool done = j - 1 >= b.z0 && j - 1 < b.zend;
        const Rsrc rd = plane_rsrc((const char*)dst.origin + (int64_t)(done ? j - 1 : b.z0) * dpb, done ? dpb : 0);
#pragma unroll
        for (int r = 0; r < P; ++r) {
            const T w = half * (pK[r + 1] + K[r + 1]);
            const T d = U[r + 1] - pU[r + 1];
            bstore<SA>(fma(dt, fma(w, d, acc[PV][r]), pU[r + 1]), rd, vo[r], sro[r]);
            acc[C][r] = fma(w, -d, a[r]);
        }
    };
    int j = jstart;
    for (; j + NB - 1 <= jend; j += NB)
        static_for<0, NB>([&](auto c) __attribute__((always_inline)) { step(j + decltype(c)::value, c); });
    static_for<0, NB - 1>([&](auto c) __attribute__((always_inline)) {
        if (j + decltype(c)::value <= jend) step(j + decltype(c)::value, c);
    });
}

// The one-step reverse in the same form as the forward step: planes, partial
// sums and the old gradient in a ring of PF + 2 slots, every step the same
// loads and stores (out-of-chunk ones through resources of no bytes).
template <typename T, typename TG, int P, int NW, int PF = 1, int SA = 0>
__global__ void __launch_bounds__(NW * 64)
k_varw_adjoint(DevGrid lnext, DevGrid lam, DevGrid ug, DevGrid kap, DevGrid gk, T dt, int chunk, int strips, int segs,
               int nwaves, int nbp) {
    constexpr int NR = P + 2, NB = PF + 2;
    constexpr unsigned kDrop = 0x80000000u;   // past every plane (planes are below 2^31 bytes)
    Brick b;
    if (!brick_of(lnext, P, chunk, strips, segs, nwaves, nbp, NW, b)) return;
    Cols<T, NR> cl, cu, ck;
    cl.init(lnext, b.x0, b.y0 - 1, P);
    cu.init(ug, b.x0, b.y0 - 1, P);
    ck.init(kap, b.x0, b.y0 - 1, P);
    const int lane = threadIdx.x & 63;
    const int nz = lnext.nz, ny = lnext.ny;
    const bool xin = b.x0 + lane < lnext.nx;   // lanes past a ragged x end store nothing
    const int64_t lpb = lam.sz * (int64_t)sizeof(T), gpb = gk.sz * (int64_t)sizeof(TG);
    const T half = (T)0.5, hdt = (T)0.5 * dt;
    unsigned vol[P], vog[P];
    int srl[P], srg[P];
#pragma unroll
    for (int r = 0; r < P; ++r) {
        const int y = b.y0 + r;
        const bool ok = xin && y < ny;
        vol[r] = ok ? (unsigned)(b.x0 + lane) * (unsigned)sizeof(T) : kDrop;
        vog[r] = ok ? (unsigned)(b.x0 + lane) * (unsigned)sizeof(TG) : kDrop;
        const int yr = y < ny ? y : 0;
        srl[r] = (int)((unsigned)yr * (unsigned)lam.sy * (unsigned)sizeof(T));
        srg[r] = (int)((unsigned)yr * (unsigned)gk.sy * (unsigned)sizeof(TG));
    }

    T l[NB][NR], u[NB][NR], k[NB][NR], el[NB], eu[NB], ek[NB];   // planes j - 1, j, PF in flight
    T al[NB][P], ag[NB][P];   // partial sums (lam, gradient) of the plane in the same slot
    TG gold[NB][P];           // kappa gradient of the plane in the same slot, read one step ahead
#pragma unroll
    for (int s = 0; s < NB; ++s) {
#pragma unroll
        for (int r = 0; r < NR; ++r) l[s][r] = u[s][r] = k[s][r] = (T)0;
#pragma unroll
        for (int r = 0; r < P; ++r) {
            al[s][r] = ag[s][r] = (T)0;
            gold[s][r] = (TG)0;
        }
        el[s] = eu[s] = ek[s] = (T)0;
    }
    const int jstart = b.z0 - 1, jend = b.zend;
    static_for<0, PF>([&](auto q) __attribute__((always_inline)) {
        constexpr int Q = decltype(q)::value;
        cl.load(jstart + Q, nz, l[Q], el[Q], jstart + Q <= jend);
        cu.load(jstart + Q, nz, u[Q], eu[Q], jstart + Q <= jend);
        ck.load(jstart + Q, nz, k[Q], ek[Q], jstart + Q <= jend);
    });

    auto step = [&](int j, auto cur_c) __attribute__((always_inline)) {
        constexpr int C = decltype(cur_c)::value, PV = (C + NB - 1) % NB, N = (C + PF) % NB;
        cl.load(j + PF, nz, l[N], el[N], j + PF <= jend);
        cu.load(j + PF, nz, u[N], eu[N], j + PF <= jend);
        ck.load(j + PF, nz, k[N], ek[N], j + PF <= jend);
        const T(&L)[NR] = l[C];
        const T(&U)[NR] = u[C];
        const T(&K)[NR] = k[C];
        const T(&pL)[NR] = l[PV];
        const T(&pU)[NR] = u[PV];
        const T(&pK)[NR] = k[PV];
        // plane j's kappa gradient (read now, updated when the plane completes)
        {
            const bool own = j >= b.z0 && j < b.zend;
            const Rsrc rgj = plane_rsrc((const char*)gk.origin + (int64_t)(own ? j : b.z0) * gpb, own ? gpb : 0);
#pragma unroll
            for (int r = 0; r < P; ++r) gold[C][r] = bload<TG>(rgj, vog[r], srg[r]);
        }
        // plane j's in-plane terms
        T a[P], g[P];
        static_for<1, P + 1>([&](auto rc) __attribute__((always_inline)) {
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
            a[r - 1] = s;
            g[r - 1] = t;
        });
        // the face between planes j-1 and j (both sides' terms are the same
        // products with opposite signs); plane j-1 completes
        const bool done = j - 1 >= b.z0 && j - 1 < b.zend;
        const int pc = done ? j - 1 : b.z0;
        const Rsrc rl = plane_rsrc((const char*)lam.origin + (int64_t)pc * lpb, done ? lpb : 0);
        const Rsrc rg = plane_rsrc((const char*)gk.origin + (int64_t)pc * gpb, done ? gpb : 0);
#pragma unroll
        for (int r = 0; r < P; ++r) {
            const T w = half * (pK[r + 1] + K[r + 1]);
            const T dl = L[r + 1] - pL[r + 1];   // lam'_j - lam'_{j-1}
            const T du = U[r + 1] - pU[r + 1];   // u_j - u_{j-1}
            bstore<SA>(fma(dt, fma(w, dl, al[PV][r]), pL[r + 1]), rl, vol[r], srl[r]);
            bstore<SA>(gold[PV][r] + (TG)(hdt * fma(du, -dl, ag[PV][r])), rg, vog[r], srg[r]);
            al[C][r] = fma(w, -dl, a[r]);
            ag[C][r] = fma(-du, dl, g[r]);
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
// those completed planes, completes plane q - 2; its face coefficient
// between planes q - 2 and q - 1 is the first level's of the step before.
//
// Every plane and every partial sum lives in a ring of three slots indexed
// by the step's phase (the march is unrolled by three), so no value moves
// between registers.  Every step is the same code: planes before and after
// the chunk are loaded (wrapped) and computed like the others, and their
// results never reach a store, because a store (and the load of the old
// gradient) whose plane lies outside the chunk goes through a resource of no
// bytes and a lane or row without an output uses the offset 2^31; the range
// check drops both.  With the same number of memory operations in every
// step the waits for a plane's loads count exactly what was issued after
// them.  The four inputs share one layout (the launcher checks), so one row
// table addresses them all.
template <typename T, typename TG, int P, int NW>
__global__ void __launch_bounds__(NW * 64)
k_varw_adjoint2(DevGrid lnext, DevGrid lam, DevGrid ut, DevGrid utm1, DevGrid kap, DevGrid gk, T dt, int chunk,
                int strips, int segs, int nwaves, int nbp) {
    constexpr int NR = P + 4;      // raw rows y0-2 .. y0+P+1
    constexpr int R1 = 1, E1 = NR - 1;   // first-level rows [R1, E1)
    constexpr int R2 = 2, E2 = NR - 2;   // second-level rows [R2, E2): the outputs
    constexpr int W = 62;
    constexpr unsigned kDrop = 0x80000000u;   // past every plane (planes are below 2^31 bytes)
    Brick b;
    if (!brick_of(lnext, P, chunk, strips, segs, nwaves, nbp, NW, b, W)) return;
    Cols<T, NR> c;
    c.init(lnext, b.x0 - 1, b.y0 - 2, E1 - R1);
    const char* const bl = (const char*)lnext.origin;
    const char* const bu = (const char*)ut.origin;
    const char* const bk = (const char*)kap.origin;
    const char* const bv = (const char*)utm1.origin;
    const int lane = threadIdx.x & 63;
    const int nz = lnext.nz, ny = lnext.ny;
    const int gx = b.x0 - 1 + lane;
    const bool xin = lane >= 1 && lane <= W && gx < lnext.nx;   // an output lane
    const int64_t lpb = lam.sz * (int64_t)sizeof(T), gpb = gk.sz * (int64_t)sizeof(TG);
    const T half = (T)0.5, hdt = (T)0.5 * dt;
    const int z0 = b.z0, zend = b.zend;
    // output rows: in-plane offsets of this lane's column (kDrop where there
    // is no output), wave-uniform row offsets
    unsigned vol[NR], vog[NR];
    int srl[NR], srg[NR];
#pragma unroll
    for (int r = R2; r < E2; ++r) {
        const int y = b.y0 + r - R2;
        const bool ok = xin && y < ny;
        vol[r] = ok ? (unsigned)gx * (unsigned)sizeof(T) : kDrop;
        vog[r] = ok ? (unsigned)gx * (unsigned)sizeof(TG) : kDrop;
        const int yr = y < ny ? y : 0;
        srl[r] = (int)((unsigned)yr * (unsigned)lam.sy * (unsigned)sizeof(T));
        srg[r] = (int)((unsigned)yr * (unsigned)gk.sy * (unsigned)sizeof(TG));
    }

    // rings of three, slot = phase of the plane's step
    T l[3][NR], u[3][NR], k[3][NR], el[3], eu[3], ek[3];   // raw lam'', u_t, kappa
    T v[3][NR];                    // u_{t-1}
    T a1[3][NR], t1[3][NR];        // first level: partial sums of its plane
    T m1[3][NR], g1[3][NR];        // first level's completed plane: lam_t, hdt*G1
    T ws[3][NR];                   // first level's face coefficient (second level's z- face)
    T a2[3][NR], t2[3][NR];        // second level: partial sums of its plane
    TG gold[3][NR];                // kappa gradient of the second level's plane
#pragma unroll
    for (int s = 0; s < 3; ++s) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            l[s][r] = u[s][r] = k[s][r] = v[s][r] = (T)0;
            a1[s][r] = t1[s][r] = m1[s][r] = g1[s][r] = ws[s][r] = a2[s][r] = t2[s][r] = (T)0;
            gold[s][r] = (TG)0;
        }
        el[s] = eu[s] = ek[s] = (T)0;
    }
    const int qstart = z0 - 2, qend = zend + 1;
    {
        const int qw = plane_wrap(qstart, nz);
        c.load_at(bl, qw, l[0], el[0]);
        c.load_at(bu, qw, u[0], eu[0]);
        c.load_at(bk, qw, k[0], ek[0]);
    }

    // step q, phase C: plane q in slot C, q - 1 in slot PV, q + 1 (and q - 2) in slot NX
    auto step = [&](int q, auto phase) __attribute__((always_inline)) {
        constexpr int C = decltype(phase)::value, PV = (C + 2) % 3, NX = (C + 1) % 3;
        const int m = q - 1;
        const int qw = plane_wrap(q, nz), qn = qw + 1 < nz ? qw + 1 : 0;
        // (planes past the march's end are loaded through a resource of no
        // bytes: the same instructions, no traffic)
        c.load_at(bl, qn, l[NX], el[NX], q + 1 <= qend);
        c.load_at(bu, qn, u[NX], eu[NX], q + 1 <= qend);
        c.load_at(bk, qn, k[NX], ek[NX], q + 1 <= qend);
        c.load_rows_at(bv, qw, v[C], q <= zend);
        {
            // the old gradient of plane m (added when m is completed, next step)
            const bool own2 = m >= z0 && m < zend;
            const Rsrc rg = plane_rsrc((const char*)gk.origin + (int64_t)(own2 ? m : z0) * gpb, own2 ? gpb : 0);
#pragma unroll
            for (int r = R2; r < E2; ++r) gold[C][r] = bload<TG>(rg, vog[r], srg[r]);
        }
        const T(&L)[NR] = l[C];
        const T(&U)[NR] = u[C];
        const T(&K)[NR] = k[C];
        const T(&pl)[NR] = l[PV];
        const T(&pu)[NR] = u[PV];
        const T(&pk)[NR] = k[PV];
        const T(&V)[NR] = v[PV];       // u_{t-1} at plane m
        const T(&V1)[NR] = v[NX];      // u_{t-1} at plane m - 1
        // first level, plane q: in-plane terms.  The face between rows r and
        // r + 1 is formed once and serves both (its difference negated for
        // row r + 1, exactly the value that row would form).
        T fw[NR], fl[NR], fu[NR];
#pragma unroll
        for (int r = R1 - 1; r < E1; ++r) {
            fw[r] = half * (K[r + 1] + K[r]);
            fl[r] = L[r + 1] - L[r];
            fu[r] = U[r + 1] - U[r];
        }
        T an[NR], tn[NR];
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
            s = fma(fw[r - 1], -fl[r - 1], s);
            t = fma(-fu[r - 1], fl[r - 1], t);
            s = fma(fw[r], fl[r], s);
            t = fma(fu[r], -fl[r], t);
            an[r] = s;
            tn[r] = t;
        });
        // first level: the face between raw planes q - 1 and q completes
        // plane m (lam_t and hdt*G1 there)
        T(&mm)[NR] = m1[C];
#pragma unroll
        for (int r = R1; r < E1; ++r) {
            const T w = half * (pk[r] + K[r]);
            const T dl = L[r] - pl[r];
            const T du = U[r] - pu[r];
            mm[r] = fma(dt, fma(w, dl, a1[PV][r]), pl[r]);
            if (r >= R2 && r < E2) {
                g1[C][r] = hdt * fma(du, -dl, t1[PV][r]);
                ws[C][r] = w;
            }
            a1[C][r] = fma(w, -dl, an[r]);
            t1[C][r] = fma(-du, dl, tn[r]);
        }
        // second level at plane m: in-plane terms (rows R2..E2, lanes 1..62).
        // Faces shared as above: along y between rows, along x with the lane
        // to the left (its x+ face is this lane's x- face; lanes 0 and 63 hold
        // no output, so their shifted values are unused).
#pragma unroll
        for (int r = R2 - 1; r < E2; ++r) {
            fw[r] = half * (pk[r + 1] + pk[r]);
            fl[r] = mm[r + 1] - mm[r];
            fu[r] = V[r + 1] - V[r];
        }
        T bn[NR], un2[NR];
#pragma unroll
        for (int r = R2; r < E2; ++r) {
            const T lc = mm[r], vc = V[r], kc = pk[r];
            const T lr = lane_shift_free<kWaveShl1>(lc), vr = lane_shift_free<kWaveShl1>(vc);
            const T kr = lane_shift_free<kWaveShl1>(kc);
            const T xw = half * (kc + kr), xl = lr - lc, xv = vr - vc;   // x+ face
            const T wl = lane_shift_free<kWaveShr1>(xw), dl = lane_shift_free<kWaveShr1>(xl);
            const T dv = lane_shift_free<kWaveShr1>(xv);                  // x- face
            T s = (T)0, t = (T)0;
            s = fma(wl, -dl, s);
            t = fma(-dv, dl, t);
            s = fma(xw, xl, s);
            t = fma(xv, -xl, t);
            s = fma(fw[r - 1], -fl[r - 1], s);
            t = fma(-fu[r - 1], fl[r - 1], t);
            s = fma(fw[r], fl[r], s);
            t = fma(fu[r], -fl[r], t);
            bn[r] = s;
            un2[r] = t;
        }
        // second level: the face between m - 1 and m completes plane m - 1
        {
            const int p = m - 1;
            const bool done = p >= z0 && p < zend;
            const int pc = done ? p : z0;
            const Rsrc rl = plane_rsrc((const char*)lam.origin + (int64_t)pc * lpb, done ? lpb : 0);
            const Rsrc rg = plane_rsrc((const char*)gk.origin + (int64_t)pc * gpb, done ? gpb : 0);
#pragma unroll
            for (int r = R2; r < E2; ++r) {
                const T w = ws[PV][r];
                const T dl = mm[r] - m1[PV][r];
                const T dv = V[r] - V1[r];
                bstore<kStreamStore>(fma(dt, fma(w, dl, a2[PV][r]), m1[PV][r]), rl, vol[r], srl[r]);
                bstore<kStreamStore>(gold[PV][r] + (TG)(g1[PV][r] + hdt * fma(dv, -dl, t2[PV][r])), rg, vog[r],
                                         srg[r]);
                a2[C][r] = fma(w, -dl, bn[r]);
                t2[C][r] = fma(-dv, dl, un2[r]);
            }
        }
    };
    int q = qstart;
    for (; q + 2 <= qend; q += 3) {
        step(q, std::integral_constant<int, 0>{});
        step(q + 1, std::integral_constant<int, 1>{});
        step(q + 2, std::integral_constant<int, 2>{});
    }
    if (q <= qend) {
        step(q, std::integral_constant<int, 0>{});
        if (q + 1 <= qend) step(q + 1, std::integral_constant<int, 1>{});
    }
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
    if (!var_pair_wave_fits(lam_next, ut, utm1, kappa, (int)sizeof(T))) return hipErrorInvalidValue;
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

bool var_pair_wave_fits(const DevGrid& a, const DevGrid& b, const DevGrid& c, const DevGrid& d, int esize) {
    const DevGrid* g[3] = {&b, &c, &d};
    for (const DevGrid* x : g)
        if (x->nx != a.nx || x->ny != a.ny || x->nz != a.nz || x->sy != a.sy || x->sz != a.sz) return false;
    return var_wave_fits(a, esize);
}

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
