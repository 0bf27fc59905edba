// One wavefront sweeping a strip of a 2D grid with a radius-1 stencil
// (box: 9 taps, star: 5 taps), TD sweeps fused: the body shared by the
// single-grid wave kernel and the batched kernel.
//
// The wave owns 64 consecutive columns of the grid (one per lane) and marches
// down the rows [y0, yend) of its strip.  Its output columns are the middle
// 64 - 2*TD, [x0, x0 + 64 - 2*TD): every fused sweep consumes one column of
// halo on each side, and the x neighbours of a lane are the values of lanes
// l-1 and l+1, moved across the wave with DPP wave shifts (the two outermost
// lanes read a neighbour the wave does not hold; their values at higher
// levels are never used by an output lane).  Each level k < TD keeps its last
// three rows in registers with their left and right neighbours (nine values);
// at march step j level 0 receives row j and level k computes row j - k from
// level k-1's rows j-k-1 .. j-k+1, all in the same step (levels ascending).
// The march is unrolled by twelve so every ring slot is a fixed register,
// and rows are prefetched twelve steps ahead (the loads in flight per wave
// are what keeps HBM busy: the wave has no other source of memory
// parallelism; twelve rather than six: 8192^2 box-9 2282-2308 -> 2346
// GPoint-updates/s, the persistent batch 3.80 -> 3.67 ms).  No LDS, no barriers.  Each point is c0*v0 followed
// by fmas in lexicographic offset order (x fastest), the same as every other
// kernel.
//
// Boundary rule: along a periodic axis the loaded column or row is the wrapped
// one; a lane outside the interior along a Dirichlet x axis (DX) holds g at
// every level (bit blend), and a row outside along a Dirichlet y axis (DY) is
// g at every level (a wave-uniform choice).
//
// With RES the strip also merges max |u_TD - u_(TD-1)| over its outputs (the
// change made by its last sweep) into the device double `residual`.  With
// STG (TD = 2) it makes one two-stage step: level 1 applies c9, level 2 the
// second table c9b plus alpha times the starting state (STG = 2).
//
// With DEV every load and store of the grid is a device-scope (agent) access,
// coherent across XCDs without cache flushes (the persistent batched launch,
// where strips of one grid run on any XCD within one kernel).
//
// Every argument must be uniform across the wave, and all 64 lanes must be
// active (the DPP shifts read every lane).
#pragma once

#include <type_traits>

#include "lope_internal.h"

namespace lope {

constexpr int kDppWaveShr1 = 0x138;   // lane l receives lane l-1
constexpr int kDppWaveShl1 = 0x130;   // lane l receives lane l+1

template <int CTRL>
__device__ __forceinline__ float wave_shift(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double wave_shift(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ float wblend(unsigned m, float v, float g) {
    return __uint_as_float((__float_as_uint(v) & m) | (__float_as_uint(g) & ~m));
}
__device__ __forceinline__ double wblend(unsigned long long m, double v, double g) {
    const unsigned long long vb = (unsigned long long)__double_as_longlong(v);
    const unsigned long long gb = (unsigned long long)__double_as_longlong(g);
    return __longlong_as_double((long long)((vb & m) | (gb & ~m)));
}

template <typename T>
struct WMask {
    typedef unsigned type;
};
template <>
struct WMask<double> {
    typedef unsigned long long type;
};

template <typename T>
struct Coef9 {
    T c[9];   // (ox + 1) + 3 * (oy + 1)
};

// f(j + P, step P) for P = 0 .. N-1 while j + P <= jend (a wave-uniform bound)
template <int P, int N, typename F>
__device__ __forceinline__ void wave_steps(int j, int jend, F& f) {
    if constexpr (P < N) {
        if (j + P > jend) return;
        f(j + P, std::integral_constant<int, P>{});
        wave_steps<P + 1, N>(j, jend, f);
    }
}

template <typename T, int TD, bool BOX, bool DX, bool DY, bool RES = false, int STG = 0, bool DEV = false>
__device__ __forceinline__ void plane2d_wave_strip(const DevGrid& src, const DevGrid& dst, T g, const T (&c9)[9],
                                                   int x0, int y0, int yend, double* residual = nullptr,
                                                   const T* c9b = nullptr, T alpha = (T)0) {
    static_assert(STG == 0 || TD == 2, "a two-stage step is two levels");
    typedef typename WMask<T>::type M;
    constexpr int G = TD;
    const int lane = threadIdx.x & 63;
    const int nx = src.nx, ny = src.ny;
    const int gx = x0 - G + lane;
    const bool ox = gx < 0 || gx >= nx;
    const int wx = DX ? min(max(gx, 0), nx - 1) : wrap_index(gx, nx);
    const M live = (DX && ox) ? (M)0 : ~(M)0;
    const bool keep = lane >= G && lane < 64 - G && gx < nx;
    const unsigned coff = (unsigned)wx * (unsigned)sizeof(T);
    const unsigned doff = keep ? (unsigned)gx * (unsigned)sizeof(T) : 0u;

    // Rows are loaded in order, one per march step: a running (wrapped) row
    // index and byte pointer avoid per-step multiplies and modulos.
    const int64_t sbytes = src.sy * (int64_t)sizeof(T);
    const char* const sbase = (const char*)src.origin;
    int lj = y0 - G;                               // next row to load
    int lw = DY ? lj : wrap_index(lj, ny);         // its wrapped index
    const char* lp = sbase + (int64_t)lw * sbytes;
    auto next_row = [&]() -> T {
        T v = g;   // raw value: the x rule is applied when the row enters level 0
        if (!DY || (lj >= 0 && lj < ny)) {
            if constexpr (DEV)
                v = __hip_atomic_load((T*)(lp + coff), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else
                v = *(const T*)(lp + coff);
        }
        ++lj;
        ++lw;
        lp += sbytes;
        if (!DY && lw == ny) {
            lw = 0;
            lp = sbase;
        }
        return v;
    };

    // ring[k][slot][0..2] = (left, centre, right) of a level-k row
    T ring[TD][3][3];
#pragma unroll
    for (int k = 0; k < TD; ++k)
#pragma unroll
        for (int s = 0; s < 3; ++s)
#pragma unroll
            for (int t = 0; t < 3; ++t) ring[k][s][t] = (T)0;

    const int jstart = y0 - G;
    const int jlast_load = yend - 1 + G;
    const int jend = yend - 1 + TD;
    // rows are loaded PF march steps ahead (PF a multiple of the ring length)
    constexpr int PF = 12;
    T pf[PF];
#pragma unroll
    for (int s = 0; s < PF; ++s) pf[s] = (jstart + s <= jlast_load) ? next_row() : g;
    // output row pointer of level TD, advanced one row per step
    const int64_t dbytes = dst.sy * (int64_t)sizeof(T);
    char* sp_out = (char*)dst.origin + (int64_t)(jstart - TD) * dbytes + doff;

    auto push = [&](int k, int slot, T v) {
        ring[k][slot][0] = wave_shift<kDppWaveShr1>(v);
        ring[k][slot][1] = v;
        ring[k][slot][2] = wave_shift<kDppWaveShl1>(v);
    };

    double rmax = 0.0;   // RES: max |last sweep - the sweep before| over this lane's outputs
    auto step = [&](int j, auto phase) {
        constexpr int PQ = decltype(phase)::value;   // 0 .. PF-1
        constexpr int PH = PQ % 3;                    // ring phase
        constexpr int S0 = (PH + 1) % 3, S1 = (PH + 2) % 3, S2 = PH;   // rows y-1, y, y+1 after the push
        push(0, PH, DX ? wblend(live, pf[PQ], g) : pf[PQ]);
        if (j + PF <= jlast_load) pf[PQ] = next_row();
#pragma unroll
        for (int k = 1; k <= TD; ++k) {
            const int yk = j - k;
            const T(*r)[3] = ring[k - 1];
            // STG: level 2 applies the second stencil, plus alpha times the
            // starting state at row yk (level 0's oldest row, still held)
            // (k is a compile-time index: each level reads one table directly)
            auto c = [&](int t) -> T { return (STG && k == 2) ? c9b[t] : c9[t]; };
            const bool with_alpha = STG == 2 && k == 2;
            const T a0 = with_alpha ? alpha * ring[0][S0][1] : (T)0;
            T v;
            if (BOX) {
                v = with_alpha ? fma(c(0), r[S0][0], a0) : c(0) * r[S0][0];
                v = fma(c(1), r[S0][1], v);
                v = fma(c(2), r[S0][2], v);
                v = fma(c(3), r[S1][0], v);
                v = fma(c(4), r[S1][1], v);
                v = fma(c(5), r[S1][2], v);
                v = fma(c(6), r[S2][0], v);
                v = fma(c(7), r[S2][1], v);
                v = fma(c(8), r[S2][2], v);
            } else {
                v = with_alpha ? fma(c(1), r[S0][1], a0) : c(1) * r[S0][1];
                v = fma(c(3), r[S1][0], v);
                v = fma(c(4), r[S1][1], v);
                v = fma(c(5), r[S1][2], v);
                v = fma(c(7), r[S2][1], v);
            }
            if (DX) v = wblend(live, v, g);
            if (DY && (yk < 0 || yk >= ny)) v = g;
            if (k == TD) {
                if (keep && yk >= y0 && yk < yend) {
                    if constexpr (DEV)
                        __hip_atomic_store((T*)sp_out, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    else
                        __builtin_nontemporal_store(v, (T*)sp_out);
                    // the centre of level TD-1 is the state before the last sweep
                    if (RES) rmax = nan_max(rmax, fabs((double)v - (double)r[S1][1]));
                }
                sp_out += dbytes;
            } else {
                push(k, PH, v);
            }
        }
    };

    for (int j = jstart; j <= jend; j += PF) wave_steps<0, PF>(j, jend, step);
    if (RES) residual_merge(rmax, residual);
}

}  // namespace lope
