// 3D radius-1 star (7 taps), TD sweeps fused per pass, one wavefront per
// brick: 64 x columns (one per lane) by P + 2*TD rows, marching a z-chunk.
// No LDS and no barriers.
//
// The 64 lanes hold 64 consecutive columns; the wave's outputs are the middle
// 64 - 2*TD columns and the middle P rows (each fused sweep consumes one
// column and one row of halo on each side, as in the 2D wave kernel).  Each
// lane keeps a column of NR = P + 2*TD rows in registers: the y neighbours of
// a row are the rows above and below in the same lane, the x neighbours come
// from lanes l-1 and l+1 as DPP operands of the fmas themselves (no separate
// moves; float32), and the z direction is the march.
//
// Instead of a ring of three input planes per level, each level keeps two
// partial sums: when level k's plane q is complete it finishes level k+1's
// plane q-1 (its z+1 tap), adds the in-plane taps to plane q (y-1, x-1,
// centre, x+1, y+1) and starts plane q+1 with its z-1 tap.  The taps of every
// point are therefore summed as c(z-1)*v followed by fmas in lexicographic
// offset order, the same chain as every other kernel.  Level k completes
// plane j - k at march step j (level 0 is the plane loaded at step j); the
// march runs from z0 - TD to zend - 1 + TD and stores level TD's planes
// [z0, zend).  Values outside the cone of the stored outputs are computed
// and thrown away (garbage lanes at the wave's edges move one lane inward per
// level and never reach an output lane).
//
// Boundary rule: a periodic axis loads the wrapped column / row / plane; a
// lane outside a Dirichlet x axis holds g at every level (bit blend, DXY), a
// row outside a Dirichlet y axis is g at every level (DXY; a wave-uniform
// choice per row) and a plane outside a Dirichlet z axis is g at every level
// (DZ).  Under Dirichlet rules only the bricks whose footprint reaches the
// edge of the interior along a Dirichlet axis run the blending march; the
// others run the march without blends (or with the z rule only), chosen per
// wave.  The z rule itself only touches the warm-up steps and the last few
// steps of a march (those that load or complete a plane past the z edge), so
// the steps in between run without it.
//
// Planes are prefetched PF steps ahead (PF = 1 or 3; the march is unrolled by
// three, the period of the partial-sum ring, so every buffer index is a
// compile-time constant and no value moves between registers).  Loads and
// stores go through a buffer resource per plane: the plane's base in scalar
// registers, a 32-bit in-plane offset per lane and row (loop-invariant), and
// the hardware's range check (the caller checks plane sizes below 2^31
// bytes; every offset is inside the plane anyway).
#include "plane2d_wave.h"

namespace lope {
namespace {

template <typename T>
struct Coef7 {
    T c[7];   // z-1, y-1, x-1, centre, x+1, y+1, z+1
};

// Buffer resource of one plane: base address, size in bytes (accesses past
// it read 0 and write nothing), the gfx9 data-format word.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buffer_load(__amdgpu_buffer_rsrc_t r, unsigned off);
// (the builtins move raw bits: the values are reinterpreted, not converted)
template <>
__device__ __forceinline__ float buffer_load<float>(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
constexpr int kBufferNontemporal = 2;   // cache-policy bits of a streaming store
__device__ __forceinline__ void buffer_store(float v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, kBufferNontemporal);
}

// a[i] + c(x-1) * v[i][lane-1] + c(x) * v[i] + c(x+1) * v[i][lane+1] for N
// rows (N <= 3), three fmas per row in that order, with the lane shifts folded
// into the fmas (DPP operands: lanes past the wave's ends read 0).  cm, cp in
// VGPRs (a DPP fma takes its second factor from a VGPR), c0 in an SGPR.  A DPP
// instruction must not read a VGPR the VALU wrote in the two wait states
// before: one s_nop covers the inputs, and with three rows interleaved every
// accumulator is two instructions old when its second DPP fma reads it (one
// or two rows add an s_nop).
__device__ __forceinline__ void fma_xrows(float& a0, float& a1, float& a2, float v0, float v1, float v2, float cm, float c0,
                                          float cp) {
    asm("s_nop 1\n\t"
        "v_fmac_f32_dpp %0, %3, %6 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %4, %6 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %2, %5, %6 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_e32 %0, %8, %3\n\t"
        "v_fmac_f32_e32 %1, %8, %4\n\t"
        "v_fmac_f32_e32 %2, %8, %5\n\t"
        "v_fmac_f32_dpp %0, %3, %7 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %4, %7 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %2, %5, %7 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "+v"(a0), "+v"(a1), "+v"(a2)
        : "v"(v0), "v"(v1), "v"(v2), "v"(cm), "v"(cp), "s"(c0));
}
__device__ __forceinline__ void fma_xrows(float& a0, float& a1, float v0, float v1, float cm, float c0, float cp) {
    asm("s_nop 1\n\t"
        "v_fmac_f32_dpp %0, %2, %4 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %3, %4 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_e32 %0, %6, %2\n\t"
        "v_fmac_f32_e32 %1, %6, %3\n\t"
        "s_nop 0\n\t"
        "v_fmac_f32_dpp %0, %2, %5 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %3, %5 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "+v"(a0), "+v"(a1)
        : "v"(v0), "v"(v1), "v"(cm), "v"(cp), "s"(c0));
}
__device__ __forceinline__ void fma_xrows(float& a0, float v0, float cm, float c0, float cp) {
    asm("s_nop 1\n\t"
        "v_fmac_f32_dpp %0, %1, %2 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_e32 %0, %4, %1\n\t"
        "s_nop 1\n\t"
        "v_fmac_f32_dpp %0, %1, %3 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "+v"(a0)
        : "v"(v0), "v"(cm), "v"(cp), "s"(c0));
}
// f(integral_constant<S>) ... f(integral_constant<E-1>), unrolled at compile time
template <int S, int E, typename F>
__device__ __forceinline__ void static_steps(F&& f) {
    if constexpr (S < E) {
        f(std::integral_constant<int, S>{});
        static_steps<S + 1, E>(f);
    }
}

// RES: also merge max |u_TD - u_(TD-1)| over the stored outputs (the change
// made by the last sweep) into the device double `residual`.
// STG: 0 = TD sweeps of one stencil; 1, 2 = TD / 2 two-stage steps: odd
// levels apply cf, even levels cf2 (plus alpha times the state two levels
// below, the state at the start of the step, when STG = 2).
// The march of the brick at (x0, y0) over planes z0 .. zend - 1.  DXY: the
// rule may put g inside the brick's footprint along x or y.
template <typename T, int TD, int P, bool DXY, bool DZ, bool RES, int STG, int PF>
__device__ __forceinline__ void wave_brick(const DevGrid& src, const DevGrid& dst, const DevRule& rule,
                                           const Coef7<T>& cf, const Coef7<T>& cf2, T alpha, int x0, int y0, int z0,
                                           int zend, double* residual) {
    static_assert(PF == 1 || PF == 3, "the march is unrolled by three");
    // float64 would need two DPP moves per lane shift (no DPP form of the
    // 64-bit fma) and twice the registers: the LDS designs serve it better
    static_assert(std::is_same<T, float>::value, "float32 only");
    static_assert(STG == 0 || (TD % 2 == 0 && !RES), "two-stage steps pair the levels");
    typedef typename WMask<T>::type M;
    constexpr int G = TD;
    constexpr int NR = P + 2 * G;
    const int nx = src.nx, ny = src.ny, nz = src.nz;
    const int yend = min(y0 + P, ny);
    const bool perx = rule.per[0] != 0, pery = rule.per[1] != 0;
    const T g = (T)rule.g;

    const int lane = threadIdx.x & 63;
    const int gx = x0 - G + lane;
    const bool ox = gx < 0 || gx >= nx;
    const int wx = perx ? wrap_index(gx, nx) : min(max(gx, 0), nx - 1);
    const M live = (DXY && !perx && ox) ? (M)0 : ~(M)0;
    const bool keep = lane >= G && lane < 64 - G && gx < nx;

    // rows: in-plane byte offsets of this lane's (wrapped or clamped) column
    // in each row, and which rows lie outside a Dirichlet y axis (g at every
    // level)
    unsigned boff[NR];
    unsigned grow = 0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int y = y0 - G + r;
        if (DXY && !pery && (y < 0 || y >= ny)) grow |= 1u << r;
        const int yw = pery ? wrap_index(y, ny) : min(max(y, 0), ny - 1);
        boff[r] = ((unsigned)yw * (unsigned)src.sy + (unsigned)wx) * (unsigned)sizeof(T);
    }
    auto is_grow = [&](int r) { return DXY && ((grow >> r) & 1u); };

    const char* sp = (const char*)src.origin;
    const char* dp = (const char*)dst.origin;
    const int64_t szb = src.sz * (int64_t)sizeof(T), dszb = dst.sz * (int64_t)sizeof(T);
    // Plane q of level 0 (every row loaded: the index is wrapped, or clamped
    // and then replaced by g outside a Dirichlet z axis).  ZR: a Dirichlet z
    // rule may apply to q (else q is inside or wrapped).
    auto load_plane = [&](int q, T (&v)[NR], auto zrule) __attribute__((always_inline)) {
        constexpr bool ZR = decltype(zrule)::value;
        const int qw = ZR ? min(max(q, 0), nz - 1) : wrap_index(q, nz);
        const __amdgpu_buffer_rsrc_t rs = plane_rsrc(sp + qw * szb, szb);
        const bool gz = ZR && (q < 0 || q >= nz);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const T t = buffer_load<T>(rs, boff[r]);
            v[r] = (is_grow(r) || gz) ? g : t;
        }
    };

    // acc[k][s][r]: partial sums of level k+1, a ring of three planes (two in
    // flight; the third slot is free between finishing one and starting one)
    T acc[TD][3][NR];
#pragma unroll
    for (int k = 0; k < TD; ++k)
#pragma unroll
        for (int s = 0; s < 3; ++s)
#pragma unroll
            for (int r = 0; r < NR; ++r) acc[k][s][r] = (T)0;

    const int jstart = z0 - TD, jend = zend - 1 + TD;
    T pf[PF][NR];
#pragma unroll
    for (int q = 0; q < PF; ++q) load_plane(jstart + q, pf[q], std::integral_constant<bool, DZ>{});

    const unsigned xoff = (unsigned)(keep ? gx : 0) * (unsigned)sizeof(T);
    double rmax = 0.0;   // RES: this lane's maximum change over its outputs
    T prev[NR];          // RES: level TD-1's previous plane (rows TD .. NR-TD-1)
#pragma unroll
    for (int r = 0; r < NR; ++r) prev[r] = (T)0;
    const unsigned dsyb = (unsigned)dst.sy * (unsigned)sizeof(T);
    // The outputs of a completed plane are stored in the next step, after its
    // first level (whose start waits for that step's plane): stored at the
    // end of their own step they would be waited for at once by the next
    // step's wait for its loads; stored one level later they have most of a
    // step to complete before that wait.
    T pend[P];
    int pend_p = -1;   // plane of the values in pend (-1: nothing to store)
#pragma unroll
    for (int i = 0; i < P; ++i) pend[i] = (T)0;
    auto store_pending = [&]() __attribute__((always_inline)) {
        if (pend_p >= 0 && keep) {
            const __amdgpu_buffer_rsrc_t rd = plane_rsrc(dp + pend_p * dszb, dszb);
#pragma unroll
            for (int i = 0; i < P; ++i)
                if (y0 + i < yend) buffer_store(pend[i], rd, (unsigned)(y0 + i) * dsyb + xoff);
        }
        pend_p = -1;
    };
    // March step j (phase u = (j - jstart) mod 3 of the three-step unroll):
    // level 0 is the plane in pf[u % PF]; once consumed, that buffer takes the
    // plane PF steps ahead (past the end: a repeat of the last plane, never
    // used).  Only levels k < KM run: during the first 2*TD steps level k+1
    // has nothing valid to start before step 2k, so those steps skip it.  ZR:
    // the step may load or complete a plane outside a Dirichlet z axis.
    auto step = [&](int j, auto phase, auto kmax, auto zrule) __attribute__((always_inline)) {
        constexpr int u = decltype(phase)::value;
        constexpr int KM = decltype(kmax)::value;
        constexpr bool ZR = decltype(zrule)::value;
        T cur[NR];
        T base[NR];   // STG = 2: the state at the start of the step (level k-1 for an even level k+1)
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            // level k's plane q = j - k, rows [k, NR - k) valid
            T(&lv)[NR] = k == 0 ? pf[u % PF] : cur;
            T(&old)[NR] = acc[k][u];             // level k+1, plane q - 1
            T(&mid)[NR] = acc[k][(u + 1) % 3];   // level k+1, plane q
            T(&nw)[NR] = acc[k][(u + 2) % 3];    // level k+1, plane q + 1
            T nxt[NR], bl[NR];
#pragma unroll
            for (int r = k; r < NR - k; ++r) bl[r] = k == 0 && DXY ? wblend(live, lv[r], g) : lv[r];
            // the stencil of level k+1 (STG: the second one on even levels)
            const bool second = STG != 0 && (k % 2) == 1;
            const Coef7<T>& c = second ? cf2 : cf;
            // STG = 2: an even level starts each plane from alpha times the
            // state at the start of the step (same plane, row), then the taps
            const bool with_alpha = STG == 2 && second;
            if (STG == 2 && !second) {
#pragma unroll
                for (int r = k; r < NR - k; ++r) base[r] = bl[r];
            }
            // rows lo .. hi-1 of level k+1: y-1 tap, x taps (three rows at a
            // time), y+1 tap; then the z+1 tap finishes plane q-1 and the z-1
            // tap starts plane q+1
            const int lo = k + 1, hi = NR - 1 - k;
#pragma unroll
            for (int r = lo; r < hi; ++r) mid[r] = fma(c.c[1], bl[r - 1], mid[r]);
#pragma unroll
            for (int r = lo; r < hi; r += 3) {
                if (r + 3 <= hi)
                    fma_xrows(mid[r], mid[r + 1], mid[r + 2], bl[r], bl[r + 1], bl[r + 2], c.c[2], c.c[3], c.c[4]);
                else if (r + 2 == hi)
                    fma_xrows(mid[r], mid[r + 1], bl[r], bl[r + 1], c.c[2], c.c[3], c.c[4]);
                else
                    fma_xrows(mid[r], bl[r], c.c[2], c.c[3], c.c[4]);
            }
#pragma unroll
            for (int r = lo; r < hi; ++r) {
                mid[r] = fma(c.c[5], bl[r + 1], mid[r]);
                nxt[r] = fma(c.c[6], bl[r], old[r]);
                // plane q+1 of level k+1 at row r; with alpha its start is
                // alpha * (that plane of level k-1), completed this step
                nw[r] = with_alpha ? fma(c.c[0], bl[r], alpha * base[r]) : c.c[0] * bl[r];
            }
            if (k == 0) {
                if (KM == TD) store_pending();
                load_plane(min(j + PF, jend), pf[u % PF], zrule);
            }
            // the rule on the completed plane p of level k+1
            const int p = j - k - 1;
            const bool gz = ZR && (p < 0 || p >= nz);
#pragma unroll
            for (int r = k + 1; r < NR - 1 - k; ++r) {
                T v = DXY ? wblend(live, nxt[r], g) : nxt[r];
                if (is_grow(r) || gz) v = g;
                nxt[r] = v;
            }
            if (k + 1 < TD) {
#pragma unroll
                for (int r = k + 1; r < NR - 1 - k; ++r) cur[r] = nxt[r];
            } else if (p >= z0 && p < zend) {
#pragma unroll
                for (int r = TD; r < NR - TD; ++r) pend[r - TD] = nxt[r];
                pend_p = p;
                if (RES && keep) {
#pragma unroll
                    for (int r = TD; r < NR - TD; ++r)
                        if (y0 + (r - TD) < yend) rmax = nan_max(rmax, fabs((double)nxt[r] - (double)prev[r]));
                }
            }
            // RES: level TD-1's plane p + 1 is the state before the last sweep
            // of the next step's outputs
            if (RES && k + 1 == TD) {
#pragma unroll
                for (int r = TD; r < NR - TD; ++r) prev[r] = bl[r];
            }
        }
    };
    // warm-up: steps jstart .. jstart + 2*TD - 1 (all exist: the chunk is not
    // empty), level k from step 2k on
    static_steps<0, 2 * TD>([&](auto st) __attribute__((always_inline)) {
        constexpr int sidx = decltype(st)::value;
        constexpr int km = sidx / 2 + 1 < TD ? sidx / 2 + 1 : TD;
        step(jstart + sidx, std::integral_constant<int, sidx % 3>{}, std::integral_constant<int, km>{},
             std::integral_constant<bool, DZ>{});
    });
    // then every level, three steps per iteration with the phases continuing
    constexpr int P0 = (2 * TD) % 3;
    const std::integral_constant<int, TD> all{};
    const std::integral_constant<int, P0> ph0{};
    const std::integral_constant<int, (P0 + 1) % 3> ph1{};
    const std::integral_constant<int, (P0 + 2) % 3> ph2{};
    // Under a Dirichlet rule, whole groups of three steps first.  After the
    // warm-up every completed plane j - k - 1 is at least z0, so a Dirichlet
    // z axis only reaches the steps that load a plane at nz or beyond, or
    // complete one there: the groups before those (the last loaded plane
    // j + 2 + PF < nz) run without the z rule.  Then the remaining steps
    // (under the rule).  The register allocation of the blending march fits
    // two waves per SIMD in this form; the plain march fits in the single
    // loop below.
    int j = jstart + 2 * TD;
    if constexpr (DXY || DZ) {
        const std::integral_constant<bool, false> inside{};
        const int jsafe = (DZ ? min(jend, nz - 1 - PF) : jend) - 2;
        for (; j <= jsafe; j += 3) {
            step(j, ph0, all, inside);
            step(j + 1, ph1, all, inside);
            step(j + 2, ph2, all, inside);
        }
    }
    const std::integral_constant<bool, DZ> zr{};
    for (; j <= jend; j += 3) {
        step(j, ph0, all, zr);
        if (j + 1 > jend) break;
        step(j + 1, ph1, all, zr);
        if (j + 2 > jend) break;
        step(j + 2, ph2, all, zr);
    }
    store_pending();
    if (RES) residual_merge(rmax, residual);
}

template <typename T, int TD, int P, int NW, bool DXY, bool DZ, bool RES, int STG, int PF, int WPE>
__global__ void __launch_bounds__(NW * 64, WPE)
k_star3d_wave(DevGrid src, DevGrid dst, DevRule rule, Coef7<T> cf, Coef7<T> cf2, T alpha, int chunk, int strips,
              int segs, int nwaves, int nblocks_padded, double* residual) {
    constexpr int G = TD;
    // the wave index is uniform: rows, planes and loop bounds stay scalar
    const int wave = xcd_logical_block(nblocks_padded) * NW + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (wave >= nwaves) return;   // whole waves leave; there is no barrier
    const int tx = wave % strips, rest = wave / strips;
    const int ty = rest % segs, tz = rest / segs;
    const int x0 = tx * (64 - 2 * G), y0 = ty * P, z0 = tz * chunk;
    const int zend = min(z0 + chunk, src.nz);
    if constexpr (DXY || DZ) {
        // a brick whose footprint (64 columns, P + 2 G rows, the chunk and G
        // planes on each side) lies inside the interior along every Dirichlet
        // axis never meets g: it runs the march without the rule's blends
        const bool xin = rule.per[0] != 0 || (x0 - G >= 0 && x0 - G + 63 < src.nx);
        const bool yin = rule.per[1] != 0 || (y0 - G >= 0 && y0 + P + G - 1 < src.ny);
        const bool zin = rule.per[2] != 0 || (z0 - G >= 0 && zend - 1 + G < src.nz);
        if (xin && yin && zin) {
            wave_brick<T, TD, P, false, false, RES, STG, PF>(src, dst, rule, cf, cf2, alpha, x0, y0, z0, zend,
                                                              residual);
            return;
        }
        if constexpr (DXY && DZ) {
            if (xin && yin) {   // only the z rule reaches this brick
                wave_brick<T, TD, P, false, true, RES, STG, PF>(src, dst, rule, cf, cf2, alpha, x0, y0, z0, zend,
                                                                 residual);
                return;
            }
        }
    }
    wave_brick<T, TD, P, DXY, DZ, RES, STG, PF>(src, dst, rule, cf, cf2, alpha, x0, y0, z0, zend, residual);
}

template <typename T>
Coef7<T> coef7(const SweepJob& j) {
    Coef7<T> cf;
    auto dense = [&](int ox, int oy, int oz) { return (T)j.dense[(ox + 1) + (oy + 1) * 3 + (oz + 1) * 9]; };
    cf.c[0] = dense(0, 0, -1);
    cf.c[1] = dense(0, -1, 0);
    cf.c[2] = dense(-1, 0, 0);
    cf.c[3] = dense(0, 0, 0);
    cf.c[4] = dense(1, 0, 0);
    cf.c[5] = dense(0, 1, 0);
    cf.c[6] = dense(0, 0, 1);
    return cf;
}

// One pass over j's grids with the kernel built for rule case (DXY, DZ) and
// residual flag RES (the stencils in cf, cf2).  The automatic z-chunk: as
// long as the resident waves (the workgroups a compute unit holds at the
// register use of this very build, on every unit) still cover every chunk in
// few rounds.
template <typename T, int TD, int P, int NW, int PF, int WPE, int STG, bool DXY, bool DZ, bool RES>
hipError_t launch_wave3_case(const SweepJob& j, const Coef7<T>& cf, const Coef7<T>& cf2, T alpha, int chunk,
                             hipStream_t s) {
    constexpr auto kernel = k_star3d_wave<T, TD, P, NW, DXY, DZ, RES, STG, PF, WPE>;
    const int out_cols = 64 - 2 * TD;
    const int strips = (j.src.nx + out_cols - 1) / out_cols;
    const int segs = (j.src.ny + P - 1) / P;
    if (chunk <= 0) {
        static const int bpc = blocks_per_cu(kernel, NW * 64);
        chunk = balanced_chunk((int64_t)strips * segs, j.src.nz, (int64_t)device_cu_count() * bpc * NW, 2 * TD + 2,
                               2 * TD);
    }
    const int chunks = (j.src.nz + chunk - 1) / chunk;
    const int64_t nw64 = (int64_t)strips * segs * chunks;
    if (nw64 > (1ll << 30)) return hipErrorInvalidConfiguration;
    const int nw = (int)nw64;
    const int nbp = padded_block_count((nw + NW - 1) / NW);
    hipLaunchKernelGGL(kernel, dim3(nbp), dim3(NW * 64), 0, s, j.src, j.dst, j.rule, cf, cf2, alpha, chunk, strips,
                       segs, nw, nbp, j.residual);
    return hipGetLastError();
}

// One pass over j's grids (its rule and residual; the stencils in cf, cf2).
template <typename T, int TD, int P, int NW, int PF, int WPE, int STG>
hipError_t launch_wave3(const SweepJob& j, const Coef7<T>& cf, const Coef7<T>& cf2, T alpha, int chunk,
                        hipStream_t s) {
    const bool dxy = !j.rule.per[0] || !j.rule.per[1], dz = !j.rule.per[2];
#define LOPE_WAVE3_RULE(C)                                                                         \
    if (dxy && dz)                                                                                 \
        return launch_wave3_case<T, TD, P, NW, PF, WPE, STG, true, true, C>(j, cf, cf2, alpha, chunk, s);   \
    else if (dxy)                                                                                  \
        return launch_wave3_case<T, TD, P, NW, PF, WPE, STG, true, false, C>(j, cf, cf2, alpha, chunk, s);  \
    else if (dz)                                                                                   \
        return launch_wave3_case<T, TD, P, NW, PF, WPE, STG, false, true, C>(j, cf, cf2, alpha, chunk, s);  \
    else                                                                                           \
        return launch_wave3_case<T, TD, P, NW, PF, WPE, STG, false, false, C>(j, cf, cf2, alpha, chunk, s)
    if (STG == 0 && j.residual) {
        LOPE_WAVE3_RULE(STG == 0);
    } else {
        LOPE_WAVE3_RULE(false);
    }
#undef LOPE_WAVE3_RULE
}

template <typename T, int TD, int P, int NW, int PF, int WPE>
hipError_t run_star3d_wave(const SweepJob& j, int chunk, hipStream_t s) {
    const Coef7<T> cf = coef7<T>(j);
    return launch_wave3<T, TD, P, NW, PF, WPE, 0>(j, cf, cf, (T)0, chunk, s);
}

// TD / 2 two-stage steps per pass (levels 1, 3, .. the first stencil; levels
// 2, 4, .. the second, plus alpha times the state at the start of the step)
template <typename T, int TD, int P, int NW, int PF, int WPE>
hipError_t run_star3d_wave_stages(const StageJob& sj, int chunk, hipStream_t s) {
    const Coef7<T> cf = coef7<T>(sj.s1), cf2 = coef7<T>(sj.s2);
    if (sj.alpha != 0.0) return launch_wave3<T, TD, P, NW, PF, WPE, 2>(sj.s1, cf, cf2, (T)sj.alpha, chunk, s);
    return launch_wave3<T, TD, P, NW, PF, WPE, 1>(sj.s1, cf, cf2, (T)0, chunk, s);
}

#define WSTAR(T, DT, TD, P, NW, PF, WPE, CH)                                                                \
    {"star3dw_" #T "_r1_t" #TD "_p" #P "_pf" #PF "_nw" #NW "_w" #WPE, FAM_STAR3D_WAVE, 3, 1, TD, DT, 0,       \
     64 - 2 * (TD), P, (NW) * 64, CH, &run_star3d_wave<T, TD, P, NW, PF, WPE>, 1,                           \
     &run_star3d_wave_stages<T, TD, P, NW, PF, WPE>}

// WPE: waves per SIMD asked of the register allocator (1 = no request);
// default z-chunk 0: the automatic (round-balanced) chunk of the launcher
const Variant kStar3dWave[] = {
    WSTAR(float, LOPE_F32, 4, 8, 4, 1, 2, 0),
    WSTAR(float, LOPE_F32, 4, 10, 4, 1, 2, 0),
    WSTAR(float, LOPE_F32, 4, 6, 4, 1, 2, 0),
};

}  // namespace

int star3d_wave_variants(const Variant** out) {
    *out = kStar3dWave;
    return (int)(sizeof(kStar3dWave) / sizeof(kStar3dWave[0]));
}

}  // namespace lope
