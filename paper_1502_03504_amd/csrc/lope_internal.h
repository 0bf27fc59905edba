// Internal declarations shared by the HIP kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lope.h"
#include "batch_queue.h"

namespace lope {

constexpr int kMaxTaps = LOPE_MAX_TAPS;
constexpr int kMaxR = LOPE_MAX_RADIUS;
constexpr int kNumXcd = 8;   // MI355X: workgroups are dealt round-robin over 8 XCDs

// Interior view of a padded grid (strides in elements; unused axes have n = 1).
struct DevGrid {
    void* origin;
    int64_t sy, sz;
    int32_t nx, ny, nz;
    int32_t pad;
};

// Boundary rule per paper axis: per[a] = 1 periodic, 0 Dirichlet.
struct DevRule {
    int32_t per[3];
    int32_t pad;
    double g;
};

// Non-zero taps in lexicographic offset order (x fastest) for the generic kernel.
template <typename T>
struct TapList {
    int32_t n;
    int32_t pad;
    int8_t off[kMaxTaps][3];
    T c[kMaxTaps];
};

// Everything a sweep launcher needs, fully validated by the ABI layer.
struct SweepJob {
    int ndim, radius, dtype;
    bool star;                      // only axis-aligned taps are non-zero
    DevGrid src, dst;
    DevRule rule;
    int ntaps;
    int8_t off[kMaxTaps][3];        // non-zero taps, lexicographic order
    double c[kMaxTaps];             // coefficients rounded to the grid dtype
    double dense[729];              // full (2r+1)^d table, rounded, x fastest
    double* residual;               // device, or null: variants with `res` merge into it the
                                    // max |last sweep - the sweep before| of their outputs
};

// ---- launchers (return hipSuccess or the launch error) ----
hipError_t launch_generic(const SweepJob& j, hipStream_t s);
// Fill the halo cells of g: lo[a] / hi[a] cells on the low / high side of axis a.
hipError_t launch_halo_fill(const DevGrid& g, const int lo[3], const int hi[3], int dtype, const DevRule& rule,
                            hipStream_t s);
hipError_t launch_accumulate(const DevGrid& part, int part_dtype, const DevGrid& total,
                             hipStream_t s);
// dL/dg of the adjoint (see lope_apply_adjoint) into *out, in a fixed order:
// per-workgroup sums into partials[0 .. min(blocks, kGbarPartials)), then one
// workgroup sums those (out may equal partials).
constexpr int kGbarPartials = LOPE_GBAR_DOUBLES;
hipError_t launch_gbar(const SweepJob& j, double* partials, double* out, hipStream_t s);
// *out (device) = max over the interior of |y - x| in float64 (x, y same extents)
hipError_t launch_residual_max(const DevGrid& x, const DevGrid& y, int dtype, double* out, hipStream_t s);
// *out (device) = +0.0, the identity of the residual maximum
hipError_t launch_residual_zero(double* out, hipStream_t s);

// Streaming copy of `bytes` (a multiple of 16; 16-byte aligned pointers).
hipError_t launch_copy16(const void* src, void* dst, int64_t bytes, hipStream_t s);

// Tuned kernel families.
enum Family {
    FAM_GENERIC = 0,
    FAM_STAR3D = 1,
    FAM_PLANE2D = 2,
    FAM_STAR3D_VEC = 3,
    FAM_STAR3D_FLAT = 4,
    FAM_STAR3D_WAVE = 5
};

typedef hipError_t (*VariantFn)(const SweepJob& j, int chunk, hipStream_t s);

// Two local-element functions per step: s1 holds the grids, the rule and the
// first stencil; s2 the second stencil (its grids and rule are s1's).
struct StageJob {
    SweepJob s1, s2;
    double alpha;   // rounded to the grid dtype
};
typedef hipError_t (*StageFn)(const StageJob& j, int chunk, hipStream_t s);
// One thread per point, both stencils from tap lists (<= kStageTaps each).
constexpr int kStageTaps = 64;
hipError_t launch_stages_generic(const StageJob& j, hipStream_t s);

struct Variant {
    const char* name;
    int family;
    int ndim, radius, tdepth, dtype;
    int box;                        // plane2d: 1 = box taps, 0 = star taps
    int bx, by, nt;                 // output tile (x, y) and threads per workgroup
    int default_chunk;
    VariantFn fn;
    int res;                        // 1: honours SweepJob::residual
    StageFn sfn;                    // tdepth / 2 two-stage steps in one pass, or null
};

// Registries filled by each kernel file.
int star3d_variants(const Variant** out);
int star3d_flat_variants(const Variant** out);
int star3d_wave_variants(const Variant** out);
int star3d_vec_variants(const Variant** out);
int plane2d_variants(const Variant** out);
int plane2d_wave_variants(const Variant** out);

// Variable-coefficient diffusion.
hipError_t launch_var_forward(const DevGrid& src, const DevGrid& dst, const DevGrid& kappa,
                              int dtype, double dt, hipStream_t s);
hipError_t launch_var_adjoint(const DevGrid& lam_next, const DevGrid& lam, const DevGrid& u,
                              const DevGrid& kappa, const DevGrid& gk, int dtype, int gk_dtype,
                              double dt, hipStream_t s);

// The same two steps with one wavefront per brick (64 columns, all outputs),
// for grids whose planes hold fewer than 2^31 bytes (var_wave_fits); the
// arithmetic per point is the same chain of fmas as the kernels above.
bool var_wave_fits(const DevGrid& g, int esize);
// The fused pair's wave kernel also needs its four inputs (lam'', u_t,
// u_{t-1}, kappa) laid out alike: one row table addresses them.
bool var_pair_wave_fits(const DevGrid& a, const DevGrid& b, const DevGrid& c, const DevGrid& d, int esize);
hipError_t launch_var_forward_wave(const DevGrid& src, const DevGrid& dst, const DevGrid& kappa, int dtype, double dt,
                                   hipStream_t s);
hipError_t launch_var_adjoint_wave(const DevGrid& lam_next, const DevGrid& lam, const DevGrid& u, const DevGrid& kappa,
                                   const DevGrid& gk, int dtype, int gk_dtype, double dt, hipStream_t s);
hipError_t launch_var_adjoint2_wave(const DevGrid& lam_next, const DevGrid& lam, const DevGrid& ut,
                                    const DevGrid& utm1, const DevGrid& kappa, const DevGrid& gk, int dtype,
                                    int gk_dtype, double dt, hipStream_t s);

// Two fused reverse steps: lam_{t-1} from lam_{t+1}, both kappa terms in one update.
hipError_t launch_var_adjoint2(const DevGrid& lam_next, const DevGrid& lam_out, const DevGrid& u_t,
                               const DevGrid& u_tm1, const DevGrid& kappa, const DevGrid& gk, int dtype,
                               int gk_dtype, double dt, hipStream_t s);

// Batched persistent sweeps (tables built by the ABI layer, read by the kernel).
struct BatchGrid {
    DevGrid src, dst;
    DevRule rule;
    double c[9];          // dense 3x3 table, rounded to the grid dtype, x fastest
    int32_t box;          // 1: all 9 taps; 0: the 5 star taps
    int32_t pad[3];
};

// One strip of one grid, swept by one wave: output columns
// [x0, x0 + batch_strip_width(tdepth)), rows [y0, y1).
struct BatchItem {
    int32_t grid;
    int32_t x0, y0, y1;
};

// Sweeps per batch pass: 1 .. kBatchMaxDepth.
constexpr int kBatchMaxDepth = 8;
// Output columns of a batch strip sweeping tdepth times per pass.
int batch_strip_width(int tdepth);
// One pass of tdepth sweeps over every listed tile; parity 0 reads src, 1 reads dst.
hipError_t launch_batch_pass(const BatchGrid* grids, const BatchItem* items, int nitems, int tdepth, int parity,
                             int dtype, hipStream_t s);

// State of the persistent batched launch (one per plan, zeroed at creation;
// the kernel's last wave leaves the queue counters, left and abort at zero
// again).  Each queue counter has a 128-byte line of its own.
struct PqCounter {
    unsigned long long next;   // next unit of the queue to hand out
    unsigned long long pad[15];
};
struct PqState {
    PqCounter queue[kPqMaxQueues];
    unsigned int left;         // waves that have left the loop
    unsigned int abort;        // set when a wait ran out of time: every wave leaves
    unsigned int timeouts;     // waits that ran out (kept; the host reads and clears it)
    unsigned int pad[29];
    PqQueue share[kPqMaxQueues];   // each queue's strips (set by the host)
};
// Per grid: strips completed in the running launch (reset by the last wave)
// and the grid's strips in the full-depth table (set by the host).
struct PqGrid {
    unsigned int done;
    int32_t full_strips;
};
// Every pass of a batch in one launch of the persistent kernel: `shape.full`
// passes of tdepth sweeps over full_items, then (rem > 0) one pass of rem
// sweeps over rem_items; `units` is the total over the queues.  wait_us bounds each dependency wait (0: a wait
// not met at its first poll runs out).
hipError_t launch_batch_persistent(const BatchGrid* grids, const BatchItem* full_items, const BatchItem* rem_items,
                                   const PqShape& shape, int64_t units, int tdepth, int rem, PqState* st,
                                   PqGrid* pg, int ngrids, long long wait_us, int dtype, hipStream_t s);

// ---- device helpers ----
__device__ __forceinline__ int wrap_index(int i, int n) {
    if ((unsigned)i < (unsigned)n) return i;
    int m = i % n;
    return m < 0 ? m + n : m;
}

// Maximum that propagates NaN (a NaN operand wins and stays).
__device__ __forceinline__ double nan_max(double a, double b) { return (b > a || b != b) ? b : a; }

// Merge a per-lane maximum of non-negative doubles (or NaN) into *out: a
// reduction across the wave, then one 64-bit unsigned atomic max per wave on
// the bit pattern (non-negative doubles and the positive NaN order like their
// bits).  Every lane of the wave must call it.
__device__ __forceinline__ void residual_merge(double m, double* out) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = nan_max(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0)
        atomicMax(reinterpret_cast<unsigned long long*>(out), (unsigned long long)__double_as_longlong(m));
}

// Barrier that orders LDS traffic only: outstanding global loads (prefetches)
// stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    __asm__ volatile("" ::: "memory");
}

// Logical block id from the hardware id so that consecutive logical tiles
// share an XCD (and its L2): XCD x gets the logical range [x*per, (x+1)*per).
__device__ __forceinline__ int xcd_logical_block(int nblocks_padded) {
    const int per = nblocks_padded / kNumXcd;
    const int b = blockIdx.x;
    return (b % kNumXcd) * per + b / kNumXcd;
}

inline int padded_block_count(int nblocks) {
    return ((nblocks + kNumXcd - 1) / kNumXcd) * kNumXcd;
}

// Compute units of the current device (queried once per device; 256 on
// MI355X if the query fails).
int device_cu_count();

// Workgroups of `kernel` (block_threads threads, no dynamic LDS) that one
// compute unit holds at once, from the compiled register and LDS use (1 if
// the query fails).
template <typename K>
inline int blocks_per_cu(K kernel, int block_threads) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, block_threads, 0) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        n = 1;
    }
    return n;
}

// Marching kernels split each column of tiles into k z-chunks of
// ceil(nz / k) planes; the launch then runs in ceil(ncols * k / slots)
// rounds of resident waves, each round costing a chunk plus `warm` march
// steps of start-up.  Returns the chunk (at least min_chunk, which bounds
// the re-read planes per chunk) of the k that minimises
// rounds * (chunk + warm), the smallest such chunk on ties.
inline int balanced_chunk(int64_t ncols, int nz, int64_t slots, int warm, int min_chunk) {
    if (nz <= 1 || ncols <= 0 || slots <= 0) return nz > 0 ? nz : 1;
    int best_chunk = nz;
    int64_t best_cost = -1;
    auto consider_chunk = [&](int chunk) {
        if (chunk < 1 || chunk > nz || (chunk < min_chunk && chunk < nz)) return;
        const int64_t kk = (nz + chunk - 1) / chunk;   // chunks actually made
        const int64_t rounds = (ncols * kk + slots - 1) / slots;
        const int64_t cost = rounds * (chunk + warm);
        if (best_cost < 0 || cost < best_cost || (cost == best_cost && chunk < best_chunk)) {
            best_cost = cost;
            best_chunk = chunk;
        }
    };
    auto consider = [&](int64_t k) {
        if (k >= 1 && k <= nz) consider_chunk((int)((nz + k - 1) / k));
    };
    // the even cuts into k chunks for every small k and for the k that fill
    // one to eight whole rounds (tall columns on few tiles need more than
    // 512 chunks), and the shortest admissible chunk (the best one wherever
    // the even cut would fall below the minimum)
    for (int k = 1; k <= 512; ++k) consider(k);
    for (int64_t m = 1; m <= 8; ++m) consider(m * slots / ncols);
    consider_chunk(min_chunk);
    return best_chunk;
}

}  // namespace lope
