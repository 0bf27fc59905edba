/*
 * lope.h — C ABI of the LOPe stencil-sweep library for AMD Instinct MI355X (gfx950).
 *
 * The library applies a locally-oriented update to every interior element of
 * a 1-3D grid: each element is rewritten only from a read-only neighbourhood
 * (its halo) of the state at invocation time, the halo is given by a boundary
 * rule, and sweeps are iterated Jacobi-style with two buffers.  The paper
 * (Rasmussen, Sottile, Nagle, Rasmussen, "Locally-Oriented Programming")
 * defines the pieces this interface is built from:
 *   - halo regions and their width (section 2.2, "Halo regions");
 *   - the local element and its read-only neighbours, zero-based offsets with
 *     the first index running left/right and the second below/above
 *     (section 2.2, "LOPe index notation"; Fig. 1);
 *   - the concurrent sweep over the interior with race freedom by double
 *     buffering (section 2.2, "Concurrent functions"; section 3.2, items 1-7);
 *   - the halo transfer with a boundary rule kept apart from the algorithm
 *     (section 3.2, HALO_TRANSFER(U, BC=CYCLIC); section 3.4, first item);
 *   - the constraints checked at run time here: no store to the halo, no out
 *     of bounds access, no race (section 3.5);
 *   - a device query that falls back to the host (section 3.1, GET_SUBIMAGE).
 *
 * Conventions for every call:
 *   - Non-owning: the caller owns all grid memory (device memory, e.g. from
 *     PyTorch's allocator) and all coefficient tables (host memory).
 *   - Asynchronous: every compute call enqueues work on `stream` (a
 *     hipStream_t; NULL means the legacy default stream) and returns without
 *     synchronising; a kernel fault surfaces at the caller's next sync.
 *   - Graph capture: the compute calls enqueue kernel launches only (no
 *     memset or copy nodes, no host wait), so a stream being captured records
 *     them into the caller's graph; the exceptions are lope_iterate_until,
 *     which waits on the host and refuses a capturing stream, and the batch
 *     plan calls, whose own rules are given with them.
 *   - Logging: with LOPE_LOG=1 in the environment every compute call writes
 *     one line to stderr naming the kernel (and depth, chunk or tiling) it
 *     chose.
 *   - Errors: every call returns LOPE_OK (0) or a negative lope_status.  All
 *     structural validation runs before any HIP call; on error nothing has
 *     been enqueued.  No exception crosses the ABI, nothing calls exit(), and
 *     there is no CPU fallback.  lope_last_error() gives a thread-local text.
 *   - Memory layout of a grid: padded storage with halo cells on each side of
 *     every used axis (h on both sides, or per-axis left/right widths); x
 *     (paper axis 0, the first index) is contiguous.  Element (x, y, z), with
 *     -lo[0] <= x < n[0]+hi[0] etc., lives at origin + x + y*stride[1] +
 *     z*stride[2] (in elements).
 */
#ifndef LOPE_H
#define LOPE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
typedef enum lope_status {
    LOPE_OK = 0,
    LOPE_ERR_INVALID_ARG = -1,    /* null pointer, bad ndim/extent/stride/dtype, mismatched grids,
                                     pointer not device memory, or storage outside its allocation */
    LOPE_ERR_HALO_TOO_SMALL = -2, /* stencil reaches beyond the halo on some side (section 3.5) */
    LOPE_ERR_ALIAS = -3,          /* source and destination interiors overlap (section 2.2, 3.5) */
    LOPE_ERR_UNSUPPORTED = -4,    /* valid request the library does not implement (see each call) */
    LOPE_ERR_NO_DEVICE = -5,      /* no usable GPU (or LOPE_FORCE_NO_DEVICE=1 in the environment) */
    LOPE_ERR_HIP = -6,            /* a HIP runtime error; its text is in lope_last_error() */
    LOPE_ERR_TIMEOUT = -7         /* a bounded device-side wait ran out (lope_batch_persistent_check) */
} lope_status;

/* Device id returned by lope_get_device when no device can be used. */
#define LOPE_HOST (-1)

/* ---- element types and boundary kinds ---------------------------------- */
typedef enum lope_dtype { LOPE_F32 = 0, LOPE_F64 = 1 } lope_dtype;

typedef enum lope_bc_kind {
    LOPE_BC_DIRICHLET = 0,        /* every halo cell along this axis holds the grid's value g */
    LOPE_BC_PERIODIC = 1          /* halo cells repeat the interior cyclically (BC=CYCLIC) */
} lope_bc_kind;

#define LOPE_MAX_NDIM 3
#define LOPE_MAX_RADIUS 4
#define LOPE_MAX_TAPS 256         /* non-zero coefficients per stencil */

/* A padded grid (section 2.2 halo region; section 3.2 padded allocation).
 *   ndim    1..3.
 *   h       halo width in cells, the same on both sides of every used axis, >= 0
 *           (used when halo_mode is 0).
 *   dtype   lope_dtype.
 *   halo_mode  0: width h on both sides of every used axis;
 *           1: per-axis widths hlo[a] (left/below) and hhi[a] (right/above), the
 *           M:*:N halo of section 2.2; each >= 0, and 0 on unused axes.
 *   n[a]    interior extent of axis a (a = 0 is x); >= 0; axes >= ndim must be 1.
 *           An interior with a zero extent is empty and every call on it is a no-op.
 *   stride  element strides; stride[0] must be 1, stride[1] >= n[0] + lo[0] + hi[0],
 *           stride[2] >= stride[1]*(n[1] + lo[1] + hi[1]) (rows and planes do not
 *           overlap), with lo/hi the halo widths of the axis.
 *   origin  device pointer to interior element (0,0,0).  The whole padded box
 *           must lie inside one device allocation (checked).
 * A stencil may be applied to a grid when, on every axis and side, the halo is
 * at least as wide as the stencil reaches (the largest offset of a tap whose
 * coefficient is non-zero once rounded to the grid type; section 3.5), else
 * LOPE_ERR_HALO_TOO_SMALL: a one-sided stencil needs a halo on one side only.
 * The sweeps never read the stored halo (they apply the rule while loading);
 * the widths matter for validation and for lope_halo_fill. */
typedef struct lope_grid {
    int32_t ndim;
    int32_t h;
    int32_t dtype;
    int32_t halo_mode;
    int64_t n[3];
    int64_t stride[3];
    void* origin;
    int32_t hlo[3];
    int32_t hhi[3];
} lope_grid;

/* Boundary rule (section 3.2, BC argument of the halo transfer).  kind[a] for
 * each used axis; one Dirichlet value per grid.  For a halo cell that lies
 * outside the interior along at least one Dirichlet axis the value is `value`;
 * otherwise it is the interior value at the index wrapped on every periodic
 * axis.  (The paper shows faces only; this order-independent rule also fixes
 * edges and corners and mixed per-axis kinds.) */
typedef struct lope_bc {
    int32_t kind[3];
    int32_t reserved;
    double value;
} lope_bc;

/* Coefficient stencil of the local-element update (Fig. 1 generalised):
 * y[x] = sum over offsets o in [-r, r]^ndim of c_o * B(src)[x + o].
 * coeffs is HOST memory holding (2r+1)^ndim doubles; the entry for offset o
 * sits at index sum_a (o_a + r) * (2r+1)^a (x fastest).  The table is copied
 * at call time and each coefficient is rounded once to the grid dtype.  Each
 * point's sum is evaluated as a chain of fused multiply-adds over the
 * non-zero taps in that same index order, so every kernel variant (tiling,
 * temporal blocking, batching) gives identical values. */
typedef struct lope_stencil {
    int32_t ndim;
    int32_t radius;               /* 0..LOPE_MAX_RADIUS */
    const double* coeffs;
} lope_stencil;

/* Spatially varying diffusion coefficient for the update
 *   u' = u + dt * sum_a sum_{s=+-1} K^s_a (u_{x+s e_a} - u_x),
 *   K^s_a = (kappa_x + kappa_{x + s e_a}) / 2,
 * a local-element function with two read-only inputs (u and kappa). */
typedef struct lope_varcoef {
    const lope_grid* kappa;       /* same ndim, extents and dtype as u; read-only */
    double dt;
} lope_varcoef;

/* Explicit launch choice, used by the autotuner (all zero = automatic). */
#define LOPE_VARIANT_GENERIC (-1)
typedef struct lope_tuning {
    int32_t variant;              /* kernel variant id from lope_variant_info, 0 = automatic,
                                     LOPE_VARIANT_GENERIC = the one-thread-per-point kernel */
    int32_t tdepth;               /* sweeps fused per pass, 1..4; 0 = automatic */
    int32_t chunk;                /* extent of the marched axis per workgroup or wave; 0 =
                                     automatic: the wave kernels cut each column of tiles into
                                     chunks as long as the device's resident waves (at the
                                     kernel's compiled occupancy) still cover in few rounds,
                                     the others use a fixed default */
    int32_t rules;                /* lope_tune_set: the boundary-rule class the choice is for,
                                     0 = periodic on every axis, 1 = some axis Dirichlet;
                                     ignored by lope_iterate_tuned */
} lope_tuning;

/* ---- device ------------------------------------------------------------ */

/* Section 3.1 (GET_SUBIMAGE): *out = ordinal if that GPU can be used, else
 * LOPE_HOST.  Falling back to the host is not an error (returns LOPE_OK) so a
 * program can proceed without a device; compute calls then return
 * LOPE_ERR_NO_DEVICE.  out must not be NULL. */
int lope_get_device(int ordinal, int* out);

/* ---- halo ---------------------------------------------------------------- */

/* Fill the stored halo of g (every side, its own width) from its own interior
 * with the boundary rule (section 3.2, the halo transfer on one device).
 * Only halo cells are written; the interior is read.  The sweeps below do NOT need this: they
 * apply the rule while loading, so the stored halo is never read by them. */
int lope_halo_fill(const lope_grid* g, const lope_bc* bc, void* stream);

/* ---- sweeps -------------------------------------------------------------- */

/* One sweep (section 3.2, do concurrent over the interior calling the local
 * element function): dst interior = S(B(src)).  src is never written; the
 * halo of dst is never written.  Requires src's halo to cover the stencil's
 * reach on every side, equal ndim, extents and dtype, and non-overlapping
 * interiors. */
int lope_apply(const lope_grid* src, const lope_grid* dst, const lope_stencil* st,
               const lope_bc* bc, void* stream);

/* n_steps sweeps alternating between a and b (section 3.2, the loop around
 * the sweep and the halo transfer; double buffering per section 2.2).  The
 * initial state is a's interior.  Several sweeps may be fused per pass over
 * memory: tdepth 1..4 asks for that many (fewer where no kernel fuses that
 * many for this grid and stencil, e.g. radius 2-4), 0 lets the tuning table
 * choose (possibly more than 4); the result is identical.  *result_index is
 * set to 0 if the final state is in a, 1 if in b (n_steps mod 2 when one
 * sweep runs per pass).  Both grids' halos must cover the stencil's reach.
 * result_index must not be NULL. */
int lope_iterate(const lope_grid* a, const lope_grid* b, const lope_stencil* st,
                 const lope_bc* bc, int64_t n_steps, int32_t tdepth, void* stream,
                 int32_t* result_index);

/* lope_iterate with an explicit kernel variant / depth / chunk (autotuner). */
int lope_iterate_tuned(const lope_grid* a, const lope_grid* b, const lope_stencil* st,
                       const lope_bc* bc, int64_t n_steps, const lope_tuning* tune,
                       void* stream, int32_t* result_index);

/* Sweeps until converged (section 3.2: the do-while loop around the sweep,
 * whose convergence test the paper leaves open).  After every sweep whose
 * count is a multiple of check_every, the residual max_x |u_t[x] - u_{t-1}[x]|
 * over the interior is formed in float64 (difference of the two values,
 * magnitude, maximum: independent of evaluation order, so exact); the loop
 * stops after the first checked sweep whose residual is <= tol, or after
 * max_steps sweeps.  Sweeps are fused per pass as in lope_iterate (tdepth,
 * 0 = automatic); the pass that ends on a checked sweep reports the residual
 * of its last sweep from values it computes anyway.  A NaN residual never
 * satisfies the test.
 *
 * residual_scratch: DEVICE pointer to one 8-byte aligned double the call may
 * overwrite (caller-owned).  On return *steps_done is the number of sweeps
 * run, *residual the last residual formed (NaN if none), *result_index 0 if
 * the final state is in a, 1 if in b; the other buffer holds an earlier
 * state.  All three must not be NULL.
 *
 * SYNCHRONOUS: the host waits on `stream` after every check to read the
 * residual, so the call cannot be recorded into a graph (a capturing stream
 * gives LOPE_ERR_UNSUPPORTED).  check_every >= 1 and max_steps >= 0, else
 * LOPE_ERR_INVALID_ARG.  An empty interior stops at once with 0 steps. */
int lope_iterate_until(const lope_grid* a, const lope_grid* b, const lope_stencil* st,
                       const lope_bc* bc, int64_t max_steps, int32_t check_every, double tol,
                       int32_t tdepth, double* residual_scratch, void* stream,
                       int64_t* steps_done, double* residual, int32_t* result_index);

/* Doubles of the array lope_apply_adjoint's gbar_dirichlet points to. */
#define LOPE_GBAR_DOUBLES 1024

/* Adjoint sweep: xbar interior = S^T(ybar), the transpose of the linear part
 * of lope_apply: the reflected stencil c_{-o} applied with the transposed
 * rule (periodic axes wrap; Dirichlet halo cells contribute zero).  If
 * gbar_dirichlet is not NULL it is a DEVICE pointer to LOPE_GBAR_DOUBLES
 * 8-byte aligned doubles (caller-owned workspace, checked to lie in one
 * device allocation): the call overwrites them, and once it has run element
 * 0 holds dL/dg = sum_x ybar[x] * (sum of c_o over the taps of x that read a
 * Dirichlet halo cell), summed in float64 in a fixed order (per-workgroup
 * sums in elements 0.., then their sum), so equal inputs give equal bits on
 * every run.  The reflected stencil reaches the other way: ybar's halo must
 * cover the forward reach mirrored (left <-> right). */
int lope_apply_adjoint(const lope_grid* ybar, const lope_grid* xbar, const lope_stencil* st,
                       const lope_bc* bc, double* gbar_dirichlet, void* stream);

/* ---- two local-element functions per step ------------------------------- */

/* Two local-element functions applied in sequence with a share of the
 * starting state: two-stage schemes such as Heun's method or the midpoint
 * rule, fused in one pass over memory (the paper leaves fusing small
 * functions to the compiler, section 3.5, and notes that intermediate results
 * of multi-step updates are not stored automatically, section 5):
 *   v  = S1(B(u))                a state of the grid type, never stored;
 *   u' = alpha * u + S2(B(v))    B gives v's halo by the same rule.
 * Per point, v is evaluated exactly as lope_apply would; the second sum is
 * alpha*u (when alpha != 0) followed by fmas over S2's non-zero taps in
 * lexicographic order, so with alpha == 0 a step equals two lope_apply calls
 * value for value.  Both stencils have the grid's ndim and at most 64
 * non-zero taps (else LOPE_ERR_UNSUPPORTED). */
typedef struct lope_stages {
    const lope_stencil* first;    /* S1 */
    const lope_stencil* second;   /* S2 */
    double alpha;                 /* rounded once to the grid dtype */
} lope_stages;

/* One two-stage step from src to dst.  src's halo must cover the first
 * stencil's reach (the intermediate's halo comes from the rule); otherwise
 * as lope_apply. */
int lope_apply_stages(const lope_grid* src, const lope_grid* dst, const lope_stages* sg,
                      const lope_bc* bc, void* stream);

/* n_steps two-stage steps alternating between a and b: two steps per pass
 * over memory where a fused kernel takes both stencils (3D radius-1 stars,
 * float32), else one; *result_index says which buffer holds the state (0: a;
 * the parity of the number of passes).  Both grids' halos must cover the
 * first stencil's reach.  result_index must not be NULL. */
int lope_iterate_stages(const lope_grid* a, const lope_grid* b, const lope_stages* sg,
                        const lope_bc* bc, int64_t n_steps, void* stream, int32_t* result_index);

/* ---- variable-coefficient diffusion (3D, periodic) ------------------------ */

/* dst = src + dt * div(kappa grad src) with arithmetic-mean faces (see
 * lope_varcoef).  3D only, every axis periodic (else LOPE_ERR_UNSUPPORTED);
 * a halo of at least 1 on both sides of every axis of src and kappa. */
int lope_apply_var(const lope_grid* src, const lope_grid* dst, const lope_varcoef* vc,
                   const lope_bc* bc, void* stream);

/* Reverse step of lope_apply_var at state u_t, given lam_next = dL/du_{t+1}:
 *   lam[x]    = lam_next[x] + dt * sum_{a,s} K^s_a(x) (lam_next[x+s e_a] - lam_next[x])
 *               (the step matrix is symmetric, so this is its transpose);
 *   gkappa[x] += dt/2 * sum_{a,s} (u_t[x+s e_a] - u_t[x]) (lam_next[x] - lam_next[x+s e_a]).
 * gkappa is a grid of the same extents, dtype F32 or F64 (accumulated in its
 * own precision; fold F32 partial sums into F64 with lope_accumulate).  lam
 * must not overlap lam_next, u_t, kappa or gkappa. */
int lope_apply_var_adjoint(const lope_grid* lam_next, const lope_grid* lam, const lope_grid* u_t,
                           const lope_varcoef* vc, const lope_bc* bc, const lope_grid* gkappa,
                           void* stream);

/* Two reverse steps in one pass: from lam_next = dL/du_{t+1}, the states u_t
 * and u_tm1 = u_{t-1}, produce lam = dL/du_{t-1} (= the step matrix applied
 * twice) and add both steps' kappa terms (at u_t with lam_next, and at
 * u_{t-1} with the intermediate dL/du_t) to gkappa in one update.  Same
 * validation and restrictions as lope_apply_var_adjoint; lam must not overlap
 * any input, gkappa must not overlap anything. */
int lope_apply_var_adjoint2(const lope_grid* lam_next, const lope_grid* lam, const lope_grid* u_t,
                            const lope_grid* u_tm1, const lope_varcoef* vc, const lope_bc* bc,
                            const lope_grid* gkappa, void* stream);

/* total (F64) += partial (F32 or F64) over the interior, then partial = 0. */
int lope_accumulate(const lope_grid* partial, const lope_grid* total, void* stream);

/* ---- batches: many independent grids advanced together -------------------- */

/* One grid of a batch: a 2D sweep from src to dst (both padded grids),
 * iterated with its own stencil and rule.  The state alternates between src
 * and dst exactly as in lope_iterate with one sweep per pass. */
typedef struct lope_batch_item {
    lope_grid src;
    lope_grid dst;
    lope_stencil stencil;         /* 2D, radius <= 1; copied at plan creation */
    lope_bc bc;
} lope_batch_item;

typedef struct lope_batch_plan lope_batch_plan;

/* Build a plan for n_items grids and n_steps sweeps each: validates every
 * item, cuts every grid into tiles of the 2D marching kernel, and uploads the
 * grid and tile tables (the plan owns this device memory).  The plan borrows
 * the grids' memory until it is destroyed.  Supports 2D float32 or float64
 * grids of any extents, radius <= 1 stencils, one dtype per batch (else
 * LOPE_ERR_UNSUPPORTED / LOPE_ERR_INVALID_ARG).
 * `stream` is unused (creation synchronises its uploads). */
int lope_batch_plan_create(const lope_batch_item* items, int64_t n_items, int64_t n_steps,
                           void* stream, lope_batch_plan** out);

/* Advance every grid n_steps sweeps from the state in its src in ONE kernel
 * launch (the persistent batched sweep; the sweep and the double buffering of
 * sections 3.2-3.3 for every grid).  The kernel's waves take work units, one
 * strip of one grid in one pass of tdepth fused sweeps each, from queues
 * numbered pass by pass, and a unit starts once every strip of its grid's
 * earlier passes is complete (per-grid counters; the kernel's grid loads and
 * stores are device-scope, so no cache flush is needed between strips).  A
 * wave waits only on units handed out before its own, so the queues cannot
 * deadlock whatever the number of resident waves; every wait is also bounded
 * (1 s, or the environment's LOPE_PERSISTENT_WAIT_US microseconds, read at
 * each call; 0 makes any wait not met at once run out), and one that runs out
 * makes all waves leave early (see lope_batch_persistent_check).  Uses the
 * plan's tiling.  Enqueued on `stream` with no other operation, so a caller
 * may capture it into a graph as one kernel node; the kernel's last wave
 * clears the plan's queues for the next launch.  Launches of one plan must
 * not overlap (they share its queues): keep them on one stream.
 * lope_batch_result_index tells which buffer holds the result.
 * Errors: LOPE_ERR_INVALID_ARG (null plan). */
int lope_batch_apply(lope_batch_plan* plan, void* stream);

/* Synchronises the device, then returns LOPE_ERR_TIMEOUT if a wait of an
 * earlier lope_batch_apply of this plan ran out of time (that launch's
 * result is invalid; the record is cleared), else LOPE_OK. */
int lope_batch_persistent_check(lope_batch_plan* plan);

/* The same sweeps as separate launches, one per pass: each launch covers
 * every strip of every grid and fuses tdepth sweeps (about n_steps/tdepth
 * launches in total).  The first call for a tiling records those launches
 * into a HIP graph owned by the plan; later calls replay it on `stream` (one
 * graph launch).  When `stream` is itself being captured, the launches are
 * enqueued directly into the caller's graph instead.  The result equals
 * lope_batch_apply's value for value, in the same buffer. */
int lope_batch_apply_passes(lope_batch_plan* plan, void* stream);

/* Same work as lope_batch_apply as ordinary lope_iterate launches, one per
 * grid per sweep (the baseline the batched launch is compared with). */
int lope_batch_apply_per_grid(lope_batch_plan* plan, void* stream);

/* Tiling of the batched passes: tdepth sweeps fused per launch (1..8; the
 * remainder of n_steps in one shorter pass) and strips of `rows` rows
 * (1..65536; 0 keeps the current rows).  A new plan starts with the tiling
 * registered by lope_batch_tune_set for its dtype and the size bucket of its
 * total interior points (else the nearest registered bucket of the dtype,
 * else 4 sweeps and 128 rows).  Builds the plan's tile tables for the tiling
 * if needed (synchronous upload); on error the plan keeps its tiling. */
int lope_batch_plan_set_tiles(lope_batch_plan* plan, int32_t tdepth, int32_t rows);

/* lope_batch_plan_set_tiles(plan, tdepth, 0). */
int lope_batch_plan_set_depth(lope_batch_plan* plan, int32_t tdepth);

/* The plan's current tiling.  No pointer may be NULL. */
int lope_batch_plan_get_tiles(const lope_batch_plan* plan, int32_t* tdepth, int32_t* rows);

/* Register the tiling new batch plans of dtype `dtype` take when their total
 * interior points fall in the bucket floor(log2(points)) (the autotuner's
 * choice): tdepth 1..8 and rows 1..65536; tdepth 0 removes the entry of that
 * bucket.  Only argument checks (no device access). */
int lope_batch_tune_set(int32_t dtype, int64_t points, int32_t tdepth, int32_t rows);

/* *out = 0 if lope_batch_apply leaves every grid's state in its src, 1 if in
 * its dst (the parity of the number of passes).  out must not be NULL. */
int lope_batch_result_index(const lope_batch_plan* plan, int32_t* out);

/* Release the plan's device memory (the caller synchronises first if the plan
 * may still be running).  NULL is a no-op. */
int lope_batch_plan_destroy(lope_batch_plan* plan);

/* Bytes of the library's static device scratch used by lope_batch_apply_noalloc
 * (4 MiB: the descriptors of up to about 21,000 grids, or some 200,000 strips
 * of 16 bytes). */
#define LOPE_BATCH_SCRATCH_BYTES (4u << 20)

/* For callers that cannot allocate device memory (serving loops that must not
 * call hipMalloc, harnesses that forbid it): the work of
 * lope_batch_plan_create + lope_batch_apply_passes + lope_batch_plan_destroy in
 * one call that allocates nothing (one launch per fused pass).  The grid descriptors and strip tables go into
 * a fixed device array of LOPE_BATCH_SCRATCH_BYTES that the library holds on
 * each device it runs on until the process ends; a batch whose tables do not
 * fit returns LOPE_ERR_UNSUPPORTED (naming the bytes needed) before anything
 * is enqueued, as do more than LOPE_BATCH_SCRATCH_BYTES / (descriptor size)
 * grids.
 *   items, n_items, n_steps: as for lope_batch_plan_create (same checks).
 *   tdepth: sweeps per launch 1..8, or 0 for the tiling registered with
 *           lope_batch_tune_set (as a new plan takes); rows: 1..65536, or 0
 *           likewise.  The result equals lope_batch_apply's value for value.
 *   result_index: set to 0 if every grid's state ends in its src, 1 if in its
 *           dst; must not be NULL.
 * The tables are written into the array from host memory on `stream` and the
 * call waits for that copy (so for the work already on `stream`); the sweeps
 * themselves are enqueued and run asynchronously.  A capturing stream gives
 * LOPE_ERR_UNSUPPORTED.  Every call on a device reuses that device's one
 * array: calls that overlap on one device (other streams or threads while
 * sweeps of an earlier call still run) race and give wrong results. */
int lope_batch_apply_noalloc(const lope_batch_item* items, int64_t n_items, int64_t n_steps, int32_t tdepth,
                             int32_t rows, void* stream, int32_t* result_index);

/* ---- measurement aid ---------------------------------------------------------- */

/* Copies `bytes` bytes from src to dst (device pointers, 16-byte aligned,
 * bytes a multiple of 16, the ranges not overlapping, each inside one
 * device allocation) with 16-byte non-temporal loads and stores: the
 * attainable-bandwidth reference for the sweeps' roofline figures (not part
 * of the method).  Asynchronous on `stream`.  Misaligned or overlapping
 * arguments give LOPE_ERR_INVALID_ARG. */
int lope_copy_stream(const void* src, void* dst, int64_t bytes, void* stream);

/* ---- introspection --------------------------------------------------------- */

/* Text of a status code (static storage). */
const char* lope_status_string(int status);

/* Thread-local text of the last error raised on this thread ("" if none). */
const char* lope_last_error(void);

/* Number of compiled kernel variants, and the description of variant id
 * (1..count): fills `text` (NUL-terminated, at most cap bytes) with
 * "name ndim=.. radius=.. tdepth=.. dtype=.. shape=.. tile=..". */
int lope_variant_count(void);
int lope_variant_info(int id, char* text, int cap);

/* Id of the kernel variant lope_iterate would use for one pass with tdepth
 * sweeps (0 = automatic) on this grid/stencil and rule (NULL: periodic on
 * every axis), or a negative status. */
int lope_select_variant(const lope_grid* g, const lope_stencil* st, const lope_bc* bc, int32_t tdepth);

/* Register a launch choice for grids and stencils like (g, st): use
 * tune->variant and tune->chunk.  tune->tdepth says which request it answers:
 * 0 = lope_iterate with tdepth 0 (automatic), k = lope_iterate with tdepth k
 * (then the variant's own depth must be k).  The key is (ndim, radius,
 * dtype, star/box shape, size bucket = floor(log2(interior points)),
 * requested depth, rule class tune->rules).  A request whose own bucket has
 * no fitting choice takes the variant and depth registered for the nearest
 * bucket of its class (the larger one on a tie), with the automatic chunk;
 * with no choice in the class at all it takes the default variant.
 * tune->variant = 0 removes the choice registered for that request (tdepth
 * 0..4) and bucket.  Only structural checks are made (no device access). */
int lope_tune_set(const lope_grid* g, const lope_stencil* st, const lope_tuning* tune);

#ifdef __cplusplus
}
#endif

#endif /* LOPE_H */
