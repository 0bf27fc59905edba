// C ABI: argument validation (the run-time form of the paper's section 3.5
// constraints), kernel selection, ping-pong iteration, tuning table.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cstddef>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "lope_internal.h"

using namespace lope;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(LOPE_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t elem_size(int dtype) { return dtype == LOPE_F64 ? 8 : 4; }

// ---- structural checks (no HIP calls) ----
// Halo widths of axis a on the low (left/below) and high (right/above) side.
int halo_lo(const lope_grid* g, int a) { return a >= g->ndim ? 0 : (g->halo_mode ? g->hlo[a] : g->h); }
int halo_hi(const lope_grid* g, int a) { return a >= g->ndim ? 0 : (g->halo_mode ? g->hhi[a] : g->h); }
bool has_halo(const lope_grid* g, int w) {
    for (int a = 0; a < g->ndim; ++a)
        if (halo_lo(g, a) < w || halo_hi(g, a) < w) return false;
    return true;
}

int check_grid(const lope_grid* g, const char* name) {
    if (!g) return fail(LOPE_ERR_INVALID_ARG, "%s: null grid", name);
    if (g->ndim < 1 || g->ndim > 3) return fail(LOPE_ERR_INVALID_ARG, "%s: ndim %d not in 1..3", name, g->ndim);
    if (g->dtype != LOPE_F32 && g->dtype != LOPE_F64)
        return fail(LOPE_ERR_INVALID_ARG, "%s: unknown dtype %d", name, g->dtype);
    if (g->halo_mode != 0 && g->halo_mode != 1)
        return fail(LOPE_ERR_INVALID_ARG, "%s: halo_mode %d not 0 or 1", name, g->halo_mode);
    if (g->halo_mode == 0 && (g->h < 0 || g->h > (1 << 20)))
        return fail(LOPE_ERR_INVALID_ARG, "%s: bad halo width %d", name, g->h);
    if (g->halo_mode == 1) {
        for (int a = 0; a < 3; ++a) {
            const bool used = a < g->ndim;
            if (g->hlo[a] < 0 || g->hhi[a] < 0 || g->hlo[a] > (1 << 20) || g->hhi[a] > (1 << 20) ||
                (!used && (g->hlo[a] || g->hhi[a])))
                return fail(LOPE_ERR_INVALID_ARG, "%s: bad halo widths (%d, %d) on axis %d", name, g->hlo[a],
                            g->hhi[a], a);
        }
    }
    for (int a = 0; a < 3; ++a) {
        if (a < g->ndim) {
            if (g->n[a] < 0 || g->n[a] > (int64_t)1 << 30)
                return fail(LOPE_ERR_INVALID_ARG, "%s: extent n[%d]=%lld out of range", name, a, (long long)g->n[a]);
        } else if (g->n[a] != 1) {
            return fail(LOPE_ERR_INVALID_ARG, "%s: unused axis %d must have extent 1", name, a);
        }
    }
    if (g->stride[0] != 1) return fail(LOPE_ERR_INVALID_ARG, "%s: stride[0] must be 1", name);
    // the padded box's element offsets must stay far from int64 overflow
    // (2^50 elements per axis span: 4 PiB of float32)
    for (int a = 0; a < g->ndim; ++a) {
        const int64_t ext = g->n[a] + halo_lo(g, a) + halo_hi(g, a);
        if (g->stride[a] > 0 && ext > ((int64_t)1 << 50) / g->stride[a])
            return fail(LOPE_ERR_INVALID_ARG, "%s: axis %d spans more than 2^50 elements", name, a);
    }
    const int64_t wx = halo_lo(g, 0) + halo_hi(g, 0), wy = halo_lo(g, 1) + halo_hi(g, 1);
    if (g->ndim >= 2 && g->stride[1] < g->n[0] + wx)
        return fail(LOPE_ERR_INVALID_ARG, "%s: stride[1]=%lld < n[0] plus the x halo", name, (long long)g->stride[1]);
    if (g->ndim >= 3 && g->stride[2] < g->stride[1] * (g->n[1] + wy))
        return fail(LOPE_ERR_INVALID_ARG, "%s: stride[2]=%lld < stride[1]*(n[1] plus the y halo)", name,
                    (long long)g->stride[2]);
    if (!g->origin) return fail(LOPE_ERR_INVALID_ARG, "%s: null origin", name);
    return LOPE_OK;
}

bool is_empty(const lope_grid* g) { return g->n[0] == 0 || g->n[1] == 0 || g->n[2] == 0; }

int check_bc(const lope_bc* bc, int ndim) {
    if (!bc) return fail(LOPE_ERR_INVALID_ARG, "null boundary rule");
    for (int a = 0; a < ndim; ++a)
        if (bc->kind[a] != LOPE_BC_DIRICHLET && bc->kind[a] != LOPE_BC_PERIODIC)
            return fail(LOPE_ERR_INVALID_ARG, "boundary kind[%d]=%d unknown", a, bc->kind[a]);
    return LOPE_OK;
}

int check_same(const lope_grid* a, const lope_grid* b, const char* an, const char* bn) {
    if (a->ndim != b->ndim || a->dtype != b->dtype)
        return fail(LOPE_ERR_INVALID_ARG, "%s and %s differ in ndim or dtype", an, bn);
    for (int k = 0; k < 3; ++k)
        if (a->n[k] != b->n[k]) return fail(LOPE_ERR_INVALID_ARG, "%s and %s differ in extents", an, bn);
    return LOPE_OK;
}

// Byte span [lo, hi) of a grid's interior or whole padded box.
void span(const lope_grid* g, bool padded, uintptr_t* lo, uintptr_t* hi) {
    const int64_t es = (int64_t)elem_size(g->dtype);
    int64_t first = 0, last = 0;
    for (int a = 0; a < g->ndim; ++a) {
        first -= (padded ? halo_lo(g, a) : 0) * g->stride[a];
        last += (g->n[a] - 1 + (padded ? halo_hi(g, a) : 0)) * g->stride[a];
    }
    *lo = (uintptr_t)((const char*)g->origin + first * es);
    *hi = (uintptr_t)((const char*)g->origin + (last + 1) * es);
}

int check_alias(const lope_grid* a, const lope_grid* b, const char* an, const char* bn) {
    uintptr_t alo, ahi, blo, bhi;
    span(a, false, &alo, &ahi);
    span(b, false, &blo, &bhi);
    if (alo < bhi && blo < ahi)
        return fail(LOPE_ERR_ALIAS, "%s and %s interiors overlap (double buffering needs two buffers)", an, bn);
    return LOPE_OK;
}

int check_stencil(const lope_stencil* st, int ndim, int* ntaps_out) {
    if (!st) return fail(LOPE_ERR_INVALID_ARG, "null stencil");
    if (st->ndim != ndim) return fail(LOPE_ERR_INVALID_ARG, "stencil ndim %d != grid ndim %d", st->ndim, ndim);
    if (st->radius < 0 || st->radius > LOPE_MAX_RADIUS)
        return fail(LOPE_ERR_INVALID_ARG, "stencil radius %d not in 0..%d", st->radius, LOPE_MAX_RADIUS);
    if (!st->coeffs) return fail(LOPE_ERR_INVALID_ARG, "null coefficient table");
    int w = 2 * st->radius + 1, count = 1, nz = 0;
    for (int a = 0; a < ndim; ++a) count *= w;
    for (int i = 0; i < count; ++i)
        if (st->coeffs[i] != 0.0) ++nz;
    if (nz > LOPE_MAX_TAPS)
        return fail(LOPE_ERR_UNSUPPORTED, "%d non-zero taps exceed the limit of %d", nz, LOPE_MAX_TAPS);
    if (ntaps_out) *ntaps_out = nz;
    return LOPE_OK;
}

double round_to(double v, int dtype) { return dtype == LOPE_F32 ? (double)(float)v : v; }

// The stencil's reach on each axis and side (section 3.5): the largest offset
// toward lower (lo) / higher (hi) indices over the taps whose coefficient is
// non-zero once rounded to `dtype`; with `reflect` the offsets are negated
// (the adjoint reads x - o).  Then the check that a grid's halo covers it.
void stencil_reach(const lope_stencil* st, int dtype, bool reflect, int lo[3], int hi[3]) {
    const int r = st->radius, w = 2 * r + 1, d = st->ndim;
    for (int a = 0; a < 3; ++a) lo[a] = hi[a] = 0;
    const int wy = d >= 2 ? w : 1, wz = d >= 3 ? w : 1;
    for (int iz = 0; iz < wz; ++iz)
        for (int iy = 0; iy < wy; ++iy)
            for (int ix = 0; ix < w; ++ix) {
                if (round_to(st->coeffs[ix + iy * w + iz * w * w], dtype) == 0.0) continue;
                const int o[3] = {ix - r, d >= 2 ? iy - r : 0, d >= 3 ? iz - r : 0};
                for (int a = 0; a < d; ++a) {
                    const int oa = reflect ? -o[a] : o[a];
                    if (-oa > lo[a]) lo[a] = -oa;
                    if (oa > hi[a]) hi[a] = oa;
                }
            }
}

int check_reach(const lope_grid* g, const lope_stencil* st, bool reflect, const char* name) {
    int lo[3], hi[3];
    stencil_reach(st, g->dtype, reflect, lo, hi);
    for (int a = 0; a < g->ndim; ++a)
        if (lo[a] > halo_lo(g, a) || hi[a] > halo_hi(g, a))
            return fail(LOPE_ERR_HALO_TOO_SMALL,
                        "%s: the stencil reaches %d left / %d right on axis %d, the halo is %d / %d", name, lo[a],
                        hi[a], a, halo_lo(g, a), halo_hi(g, a));
    return LOPE_OK;
}

// ---- device checks ----
int device_ready() {
    const char* f = getenv("LOPE_FORCE_NO_DEVICE");
    if (f && f[0] == '1') return fail(LOPE_ERR_NO_DEVICE, "no device (LOPE_FORCE_NO_DEVICE=1)");
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return fail(LOPE_ERR_NO_DEVICE, "no HIP device available");
    }
    return LOPE_OK;
}

// LOPE_LOG=1 in the environment: one line on stderr per compute call naming
// the kernel chosen (read once per process).
bool log_enabled() {
    static const bool on = [] {
        const char* v = getenv("LOPE_LOG");
        return v && v[0] == '1';
    }();
    return on;
}

void log_line(const char* fmt, ...) {
    if (!log_enabled()) return;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    fprintf(stderr, "lope: %s\n", buf);
}

// The whole padded box must be device memory inside one allocation, on the
// current device.
int check_memory(const lope_grid* g, const char* name) {
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, g->origin);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(LOPE_ERR_INVALID_ARG, "%s: origin is not a HIP allocation (%s)", name, hipGetErrorString(e));
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return fail(LOPE_ERR_INVALID_ARG, "%s: origin is not device memory", name);
    int dev = -1;
    if (hipGetDevice(&dev) == hipSuccess && attr.device != dev)
        return fail(LOPE_ERR_INVALID_ARG, "%s: memory is on device %d, current device is %d", name, attr.device, dev);
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)g->origin);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(LOPE_ERR_INVALID_ARG, "%s: cannot query allocation range (%s)", name, hipGetErrorString(e));
    }
    uintptr_t lo, hi;
    span(g, true, &lo, &hi);
    const uintptr_t b = (uintptr_t)base;
    if (lo < b || hi > b + size)
        return fail(LOPE_ERR_INVALID_ARG, "%s: padded box [%p, %p) lies outside its allocation [%p, %p)", name,
                    (void*)lo, (void*)hi, (void*)b, (void*)(b + size));
    return LOPE_OK;
}

// `bytes` bytes at p lie in one device allocation of the current device.
int check_device_pointer(const void* p, size_t bytes, const char* name) {
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess || (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)) {
        (void)hipGetLastError();
        return fail(LOPE_ERR_INVALID_ARG, "%s must be a device pointer", name);
    }
    int dev = -1;
    if (hipGetDevice(&dev) == hipSuccess && attr.device != dev)
        return fail(LOPE_ERR_INVALID_ARG, "%s: memory is on device %d, current device is %d", name, attr.device, dev);
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if ((e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(LOPE_ERR_INVALID_ARG, "%s: cannot query allocation range (%s)", name, hipGetErrorString(e));
    }
    if ((uintptr_t)p + bytes > (uintptr_t)base + size)
        return fail(LOPE_ERR_INVALID_ARG, "%s: %zu bytes do not fit its allocation", name, bytes);
    return LOPE_OK;
}

DevGrid dev_grid(const lope_grid* g) {
    DevGrid d;
    d.origin = g->origin;
    d.sy = g->ndim >= 2 ? g->stride[1] : 0;
    d.sz = g->ndim >= 3 ? g->stride[2] : 0;
    d.nx = (int32_t)g->n[0];
    d.ny = (int32_t)g->n[1];
    d.nz = (int32_t)g->n[2];
    d.pad = 0;
    return d;
}

DevRule dev_rule(const lope_bc* bc, int ndim, bool zero_value) {
    DevRule r;
    for (int a = 0; a < 3; ++a) r.per[a] = (a < ndim) ? (bc->kind[a] == LOPE_BC_PERIODIC) : 1;
    r.pad = 0;
    r.g = zero_value ? 0.0 : bc->value;
    return r;
}


// Build the job: coefficients rounded once to the grid dtype, taps in
// lexicographic order, optionally reflected (adjoint: c'_o = c_{-o}).
void build_job(SweepJob& j, const lope_grid* src, const lope_grid* dst, const lope_stencil* st,
               const lope_bc* bc, bool reflect) {
    j.ndim = src->ndim;
    j.radius = st->radius;
    j.dtype = src->dtype;
    j.src = dev_grid(src);
    j.dst = dev_grid(dst);
    j.rule = dev_rule(bc, src->ndim, reflect);
    j.residual = nullptr;
    const int r = st->radius, w = 2 * r + 1;
    const int wy = src->ndim >= 2 ? w : 1, wz = src->ndim >= 3 ? w : 1;
    memset(j.dense, 0, sizeof j.dense);
    j.ntaps = 0;
    j.star = true;
    for (int iz = 0; iz < wz; ++iz)
        for (int iy = 0; iy < wy; ++iy)
            for (int ix = 0; ix < w; ++ix) {
                const int ox = ix - r, oy = src->ndim >= 2 ? iy - r : 0, oz = src->ndim >= 3 ? iz - r : 0;
                // the coefficient used at offset o: c_o, or c_{-o} when reflected
                const int sx = reflect ? -ox : ox, sy = reflect ? -oy : oy, sz = reflect ? -oz : oz;
                const int src_idx = (sx + r) + (src->ndim >= 2 ? (sy + r) * w : 0) +
                                    (src->ndim >= 3 ? (sz + r) * w * w : 0);
                const double c = round_to(st->coeffs[src_idx], src->dtype);
                const int idx = ix + iy * w + iz * w * w;
                j.dense[idx] = c;
                if (c != 0.0) {
                    j.off[j.ntaps][0] = (int8_t)ox;
                    j.off[j.ntaps][1] = (int8_t)oy;
                    j.off[j.ntaps][2] = (int8_t)oz;
                    j.c[j.ntaps] = c;
                    ++j.ntaps;
                    if ((ox != 0) + (oy != 0) + (oz != 0) > 1) j.star = false;
                }
            }
}

// ---- variant table and tuning ----
struct Registry {
    std::vector<Variant> v;
    Registry() {
        const Variant* p;
        int n = star3d_vec_variants(&p);
        for (int i = 0; i < n; ++i) v.push_back(p[i]);
        n = star3d_variants(&p);
        for (int i = 0; i < n; ++i) v.push_back(p[i]);
        n = star3d_flat_variants(&p);
        for (int i = 0; i < n; ++i) v.push_back(p[i]);
        n = plane2d_variants(&p);
        for (int i = 0; i < n; ++i) v.push_back(p[i]);
        n = plane2d_wave_variants(&p);
        for (int i = 0; i < n; ++i) v.push_back(p[i]);
        n = star3d_wave_variants(&p);
        for (int i = 0; i < n; ++i) v.push_back(p[i]);
    }
};
Registry& registry() {
    static Registry r;
    return r;
}

struct TuneChoice {
    int variant, tdepth, chunk;
};
std::mutex g_tune_mu;
typedef std::tuple<int, int, int, int, int, int, int> TuneKey;
std::map<TuneKey, TuneChoice> g_tune;

// (ndim, radius, dtype, star, floor(log2 points), requested sweeps per pass (0 = automatic),
// rule class: 0 = periodic on every axis, 1 = some axis Dirichlet)
// The tuning table's rule class of a job: 1 if some axis is Dirichlet (kernels
// that bit-blend the boundary value run differently from all-periodic ones).
int rule_class(const SweepJob& j) {
    for (int a = 0; a < j.ndim; ++a)
        if (!j.rule.per[a]) return 1;
    return 0;
}

TuneKey tune_key(int ndim, int radius, int dtype, bool star, int64_t points, int tdepth_req, int rules) {
    int bucket = 0;
    while (bucket < 62 && ((int64_t)1 << (bucket + 1)) <= points) ++bucket;
    return std::make_tuple(ndim, radius, dtype, star ? 1 : 0, bucket, tdepth_req, rules);
}

bool variant_fits(const Variant& v, const SweepJob& j, int tdepth) {
    if (v.ndim != j.ndim || v.radius != j.radius || v.dtype != j.dtype || v.tdepth != tdepth) return false;
    if (v.family == FAM_STAR3D) return j.star;
    if (v.family == FAM_STAR3D_FLAT || v.family == FAM_STAR3D_WAVE) {   // in-plane byte offsets within 31 bits
        const int64_t esize = j.dtype == LOPE_F64 ? 8 : 4;
        return j.star && j.src.sz * esize < ((int64_t)1 << 31) && j.dst.sz * esize < ((int64_t)1 << 31);
    }
    if (v.family == FAM_PLANE2D) return v.box ? true : j.star;
    if (v.family == FAM_STAR3D_VEC) {
        // 16-byte vectors: aligned origins, strides in whole vectors
        const int64_t vec = j.dtype == LOPE_F64 ? 2 : 4;
        auto aligned = [&](const DevGrid& g) {
            return ((uintptr_t)g.origin % 16) == 0 && g.sy % vec == 0 && g.sz % vec == 0;
        };
        return j.star && aligned(j.src) && aligned(j.dst);
    }
    return false;
}

// Default variant for a (job, depth): the first fitting entry in table order
// (each table lists its preferred tile first); a 2D star stencil prefers a
// star-shaped kernel when one fits.
int default_variant(const SweepJob& j, int tdepth) {
    auto& R = registry().v;
    int first = 0;
    for (size_t i = 0; i < R.size(); ++i) {
        if (!variant_fits(R[i], j, tdepth)) continue;
        const bool plane_star_job = R[i].family == FAM_PLANE2D && j.star;
        if (plane_star_job && !R[i].box) return (int)i + 1;
        if (!first) first = (int)i + 1;
        if (!plane_star_job) return first;
    }
    return first;
}

// A chunk longer than every extent marches the whole axis; clamping keeps the
// launchers' chunk-count arithmetic far from int overflow.
int clamp_chunk(const SweepJob& j, int chunk) {
    return std::min(chunk, std::max(j.src.nx, std::max(j.src.ny, j.src.nz)));
}

// One pass of `depth` sweeps from job.src to job.dst with variant id (0 = generic, depth 1).
int run_pass(const SweepJob& j, int variant, int chunk, hipStream_t s) {
    hipError_t e;
    if (variant <= 0) {
        e = launch_generic(j, s);
    } else {
        const Variant& v = registry().v[variant - 1];
        e = v.fn(j, chunk > 0 ? clamp_chunk(j, chunk) : v.default_chunk, s);
    }
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return LOPE_OK;
}

struct Plan {
    int variant;  // 0 = generic
    int tdepth;
    int chunk;
};

const char* variant_name(int variant) { return variant > 0 ? registry().v[variant - 1].name : "generic"; }

// The registered choice for a request of `req` sweeps per pass (0 = automatic)
// on a job like j: the entry of j's own size bucket if its variant fits j,
// else the fitting entry of the same class (ndim, radius, dtype, shape, request,
// rule class) whose bucket is nearest (the larger on a tie); *exact says
// which.  Caller holds g_tune_mu.
const TuneChoice* tune_lookup(const SweepJob& j, int req, bool* exact) {
    const int64_t pts = (int64_t)j.src.nx * j.src.ny * j.src.nz;
    const TuneKey key = tune_key(j.ndim, j.radius, j.dtype, j.star, pts, req, rule_class(j));
    auto fits = [&](const TuneChoice& c) {
        return c.variant > 0 && variant_fits(registry().v[c.variant - 1], j, c.tdepth);
    };
    auto it = g_tune.find(key);
    if (it != g_tune.end() && fits(it->second)) {
        *exact = true;
        return &it->second;
    }
    *exact = false;
    const int bucket = std::get<4>(key);
    const TuneChoice* best = nullptr;
    int best_dist = 0, best_bucket = 0;
    for (const auto& kv : g_tune) {
        const TuneKey& k = kv.first;
        if (std::get<0>(k) != std::get<0>(key) || std::get<1>(k) != std::get<1>(key) ||
            std::get<2>(k) != std::get<2>(key) || std::get<3>(k) != std::get<3>(key) ||
            std::get<5>(k) != std::get<5>(key) || std::get<6>(k) != std::get<6>(key) || !fits(kv.second))
            continue;
        const int b = std::get<4>(k), dist = b > bucket ? b - bucket : bucket - b;
        if (!best || dist < best_dist || (dist == best_dist && b > best_bucket)) {
            best = &kv.second;
            best_dist = dist;
            best_bucket = b;
        }
    }
    return best;
}

Plan choose(const SweepJob& j, int tdepth_req, int variant_req, int chunk_req) {
    Plan p{0, 1, chunk_req};
    if (variant_req == LOPE_VARIANT_GENERIC) return p;
    if (variant_req > 0) {
        const Variant& v = registry().v[variant_req - 1];
        p.variant = variant_req;
        p.tdepth = v.tdepth;
        return p;
    }
    int td = tdepth_req;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        bool exact = false;
        if (const TuneChoice* c = tune_lookup(j, td > 0 ? td : 0, &exact)) {
            p.variant = c->variant;
            p.tdepth = c->tdepth;
            // a chunk length was tuned for its own size; other sizes take
            // the launcher's automatic chunk
            if (p.chunk <= 0) p.chunk = exact ? c->chunk : 0;
            return p;
        }
    }
    if (td <= 0) td = 1;
    for (; td >= 1; --td) {
        const int v = default_variant(j, td);
        if (v) {
            p.variant = v;
            p.tdepth = td;
            return p;
        }
    }
    p.variant = 0;
    p.tdepth = 1;
    return p;
}

// A variant of `depth` sweeps per pass that reports the residual of its last
// sweep (Variant::res): the tuned choice for that depth if it has one, else the
// first fitting entry of the table.  0 if none fits.
int residual_variant(const SweepJob& j, int depth, int* chunk) {
    *chunk = 0;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        bool exact = false;
        const TuneChoice* c = tune_lookup(j, depth, &exact);
        if (c && c->tdepth == depth && registry().v[c->variant - 1].res) {
            *chunk = exact ? c->chunk : 0;
            return c->variant;
        }
    }
    auto& R = registry().v;
    for (size_t i = 0; i < R.size(); ++i)
        if (R[i].res && variant_fits(R[i], j, depth)) return (int)i + 1;
    return 0;
}

int iterate_impl(const lope_grid* a, const lope_grid* b, const lope_stencil* st, const lope_bc* bc,
                 int64_t n_steps, int32_t tdepth, int variant_req, int chunk_req, void* stream,
                 int32_t* result_index) {
    if (!result_index) return fail(LOPE_ERR_INVALID_ARG, "null result_index");
    int rc;
    if ((rc = check_grid(a, "a")) || (rc = check_grid(b, "b")) || (rc = check_same(a, b, "a", "b")) ||
        (rc = check_bc(bc, a->ndim)) || (rc = check_stencil(st, a->ndim, nullptr)))
        return rc;
    if (n_steps < 0) return fail(LOPE_ERR_INVALID_ARG, "n_steps %lld < 0", (long long)n_steps);
    if (tdepth < 0 || tdepth > 4) return fail(LOPE_ERR_INVALID_ARG, "tdepth %d not in 0..4", tdepth);
    if ((rc = check_reach(a, st, false, "a")) || (rc = check_reach(b, st, false, "b"))) return rc;
    if ((rc = check_alias(a, b, "a", "b"))) return rc;
    if (variant_req < LOPE_VARIANT_GENERIC || variant_req > (int)registry().v.size())
        return fail(LOPE_ERR_INVALID_ARG, "variant %d out of range", variant_req);
    *result_index = 0;
    if ((rc = device_ready())) return rc;
    if ((rc = check_memory(a, "a")) || (rc = check_memory(b, "b"))) return rc;
    if (is_empty(a) || n_steps == 0) return LOPE_OK;

    static thread_local SweepJob job;
    build_job(job, a, b, st, bc, false);
    if (variant_req > 0 && !variant_fits(registry().v[variant_req - 1], job, registry().v[variant_req - 1].tdepth))
        return fail(LOPE_ERR_UNSUPPORTED, "variant %d does not fit this grid/stencil", variant_req);
    const Plan plan = choose(job, tdepth, variant_req, chunk_req);
    log_line("iterate %lld sweeps on %dx%dx%d %s radius %d: %s, %d per pass, chunk %d", (long long)n_steps, job.src.nx,
             job.src.ny, job.src.nz, job.dtype == LOPE_F64 ? "f64" : "f32", job.radius, variant_name(plan.variant),
             plan.tdepth, plan.chunk);
    const hipStream_t s = (hipStream_t)stream;
    const DevGrid ga = dev_grid(a), gb = dev_grid(b);
    int64_t done = 0, passes = 0;
    while (done < n_steps) {
        int64_t left = n_steps - done;
        int variant = plan.variant, chunk = plan.chunk;
        if (left < plan.tdepth && variant > 0) {
            // remainder: the tuned (else the first fitting) variant of at most `left` sweeps
            const Plan rp = choose(job, (int)left, 0, 0);
            variant = rp.variant;
            chunk = rp.chunk;
        }
        job.src = (passes & 1) ? gb : ga;
        job.dst = (passes & 1) ? ga : gb;
        if ((rc = run_pass(job, variant, chunk, s))) return rc;
        done += variant > 0 ? registry().v[variant - 1].tdepth : 1;
        ++passes;
    }
    *result_index = (int32_t)(passes & 1);
    return LOPE_OK;
}


// ---- batch plans ----
constexpr int kBatchRows = 128;       // rows per batch strip unless tuned or set
constexpr int kBatchDefaultDepth = 4; // sweeps per pass unless tuned or set
constexpr int kBatchMaxRows = 1 << 16;

// Batch tiling table: (dtype, floor(log2 interior points of the whole batch))
// -> (sweeps per pass, rows per strip), registered by lope_batch_tune_set.
std::mutex g_batch_tune_mu;
std::map<std::pair<int, int>, std::pair<int, int>> g_batch_tune;

int log2_bucket(int64_t points) {
    int bucket = 0;
    while (bucket < 62 && ((int64_t)1 << (bucket + 1)) <= points) ++bucket;
    return bucket;
}

// The registered tiling for a batch of `points` interior points: its own
// bucket, else the nearest registered bucket of the dtype (the larger on a
// tie), else the defaults.
void batch_tiling(int dtype, int64_t points, int* tdepth, int* rows) {
    *tdepth = kBatchDefaultDepth;
    *rows = kBatchRows;
    const int bucket = log2_bucket(points);
    std::lock_guard<std::mutex> lk(g_batch_tune_mu);
    int best_dist = -1, best_bucket = 0;
    for (const auto& kv : g_batch_tune) {
        if (kv.first.first != dtype) continue;
        const int b = kv.first.second, dist = b > bucket ? b - bucket : bucket - b;
        if (best_dist < 0 || dist < best_dist || (dist == best_dist && b > best_bucket)) {
            best_dist = dist;
            best_bucket = b;
            *tdepth = kv.second.first;
            *rows = kv.second.second;
        }
    }
}

struct PlanGrid {
    lope_grid src, dst;
    lope_bc bc;
    std::vector<double> coeffs;
    lope_stencil st;
};

// Byte span of one interior of a batch: [lo, hi), the item and which buffer.
struct BatchSpan {
    uintptr_t lo, hi;
    int64_t item;
    int dst;
};

// Structural, device and memory checks of a batch (before anything is
// allocated or enqueued); *dtype receives the batch's element type.  Every
// pass writes one buffer of every item while it reads the other, so the
// interiors of all 2 n_items buffers must be disjoint: their spans are sorted
// into `spans` (room for 2 n_items entries) and neighbours compared.
int batch_check(const lope_batch_item* items, int64_t n_items, int64_t n_steps, int* dtype, BatchSpan* spans) {
    int rc;
    if (!items && n_items > 0) return fail(LOPE_ERR_INVALID_ARG, "null item array");
    if (n_items < 0 || n_items > (1 << 20)) return fail(LOPE_ERR_INVALID_ARG, "n_items %lld out of range", (long long)n_items);
    if (n_steps < 0 || n_steps > (1 << 24)) return fail(LOPE_ERR_INVALID_ARG, "n_steps %lld out of range", (long long)n_steps);
    *dtype = n_items > 0 ? items[0].src.dtype : LOPE_F32;
    for (int64_t i = 0; i < n_items; ++i) {
        const lope_batch_item& it = items[i];
        char a[32], b[32];
        snprintf(a, sizeof a, "items[%lld].src", (long long)i);
        snprintf(b, sizeof b, "items[%lld].dst", (long long)i);
        if ((rc = check_grid(&it.src, a)) || (rc = check_grid(&it.dst, b)) || (rc = check_same(&it.src, &it.dst, a, b)) ||
            (rc = check_bc(&it.bc, it.src.ndim)) || (rc = check_stencil(&it.stencil, it.src.ndim, nullptr)))
            return rc;
        if (it.src.ndim != 2) return fail(LOPE_ERR_UNSUPPORTED, "%s: batches hold 2D grids", a);
        if (it.src.dtype != *dtype) return fail(LOPE_ERR_INVALID_ARG, "%s: all grids of a batch share one dtype", a);
        if (it.stencil.radius > 1) return fail(LOPE_ERR_UNSUPPORTED, "%s: batch stencils have radius <= 1", a);
        if ((rc = check_reach(&it.src, &it.stencil, false, a)) || (rc = check_reach(&it.dst, &it.stencil, false, b)))
            return rc;
        if ((rc = check_alias(&it.src, &it.dst, a, b))) return rc;
    }
    for (int64_t i = 0; i < n_items; ++i) {
        for (int d = 0; d < 2; ++d) {
            BatchSpan& sp = spans[2 * i + d];
            span(d ? &items[i].dst : &items[i].src, false, &sp.lo, &sp.hi);
            sp.item = i;
            sp.dst = d;
        }
    }
    std::sort(spans, spans + 2 * n_items, [](const BatchSpan& x, const BatchSpan& y) {
        return x.lo < y.lo || (x.lo == y.lo && (x.item < y.item || (x.item == y.item && x.dst < y.dst)));
    });
    for (int64_t k = 0; k + 1 < 2 * n_items; ++k) {
        const BatchSpan &x = spans[k], &y = spans[k + 1];
        if (x.lo < x.hi && y.lo < y.hi && y.lo < x.hi)
            return fail(LOPE_ERR_ALIAS, "items[%lld].%s and items[%lld].%s overlap (every grid of a batch needs "
                        "buffers of its own)", (long long)x.item, x.dst ? "dst" : "src", (long long)y.item,
                        y.dst ? "dst" : "src");
    }
    if ((rc = device_ready())) return rc;
    for (int64_t i = 0; i < n_items; ++i) {
        if ((rc = check_memory(&items[i].src, "batch src")) || (rc = check_memory(&items[i].dst, "batch dst"))) return rc;
    }
    return LOPE_OK;
}

// The kernel's descriptor of one grid: views, rule, the 3x3 coefficient table
// rounded to the grid dtype, star or box.  `job` is working storage.
void batch_grid_desc(const lope_grid* src, const lope_grid* dst, const lope_stencil* st, const lope_bc* bc,
                     SweepJob& job, BatchGrid& bg) {
    build_job(job, src, dst, st, bc, false);
    bg = BatchGrid{};
    bg.src = dev_grid(src);
    bg.dst = dev_grid(dst);
    bg.rule = dev_rule(bc, 2, false);
    const int r = st->radius;
    for (int oy = -r; oy <= r; ++oy)
        for (int ox = -r; ox <= r; ++ox) bg.c[(ox + 1) + (oy + 1) * 3] = job.dense[(ox + r) + (oy + r) * (2 * r + 1)];
    bg.box = job.star ? 0 : 1;
}

// Grids in tile-table order: dealt to the 8 XCD ranges largest first, each to
// the least-loaded range, then listed range by range, so a grid's tiles get
// consecutive workgroup ids (one XCD).  order and sorted hold n entries,
// range holds n (working storage; nothing is allocated).
void batch_order(const lope_batch_item* items, int64_t n, int64_t* order, int64_t* sorted, int8_t* range) {
    auto points = [&](int64_t i) { return items[i].src.n[0] * items[i].src.n[1]; };
    for (int64_t i = 0; i < n; ++i) sorted[i] = i;
    std::sort(sorted, sorted + n, [&](int64_t x, int64_t y) {
        return points(x) > points(y) || (points(x) == points(y) && x < y);
    });
    int64_t load[kNumXcd] = {};
    for (int64_t k = 0; k < n; ++k) {
        int best = 0;
        for (int q = 1; q < kNumXcd; ++q)
            if (load[q] < load[best]) best = q;
        range[sorted[k]] = (int8_t)best;
        load[best] += points(sorted[k]);
    }
    int64_t m = 0;
    for (int q = 0; q < kNumXcd; ++q)
        for (int64_t k = 0; k < n; ++k)
            if (range[sorted[k]] == q) order[m++] = sorted[k];
}

// Work-table entries of passes of `depth` sweeps: per grid in `order`, strips
// of batch_strip_width(depth) output columns by chunks of `rows` rows.  Writes
// the first `cap` entries to out (if not null) and returns how many there are.
int64_t batch_strips(const lope_batch_item* items, const int64_t* order, int64_t n, int depth, int rows,
                     BatchItem* out, int64_t cap) {
    const int64_t bw = batch_strip_width(depth);
    int64_t count = 0;
    for (int64_t k = 0; k < n; ++k) {
        const int64_t gi = order[k];
        const int64_t nx = items[gi].src.n[0], ny = items[gi].src.n[1];
        if (nx == 0 || ny == 0) continue;
        for (int64_t y0 = 0; y0 < ny; y0 += rows)
            for (int64_t x0 = 0; x0 < nx; x0 += bw) {
                if (out && count < cap) {
                    BatchItem& it = out[count];
                    it = BatchItem{};
                    it.grid = (int32_t)gi;
                    it.x0 = (int32_t)x0;
                    it.y0 = (int32_t)y0;
                    it.y1 = (int32_t)std::min(ny, y0 + rows);
                }
                ++count;
            }
    }
    return count;
}

// Passes of n_steps sweeps at `depth` per launch on stream s: full passes
// alternating src->dst and dst->src, then one pass of the remaining sweeps.
hipError_t enqueue_passes(const BatchGrid* grids, const BatchItem* full_items, int n_full_items,
                          const BatchItem* rem_items, int n_rem_items, int64_t n_steps, int depth, int dtype,
                          hipStream_t s) {
    const int64_t full = n_steps / depth;
    const int rem = (int)(n_steps % depth);
    int64_t pass = 0;
    for (; pass < full; ++pass) {
        const hipError_t e = launch_batch_pass(grids, full_items, n_full_items, depth, (int)(pass & 1), dtype, s);
        if (e != hipSuccess) return e;
    }
    if (rem) return launch_batch_pass(grids, rem_items, n_rem_items, rem, (int)(pass & 1), dtype, s);
    return hipSuccess;
}

}  // namespace

struct lope_batch_plan {
    int dtype = LOPE_F32;
    int64_t n_steps = 0;
    int device = 0;
    int tdepth = kBatchDefaultDepth;
    int rows = kBatchRows;            // rows per strip of the tile tables
    std::vector<PlanGrid> grids;
    std::vector<lope_batch_item> items;   // the items as given, coefficients pointing into grids[i].coeffs
    std::vector<int64_t> order;       // grids in tile-table order (largest first, dealt to XCD ranges)
    std::vector<int8_t> range;        // each grid's XCD range (the order lists range 0's grids first)
    std::vector<SweepJob> jobs;       // per-grid launches (the comparison path)
    std::vector<int> job_variant;
    BatchGrid* d_grids = nullptr;
    BatchItem* d_items[kBatchMaxDepth + 1] = {};   // tile tables per depth
    int nitems[kBatchMaxDepth + 1] = {};
    int items_rows[kBatchMaxDepth + 1] = {};   // rows per strip each table was built with
    hipGraphExec_t graph = nullptr;   // every pass of lope_batch_apply, recorded for (graph_depth, graph_rows)
    int graph_depth = 0, graph_rows = 0;
    // persistent launch: queue state followed by one PqGrid per grid (zeroed at
    // creation); the strip counts are those of the tiling (pq_depth, pq_rows)
    PqState* d_pq = nullptr;
    PqGrid* d_pqg = nullptr;
    int pq_depth = 0, pq_rows = 0;
    int pq_nq = 1;                    // queues of the persistent launch
};

namespace {

void plan_free(lope_batch_plan* p) {
    if (!p) return;
    if (p->graph) (void)hipGraphExecDestroy(p->graph);
    if (p->d_grids) (void)hipFree(p->d_grids);
    if (p->d_pq) (void)hipFree(p->d_pq);
    for (int d = 0; d <= kBatchMaxDepth; ++d)
        if (p->d_items[d]) (void)hipFree(p->d_items[d]);
    delete p;
}

// Work table for passes of `depth` sweeps: per grid (in plan order), strips
// of batch_strip_width(depth) output columns by chunks of p->rows rows, one
// entry per wave.  Built and uploaded once per (depth, rows).
int plan_items(lope_batch_plan* p, int depth) {
    if (p->d_items[depth] && p->items_rows[depth] == p->rows) return LOPE_OK;
    if (p->d_items[depth]) {
        (void)hipFree(p->d_items[depth]);
        p->d_items[depth] = nullptr;
    }
    const int64_t n = (int64_t)p->order.size();
    const int64_t count = batch_strips(p->items.data(), p->order.data(), n, depth, p->rows, nullptr, 0);
    if (count > (int64_t)(1 << 30)) return fail(LOPE_ERR_UNSUPPORTED, "batch tile table too long");
    std::vector<BatchItem> items((size_t)count);
    batch_strips(p->items.data(), p->order.data(), n, depth, p->rows, items.data(), count);
    p->nitems[depth] = (int)items.size();
    p->items_rows[depth] = p->rows;
    if (items.empty()) return LOPE_OK;
    hipError_t e = hipMalloc(&p->d_items[depth], items.size() * sizeof(BatchItem));
    if (e == hipSuccess)
        e = hipMemcpy(p->d_items[depth], items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (p->d_items[depth]) (void)hipFree(p->d_items[depth]);
        p->d_items[depth] = nullptr;
        p->nitems[depth] = 0;
        return hip_fail(e, "batch tile table upload");
    }
    return LOPE_OK;
}

// Queue state of the persistent launch for the plan's tiling: allocated and
// zeroed once, and each grid's strip count in the full-depth table uploaded
// whenever the tiling changes (after the device is idle, since a running
// launch reads them).
int plan_pq(lope_batch_plan* p) {
    if (p->d_pq && p->pq_depth == p->tdepth && p->pq_rows == p->rows) return LOPE_OK;
    const size_t n = p->grids.size();
    hipError_t e = hipSuccess;
    if (!p->d_pq) {
        const size_t bytes = sizeof(PqState) + std::max<size_t>(n, 1) * sizeof(PqGrid);
        e = hipMalloc(&p->d_pq, bytes);
        if (e == hipSuccess) e = hipMemset(p->d_pq, 0, bytes);
        if (e != hipSuccess) {
            if (p->d_pq) (void)hipFree(p->d_pq);
            p->d_pq = nullptr;
            return hip_fail(e, "persistent batch state");
        }
        p->d_pqg = reinterpret_cast<PqGrid*>(p->d_pq + 1);
    } else if ((e = hipDeviceSynchronize()) != hipSuccess) {
        return hip_fail(e, "device synchronisation before the persistent batch tables");
    }
    const int64_t bw = batch_strip_width(p->tdepth), full = p->n_steps / p->tdepth;
    const int rem = (int)(p->n_steps % p->tdepth);
    const int64_t bwr = rem ? batch_strip_width(rem) : 1;
    std::vector<PqGrid> hg(std::max<size_t>(n, 1));
    std::vector<int64_t> rstrips(n);
    for (size_t i = 0; i < n; ++i) {
        const int64_t nx = p->items[i].src.n[0], ny = p->items[i].src.n[1];
        const int64_t ry = (ny + p->rows - 1) / p->rows;
        const int64_t fs = (nx && ny) ? ry * ((nx + bw - 1) / bw) : 0;
        const int64_t rs = (nx && ny && rem) ? ry * ((nx + bwr - 1) / bwr) : 0;
        // the per-grid counter reaches full * fs + rs in one launch
        if (full * fs + rs > (int64_t)INT32_MAX)
            return fail(LOPE_ERR_UNSUPPORTED, "grid %zu has too many strips for one persistent launch", i);
        hg[i].done = 0;
        hg[i].full_strips = (int32_t)fs;
        rstrips[i] = rs;
    }
    // one queue per XCD range: the tables list each range's grids together,
    // so a queue's strips are one contiguous span of each table
    const int nq = kPqMaxQueues;
    PqQueue share[kPqMaxQueues] = {};
    {
        int64_t fpos = 0, rpos = 0;
        int last = -1;
        for (size_t k = 0; k < n; ++k) {
            const int64_t gi = p->order[k];
            const int q = (int)p->range[(size_t)gi];
            if (q < last || q >= nq) return fail(LOPE_ERR_UNSUPPORTED, "batch grids not grouped by queue");
            if (q != last) {
                share[q].full_begin = fpos;
                share[q].rem_begin = rpos;
                last = q;
            }
            share[q].full_count += hg[(size_t)gi].full_strips;
            share[q].rem_count += rstrips[(size_t)gi];
            fpos += hg[(size_t)gi].full_strips;
            rpos += rstrips[(size_t)gi];
        }
        if (fpos != p->nitems[p->tdepth] || (rem && rpos != p->nitems[rem]))
            return fail(LOPE_ERR_UNSUPPORTED, "persistent batch queues do not cover the strip tables");
    }
    e = hipMemcpy(p->d_pqg, hg.data(), n * sizeof(PqGrid), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(&p->d_pq->share[0], share, sizeof(share), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "persistent batch table upload");
    p->pq_nq = nq;
    p->pq_depth = p->tdepth;
    p->pq_rows = p->rows;
    return LOPE_OK;
}

// Passes of lope_batch_apply: full passes of tdepth sweeps, then one pass of
// the remaining n mod tdepth sweeps.
int64_t plan_passes(const lope_batch_plan* p) {
    return p->n_steps / p->tdepth + (p->n_steps % p->tdepth ? 1 : 0);
}

// Every pass of lope_batch_apply on stream s: full passes of tdepth sweeps
// alternating src->dst and dst->src, then the remainder pass.
hipError_t enqueue_batch_passes(const lope_batch_plan* p, hipStream_t s) {
    const int rem = (int)(p->n_steps % p->tdepth);
    return enqueue_passes(p->d_grids, p->d_items[p->tdepth], p->nitems[p->tdepth], rem ? p->d_items[rem] : nullptr,
                          rem ? p->nitems[rem] : 0, p->n_steps, p->tdepth, p->dtype, s);
}

// Records the passes once into an executable graph (kernel nodes only) on a
// private stream; replaying it costs one launch per lope_batch_apply.
hipError_t record_batch_graph(const lope_batch_plan* p, hipGraphExec_t* out) {
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t le = enqueue_batch_passes(p, cs);
        e = hipStreamEndCapture(cs, &g);
        if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    return e;
}

}  // namespace

// ---- batches without device allocation ----
// The grid descriptors and strip tables of lope_batch_apply_noalloc live in
// this fixed array (one copy per device, kept until the process ends).  Host
// code never passes the symbol itself to a kernel or copy: it uses the device
// address hipGetSymbolAddress gives for the current device.
static __device__ __align__(256) unsigned char scratch[LOPE_BATCH_SCRATCH_BYTES];

namespace {

constexpr int kNoallocMaxDevices = 64;
constexpr int64_t kNoallocMaxGrids = LOPE_BATCH_SCRATCH_BYTES / sizeof(BatchGrid);
std::mutex g_noalloc_mu;                             // one call at a time builds and uploads tables
void* g_scratch_dev[kNoallocMaxDevices] = {};        // device address of `scratch` per device
// host staging and working storage (static: the call allocates nothing)
alignas(256) unsigned char g_noalloc_stage[LOPE_BATCH_SCRATCH_BYTES];
int64_t g_noalloc_order[kNoallocMaxGrids], g_noalloc_sorted[kNoallocMaxGrids];
BatchSpan g_noalloc_spans[2 * kNoallocMaxGrids];
int8_t g_noalloc_range[kNoallocMaxGrids];

// Device address of `scratch` on the current device, looked up once per
// device with that device current.  Caller holds g_noalloc_mu.
int noalloc_scratch(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "current device");
    if (dev < 0 || dev >= kNoallocMaxDevices) return fail(LOPE_ERR_UNSUPPORTED, "device %d out of range", dev);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "address of the static batch scratch");
        if (!p) return fail(LOPE_ERR_HIP, "address of the static batch scratch: null");
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return LOPE_OK;
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

int lope_get_device(int ordinal, int* out) {
    if (!out) return fail(LOPE_ERR_INVALID_ARG, "null output pointer");
    *out = LOPE_HOST;
    const char* f = getenv("LOPE_FORCE_NO_DEVICE");
    if (f && f[0] == '1') return LOPE_OK;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) {
        (void)hipGetLastError();
        return LOPE_OK;
    }
    if (ordinal >= 0 && ordinal < n) *out = ordinal;
    return LOPE_OK;
}

int lope_halo_fill(const lope_grid* g, const lope_bc* bc, void* stream) {
    int rc;
    if ((rc = check_grid(g, "grid")) || (rc = check_bc(bc, g->ndim))) return rc;
    if ((rc = device_ready())) return rc;
    if ((rc = check_memory(g, "grid"))) return rc;
    if (is_empty(g)) return LOPE_OK;
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = halo_lo(g, a);
        hi[a] = halo_hi(g, a);
    }
    const hipError_t e = launch_halo_fill(dev_grid(g), lo, hi, g->dtype, dev_rule(bc, g->ndim, false),
                                          (hipStream_t)stream);
    return e == hipSuccess ? LOPE_OK : hip_fail(e, "halo fill launch");
}

int lope_apply(const lope_grid* src, const lope_grid* dst, const lope_stencil* st, const lope_bc* bc,
               void* stream) {
    int32_t idx = 0;
    return iterate_impl(src, dst, st, bc, 1, 1, 0, 0, stream, &idx);
}

int lope_iterate(const lope_grid* a, const lope_grid* b, const lope_stencil* st, const lope_bc* bc,
                 int64_t n_steps, int32_t tdepth, void* stream, int32_t* result_index) {
    return iterate_impl(a, b, st, bc, n_steps, tdepth, 0, 0, stream, result_index);
}

int lope_iterate_until(const lope_grid* a, const lope_grid* b, const lope_stencil* st, const lope_bc* bc,
                       int64_t max_steps, int32_t check_every, double tol, int32_t tdepth, double* residual_scratch,
                       void* stream, int64_t* steps_done, double* residual, int32_t* result_index) {
    if (!steps_done || !residual || !result_index) return fail(LOPE_ERR_INVALID_ARG, "null output pointer");
    *steps_done = 0;
    *residual = std::nan("");
    *result_index = 0;
    if (check_every < 1) return fail(LOPE_ERR_INVALID_ARG, "check_every %d < 1", check_every);
    if (max_steps < 0) return fail(LOPE_ERR_INVALID_ARG, "max_steps %lld < 0", (long long)max_steps);
    if (!residual_scratch || ((uintptr_t)residual_scratch & 7))
        return fail(LOPE_ERR_INVALID_ARG, "residual_scratch must be an 8-byte aligned device pointer");
    int rc;
    int32_t idx = 0;
    // full validation of the grids, stencil and rule (zero sweeps launch nothing)
    if ((rc = iterate_impl(a, b, st, bc, 0, tdepth, 0, 0, stream, &idx))) return rc;
    if ((rc = check_device_pointer(residual_scratch, sizeof(double), "residual_scratch"))) return rc;
    if (is_empty(a)) return LOPE_OK;
    const hipStream_t s = (hipStream_t)stream;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cap);
    if (e != hipSuccess) return hip_fail(e, "stream capture query");
    if (cap != hipStreamCaptureStatusNone)
        return fail(LOPE_ERR_UNSUPPORTED, "lope_iterate_until waits on the host; it cannot be captured");
    const DevGrid ga = dev_grid(a), gb = dev_grid(b);
    // The last sweeps before each check run as one pass of a variant that also
    // reports the residual of its last sweep (no extra pass over memory); with
    // no such variant, the checked sweep runs alone and k_residual_max
    // compares the two buffers.
    static thread_local SweepJob rjob;
    build_job(rjob, a, b, st, bc, false);
    const int want = choose(rjob, tdepth, 0, 0).tdepth;
    int cur = 0;   // buffer holding the state: 0 = a, 1 = b
    int64_t done = 0;
    while (done < max_steps) {
        const int64_t to_check = check_every - done % check_every;
        const int64_t left = max_steps - done;
        if (to_check > left) {   // no check within the budget: plain sweeps
            if ((rc = iterate_impl(cur ? b : a, cur ? a : b, st, bc, left, tdepth, 0, 0, stream, &idx))) return rc;
            cur ^= idx;
            done = max_steps;
            break;
        }
        int rd = (int)std::min<int64_t>(want, to_check), rv = 0, rchunk = 0;
        for (; rd >= 1 && !(rv = residual_variant(rjob, rd, &rchunk)); --rd) {
        }
        const int last = rv ? rd : 1;   // sweeps of the checked pass
        if (to_check > last) {
            if ((rc = iterate_impl(cur ? b : a, cur ? a : b, st, bc, to_check - last, tdepth, 0, 0, stream, &idx)))
                return rc;
            cur ^= idx;
        }
        if (rv) {
            build_job(rjob, cur ? b : a, cur ? a : b, st, bc, false);
            rjob.residual = residual_scratch;
            if ((e = launch_residual_zero(residual_scratch, s)) != hipSuccess) return hip_fail(e, "residual reset");
            if ((rc = run_pass(rjob, rv, rchunk, s))) return rc;
            rjob.residual = nullptr;
            cur ^= 1;
        } else {
            // the checked sweep alone, then the residual between the two buffers
            if ((rc = iterate_impl(cur ? b : a, cur ? a : b, st, bc, 1, 1, 0, 0, stream, &idx))) return rc;
            const DevGrid& prev = cur ? gb : ga;
            const DevGrid& next = cur ? ga : gb;
            cur ^= 1;
            if ((e = launch_residual_max(prev, next, a->dtype, residual_scratch, s)) != hipSuccess)
                return hip_fail(e, "residual launch");
        }
        done += to_check;
        double r = 0.0;
        if ((e = hipMemcpyAsync(&r, residual_scratch, sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return hip_fail(e, "residual read-back");
        *residual = r;
        *steps_done = done;
        *result_index = cur;
        if (r <= tol) return LOPE_OK;
    }
    *steps_done = done;
    *result_index = cur;
    return LOPE_OK;
}

namespace {

// Two-stage steps: validation, then passes of two steps with a fused
// four-level variant while two or more steps remain, the rest one per pass
// with a fused two-level variant (each the tuned choice of its depth for the
// first stencil if it can also take the second, else the first that can) or
// the one-thread-per-point kernel.
int stages_impl(const lope_grid* a, const lope_grid* b, const lope_stages* sg, const lope_bc* bc, int64_t n_steps,
                void* stream, int32_t* result_index) {
    if (!result_index) return fail(LOPE_ERR_INVALID_ARG, "null result_index");
    *result_index = 0;
    if (!sg || !sg->first || !sg->second) return fail(LOPE_ERR_INVALID_ARG, "null stages or stencil");
    int rc;
    if ((rc = check_grid(a, "a")) || (rc = check_grid(b, "b")) || (rc = check_same(a, b, "a", "b")) ||
        (rc = check_bc(bc, a->ndim)) || (rc = check_stencil(sg->first, a->ndim, nullptr)) ||
        (rc = check_stencil(sg->second, a->ndim, nullptr)))
        return rc;
    if (n_steps < 0) return fail(LOPE_ERR_INVALID_ARG, "n_steps %lld < 0", (long long)n_steps);
    if ((rc = check_reach(a, sg->first, false, "a")) || (rc = check_reach(b, sg->first, false, "b"))) return rc;
    if ((rc = check_alias(a, b, "a", "b"))) return rc;
    static thread_local StageJob sj;
    build_job(sj.s1, a, b, sg->first, bc, false);
    build_job(sj.s2, a, b, sg->second, bc, false);
    if (sj.s1.ntaps > kStageTaps || sj.s2.ntaps > kStageTaps)
        return fail(LOPE_ERR_UNSUPPORTED, "two-stage steps take stencils of at most %d non-zero taps", kStageTaps);
    sj.alpha = round_to(sg->alpha, a->dtype);
    if ((rc = device_ready())) return rc;
    if ((rc = check_memory(a, "a")) || (rc = check_memory(b, "b"))) return rc;
    if (is_empty(a) || n_steps == 0) return LOPE_OK;
    auto& R = registry().v;
    // a variant making depth / 2 steps per pass that takes both stencils
    auto takes = [&](int v, int depth) {
        return v > 0 && R[v - 1].sfn && variant_fits(R[v - 1], sj.s1, depth) && variant_fits(R[v - 1], sj.s2, depth);
    };
    // the tuned choice for that depth if it takes both, else the first that does
    auto pick = [&](int depth, int* chunk) {
        *chunk = 0;
        const Plan p = choose(sj.s1, depth, 0, 0);
        if (p.tdepth == depth && takes(p.variant, depth)) {
            *chunk = p.chunk;
            return p.variant;
        }
        for (size_t i = 0; i < R.size(); ++i)
            if (takes((int)i + 1, depth)) return (int)i + 1;
        return 0;
    };
    int chunk2 = 0, chunk1 = 0;
    const int v2 = pick(4, &chunk2);   // two steps per pass
    const int v1 = pick(2, &chunk1);   // one step per pass
    log_line("two-stage steps (%lld) on %dx%dx%d: two per pass %s, one per pass %s", (long long)n_steps, sj.s1.src.nx,
             sj.s1.src.ny, sj.s1.src.nz, v2 ? variant_name(v2) : "none", v1 ? variant_name(v1) : "k_stages");
    const DevGrid ga = dev_grid(a), gb = dev_grid(b);
    const hipStream_t s = (hipStream_t)stream;
    int64_t done = 0, passes = 0;
    while (done < n_steps) {
        sj.s1.src = (passes & 1) ? gb : ga;
        sj.s1.dst = (passes & 1) ? ga : gb;
        hipError_t e;
        if (v2 && n_steps - done >= 2) {
            e = R[v2 - 1].sfn(sj, chunk2 > 0 ? clamp_chunk(sj.s1, chunk2) : R[v2 - 1].default_chunk, s);
            done += 2;
        } else {
            e = v1 ? R[v1 - 1].sfn(sj, chunk1 > 0 ? clamp_chunk(sj.s1, chunk1) : R[v1 - 1].default_chunk, s)
                   : launch_stages_generic(sj, s);
            done += 1;
        }
        if (e != hipSuccess) return hip_fail(e, "two-stage launch");
        ++passes;
    }
    *result_index = (int32_t)(passes & 1);
    return LOPE_OK;
}

}  // namespace

int lope_apply_stages(const lope_grid* src, const lope_grid* dst, const lope_stages* sg, const lope_bc* bc,
                      void* stream) {
    int32_t idx = 0;
    return stages_impl(src, dst, sg, bc, 1, stream, &idx);
}

int lope_iterate_stages(const lope_grid* a, const lope_grid* b, const lope_stages* sg, const lope_bc* bc,
                        int64_t n_steps, void* stream, int32_t* result_index) {
    return stages_impl(a, b, sg, bc, n_steps, stream, result_index);
}

int lope_iterate_tuned(const lope_grid* a, const lope_grid* b, const lope_stencil* st, const lope_bc* bc,
                       int64_t n_steps, const lope_tuning* tune, void* stream, int32_t* result_index) {
    if (!tune) return fail(LOPE_ERR_INVALID_ARG, "null tuning");
    if (tune->chunk < 0) return fail(LOPE_ERR_INVALID_ARG, "chunk %d < 0", tune->chunk);
    return iterate_impl(a, b, st, bc, n_steps, tune->tdepth, tune->variant, tune->chunk, stream, result_index);
}

int lope_apply_adjoint(const lope_grid* ybar, const lope_grid* xbar, const lope_stencil* st, const lope_bc* bc,
                       double* gbar_dirichlet, void* stream) {
    int rc;
    if ((rc = check_grid(ybar, "ybar")) || (rc = check_grid(xbar, "xbar")) ||
        (rc = check_same(ybar, xbar, "ybar", "xbar")) || (rc = check_bc(bc, ybar->ndim)) ||
        (rc = check_stencil(st, ybar->ndim, nullptr)))
        return rc;
    if ((rc = check_reach(ybar, st, true, "ybar"))) return rc;
    if ((rc = check_alias(ybar, xbar, "ybar", "xbar"))) return rc;
    if ((rc = device_ready())) return rc;
    if ((rc = check_memory(ybar, "ybar")) || (rc = check_memory(xbar, "xbar"))) return rc;
    if (gbar_dirichlet && ((uintptr_t)gbar_dirichlet & 7))
        return fail(LOPE_ERR_INVALID_ARG, "gbar_dirichlet must be 8-byte aligned");
    if (gbar_dirichlet &&
        (rc = check_device_pointer(gbar_dirichlet, LOPE_GBAR_DOUBLES * sizeof(double), "gbar_dirichlet")))
        return rc;
    const hipStream_t s = (hipStream_t)stream;
    static thread_local SweepJob job;
    if (is_empty(ybar)) {
        if (gbar_dirichlet) {
            build_job(job, ybar, xbar, st, bc, false);
            job.src.nx = 0;
            const hipError_t e = launch_gbar(job, gbar_dirichlet, gbar_dirichlet, s);
            if (e != hipSuccess) return hip_fail(e, "gbar launch");
        }
        return LOPE_OK;
    }
    if (gbar_dirichlet) {
        build_job(job, ybar, xbar, st, bc, false);
        const hipError_t e = launch_gbar(job, gbar_dirichlet, gbar_dirichlet, s);
        if (e != hipSuccess) return hip_fail(e, "gbar launch");
    }
    build_job(job, ybar, xbar, st, bc, true);
    const Plan plan = choose(job, 1, 0, 0);
    log_line("adjoint on %dx%dx%d: %s%s", job.src.nx, job.src.ny, job.src.nz,
             variant_name(plan.tdepth == 1 ? plan.variant : 0), gbar_dirichlet ? ", gbar" : "");
    return run_pass(job, plan.tdepth == 1 ? plan.variant : 0, plan.chunk, s);
}

int lope_apply_var(const lope_grid* src, const lope_grid* dst, const lope_varcoef* vc, const lope_bc* bc,
                   void* stream) {
    int rc;
    if (!vc) return fail(LOPE_ERR_INVALID_ARG, "null varcoef");
    if ((rc = check_grid(src, "src")) || (rc = check_grid(dst, "dst")) || (rc = check_grid(vc->kappa, "kappa")) ||
        (rc = check_same(src, dst, "src", "dst")) || (rc = check_same(src, vc->kappa, "src", "kappa")) ||
        (rc = check_bc(bc, src->ndim)))
        return rc;
    if (src->ndim != 3) return fail(LOPE_ERR_UNSUPPORTED, "variable-coefficient diffusion is 3D only");
    for (int a = 0; a < 3; ++a)
        if (bc->kind[a] != LOPE_BC_PERIODIC)
            return fail(LOPE_ERR_UNSUPPORTED, "variable-coefficient diffusion supports periodic boundaries only");
    if (!has_halo(src, 1) || !has_halo(vc->kappa, 1))
        return fail(LOPE_ERR_HALO_TOO_SMALL, "src and kappa need a halo of 1 on every side");
    if ((rc = check_alias(src, dst, "src", "dst")) || (rc = check_alias(vc->kappa, dst, "kappa", "dst"))) return rc;
    if ((rc = device_ready())) return rc;
    if ((rc = check_memory(src, "src")) || (rc = check_memory(dst, "dst")) || (rc = check_memory(vc->kappa, "kappa")))
        return rc;
    if (is_empty(src)) return LOPE_OK;
    const DevGrid gs = dev_grid(src), gd = dev_grid(dst), gk = dev_grid(vc->kappa);
    const int es = (int)elem_size(src->dtype);
    const bool wave = var_wave_fits(gs, es) && var_wave_fits(gd, es) && var_wave_fits(gk, es);
    log_line("diffusion step on %dx%dx%d: %s", gs.nx, gs.ny, gs.nz, wave ? "k_varw_forward" : "k_var_forward");
    const hipError_t e = wave ? launch_var_forward_wave(gs, gd, gk, src->dtype, vc->dt, (hipStream_t)stream)
                              : launch_var_forward(gs, gd, gk, src->dtype, vc->dt, (hipStream_t)stream);
    return e == hipSuccess ? LOPE_OK : hip_fail(e, "diffusion launch");
}

int lope_apply_var_adjoint(const lope_grid* lam_next, const lope_grid* lam, const lope_grid* u_t,
                           const lope_varcoef* vc, const lope_bc* bc, const lope_grid* gkappa, void* stream) {
    int rc;
    if (!vc) return fail(LOPE_ERR_INVALID_ARG, "null varcoef");
    if ((rc = check_grid(lam_next, "lam_next")) || (rc = check_grid(lam, "lam")) || (rc = check_grid(u_t, "u_t")) ||
        (rc = check_grid(vc->kappa, "kappa")) || (rc = check_grid(gkappa, "gkappa")) ||
        (rc = check_same(lam_next, lam, "lam_next", "lam")) || (rc = check_same(lam_next, u_t, "lam_next", "u_t")) ||
        (rc = check_same(lam_next, vc->kappa, "lam_next", "kappa")) || (rc = check_bc(bc, lam_next->ndim)))
        return rc;
    if (gkappa->ndim != lam_next->ndim || gkappa->n[0] != lam_next->n[0] || gkappa->n[1] != lam_next->n[1] ||
        gkappa->n[2] != lam_next->n[2])
        return fail(LOPE_ERR_INVALID_ARG, "gkappa extents differ");
    if (lam_next->ndim != 3) return fail(LOPE_ERR_UNSUPPORTED, "variable-coefficient diffusion is 3D only");
    for (int a = 0; a < 3; ++a)
        if (bc->kind[a] != LOPE_BC_PERIODIC)
            return fail(LOPE_ERR_UNSUPPORTED, "variable-coefficient diffusion supports periodic boundaries only");
    if (!has_halo(lam_next, 1) || !has_halo(u_t, 1) || !has_halo(vc->kappa, 1))
        return fail(LOPE_ERR_HALO_TOO_SMALL, "lam_next, u_t and kappa need a halo of 1 on every side");
    if ((rc = check_alias(lam_next, lam, "lam_next", "lam")) || (rc = check_alias(u_t, lam, "u_t", "lam")) ||
        (rc = check_alias(vc->kappa, lam, "kappa", "lam")) || (rc = check_alias(gkappa, lam, "gkappa", "lam")) ||
        (rc = check_alias(gkappa, lam_next, "gkappa", "lam_next")) || (rc = check_alias(gkappa, u_t, "gkappa", "u_t")) ||
        (rc = check_alias(gkappa, vc->kappa, "gkappa", "kappa")))
        return rc;
    if ((rc = device_ready())) return rc;
    if ((rc = check_memory(lam_next, "lam_next")) || (rc = check_memory(lam, "lam")) ||
        (rc = check_memory(u_t, "u_t")) || (rc = check_memory(vc->kappa, "kappa")) ||
        (rc = check_memory(gkappa, "gkappa")))
        return rc;
    if (is_empty(lam_next)) return LOPE_OK;
    const DevGrid gn = dev_grid(lam_next), gl = dev_grid(lam), gu = dev_grid(u_t), gk = dev_grid(vc->kappa),
                  gg = dev_grid(gkappa);
    const int es = (int)elem_size(lam_next->dtype);
    const bool wave = var_wave_fits(gn, es) && var_wave_fits(gl, es) && var_wave_fits(gu, es) &&
                      var_wave_fits(gk, es) && var_wave_fits(gg, (int)elem_size(gkappa->dtype));
    log_line("diffusion reverse step on %dx%dx%d: %s", gn.nx, gn.ny, gn.nz, wave ? "k_varw_adjoint" : "k_var_adjoint");
    const hipError_t e =
        wave ? launch_var_adjoint_wave(gn, gl, gu, gk, gg, lam_next->dtype, gkappa->dtype, vc->dt, (hipStream_t)stream)
             : launch_var_adjoint(gn, gl, gu, gk, gg, lam_next->dtype, gkappa->dtype, vc->dt, (hipStream_t)stream);
    return e == hipSuccess ? LOPE_OK : hip_fail(e, "diffusion adjoint launch");
}

int lope_apply_var_adjoint2(const lope_grid* lam_next, const lope_grid* lam, const lope_grid* u_t,
                            const lope_grid* u_tm1, const lope_varcoef* vc, const lope_bc* bc,
                            const lope_grid* gkappa, void* stream) {
    int rc;
    if (!vc) return fail(LOPE_ERR_INVALID_ARG, "null varcoef");
    if ((rc = check_grid(lam_next, "lam_next")) || (rc = check_grid(lam, "lam")) || (rc = check_grid(u_t, "u_t")) ||
        (rc = check_grid(u_tm1, "u_tm1")) || (rc = check_grid(vc->kappa, "kappa")) ||
        (rc = check_grid(gkappa, "gkappa")) || (rc = check_same(lam_next, lam, "lam_next", "lam")) ||
        (rc = check_same(lam_next, u_t, "lam_next", "u_t")) || (rc = check_same(lam_next, u_tm1, "lam_next", "u_tm1")) ||
        (rc = check_same(lam_next, vc->kappa, "lam_next", "kappa")) || (rc = check_bc(bc, lam_next->ndim)))
        return rc;
    if (gkappa->ndim != lam_next->ndim || gkappa->n[0] != lam_next->n[0] || gkappa->n[1] != lam_next->n[1] ||
        gkappa->n[2] != lam_next->n[2])
        return fail(LOPE_ERR_INVALID_ARG, "gkappa extents differ");
    if (lam_next->ndim != 3) return fail(LOPE_ERR_UNSUPPORTED, "variable-coefficient diffusion is 3D only");
    for (int a = 0; a < 3; ++a)
        if (bc->kind[a] != LOPE_BC_PERIODIC)
            return fail(LOPE_ERR_UNSUPPORTED, "variable-coefficient diffusion supports periodic boundaries only");
    if (!has_halo(lam_next, 1) || !has_halo(u_t, 1) || !has_halo(u_tm1, 1) || !has_halo(vc->kappa, 1))
        return fail(LOPE_ERR_HALO_TOO_SMALL, "lam_next, u_t, u_tm1 and kappa need a halo of 1 on every side");
    const lope_grid* ins[4] = {lam_next, u_t, u_tm1, vc->kappa};
    const char* names[4] = {"lam_next", "u_t", "u_tm1", "kappa"};
    for (int i = 0; i < 4; ++i)
        if ((rc = check_alias(ins[i], lam, names[i], "lam")) || (rc = check_alias(ins[i], gkappa, names[i], "gkappa")))
            return rc;
    if ((rc = check_alias(gkappa, lam, "gkappa", "lam"))) return rc;
    if ((rc = device_ready())) return rc;
    for (int i = 0; i < 4; ++i)
        if ((rc = check_memory(ins[i], names[i]))) return rc;
    if ((rc = check_memory(lam, "lam")) || (rc = check_memory(gkappa, "gkappa"))) return rc;
    if (is_empty(lam_next)) return LOPE_OK;
    const DevGrid gn = dev_grid(lam_next), gl = dev_grid(lam), gu = dev_grid(u_t), gv = dev_grid(u_tm1),
                  gk = dev_grid(vc->kappa), gg = dev_grid(gkappa);
    const int es = (int)elem_size(lam_next->dtype);
    const bool wave = var_pair_wave_fits(gn, gu, gv, gk, es) && var_wave_fits(gl, es) &&
                      var_wave_fits(gg, (int)elem_size(gkappa->dtype));
    log_line("diffusion reverse pair on %dx%dx%d: %s", gn.nx, gn.ny, gn.nz, wave ? "k_varw_adjoint2" : "k_var_adjoint2");
    const hipError_t e =
        wave ? launch_var_adjoint2_wave(gn, gl, gu, gv, gk, gg, lam_next->dtype, gkappa->dtype, vc->dt, (hipStream_t)stream)
             : launch_var_adjoint2(gn, gl, gu, gv, gk, gg, lam_next->dtype, gkappa->dtype, vc->dt, (hipStream_t)stream);
    return e == hipSuccess ? LOPE_OK : hip_fail(e, "diffusion two-step adjoint launch");
}

int lope_accumulate(const lope_grid* partial, const lope_grid* total, void* stream) {
    int rc;
    if ((rc = check_grid(partial, "partial")) || (rc = check_grid(total, "total"))) return rc;
    if (total->dtype != LOPE_F64) return fail(LOPE_ERR_INVALID_ARG, "total must be F64");
    if (partial->ndim != total->ndim || partial->n[0] != total->n[0] || partial->n[1] != total->n[1] ||
        partial->n[2] != total->n[2])
        return fail(LOPE_ERR_INVALID_ARG, "partial and total extents differ");
    if ((rc = check_alias(partial, total, "partial", "total"))) return rc;
    if ((rc = device_ready())) return rc;
    if ((rc = check_memory(partial, "partial")) || (rc = check_memory(total, "total"))) return rc;
    if (is_empty(partial)) return LOPE_OK;
    const hipError_t e = launch_accumulate(dev_grid(partial), partial->dtype, dev_grid(total), (hipStream_t)stream);
    return e == hipSuccess ? LOPE_OK : hip_fail(e, "accumulate launch");
}


int lope_batch_plan_create(const lope_batch_item* items, int64_t n_items, int64_t n_steps, void* stream,
                           lope_batch_plan** out) {
    int rc, dtype = LOPE_F32;
    if (!out) return fail(LOPE_ERR_INVALID_ARG, "null plan output");
    *out = nullptr;
    if (n_items < 0 || n_items > (1 << 20)) return fail(LOPE_ERR_INVALID_ARG, "n_items %lld out of range", (long long)n_items);
    {
        std::vector<BatchSpan> spans((size_t)(2 * n_items));
        if ((rc = batch_check(items, n_items, n_steps, &dtype, spans.data()))) return rc;
    }
    lope_batch_plan* p = new lope_batch_plan();
    p->dtype = dtype;
    p->n_steps = n_steps;
    {
        int64_t points = 0;
        for (int64_t i = 0; i < n_items; ++i) points += items[i].src.n[0] * items[i].src.n[1];
        batch_tiling(dtype, points, &p->tdepth, &p->rows);
    }
    (void)hipGetDevice(&p->device);
    // copy items (the stencil table is copied; grids are borrowed)
    p->grids.resize((size_t)n_items);
    p->items.resize((size_t)n_items);
    for (int64_t i = 0; i < n_items; ++i) {
        PlanGrid& g = p->grids[(size_t)i];
        g.src = items[i].src;
        g.dst = items[i].dst;
        g.bc = items[i].bc;
        const int r = items[i].stencil.radius, w = 2 * r + 1;
        g.coeffs.assign(items[i].stencil.coeffs, items[i].stencil.coeffs + w * w);
        g.st = items[i].stencil;
        g.st.coeffs = g.coeffs.data();
        p->items[(size_t)i] = lope_batch_item{g.src, g.dst, g.st, g.bc};
    }
    // per-grid jobs for the one-launch-per-grid path
    p->jobs.resize((size_t)n_items);
    p->job_variant.resize((size_t)n_items);
    for (int64_t i = 0; i < n_items; ++i) {
        PlanGrid& g = p->grids[(size_t)i];
        build_job(p->jobs[(size_t)i], &g.src, &g.dst, &g.st, &g.bc, false);
        p->job_variant[(size_t)i] = default_variant(p->jobs[(size_t)i], 1);
    }
    p->order.resize((size_t)n_items);
    p->range.resize((size_t)n_items);
    {
        std::vector<int64_t> sorted((size_t)n_items);
        batch_order(p->items.data(), n_items, p->order.data(), sorted.data(), p->range.data());
    }
    std::vector<BatchGrid> hg((size_t)n_items);
    {
        static thread_local SweepJob job;
        for (int64_t i = 0; i < n_items; ++i) {
            const PlanGrid& g = p->grids[(size_t)i];
            batch_grid_desc(&g.src, &g.dst, &g.st, &g.bc, job, hg[(size_t)i]);
        }
    }
    hipError_t e = hipMalloc(&p->d_grids, (hg.empty() ? 1 : hg.size()) * sizeof(BatchGrid));
    if (e == hipSuccess && !hg.empty())
        e = hipMemcpy(p->d_grids, hg.data(), hg.size() * sizeof(BatchGrid), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        plan_free(p);
        return hip_fail(e, "batch plan upload");
    }
    if ((rc = plan_items(p, p->tdepth)) || (n_steps % p->tdepth && (rc = plan_items(p, (int)(n_steps % p->tdepth)))) ||
        (rc = plan_pq(p))) {
        plan_free(p);
        return rc;
    }
    (void)stream;
    *out = p;
    return LOPE_OK;
}

int lope_batch_plan_set_tiles(lope_batch_plan* plan, int32_t tdepth, int32_t rows) {
    if (!plan) return fail(LOPE_ERR_INVALID_ARG, "null plan");
    if (tdepth < 1 || tdepth > kBatchMaxDepth)
        return fail(LOPE_ERR_INVALID_ARG, "tdepth %d not in 1..%d", tdepth, kBatchMaxDepth);
    if (rows < 0 || rows > kBatchMaxRows) return fail(LOPE_ERR_INVALID_ARG, "rows %d not in 0..%d", rows, kBatchMaxRows);
    int rc;
    if ((rc = device_ready())) return rc;
    const int old_depth = plan->tdepth, old_rows = plan->rows;
    plan->tdepth = tdepth;
    if (rows > 0) plan->rows = rows;
    if ((rc = plan_items(plan, tdepth)) ||
        (plan->n_steps % tdepth && (rc = plan_items(plan, (int)(plan->n_steps % tdepth)))) || (rc = plan_pq(plan))) {
        plan->tdepth = old_depth;
        plan->rows = old_rows;
        return rc;
    }
    return LOPE_OK;
}

int lope_batch_plan_set_depth(lope_batch_plan* plan, int32_t tdepth) { return lope_batch_plan_set_tiles(plan, tdepth, 0); }

int lope_batch_plan_get_tiles(const lope_batch_plan* plan, int32_t* tdepth, int32_t* rows) {
    if (!plan || !tdepth || !rows) return fail(LOPE_ERR_INVALID_ARG, "null plan or output");
    *tdepth = plan->tdepth;
    *rows = plan->rows;
    return LOPE_OK;
}

int lope_batch_tune_set(int32_t dtype, int64_t points, int32_t tdepth, int32_t rows) {
    if (dtype != LOPE_F32 && dtype != LOPE_F64) return fail(LOPE_ERR_INVALID_ARG, "unknown dtype %d", dtype);
    if (points < 1) return fail(LOPE_ERR_INVALID_ARG, "points %lld < 1", (long long)points);
    if (tdepth < 0 || tdepth > kBatchMaxDepth)
        return fail(LOPE_ERR_INVALID_ARG, "tdepth %d not in 0..%d", tdepth, kBatchMaxDepth);
    if (tdepth > 0 && (rows < 1 || rows > kBatchMaxRows))
        return fail(LOPE_ERR_INVALID_ARG, "rows %d not in 1..%d", rows, kBatchMaxRows);
    std::lock_guard<std::mutex> lk(g_batch_tune_mu);
    const std::pair<int, int> key(dtype, log2_bucket(points));
    if (tdepth == 0)
        g_batch_tune.erase(key);
    else
        g_batch_tune[key] = std::make_pair((int)tdepth, (int)rows);
    return LOPE_OK;
}

int lope_batch_result_index(const lope_batch_plan* plan, int32_t* out) {
    if (!plan || !out) return fail(LOPE_ERR_INVALID_ARG, "null plan or output");
    *out = (int32_t)(plan_passes(plan) & 1);
    return LOPE_OK;
}

int lope_batch_apply_passes(lope_batch_plan* plan, void* stream) {
    if (!plan) return fail(LOPE_ERR_INVALID_ARG, "null plan");
    int rc;
    if ((rc = device_ready())) return rc;
    if (plan_passes(plan) == 0) return LOPE_OK;
    const hipStream_t s = (hipStream_t)stream;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cap);
    if (e != hipSuccess) return hip_fail(e, "stream capture query");
    log_line("batch of %zu grids, %lld sweeps as passes: %d per launch, %d-row strips, %lld launches%s", plan->grids.size(),
             (long long)plan->n_steps, plan->tdepth, plan->rows, (long long)plan_passes(plan),
             cap != hipStreamCaptureStatusNone ? " (into the caller's graph)" : "");
    if (cap != hipStreamCaptureStatusNone) {
        // the caller is recording a graph: its graph takes the launches
        e = enqueue_batch_passes(plan, s);
        return e == hipSuccess ? LOPE_OK : hip_fail(e, "batch pass launch");
    }
    if (!plan->graph || plan->graph_depth != plan->tdepth || plan->graph_rows != plan->rows) {
        if (plan->graph) (void)hipGraphExecDestroy(plan->graph);
        plan->graph = nullptr;
        if ((e = record_batch_graph(plan, &plan->graph)) != hipSuccess) return hip_fail(e, "batch graph recording");
        plan->graph_depth = plan->tdepth;
        plan->graph_rows = plan->rows;
    }
    e = hipGraphLaunch(plan->graph, s);
    return e == hipSuccess ? LOPE_OK : hip_fail(e, "batch graph launch");
}

int lope_batch_apply(lope_batch_plan* plan, void* stream) {
    if (!plan) return fail(LOPE_ERR_INVALID_ARG, "null plan");
    int rc;
    if ((rc = device_ready())) return rc;
    if (plan_passes(plan) == 0) return LOPE_OK;
    if (!plan->d_pq || plan->pq_depth != plan->tdepth || plan->pq_rows != plan->rows)
        return fail(LOPE_ERR_INVALID_ARG, "persistent batch state does not match the plan's tiling");
    const int rem = (int)(plan->n_steps % plan->tdepth);
    PqShape shape{};
    shape.full = (int32_t)(plan->n_steps / plan->tdepth);
    shape.nq = plan->pq_nq;
    shape.take = 1;   // one unit per take
    const int64_t units = (int64_t)shape.full * plan->nitems[plan->tdepth] + (rem ? plan->nitems[rem] : 0);
    log_line("batch of %zu grids, %lld sweeps in one persistent launch: %d per pass, %d-row strips, %lld passes, "
             "%lld units",
             plan->grids.size(), (long long)plan->n_steps, plan->tdepth, plan->rows, (long long)plan_passes(plan),
             (long long)units);
    // time limit of one dependency wait: 1 s, or LOPE_PERSISTENT_WAIT_US
    // microseconds (read at each launch; 0 makes any wait not met at once run
    // out, which exercises the abort path)
    long long wait_us = 1000000;
    if (const char* w = getenv("LOPE_PERSISTENT_WAIT_US")) {
        char* end = nullptr;
        const long long v = strtoll(w, &end, 10);
        if (end == w || *end != '\0' || v < 0 || v > 1000000000ll)
            return fail(LOPE_ERR_INVALID_ARG, "LOPE_PERSISTENT_WAIT_US=%s is not 0..1000000000", w);
        wait_us = v;
    }
    const hipError_t e = launch_batch_persistent(plan->d_grids, plan->d_items[plan->tdepth],
                                                 rem ? plan->d_items[rem] : nullptr, shape, units, plan->tdepth, rem,
                                                 plan->d_pq, plan->d_pqg, (int)plan->grids.size(), wait_us,
                                                 plan->dtype, (hipStream_t)stream);
    return e == hipSuccess ? LOPE_OK : hip_fail(e, "persistent batch launch");
}

int lope_batch_persistent_check(lope_batch_plan* plan) {
    if (!plan) return fail(LOPE_ERR_INVALID_ARG, "null plan");
    int rc;
    if ((rc = device_ready())) return rc;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "device synchronisation");
    if (!plan->d_pq) return LOPE_OK;
    unsigned int timeouts = 0;
    e = hipMemcpy(&timeouts, &plan->d_pq->timeouts, sizeof(timeouts), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "persistent batch status");
    if (timeouts == 0) return LOPE_OK;
    const unsigned int zero = 0;
    e = hipMemcpy(&plan->d_pq->timeouts, &zero, sizeof(zero), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "persistent batch status reset");
    return fail(LOPE_ERR_TIMEOUT, "%u wait(s) of a persistent batch launch ran out of time; its result is invalid",
                timeouts);
}

int lope_batch_apply_per_grid(lope_batch_plan* plan, void* stream) {
    if (!plan) return fail(LOPE_ERR_INVALID_ARG, "null plan");
    int rc;
    if ((rc = device_ready())) return rc;
    const hipStream_t s = (hipStream_t)stream;
    for (size_t i = 0; i < plan->jobs.size(); ++i) {
        SweepJob& j = plan->jobs[i];
        if (j.src.nx == 0 || j.src.ny == 0) continue;
        const DevGrid a = dev_grid(&plan->grids[i].src), b = dev_grid(&plan->grids[i].dst);
        for (int64_t t = 0; t < plan->n_steps; ++t) {
            j.src = (t & 1) ? b : a;
            j.dst = (t & 1) ? a : b;
            if ((rc = run_pass(j, plan->job_variant[i], 0, s))) return rc;
        }
        j.src = a;
        j.dst = b;
    }
    return LOPE_OK;
}

int lope_batch_plan_destroy(lope_batch_plan* plan) {
    plan_free(plan);
    return LOPE_OK;
}

int lope_batch_apply_noalloc(const lope_batch_item* items, int64_t n_items, int64_t n_steps, int32_t tdepth,
                             int32_t rows, void* stream, int32_t* result_index) {
    if (!result_index) return fail(LOPE_ERR_INVALID_ARG, "null result_index");
    *result_index = 0;
    if (tdepth < 0 || tdepth > kBatchMaxDepth)
        return fail(LOPE_ERR_INVALID_ARG, "tdepth %d not in 0..%d", tdepth, kBatchMaxDepth);
    if (rows < 0 || rows > kBatchMaxRows) return fail(LOPE_ERR_INVALID_ARG, "rows %d not in 0..%d", rows, kBatchMaxRows);
    if (n_items > kNoallocMaxGrids)
        return fail(LOPE_ERR_UNSUPPORTED, "%lld grids: the static scratch holds the descriptors of at most %lld",
                    (long long)n_items, (long long)kNoallocMaxGrids);
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    int rc, dtype = LOPE_F32;
    if ((rc = batch_check(items, n_items, n_steps, &dtype, g_noalloc_spans))) return rc;
    const hipStream_t s = (hipStream_t)stream;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cap);
    if (e != hipSuccess) return hip_fail(e, "stream capture query");
    if (cap != hipStreamCaptureStatusNone)
        return fail(LOPE_ERR_UNSUPPORTED, "lope_batch_apply_noalloc uploads its tables and waits; it cannot be captured");
    int64_t points = 0;
    for (int64_t i = 0; i < n_items; ++i) points += items[i].src.n[0] * items[i].src.n[1];
    int depth = 0, nrows = 0;
    batch_tiling(dtype, points, &depth, &nrows);
    if (tdepth > 0) depth = tdepth;
    if (rows > 0) nrows = rows;
    const int64_t passes = n_steps / depth + (n_steps % depth ? 1 : 0);
    if (n_items == 0 || passes == 0) return LOPE_OK;
    const int rem = (int)(n_steps % depth);
    void* dev = nullptr;
    if ((rc = noalloc_scratch(&dev))) return rc;
    batch_order(items, n_items, g_noalloc_order, g_noalloc_sorted, g_noalloc_range);
    const int64_t nfull = batch_strips(items, g_noalloc_order, n_items, depth, nrows, nullptr, 0);
    const int64_t nrem = rem ? batch_strips(items, g_noalloc_order, n_items, rem, nrows, nullptr, 0) : 0;
    const size_t gbytes = round256((size_t)n_items * sizeof(BatchGrid));
    const size_t fbytes = round256((size_t)nfull * sizeof(BatchItem));
    const size_t need = gbytes + fbytes + (size_t)nrem * sizeof(BatchItem);
    if (need > (size_t)LOPE_BATCH_SCRATCH_BYTES)
        return fail(LOPE_ERR_UNSUPPORTED,
                    "the batch's tables need %zu bytes (%lld grids, %lld + %lld strips); the static scratch holds %zu",
                    need, (long long)n_items, (long long)nfull, (long long)nrem, (size_t)LOPE_BATCH_SCRATCH_BYTES);
    log_line("batch without allocation, %lld grids, %lld sweeps: %d per launch, %d-row strips, %lld launches, %zu "
             "bytes of tables", (long long)n_items, (long long)n_steps, depth, nrows, (long long)passes, need);
    // the tables, laid out as on the device: descriptors, full-pass strips, remainder strips
    BatchGrid* hg = reinterpret_cast<BatchGrid*>(g_noalloc_stage);
    BatchItem* hfull = reinterpret_cast<BatchItem*>(g_noalloc_stage + gbytes);
    BatchItem* hrem = reinterpret_cast<BatchItem*>(g_noalloc_stage + gbytes + fbytes);
    {
        static thread_local SweepJob job;
        for (int64_t i = 0; i < n_items; ++i)
            batch_grid_desc(&items[i].src, &items[i].dst, &items[i].stencil, &items[i].bc, job, hg[i]);
    }
    batch_strips(items, g_noalloc_order, n_items, depth, nrows, hfull, nfull);
    if (rem) batch_strips(items, g_noalloc_order, n_items, rem, nrows, hrem, nrem);
    // ordered after earlier work on `stream`; the wait frees the staging
    // memory for the next call
    unsigned char* d = static_cast<unsigned char*>(dev);
    if ((e = hipMemcpyAsync(d, g_noalloc_stage, need, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "batch table upload to the static scratch");
    e = enqueue_passes(reinterpret_cast<const BatchGrid*>(d), reinterpret_cast<const BatchItem*>(d + gbytes), (int)nfull,
                       rem ? reinterpret_cast<const BatchItem*>(d + gbytes + fbytes) : nullptr, (int)nrem, n_steps,
                       depth, dtype, s);
    if (e != hipSuccess) return hip_fail(e, "batch pass launch");
    *result_index = (int32_t)(passes & 1);
    return LOPE_OK;
}

int lope_copy_stream(const void* src, void* dst, int64_t bytes, void* stream) {
    if (!src || !dst) return fail(LOPE_ERR_INVALID_ARG, "null pointer");
    if (bytes < 0 || bytes % 16) return fail(LOPE_ERR_INVALID_ARG, "bytes %lld: a non-negative multiple of 16", (long long)bytes);
    if (((uintptr_t)src | (uintptr_t)dst) & 15) return fail(LOPE_ERR_INVALID_ARG, "pointers must be 16-byte aligned");
    const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
    if (bytes > 0 && a < b + (uintptr_t)bytes && b < a + (uintptr_t)bytes)
        return fail(LOPE_ERR_ALIAS, "source and destination ranges overlap");
    int rc;
    if ((rc = device_ready())) return rc;
    if (bytes == 0) return LOPE_OK;
    if ((rc = check_device_pointer(src, (size_t)bytes, "src")) || (rc = check_device_pointer(dst, (size_t)bytes, "dst")))
        return rc;
    const hipError_t e = launch_copy16(src, dst, bytes, (hipStream_t)stream);
    return e == hipSuccess ? LOPE_OK : hip_fail(e, "copy launch");
}

const char* lope_status_string(int status) {
    switch (status) {
        case LOPE_OK: return "ok";
        case LOPE_ERR_INVALID_ARG: return "invalid argument";
        case LOPE_ERR_HALO_TOO_SMALL: return "halo too small for stencil radius";
        case LOPE_ERR_ALIAS: return "source and destination overlap";
        case LOPE_ERR_UNSUPPORTED: return "unsupported";
        case LOPE_ERR_NO_DEVICE: return "no device";
        case LOPE_ERR_HIP: return "HIP runtime error";
        case LOPE_ERR_TIMEOUT: return "device wait timed out";
        default: return "unknown status";
    }
}

const char* lope_last_error(void) { return g_last_error.c_str(); }

int lope_variant_count(void) { return (int)registry().v.size(); }

int lope_variant_info(int id, char* text, int cap) {
    if (id < 1 || id > (int)registry().v.size()) return fail(LOPE_ERR_INVALID_ARG, "variant %d out of range", id);
    if (!text || cap <= 0) return fail(LOPE_ERR_INVALID_ARG, "null text buffer");
    const Variant& v = registry().v[id - 1];
    snprintf(text, (size_t)cap, "%s ndim=%d radius=%d tdepth=%d dtype=%s shape=%s tile=%dx%d nt=%d chunk=%d", v.name,
             v.ndim, v.radius, v.tdepth, v.dtype == LOPE_F64 ? "f64" : "f32",
             v.family == FAM_PLANE2D ? (v.box ? "box" : "star") : "star", v.bx, v.by, v.nt, v.default_chunk);
    return LOPE_OK;
}

int lope_select_variant(const lope_grid* g, const lope_stencil* st, const lope_bc* bc, int32_t tdepth) {
    int rc;
    if ((rc = check_grid(g, "grid")) || (rc = check_stencil(st, g->ndim, nullptr))) return rc;
    if (bc && (rc = check_bc(bc, g->ndim))) return rc;
    if (tdepth < 0 || tdepth > 4) return fail(LOPE_ERR_INVALID_ARG, "tdepth %d not in 0..4", tdepth);
    static thread_local SweepJob job;
    lope_bc periodic{};
    for (int a = 0; a < 3; ++a) periodic.kind[a] = LOPE_BC_PERIODIC;
    build_job(job, g, g, st, bc ? bc : &periodic, false);
    return choose(job, tdepth, 0, 0).variant;
}

int lope_tune_set(const lope_grid* g, const lope_stencil* st, const lope_tuning* tune) {
    int rc;
    if (!tune) return fail(LOPE_ERR_INVALID_ARG, "null tuning");
    if ((rc = check_grid(g, "grid")) || (rc = check_stencil(st, g->ndim, nullptr))) return rc;
    if (tune->variant < 0 || tune->variant > (int)registry().v.size())
        return fail(LOPE_ERR_INVALID_ARG, "variant %d out of range", tune->variant);
    if (tune->rules != 0 && tune->rules != 1)
        return fail(LOPE_ERR_INVALID_ARG, "rules %d: 0 (every axis periodic) or 1 (some axis Dirichlet)", tune->rules);
    if (tune->chunk < 0) return fail(LOPE_ERR_INVALID_ARG, "chunk %d < 0", tune->chunk);
    static thread_local SweepJob job;
    lope_bc bc{};
    for (int a = 0; a < 3; ++a) bc.kind[a] = tune->rules && a == 0 ? LOPE_BC_DIRICHLET : LOPE_BC_PERIODIC;
    build_job(job, g, g, st, &bc, false);
    if (tune->variant == 0) {   // remove the choice for this request
        if (tune->tdepth < 0 || tune->tdepth > 4) return fail(LOPE_ERR_INVALID_ARG, "tdepth %d not in 0..4", tune->tdepth);
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune.erase(tune_key(job.ndim, job.radius, job.dtype, job.star, (int64_t)job.src.nx * job.src.ny * job.src.nz,
                              tune->tdepth, tune->rules));
        return LOPE_OK;
    }
    const int td = registry().v[tune->variant - 1].tdepth;
    if (!variant_fits(registry().v[tune->variant - 1], job, td))
        return fail(LOPE_ERR_UNSUPPORTED, "variant %d does not fit this grid/stencil", tune->variant);
    if (tune->tdepth < 0 || tune->tdepth > 4 || (tune->tdepth > 0 && tune->tdepth != td))
        return fail(LOPE_ERR_INVALID_ARG, "tdepth %d: 0 (automatic) or the variant's own depth %d", tune->tdepth, td);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[tune_key(job.ndim, job.radius, job.dtype, job.star, (int64_t)job.src.nx * job.src.ny * job.src.nz,
                    tune->tdepth, tune->rules)] = TuneChoice{tune->variant, td, tune->chunk};
    return LOPE_OK;
}

}  // extern "C"
