// The persistent batched launch: one kernel advances every grid of a batch
// through all of its passes.
//
// Each wave is an independent worker running the loop of batch_queue.h: it
// takes the next unit (one strip of one grid in one pass), waits until the
// grid's earlier passes are complete, sweeps the strip with the same body as
// the per-pass kernel (batch_strip, TD fused sweeps, or the remainder depth
// in the last pass) and counts it complete.  Units are handed out pass-major,
// so waves of one launch work on several passes at once wherever the grids'
// dependencies allow, with no kernel boundary between passes.
//
// Memory ordering: a grid's strips run on any XCD, and the XCDs' L2 caches
// are not coherent with each other, so every load and store of grid data in
// this kernel is a device-scope (agent) access (batch_strip with DEV): loads
// read past every cache that could hold an older copy, and a store is
// complete only once every XCD can see it.  A wave then publishes its strip
// by waiting for its stores to complete before adding to the grid's counter
// (an agent-scope atomic), and a waiting wave polls the counter with relaxed
// agent-scope loads; no cache write-back or invalidation is needed per strip.
// (The same ordering by agent-scope release and acquire fences around plain
// accesses, which flush and invalidate the L2 at every strip, is 3-6x slower
// here.)  Every wait is bounded (wall clock and poll count); one that runs
// out sets the abort flag and counts a timeout, and every wave leaves.
#include "batch_strip.h"

#include <algorithm>

namespace lope {
namespace {

constexpr int kPqWaves = 4;                  // waves per workgroup
constexpr unsigned long long kPqTicksPerUs = 100;   // the real-time clock runs at 100 MHz
constexpr unsigned kPqMaxPolls = 1u << 22;    // polls of one wait (each sleeps about 128 clocks)

__device__ __forceinline__ bool lane0() { return (threadIdx.x & 63) == 0; }
__device__ __forceinline__ unsigned uniform(unsigned v) { return (unsigned)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ unsigned long long uniform(unsigned long long v) {
    const unsigned lo = uniform((unsigned)(v & 0xffffffffu)), hi = uniform((unsigned)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// Strip body at a run-time depth (the remainder pass sweeps fewer times than
// the full passes); depth is wave-uniform and at most TD.
template <typename T, int TD>
__device__ __forceinline__ void strip_at_depth(const BatchGrid& gr, int parity, const BatchItem& it, int depth) {
    if constexpr (TD > 1) {
        if (depth < TD) {
            strip_at_depth<T, TD - 1>(gr, parity, it, depth);
            return;
        }
    }
    batch_strip<T, TD, true>(gr, parity, it);
}

// The worker policy of one wave (every member function is called by all 64
// lanes with wave-uniform arguments; single-lane atomics are broadcast).
template <typename T, int TD>
struct WaveOps {
    const BatchGrid* grids;
    const BatchItem* full_items;
    const BatchItem* rem_items;
    PqState* st;
    PqGrid* pg;
    int ngrids;
    int nq;
    int rem;
    unsigned nwaves;
    unsigned long long wait_ticks;   // time limit of one wait
    unsigned max_polls;              // poll limit of one wait
    BatchItem it;

    __device__ __forceinline__ int32_t first_queue() { return (int32_t)(blockIdx.x % (unsigned)nq); }
    __device__ __forceinline__ PqQueue queue(int32_t q) {
        PqQueue r;
        r.full_begin = (int64_t)uniform((unsigned long long)st->share[q].full_begin);
        r.full_count = (int64_t)uniform((unsigned long long)st->share[q].full_count);
        r.rem_begin = (int64_t)uniform((unsigned long long)st->share[q].rem_begin);
        r.rem_count = (int64_t)uniform((unsigned long long)st->share[q].rem_count);
        return r;
    }
    __device__ __forceinline__ bool aborted() {
        return uniform(__hip_atomic_load(&st->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0;
    }
    __device__ __forceinline__ int64_t take(int32_t q, int32_t n) {
        unsigned long long u = 0;
        if (lane0())
            u = __hip_atomic_fetch_add(&st->queue[q].next, (unsigned long long)n, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        return (int64_t)uniform(u);
    }
    __device__ __forceinline__ int32_t grid_of(const PqUnit& un) {
        const BatchItem* tab = un.rem ? rem_items : full_items;
        const BatchItem& src = tab[un.strip];
        it.grid = uniform(src.grid);
        it.x0 = uniform(src.x0);
        it.y0 = uniform(src.y0);
        it.y1 = uniform(src.y1);
        return it.grid;
    }
    __device__ __forceinline__ int32_t full_strips(int32_t g) { return uniform(pg[g].full_strips); }
    __device__ __forceinline__ bool wait(int32_t g, int64_t need) {
        const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
        for (unsigned polls = 0;; ++polls) {
            const unsigned d = uniform(__hip_atomic_load(&pg[g].done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            if ((int64_t)d >= need) break;
            if (aborted()) return false;
            if (polls >= max_polls || __builtin_amdgcn_s_memrealtime() - t0 > wait_ticks) {
                if (lane0()) {
                    __hip_atomic_fetch_add(&st->timeouts, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&st->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                return false;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        // the strip's loads are device-scope: they read past every cache that
        // could hold an older copy; only the compiler must keep them after the poll
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        return true;
    }
    __device__ __forceinline__ void run(const PqUnit& un) {
        strip_at_depth<T, TD>(grids[it.grid], un.pass & 1, it, un.rem ? rem : TD);
    }
    __device__ __forceinline__ void complete(int32_t g) {
        // the strip's stores are device-scope: once complete they are visible
        // to every XCD, so waiting for them is the whole release
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        // every lane adds (lane 0 adds the one), so each lane's stores are
        // ordered before the count by its own fence
        __hip_atomic_fetch_add(&pg[g].done, lane0() ? 1u : 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ __forceinline__ void leave() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        unsigned old = 0;
        if (lane0()) old = __hip_atomic_fetch_add(&st->left, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (uniform(old) + 1 != nwaves) return;
        // the last wave: every other wave has left; clear for the next launch
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        for (int g = (int)(threadIdx.x & 63); g < ngrids; g += 64)
            __hip_atomic_store(&pg[g].done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int q = (int)(threadIdx.x & 63); q < nq; q += 64)
            __hip_atomic_store(&st->queue[q].next, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (lane0()) {
            __hip_atomic_store(&st->abort, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&st->left, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
};

template <typename T, int TD>
__global__ void __launch_bounds__(kPqWaves * 64)
k_batch_persistent(const BatchGrid* __restrict__ grids, const BatchItem* __restrict__ full_items,
                   const BatchItem* __restrict__ rem_items, PqState* st, PqGrid* pg, PqShape shape, int rem,
                   int ngrids, unsigned nwaves, unsigned long long wait_ticks, unsigned max_polls) {
    WaveOps<T, TD> ops{grids, full_items, rem_items, st,         pg,        ngrids,
                       shape.nq, rem,        nwaves,    wait_ticks, max_polls, BatchItem{}};
    pq_worker(ops, shape);
}

template <typename T, int TD>
hipError_t launch_p(const BatchGrid* grids, const BatchItem* full_items, const BatchItem* rem_items,
                    const PqShape& shape, int64_t units, int rem, PqState* st, PqGrid* pg, int ngrids,
                    long long wait_us, hipStream_t s) {
    const auto kernel = k_batch_persistent<T, TD>;
    static const int bpc = blocks_per_cu(kernel, kPqWaves * 64);
    // as many workgroups as the device holds at once (more would only queue)
    const int64_t takes = (units + shape.take - 1) / shape.take;
    int64_t nb = std::min<int64_t>((takes + kPqWaves - 1) / kPqWaves, (int64_t)bpc * device_cu_count());
    // workgroup b runs on XCD b mod 8: a multiple of the queue count starts
    // waves at every queue
    nb = (nb + shape.nq - 1) / shape.nq * shape.nq;
    // a limit of 0 makes the first poll that finds a wait unmet run out
    const unsigned long long ticks = (unsigned long long)wait_us * kPqTicksPerUs;
    const unsigned polls = wait_us > 0 ? kPqMaxPolls : 0u;
    hipLaunchKernelGGL(kernel, dim3((unsigned)nb), dim3(kPqWaves * 64), 0, s, grids, full_items, rem_items, st, pg,
                       shape, rem, ngrids, (unsigned)(nb * kPqWaves), ticks, polls);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_typed(const BatchGrid* grids, const BatchItem* full_items, const BatchItem* rem_items,
                        const PqShape& shape, int64_t units, int tdepth, int rem, PqState* st, PqGrid* pg,
                        int ngrids, long long wait_us, hipStream_t s) {
    switch (tdepth) {
        case 1: return launch_p<T, 1>(grids, full_items, rem_items, shape, units, rem, st, pg, ngrids, wait_us, s);
        case 2: return launch_p<T, 2>(grids, full_items, rem_items, shape, units, rem, st, pg, ngrids, wait_us, s);
        case 3: return launch_p<T, 3>(grids, full_items, rem_items, shape, units, rem, st, pg, ngrids, wait_us, s);
        case 4: return launch_p<T, 4>(grids, full_items, rem_items, shape, units, rem, st, pg, ngrids, wait_us, s);
        case 5: return launch_p<T, 5>(grids, full_items, rem_items, shape, units, rem, st, pg, ngrids, wait_us, s);
        case 6: return launch_p<T, 6>(grids, full_items, rem_items, shape, units, rem, st, pg, ngrids, wait_us, s);
        case 7: return launch_p<T, 7>(grids, full_items, rem_items, shape, units, rem, st, pg, ngrids, wait_us, s);
        case 8: return launch_p<T, 8>(grids, full_items, rem_items, shape, units, rem, st, pg, ngrids, wait_us, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_batch_persistent(const BatchGrid* grids, const BatchItem* full_items, const BatchItem* rem_items,
                                   const PqShape& shape, int64_t units, int tdepth, int rem, PqState* st,
                                   PqGrid* pg, int ngrids, long long wait_us, int dtype, hipStream_t s) {
    if (units <= 0) return hipSuccess;
    if (rem < 0 || rem >= tdepth || shape.nq < 1 || shape.nq > kPqMaxQueues || shape.take < 1)
        return hipErrorInvalidValue;
    if (wait_us < 0 || wait_us > (1ll << 40)) return hipErrorInvalidValue;
    if (dtype == LOPE_F32)
        return launch_typed<float>(grids, full_items, rem_items, shape, units, tdepth, rem, st, pg, ngrids, wait_us, s);
    return launch_typed<double>(grids, full_items, rem_items, shape, units, tdepth, rem, st, pg, ngrids, wait_us, s);
}

}  // namespace lope
