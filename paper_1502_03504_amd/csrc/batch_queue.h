// Scheduling of the persistent batched launch: one kernel runs every pass of
// every grid of a batch, each wave taking work units from one queue.
//
// A unit is one strip of one grid in one pass (a pass fuses TD sweeps).
// Units are numbered pass-major: the strips of the full-depth table for pass
// 0, then for pass 1, ..., then the strips of the remainder table (the last,
// shorter pass).  A strip of pass p of grid g reads the state pass p-1 wrote
// and overwrites the buffer pass p-1 read, so it may start only when every
// strip of grid g in passes 0 .. p-1 is complete; a per-grid counter of
// completed strips records that (the first p passes of g hold p times g's
// strips of the full-depth table).
//
// Why the queue cannot deadlock: a unit waits only on units with smaller
// numbers, and units are handed out in increasing order, so every unit a wave
// waits on was handed out before, to a wave that is running (a wave takes a
// unit only once it runs).  The smallest unfinished unit therefore has all of
// its dependencies complete, and its wave finishes it; by induction every
// unit finishes, whatever the number of resident waves.  Each wait is also
// bounded in time: a wave whose wait runs out sets an abort flag, every wave
// then leaves at its next check, and the host reports the failure.
//
// The last wave to leave clears the queue, the flags and the per-grid
// counters, so the next launch starts from zero without any other kernel or
// memory operation (one kernel node when recorded in a graph).
//
// The same worker loop runs in the kernel and in a CPU emulation of it (plain
// C++ with host threads for waves): the policy object supplies the atomics,
// the waits and the strip body.
#pragma once

#include <stdint.h>

// Inlined into the kernel (a call would need a stack) and plain inline C++
// elsewhere.
#if defined(__HIPCC__) || defined(__HIP__)
#define LOPE_HD __host__ __device__ __forceinline__
#else
#define LOPE_HD inline __attribute__((always_inline))
#endif

namespace lope {

// Units of one launch.
struct PqShape {
    int64_t n_full;   // strips in the full-depth table (one pass)
    int64_t n_rem;    // strips in the remainder table (0: no remainder pass)
    int32_t full;     // full passes
};

// Which strip a unit is.
struct PqUnit {
    int32_t pass;     // 0-based pass
    int32_t strip;    // index into that pass's table
    int32_t rem;      // 1: the remainder table (pass == full)
};

LOPE_HD int64_t pq_total(const PqShape& s) { return (int64_t)s.full * s.n_full + s.n_rem; }

LOPE_HD PqUnit pq_unit(const PqShape& s, int64_t u) {
    const int64_t f = (int64_t)s.full * s.n_full;
    PqUnit r;
    if (u < f) {
        r.pass = (int32_t)(u / s.n_full);
        r.strip = (int32_t)(u - (int64_t)r.pass * s.n_full);
        r.rem = 0;
    } else {
        r.pass = s.full;
        r.strip = (int32_t)(u - f);
        r.rem = 1;
    }
    return r;
}

// Completed strips grid g needs before a strip of `pass` may start: all of
// its strips of the earlier passes, which are full passes.
LOPE_HD int64_t pq_need(int32_t pass, int32_t grid_full_strips) {
    return (int64_t)pass * (int64_t)grid_full_strips;
}

// One wave's loop.  Ops provides (all wave-uniform):
//   bool aborted()                 the abort flag is set
//   int64_t take()                 next unit number (one per call per wave)
//   int32_t grid_of(const PqUnit&) the unit's grid (and remembers its strip)
//   int32_t full_strips(int32_t g) g's strips in the full-depth table
//   bool wait(int32_t g, int64_t need)  until g's counter >= need; false if
//                                  the abort flag is set or the wait ran out
//                                  (which sets the flag)
//   void run(const PqUnit&)        the strip's sweeps
//   void complete(int32_t g)       publish the strip's stores, then count it
//   void leave()                   count this wave out; the last one resets
template <class Ops>
LOPE_HD void pq_worker(Ops& ops, const PqShape& s) {
    const int64_t total = pq_total(s);
    for (;;) {
        if (ops.aborted()) break;
        const int64_t u = ops.take();
        if (u >= total) break;
        const PqUnit un = pq_unit(s, u);
        const int32_t g = ops.grid_of(un);
        const int64_t need = pq_need(un.pass, ops.full_strips(g));
        if (need > 0 && !ops.wait(g, need)) break;
        ops.run(un);
        ops.complete(g);
    }
    ops.leave();
}

}  // namespace lope
