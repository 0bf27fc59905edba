// Scheduling of the persistent batched launch: one kernel runs every pass of
// every grid of a batch, each wave taking work units from a few queues.
//
// A unit is one strip of one grid in one pass (a pass fuses TD sweeps).  The
// grids are dealt to NQ queues (the plan's XCD ranges: each queue owns a
// contiguous range of the full-depth strip table and of the remainder table).
// A queue numbers its units pass-major: its strips of the full-depth table
// for pass 0, then for pass 1, ..., then its strips of the remainder table
// (the last, shorter pass).  A strip of pass p of grid g reads the state pass
// p-1 wrote and overwrites the buffer pass p-1 read, so it may start only
// when every strip of grid g in passes 0 .. p-1 is complete; a per-grid
// counter of completed strips records that (the first p passes of g hold p
// times g's strips of the full-depth table).
//
// A wave starts at one queue (workgroup id mod NQ: the XCD it runs on, so a
// queue's strips mostly share one L2), takes TAKE consecutive units at a time
// and runs them in order; when its queue is drained it moves on to the next
// queue, until every queue is drained.
//
// Why the queues cannot deadlock: a unit depends only on units of its own
// grid, hence of its own queue, with smaller numbers.  A queue hands out its
// units in increasing order, and a wave runs the units it took in increasing
// order before taking any others.  Take the smallest unfinished unit m of a
// queue: every unit it depends on is smaller, hence finished; the wave that
// took m has finished its earlier units of the same take (also smaller), so
// it is running m and finishes it.  By induction every unit finishes,
// whatever the number of resident waves (a wave takes units only once it
// runs).  Each wait is also bounded in time: a wave whose wait runs out sets
// an abort flag, every wave then leaves at its next check, and the host
// reports the failure.
//
// The last wave to leave clears the queues, the flags and the per-grid
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

constexpr int kPqMaxQueues = 8;

// Units of one launch.
struct PqShape {
    int32_t full;     // full passes
    int32_t nq;       // queues (1 .. kPqMaxQueues)
    int32_t take;     // units a wave takes at once (>= 1)
    int32_t pad;
};

// One queue's share of the two strip tables.
struct PqQueue {
    int64_t full_begin, full_count;   // strips [full_begin, +full_count) of the full-depth table
    int64_t rem_begin, rem_count;     // strips [rem_begin, +rem_count) of the remainder table
};

// Which strip a unit is.
struct PqUnit {
    int32_t pass;     // 0-based pass
    int32_t rem;      // 1: the remainder table (pass == full)
    int64_t strip;    // index into that pass's table
};

LOPE_HD int64_t pq_total(const PqQueue& q, int32_t full) { return (int64_t)full * q.full_count + q.rem_count; }

LOPE_HD PqUnit pq_unit(const PqQueue& q, int32_t full, int64_t u) {
    const int64_t f = (int64_t)full * q.full_count;
    PqUnit r;
    if (u < f) {
        r.pass = (int32_t)(u / q.full_count);
        r.rem = 0;
        r.strip = q.full_begin + (u - (int64_t)r.pass * q.full_count);
    } else {
        r.pass = full;
        r.rem = 1;
        r.strip = q.rem_begin + (u - f);
    }
    return r;
}

// Completed strips grid g needs before a strip of `pass` may start: all of
// its strips of the earlier passes, which are full passes.
LOPE_HD int64_t pq_need(int32_t pass, int32_t grid_full_strips) {
    return (int64_t)pass * (int64_t)grid_full_strips;
}

// One wave's loop.  Ops provides (all wave-uniform):
//   int32_t first_queue()          where this wave starts (0 .. nq-1)
//   PqQueue queue(int32_t q)       queue q's share of the tables
//   bool aborted()                 the abort flag is set
//   int64_t take(int32_t q, int32_t n)  first of the next n unit numbers of q
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
    const int32_t q0 = ops.first_queue();
    for (int32_t k = 0; k < s.nq; ++k) {
        const int32_t q = (q0 + k) % s.nq;
        const PqQueue qs = ops.queue(q);
        const int64_t total = pq_total(qs, s.full);
        for (;;) {
            if (ops.aborted()) {
                ops.leave();
                return;
            }
            const int64_t u0 = ops.take(q, s.take);
            if (u0 >= total) break;
            const int64_t u1 = u0 + s.take < total ? u0 + s.take : total;
            for (int64_t u = u0; u < u1; ++u) {
                const PqUnit un = pq_unit(qs, s.full, u);
                const int32_t g = ops.grid_of(un);
                const int64_t need = pq_need(un.pass, ops.full_strips(g));
                if (need > 0 && !ops.wait(g, need)) {
                    ops.leave();
                    return;
                }
                ops.run(un);
                ops.complete(g);
            }
        }
    }
    ops.leave();
}

}  // namespace lope
