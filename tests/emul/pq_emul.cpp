// CPU emulation of the persistent batched launch's scheduling: the worker
// loop of batch_queue.h (the code the kernel runs) driven by host threads
// standing in for waves, with std::atomic in place of the device atomics.
//
// A launch has W waves but only R run at a time (R threads, each running
// waves one after another, as workgroups that are not yet resident start when
// others leave).  The strip body checks, against shadow counters, that every
// strip of the grid's earlier passes is complete and that no strip of a later
// pass of the grid has started; every unit must run exactly once, no wait may
// run out, and after the launch the queue state must be back at zero (checked
// by running several launches on one state).  A planted mistake (each grid
// claims one strip more per pass than it has, so a unit of pass 1 or later
// waits for completions that cannot come) must end every wave through the
// time limit and the abort flag, with the state reset as well; one strip too
// few per pass must show up as dependency violations.
//
// Usage: pq_emul  (prints "ok" and exits 0, else prints the failures and exits 1)
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "batch_queue.h"

namespace {

using namespace lope;

struct Item {
    int32_t grid;
};

struct Launch {
    std::vector<int32_t> full_strips;   // per grid, strips of one full pass
    std::vector<int32_t> rem_strips;    // per grid, strips of the remainder pass
    std::vector<Item> full_items;       // grid-major and grouped by queue, as the plan builds them
    std::vector<Item> rem_items;
    PqQueue share[kPqMaxQueues] = {};
    PqShape shape{};
    int ngrids = 0;
    int64_t units = 0;
};

// Grid g goes to queue g mod nq; the tables list queue 0's grids first.
Launch make_launch(std::mt19937& rng, int ngrids, int full, bool with_rem, int max_strips, int nq, int take) {
    Launch L;
    L.ngrids = ngrids;
    std::uniform_int_distribution<int> ns(0, max_strips);
    for (int g = 0; g < ngrids; ++g) {
        const int fs = ns(rng);   // 0: an empty grid
        L.full_strips.push_back(fs);
        L.rem_strips.push_back((with_rem && fs) ? 1 + (fs * 3) / 4 : 0);
    }
    for (int q = 0; q < nq; ++q) {
        L.share[q].full_begin = (int64_t)L.full_items.size();
        L.share[q].rem_begin = (int64_t)L.rem_items.size();
        for (int g = q; g < ngrids; g += nq) {
            for (int k = 0; k < L.full_strips[(size_t)g]; ++k) L.full_items.push_back(Item{g});
            for (int k = 0; k < L.rem_strips[(size_t)g]; ++k) L.rem_items.push_back(Item{g});
        }
        L.share[q].full_count = (int64_t)L.full_items.size() - L.share[q].full_begin;
        L.share[q].rem_count = (int64_t)L.rem_items.size() - L.share[q].rem_begin;
    }
    L.shape.full = full;
    L.shape.nq = nq;
    L.shape.take = take;
    L.units = (int64_t)full * (int64_t)L.full_items.size() + (int64_t)L.rem_items.size();
    return L;
}

// Device state of one plan (kept across launches, as on the device).
struct State {
    std::atomic<uint64_t> next[kPqMaxQueues];
    std::atomic<uint32_t> left{0};
    std::atomic<uint32_t> abort{0};
    std::atomic<uint32_t> timeouts{0};
    std::vector<std::atomic<uint32_t>> done;
    explicit State(int ngrids) : done((size_t)ngrids) {
        for (auto& d : done) d.store(0);
        for (auto& n : next) n.store(0);
    }
};

// Shadow bookkeeping of one launch (checks only).
struct Shadow {
    int npasses;
    std::vector<std::atomic<int32_t>> started, finished;   // [grid * npasses + pass]
    std::vector<std::atomic<int32_t>> runs;                // per (table, strip, pass)
    std::atomic<int64_t> violations{0};
    Shadow(int ngrids, int npasses, int64_t units)
        : npasses(npasses), started((size_t)ngrids * npasses), finished((size_t)ngrids * npasses),
          runs((size_t)units) {
        for (auto& v : started) v.store(0);
        for (auto& v : finished) v.store(0);
        for (auto& v : runs) v.store(0);
    }
};

struct HostOps {
    const Launch* L;
    State* st;
    Shadow* sh;
    uint32_t nwaves;
    std::chrono::microseconds limit;
    int mistake;          // planted: 1 one strip too many per pass (a wait never satisfied),
                          // 2 one too few (a unit may start before its inputs are complete)
    std::mt19937* rng;
    int32_t first;
    int64_t unit = -1;   // the unit's slot in Shadow::runs
    int32_t grid = -1;

    int32_t first_queue() { return first; }
    PqQueue queue(int32_t q) { return L->share[q]; }
    bool aborted() { return st->abort.load(std::memory_order_relaxed) != 0; }
    int64_t take(int32_t q, int32_t n) { return (int64_t)st->next[q].fetch_add((uint64_t)n, std::memory_order_relaxed); }
    int32_t grid_of(const PqUnit& un) {
        grid = un.rem ? L->rem_items[(size_t)un.strip].grid : L->full_items[(size_t)un.strip].grid;
        unit = un.rem ? (int64_t)L->shape.full * (int64_t)L->full_items.size() + un.strip
                      : (int64_t)un.pass * (int64_t)L->full_items.size() + un.strip;
        return grid;
    }
    int32_t full_strips(int32_t g) {
        const int32_t fs = L->full_strips[(size_t)g];
        return fs + (mistake == 1 ? 1 : 0) - (mistake == 2 && fs > 1 ? 1 : 0);
    }
    bool wait(int32_t g, int64_t need) {
        const auto t0 = std::chrono::steady_clock::now();
        for (;;) {
            if ((int64_t)st->done[(size_t)g].load(std::memory_order_relaxed) >= need) break;
            if (aborted()) return false;
            if (std::chrono::steady_clock::now() - t0 > limit) {
                st->timeouts.fetch_add(1, std::memory_order_relaxed);
                st->abort.store(1, std::memory_order_relaxed);
                return false;
            }
            std::this_thread::yield();
        }
        std::atomic_thread_fence(std::memory_order_acquire);
        return true;
    }
    int32_t strips_in(int32_t g, int32_t pass) const {
        return pass < L->shape.full ? L->full_strips[(size_t)g] : L->rem_strips[(size_t)g];
    }
    void run(const PqUnit& un) {
        const int P = sh->npasses;
        if (sh->runs[(size_t)unit].fetch_add(1) != 0) sh->violations.fetch_add(1);
        for (int q = 0; q < un.pass; ++q)
            if (sh->finished[(size_t)grid * P + q].load() != strips_in(grid, q)) sh->violations.fetch_add(1);
        for (int q = un.pass + 1; q < P; ++q)
            if (sh->started[(size_t)grid * P + q].load() != 0) sh->violations.fetch_add(1);
        sh->started[(size_t)grid * P + un.pass].fetch_add(1);
        if (((*rng)() & 7) == 0) std::this_thread::sleep_for(std::chrono::microseconds((*rng)() % 50));
        sh->finished[(size_t)grid * P + un.pass].fetch_add(1);
    }
    void complete(int32_t g) { st->done[(size_t)g].fetch_add(1, std::memory_order_release); }
    void leave() {
        const uint32_t old = st->left.fetch_add(1, std::memory_order_acq_rel);
        if (old + 1 != nwaves) return;
        for (auto& d : st->done) d.store(0, std::memory_order_relaxed);
        for (auto& n : st->next) n.store(0, std::memory_order_relaxed);
        st->abort.store(0, std::memory_order_relaxed);
        st->left.store(0, std::memory_order_relaxed);
    }
};

// One launch of W waves on R resident slots; returns the failures found
// (with mistake 2, adds the dependency violations seen to *violations).
int run_launch(const Launch& L, State& st, int W, int R, int mistake, unsigned seed, const char* name,
               int64_t* violations = nullptr) {
    const int npasses = L.shape.full + (L.rem_items.empty() ? 0 : 1);
    const int64_t units = L.units;
    Shadow sh(L.ngrids, npasses > 0 ? npasses : 1, units > 0 ? units : 1);
    std::atomic<int> next_wave{0};
    const auto limit = std::chrono::microseconds(mistake == 1 ? 20000 : 5000000);
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<std::thread> slots;
    for (int r = 0; r < R; ++r)
        slots.emplace_back([&, r]() {
            std::mt19937 rng(seed * 7919u + (unsigned)r);
            for (;;) {
                const int w = next_wave.fetch_add(1);
                if (w >= W) break;
                HostOps ops{&L, &st, &sh, (uint32_t)W, limit, mistake, &rng, w % L.shape.nq};
                pq_worker(ops, L.shape);
            }
        });
    for (auto& t : slots) t.join();
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int bad = 0;
    auto failf = [&](const char* what, long long v) {
        std::printf("FAIL %s: %s (%lld)\n", name, what, v);
        ++bad;
    };
    for (auto& n : st.next)
        if (n.load() != 0) failf("queue counter not reset", (long long)n.load());
    if (st.left.load() != 0 || st.abort.load() != 0) failf("queue state not reset", 0);
    for (auto& d : st.done)
        if (d.load() != 0) {
            failf("grid counter not reset", (long long)d.load());
            break;
        }
    if (mistake == 2) {
        *violations += sh.violations.load();
        return bad;
    }
    if (mistake == 1) {
        // a unit of a second pass whose grid has strips waits in vain
        const bool waits = !L.full_items.empty() && (L.shape.full >= 2 || (L.shape.full >= 1 && !L.rem_items.empty()));
        if (waits && st.timeouts.load() == 0) failf("planted wait did not time out", 0);
        if (secs > 5.0) failf("abort took too long (ms)", (long long)(secs * 1000));
        st.timeouts.store(0);
        return bad;
    }
    if (st.timeouts.load() != 0) failf("waits ran out", (long long)st.timeouts.load());
    if (sh.violations.load() != 0) failf("dependency violations", (long long)sh.violations.load());
    for (int64_t u = 0; u < units; ++u)
        if (sh.runs[(size_t)u].load() != 1) {
            failf("unit not run exactly once", (long long)u);
            break;
        }
    return bad;
}

}  // namespace

int main() {
    std::mt19937 rng(12345);
    int bad = 0, launches = 0;
    int64_t under = 0;
    struct Case {
        int ngrids, full;
        bool rem;
        int max_strips, W, R, nq, take;
    };
    const Case cases[] = {
        {1, 1, false, 1, 1, 1, 1, 1},      {1, 3, true, 4, 8, 2, 8, 2},       {5, 0, true, 6, 16, 4, 8, 1},
        {7, 8, true, 9, 64, 8, 8, 3},      {24, 9, false, 12, 200, 16, 8, 1}, {64, 2, true, 30, 256, 12, 1, 4},
        {3, 50, false, 3, 40, 6, 2, 1},    {200, 4, true, 5, 512, 16, 8, 8},  {2, 6, true, 40, 3, 3, 8, 5},
        {16, 5, false, 0, 32, 4, 8, 2},    {40, 7, true, 20, 1000, 9, 8, 1},  {9, 6, true, 25, 7, 2, 3, 64},
        {24, 3, true, 12, 5, 3, 8, 1},     {1, 2, true, 4, 1, 1, 8, 1},
    };
    for (const Case& c : cases) {
        const Launch L = make_launch(rng, c.ngrids, c.full, c.rem, c.max_strips, c.nq, c.take);
        State st(c.ngrids);
        char name[160];
        auto label = [&](const char* what) {
            std::snprintf(name, sizeof(name), "grids=%d full=%d rem=%d W=%d R=%d nq=%d take=%d %s", c.ngrids, c.full,
                          (int)c.rem, c.W, c.R, c.nq, c.take, what);
            return name;
        };
        // three launches on one state: each must find it cleared by the last wave
        for (int k = 0; k < 3; ++k) {
            bad += run_launch(L, st, c.W, c.R, 0, 100u * (unsigned)launches + (unsigned)k, label("launch"));
            ++launches;
        }
        bad += run_launch(L, st, c.W, c.R, 1, 7u, label("planted"));
        bad += run_launch(L, st, c.W, c.R, 0, 9u, label("after planted"));
        bad += run_launch(L, st, c.W, c.R, 2, 11u, label("too few"), &under);
    }
    // the checks themselves: counting one strip too few must be caught
    if (under == 0) {
        std::printf("FAIL the dependency check missed a planted undercount\n");
        ++bad;
    }
    if (bad) {
        std::printf("%d failure(s)\n", bad);
        return 1;
    }
    std::printf("ok (%d launches)\n", launches);
    return 0;
}
