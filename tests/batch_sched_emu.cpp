// CPU emulation of the batched form's persistent single-launch scheduler.
//
// The persistent mode (switched off in the library) runs one kernel per step
// whose workgroups take work items from an atomic queue head, wait (bounded
// in time) until the counter of their domain's previous stage reaches that
// stage's item count, do the item and count it with a release.  This program
// builds the same programs as the library (batch_program.hpp) for a list of
// domains and checks the protocol on the host:
//   1. the layout: every item's dependency names an earlier non-empty stage
//      of its own domain whose item count equals the item's `need`, and
//      every item it depends on sits earlier in the queue;
//   2. emulation with host threads standing in for resident workgroups,
//      with the kernel's atomics and memory orders: every item runs once,
//      every wait that succeeds finds its previous stage complete, and no
//      wait reaches the time bound (no deadlock), for several worker counts
//      and random delays, twice in a row after a counter reset (replays);
//   3. the error exit: with one item made slower than the wait bound, the
//      waits behind it fail, the error flag is raised, and every worker
//      still drains the queue and ends.
//
// Input (stdin): lines "nx ny nz S dtype nsrc ndir"; output: one line per
// check, "ok ..." or "FAIL ...", and exit status 0 only if all passed.
#include <atomic>
#include <cstdlib>
#include <chrono>
#include <cstdio>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "batch_program.hpp"

using namespace bfvm;
using Clock = std::chrono::steady_clock;

static int g_fail = 0;

static void report(bool ok, const std::string& what)
{
    std::printf("%s %s\n", ok ? "ok" : "FAIL", what.c_str());
    if (!ok) ++g_fail;
}

// 1. the layout
static bool check_layout(const ProgramLayout& P, std::string* why)
{
    const int64_t nc = P.ncounters;
    std::vector<int64_t> count(nc, 0), last_index(nc, -1);
    std::vector<int32_t> dom_of(nc, -1);
    for (size_t i = 0; i < P.items.size(); ++i) {
        const BItem& it = P.items[i];
        if (it.done < 0 || it.done >= nc) { *why = "done counter out of range"; return false; }
        if (dom_of[it.done] >= 0 && dom_of[it.done] != it.dom) { *why = "counter shared by two domains"; return false; }
        dom_of[it.done] = it.dom;
        ++count[it.done];
        last_index[it.done] = (int64_t)i;
    }
    for (size_t i = 0; i < P.items.size(); ++i) {
        const BItem& it = P.items[i];
        if (it.dep < 0) continue;
        if (it.dep >= nc) { *why = "dep counter out of range"; return false; }
        if (dom_of[it.dep] != it.dom) { *why = "dependency on another domain's stage"; return false; }
        if (it.dep >= it.done) { *why = "dependency on a later stage"; return false; }
        if ((int64_t)it.need != count[it.dep]) { *why = "need differs from the stage's item count"; return false; }
        if (last_index[it.dep] >= (int64_t)i) { *why = "a depended-on item is queued after its dependent"; return false; }
    }
    // per domain, each non-empty stage but the first depends on the one before
    for (int64_t c = 0; c < nc; ++c) {
        for (const BItem& it : P.items) {
            if (it.done != c) continue;
            int64_t prev = -1;
            for (int64_t k = c - 1; k >= 0; --k)
                if (dom_of[k] == it.dom) { prev = k; break; }
            if (it.dep != prev) { *why = "dependency is not the domain's previous stage"; return false; }
            break;
        }
    }
    return true;
}

// 2./3. emulation of the kernel loop
struct Run {
    bool finished = false;   // every worker ended before the watchdog
    uint32_t err = 0;
    int64_t twice = 0;       // items run more than once
    int64_t missed = 0;      // items never run
    int64_t early = 0;       // items that passed a successful wait before their stage was complete
    int64_t timeouts = 0;    // waits that reached the bound
    double seconds = 0;
};

static Run emulate(const ProgramLayout& P, int workers, double bound_s, int64_t slow_item, double slow_s,
                   unsigned seed, int replays)
{
    Run R;
    const int64_t n = (int64_t)P.items.size();
    std::vector<std::atomic<uint32_t>> cnt(P.ncounters);
    std::vector<std::atomic<int>> runs(n);
    std::vector<std::vector<int64_t>> members(P.ncounters);
    for (int64_t i = 0; i < n; ++i) members[P.items[i].done].push_back(i);
    std::atomic<int64_t> early{0}, timeouts{0};
    for (auto& r : runs) r.store(0);
    const auto t_start = Clock::now();
    for (int rep = 0; rep < replays; ++rep) {
        // the reset kernel that precedes every launch
        std::atomic<uint32_t> head{0}, err{0};
        for (auto& c : cnt) c.store(0);
        for (auto& r : runs) r.store(0);
        std::atomic<int> alive{workers};
        std::vector<std::thread> pool;
        for (int w = 0; w < workers; ++w) {
            pool.emplace_back([&, w]() {
                std::mt19937 rng(seed * 7919u + (unsigned)w * 104729u + (unsigned)rep);
                std::uniform_int_distribution<int> jitter(0, 40);
                for (;;) {
                    const int64_t idx = (int64_t)head.fetch_add(1u, std::memory_order_relaxed);
                    if (idx >= n) break;
                    const BItem& it = P.items[idx];
                    bool ok = true;
                    if (it.dep >= 0) {
                        const auto t0 = Clock::now();
                        while (cnt[it.dep].load(std::memory_order_relaxed) < it.need) {
                            if (err.load(std::memory_order_relaxed)) { ok = false; break; }
                            std::this_thread::yield();
                            if (std::chrono::duration<double>(Clock::now() - t0).count() > bound_s) {
                                err.fetch_or(1u, std::memory_order_relaxed);
                                timeouts.fetch_add(1);
                                ok = false;
                                break;
                            }
                        }
                        if (ok) std::atomic_thread_fence(std::memory_order_acquire);
                        if (ok)
                            for (int64_t j : members[it.dep])
                                if (runs[j].load(std::memory_order_relaxed) == 0) { early.fetch_add(1); break; }
                    }
                    // the item's work
                    if (idx == slow_item) std::this_thread::sleep_for(std::chrono::duration<double>(slow_s));
                    else if (jitter(rng) == 0) std::this_thread::sleep_for(std::chrono::microseconds(jitter(rng)));
                    runs[idx].fetch_add(1, std::memory_order_relaxed);
                    // publish, then count
                    std::atomic_thread_fence(std::memory_order_release);
                    cnt[it.done].fetch_add(1u, std::memory_order_relaxed);
                }
                alive.fetch_sub(1);
            });
        }
        // watchdog: a worker stuck for good would keep `alive` above zero
        const auto tw = Clock::now();
        while (alive.load() > 0 && std::chrono::duration<double>(Clock::now() - tw).count() < 60.0)
            std::this_thread::sleep_for(std::chrono::milliseconds(1));
        if (alive.load() > 0) {
            // a worker that never ends: the protocol can hang; stop here
            std::printf("FAIL a worker did not end within 60 s (%d workers)\n", workers);
            std::fflush(stdout);
            std::_Exit(2);
        }
        for (auto& t : pool) t.join();
        R.err |= err.load();
        for (int64_t i = 0; i < n; ++i) {
            const int r = runs[i].load();
            if (r == 0) ++R.missed;
            if (r > 1) ++R.twice;
        }
    }
    R.finished = true;
    R.early = early.load();
    R.timeouts = timeouts.load();
    R.seconds = std::chrono::duration<double>(Clock::now() - t_start).count();
    return R;
}

int main()
{
    std::vector<BDomain> doms;
    int nx, ny, nz, S, dt;
    long long nsrc, ndir;
    while (std::scanf("%d %d %d %d %d %lld %lld", &nx, &ny, &nz, &S, &dt, &nsrc, &ndir) == 7) {
        BDomain d{};
        d.dtype = dt;
        d.S = S;
        d.nx = nx;
        d.ny = ny;
        d.nz = nz;
        d.nsrc = nsrc;
        d.ndir = ndir;
        default_batch_plan(d, BFVM_BATCH_PERSISTENT);
        doms.push_back(d);
    }
    if (doms.empty()) {
        std::printf("FAIL no domains read\n");
        return 1;
    }
    std::vector<int32_t> all(doms.size()), subset;
    for (size_t i = 0; i < doms.size(); ++i) all[i] = (int32_t)i;
    for (size_t i = 0; i < doms.size() && i < 32; ++i) subset.push_back((int32_t)i);
    struct Case {
        std::string name;
        ProgramLayout P;
    };
    std::vector<Case> cases;
    for (int64_t chunk : {int64_t(1) << 12, int64_t(1) << 14, int64_t(1) << 17}) {
        Case f{"forward, " + std::to_string(doms.size()) + " domains, chunk " + std::to_string(chunk), {}};
        build_layout(doms, chunk, all, forward_program(), f.P);
        cases.push_back(std::move(f));
        Case a{"reverse step of domains 0.." + std::to_string(subset.size() - 1) + ", chunk " + std::to_string(chunk),
               {}};
        build_layout(doms, chunk, subset, adjoint_program(), a.P);
        cases.push_back(std::move(a));
    }
    for (const Case& c : cases) {
        std::string why;
        const bool ok = check_layout(c.P, &why);
        report(ok, "layout: " + c.name + " (" + std::to_string(c.P.items.size()) + " items, " +
                       std::to_string(c.P.ncounters) + " counters)" + (ok ? "" : ": " + why));
    }
    unsigned seed = 1;
    for (const Case& c : cases) {
        for (int workers : {1, 3, 16, 64, 512}) {
            const Run r = emulate(c.P, workers, 10.0, -1, 0.0, seed++, 2);
            const bool ok = r.finished && r.err == 0 && r.twice == 0 && r.missed == 0 && r.early == 0 &&
                            r.timeouts == 0;
            report(ok, "protocol: " + c.name + ", " + std::to_string(workers) + " workers, 2 launches: " +
                           (r.finished ? "ended" : "did not end") + ", timeouts " + std::to_string(r.timeouts) +
                           ", early " + std::to_string(r.early) + ", missed " + std::to_string(r.missed) +
                           ", twice " + std::to_string(r.twice));
        }
    }
    // the error exit: one item in the middle sleeps past the wait bound
    for (const Case& c : cases) {
        const int64_t slow = (int64_t)c.P.items.size() / 2;
        const Run r = emulate(c.P, 16, 0.02, slow, 0.2, seed++, 1);
        const bool ok = r.finished && r.err == 1 && r.twice == 0 && r.missed == 0 && r.timeouts >= 1 &&
                        r.seconds < 30.0;
        report(ok, "error exit: " + c.name + ": " + (r.finished ? "ended" : "did not end") + ", flag " +
                       std::to_string(r.err) + ", timeouts " + std::to_string(r.timeouts) + ", missed " +
                       std::to_string(r.missed) + ", " + std::to_string(r.seconds) + " s");
    }
    std::printf("%d failed\n", g_fail);
    return g_fail ? 1 : 0;
}
