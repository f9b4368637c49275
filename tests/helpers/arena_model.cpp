// Host model of the asynchronous scheduler's work-link protocol: per-worker
// stashes (free / ready / one partial link per event), spills to and refills
// from a global arena of links held in lock-free (head, tail) queues that are
// claimed by atomic exchange, and the drained-stash exit rules.  Particles are
// counters of remaining events; the model checks that every particle finishes
// exactly once, for many workers running concurrently on host threads.
//
// Bounded waits: every wait (for a queue, an empty link, links in flight)
// gives up once the arena's fill count has not changed for a wall-clock
// budget (no worker anywhere spilled or refilled: nothing can free what the
// wait needs), or at once when the run has already failed for capacity (a
// worker that fails publishes it at once), so an exhausted arena is reported
// within milliseconds while a slow but moving arena is waited for; a failed
// run stops sourcing.
//
// Build: g++ -O1 -std=c++17 -pthread [-fsanitize=thread] arena_model.cpp
// Run:   ./a.out <workers> <particles> <links> <force_spill> <consolidate> <seed> [arena_links] [budget_ms]
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

namespace {

constexpr uint32_t NIL = 0xFFFFFFFFu;
constexpr uint64_t Q_EMPTY = ~0ull;
constexpr uint64_t Q_CLAIMED = 0xFFFFFFFEFFFFFFFEull;
constexpr int Q = 64, SLOTS = 64, E = 2, DONATE_BELOW = 32;

uint32_t qh(uint64_t q) { return (uint32_t)(q >> 32); }
uint32_t qt(uint64_t q) { return (uint32_t)q; }
uint64_t qp(uint32_t h, uint32_t t) { return ((uint64_t)h << 32) | t; }

struct Particle {
    int32_t id;
    int32_t left;   // events still to run
};

using Clock = std::chrono::steady_clock;

struct Arena {
    int n;
    std::atomic<uint32_t> failed{0};             // the run has failed for capacity
    Clock::duration budget = std::chrono::milliseconds(20);
    // keep waiting: the run has not failed and the fill count changed within
    // the budget (w holds the start of the wait and the count last seen)
    struct Wait {
        Clock::time_point t0{};
        uint32_t seen = 0;
        bool started = false;
    };
    bool wait_on(Wait &w) const
    {
        if (failed.load(std::memory_order_relaxed) != 0) return false;
        Clock::time_point now = Clock::now();
        uint32_t f = fill.load(std::memory_order_relaxed);
        if (!w.started || f != w.seen) {
            w.started = true;
            w.t0 = now;
            w.seen = f;
            return true;
        }
        return now - w.t0 < budget;
    }
    void fail()
    {
        err.fetch_add(1);
        failed.store(1, std::memory_order_relaxed);
    }
    std::vector<std::vector<Particle>> data;   // link contents
    std::vector<std::atomic<uint32_t>> hdr, next;
    std::atomic<uint64_t> qfull[Q], qempty[Q];
    std::atomic<uint32_t> fill{0};
    std::atomic<uint32_t> active{0};
    std::atomic<uint64_t> cursor{0};
    std::atomic<uint64_t> spills{0}, refills{0}, err{0};
    explicit Arena(int links) : n(links), data(links, std::vector<Particle>(SLOTS)), hdr(links), next(links)
    {
        for (int i = 0; i < n; ++i) next[i].store(i + Q < n ? (uint32_t)(i + Q) : NIL);
        for (int q = 0; q < Q; ++q) {
            qfull[q].store(Q_EMPTY);
            if (q < n) qempty[q].store(qp((uint32_t)q, (uint32_t)(q + Q * ((n - 1 - q) / Q))));
            else qempty[q].store(Q_EMPTY);
        }
    }
    uint32_t pop(std::atomic<uint64_t> *slots, uint32_t start)
    {
        for (int i = 0; i < Q; ++i) {
            int s = (int)((start + i) % Q);
            uint64_t peek = slots[s].load(std::memory_order_relaxed);
            if (peek == Q_CLAIMED || qh(peek) == NIL) continue;
            uint64_t v = slots[s].exchange(Q_CLAIMED, std::memory_order_acq_rel);
            if (v == Q_CLAIMED) continue;
            if (qh(v) == NIL) {
                slots[s].exchange(v, std::memory_order_acq_rel);
                continue;
            }
            uint32_t a = qh(v);
            uint32_t nh = next[a].load(std::memory_order_relaxed);
            slots[s].exchange(nh == NIL ? Q_EMPTY : qp(nh, qt(v)), std::memory_order_acq_rel);
            return a;
        }
        return NIL;
    }
    bool push(std::atomic<uint64_t> *slots, uint32_t start, uint32_t a)
    {
        next[a].store(NIL, std::memory_order_relaxed);
        for (Wait w; wait_on(w);) {
            for (int i = 0; i < Q; ++i) {
                int s = (int)((start + i) % Q);
                uint64_t v = slots[s].exchange(Q_CLAIMED, std::memory_order_acq_rel);
                if (v == Q_CLAIMED) continue;
                uint64_t nv;
                if (qh(v) == NIL) {
                    nv = qp(a, a);
                } else {
                    next[qt(v)].store(a, std::memory_order_relaxed);
                    nv = qp(qh(v), a);
                }
                slots[s].exchange(nv, std::memory_order_acq_rel);
                return true;
            }
            std::this_thread::yield();
        }
        return false;
    }
};

struct Link {
    std::vector<Particle> p = std::vector<Particle>(SLOTS);
    int cnt = 0, ev = 0;
};

struct Worker {
    Arena &A;
    uint64_t total;
    int L, force_spill, consolidate;
    uint32_t start;
    std::vector<Link> link;
    uint32_t freem, readym = 0;
    int part[E];
    uint32_t tick = 0;
    std::vector<int> &done;
    std::mt19937 rng;

    Worker(Arena &a, uint64_t tot, int links, int fs, int cons, uint32_t st, std::vector<int> &d, uint32_t seed)
        : A(a), total(tot), L(links), force_spill(fs), consolidate(cons), start(st), link(links),
          freem((1u << links) - 1u), done(d), rng(seed)
    {
        for (int k = 0; k < E; ++k) part[k] = -1;
    }

    bool spill(int v)
    {
        uint32_t a = NIL;
        for (Arena::Wait w; a == NIL && A.wait_on(w);) {
            a = A.pop(A.qempty, start);
            if (a == NIL) std::this_thread::yield();
        }
        if (a == NIL) return false;
        A.data[a] = link[v].p;
        A.hdr[a].store((uint32_t)link[v].ev | ((uint32_t)link[v].cnt << 8), std::memory_order_relaxed);
        std::atomic_thread_fence(std::memory_order_release);
        if (!A.push(A.qfull, start, a)) return false;
        A.fill.fetch_add(1);
        A.spills.fetch_add(1);
        return true;
    }

    int alloc()
    {
        if (freem == 0) {
            if (readym == 0) { A.fail(); return -1; }
            int v = __builtin_ctz(readym);
            if (!spill(v)) { A.fail(); return -1; }
            readym &= ~(1u << v);
            freem |= 1u << v;
        }
        int l = __builtin_ctz(freem);
        freem &= ~(1u << l);
        return l;
    }

    // deposit particles (all of event k)
    void deposit(int k, const std::vector<Particle> &ps)
    {
        int n = (int)ps.size();
        if (n == 0) return;
        int pl = part[k], f = 0;
        if (pl < 0) {
            pl = alloc();
            if (pl < 0) return;
            link[pl].ev = k;
            link[pl].cnt = 0;
            part[k] = pl;
        } else {
            f = link[pl].cnt;
        }
        int take = n < SLOTS - f ? n : SLOTS - f;
        for (int r = 0; r < take; ++r) link[pl].p[f + r] = ps[r];
        if (f + take < SLOTS) { link[pl].cnt = f + take; return; }
        link[pl].cnt = SLOTS;
        readym |= 1u << pl;
        part[k] = -1;
        if (force_spill > 0 && ++tick % (uint32_t)force_spill == 0) {
            if (spill(pl)) { readym &= ~(1u << pl); freem |= 1u << pl; }
            else A.fail();
        }
        if (n > take) {
            int p2 = alloc();
            if (p2 < 0) return;
            link[p2].ev = k;
            link[p2].cnt = n - take;
            part[k] = p2;
            for (int r = take; r < n; ++r) link[p2].p[r - take] = ps[r];
        }
    }

    void run_link(int l)
    {
        std::vector<Particle> out[E];
        Link &lk = link[l];
        int ev = lk.ev, c = lk.cnt;
        std::vector<Particle> ps(lk.p.begin(), lk.p.begin() + c);
        freem |= 1u << l;
        for (auto &p : ps) {
            p.left -= 1;
            if (p.left <= 0) {
                if (done[p.id] != 0) A.err.fetch_add(1);   // finished twice
                done[p.id] += 1;
            } else {
                out[(ev + 1) % E].push_back(p);
            }
        }
        for (int k = 0; k < E; ++k) deposit(k, out[k]);
    }

    bool refill()
    {
        if (freem == 0 || A.fill.load() == 0) return false;
        uint32_t a = A.pop(A.qfull, start);
        if (a == NIL) return false;
        A.fill.fetch_sub(1);
        std::atomic_thread_fence(std::memory_order_acquire);
        uint32_t h = A.hdr[a].load(std::memory_order_relaxed);
        int ev = (int)(h & 0xff), c = (int)(h >> 8);
        std::vector<Particle> ps(A.data[a].begin(), A.data[a].begin() + c);
        A.refills.fetch_add(1);
        if (!A.push(A.qempty, start, a)) A.fail();
        if (!consolidate || c == SLOTS) {
            int l = __builtin_ctz(freem);
            freem &= ~(1u << l);
            link[l].ev = ev;
            link[l].cnt = c;
            for (int i = 0; i < c; ++i) link[l].p[i] = ps[i];
            readym |= 1u << l;
        } else {
            deposit(ev, ps);
        }
        return true;
    }

    bool last_with_work()
    {
        uint32_t old = A.active.fetch_sub(1, std::memory_order_acq_rel);
        if (old != 1u) return false;
        if (A.fill.load() == 0) return false;
        A.active.fetch_add(1, std::memory_order_acq_rel);
        return true;
    }

    void main_loop()
    {
        bool src_done = false, may_donate = true;
        Arena::Wait idle;                   // the current idle spell's wait
        std::uniform_int_distribution<int> len(1, 40);
        for (;;) {
            int l = -1;
            if (readym) {
                l = __builtin_ctz(readym);
                readym &= ~(1u << l);
            } else if (!src_done) {
                if (A.failed.load(std::memory_order_relaxed)) { src_done = true; continue; }
                uint64_t b = A.cursor.fetch_add(SLOTS);
                if (b >= total) { src_done = true; continue; }
                std::vector<Particle> ps;
                for (uint64_t g = b; g < b + SLOTS && g < total; ++g)
                    ps.push_back(Particle{(int32_t)g, (int32_t)(1 + (g * 2654435761u) % 37)});
                deposit(0, ps);
                continue;
            } else if (refill()) {
                idle = Arena::Wait{};
                continue;
            } else {
                int best = -1, bc = 0, tot = 0;
                for (int k = 0; k < E; ++k)
                    if (part[k] >= 0) {
                        int c = link[part[k]].cnt;
                        tot += c;
                        if (c > bc) { bc = c; best = k; }
                    }
                if (!consolidate) {
                    if (tot > 0) {
                        l = part[best];
                        part[best] = -1;
                    } else {
                        if (A.fill.load() != 0 && A.wait_on(idle)) {
                            std::this_thread::yield();
                            continue;
                        }
                        break;
                    }
                } else if (tot > 0 && (tot >= DONATE_BELOW || !may_donate)) {
                    l = part[best];
                    part[best] = -1;
                } else {
                    if (tot > 0) {
                        for (int k = 0; k < E; ++k) {
                            int pl = part[k];
                            if (pl < 0) continue;
                            if (spill(pl)) { part[k] = -1; freem |= 1u << pl; }
                            else { A.fail(); may_donate = false; }
                        }
                        if (!may_donate) continue;
                    }
                    if (last_with_work()) {
                        may_donate = false;
                        if (A.wait_on(idle)) continue;
                        A.fail();
                    }
                    break;
                }
            }
            idle = Arena::Wait{};           // the wait budget is per idle spell
            run_link(l);
        }
        if (!consolidate) A.active.fetch_sub(1);
    }
};

}  // namespace

int main(int argc, char **argv)
{
    int workers = argc > 1 ? atoi(argv[1]) : 8;
    uint64_t particles = argc > 2 ? strtoull(argv[2], nullptr, 10) : 20000;
    int links = argc > 3 ? atoi(argv[3]) : 3;
    int force = argc > 4 ? atoi(argv[4]) : 0;
    int cons = argc > 5 ? atoi(argv[5]) : 0;
    uint32_t seed = argc > 6 ? (uint32_t)atoi(argv[6]) : 1;
    int arena_links = argc > 7 ? atoi(argv[7]) : workers * (E + 2) + 1024;
    int budget_ms = argc > 8 ? atoi(argv[8]) : 20;
    Arena A(arena_links);
    A.budget = std::chrono::milliseconds(budget_ms);
    Clock::time_point t_start = Clock::now();
    A.active.store((uint32_t)workers);
    std::vector<int> done(particles, 0);
    std::vector<std::thread> th;
    std::vector<Worker *> ws;
    for (int w = 0; w < workers; ++w)
        ws.push_back(new Worker(A, particles, links, force, cons, (uint32_t)w * 2654435761u, done, seed + w));
    for (int w = 0; w < workers; ++w) th.emplace_back([&, w] { ws[w]->main_loop(); });
    for (auto &t : th) t.join();
    double ms = std::chrono::duration<double, std::milli>(Clock::now() - t_start).count();
    uint64_t missing = 0, twice = 0;
    for (uint64_t i = 0; i < particles; ++i) {
        if (done[i] == 0) ++missing;
        if (done[i] > 1) ++twice;
    }
    printf("workers=%d particles=%llu links=%d force=%d consolidate=%d spills=%llu refills=%llu fill=%u "
           "missing=%llu twice=%llu err=%llu failed=%u ms=%.1f\n",
           workers, (unsigned long long)particles, links, force, cons, (unsigned long long)A.spills.load(),
           (unsigned long long)A.refills.load(), A.fill.load(), (unsigned long long)missing,
           (unsigned long long)twice, (unsigned long long)A.err.load(), A.failed.load(), ms);
    for (auto *w : ws) delete w;
    return (missing || twice || A.err.load()) ? 1 : 0;
}
