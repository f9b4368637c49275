// Host model of the block-shared stash of the asynchronous scheduler: the
// wavefronts of a block (host threads here) share one pool of work links
// through lock-free transactions, and spill to / refill from a global arena
// of links held in lock-free (head, tail) queues.  Particles are counters of
// remaining events; every particle must finish exactly once.
//
// Shared stash (one per block):
//  free, ready   bit masks of links; a bit is claimed by an atomic AND whose
//                returned old value shows it was still set
//  part[k]       the link being filled with particles of event k, tagged:
//                (tag << 8) | link, or NONE
//  resv[l]       (tag << 16) | slots reserved; a depositor reserves with a
//                compare-and-swap that requires the tag it read from part[k]
//                and fewer than 64 reserved, so a reservation on a link that
//                has since been recycled fails instead of corrupting it
//  wrt[l]        slots written; the writer that brings it to 64 publishes the
//                link as ready
//  a depositor that fills the last slot takes the link out of part[k]; a
//  drained wavefront closes a partial link (takes it out of part[k], then
//  adds 64 to its reservation), waits until the reserved slots are written
//  and runs it
//  busy          wavefronts of the block holding particles outside the stash
//                (raised once work is taken, so idle wavefronts looking for
//                work never keep each other from seeing the block drained)
//
// Build: g++ -O1 -std=c++17 -pthread [-fsanitize=thread] shared_stash_model.cpp
// Run:   ./a.out <blocks> <waves_per_block> <links> <particles> <force_spill> <arena_links> <seed>
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

namespace {

constexpr uint32_t NIL = 0xFFFFFFFFu;
constexpr uint32_t NONE = 0xFFFFFFFFu;
constexpr uint64_t Q_EMPTY = ~0ull;
constexpr uint64_t Q_CLAIMED = 0xFFFFFFFEFFFFFFFEull;
constexpr int Q = 64, SLOTS = 64, E = 2, MAXL = 32;
using Clock = std::chrono::steady_clock;

uint32_t qh(uint64_t q) { return (uint32_t)(q >> 32); }
uint32_t qt(uint64_t q) { return (uint32_t)q; }
uint64_t qp(uint32_t h, uint32_t t) { return ((uint64_t)h << 32) | t; }

struct Particle {
    int32_t id;
    int32_t left;
};

// global arena: links in lock-free queues of empty and filled links
struct Arena {
    int n;
    std::vector<std::vector<Particle>> data;
    std::vector<std::atomic<uint32_t>> hdr, next;
    std::atomic<uint64_t> qfull[Q], qempty[Q];
    std::atomic<uint32_t> fill{0};
    std::atomic<uint32_t> failed{0};
    std::atomic<uint64_t> cursor{0};
    std::atomic<uint64_t> spills{0}, refills{0}, err{0};
    Clock::duration budget = std::chrono::milliseconds(50);
    explicit Arena(int links) : n(links), data(links, std::vector<Particle>(SLOTS)), hdr(links), next(links)
    {
        for (int i = 0; i < n; ++i) next[i].store(i + Q < n ? (uint32_t)(i + Q) : NIL);
        for (int q = 0; q < Q; ++q) {
            qfull[q].store(Q_EMPTY);
            qempty[q].store(q < n ? qp((uint32_t)q, (uint32_t)(q + Q * ((n - 1 - q) / Q))) : Q_EMPTY);
        }
    }
    struct Wait {
        Clock::time_point t0{};
        uint32_t seen = 0;
        bool started = false;
    };
    bool wait_on(Wait &w)
    {
        if (failed.load(std::memory_order_relaxed)) return false;
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
        failed.store(1);
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

// one block's shared stash
struct Shared {
    int L;
    std::vector<std::vector<Particle>> link;       // slot data (plain: published by the counters)
    std::atomic<uint32_t> freem{0}, readym{0};
    std::atomic<uint32_t> part[E];
    std::atomic<uint32_t> resv[MAXL], wrt[MAXL], ev[MAXL];
    std::atomic<uint32_t> busy{0};
    explicit Shared(int links) : L(links), link(links, std::vector<Particle>(SLOTS))
    {
        freem.store(links >= 32 ? 0xFFFFFFFFu : ((1u << links) - 1u));
        for (int k = 0; k < E; ++k) part[k].store(NONE);
        for (int l = 0; l < MAXL; ++l) {
            resv[l].store(0);
            wrt[l].store(0);
            ev[l].store(0);
        }
    }
    // claim one set bit of m (-1 if none)
    static int claim(std::atomic<uint32_t> &m)
    {
        for (;;) {
            uint32_t v = m.load(std::memory_order_acquire);
            if (v == 0) return -1;
            int l = __builtin_ctz(v);
            uint32_t old = m.fetch_and(~(1u << l), std::memory_order_acq_rel);
            if (old & (1u << l)) return l;
        }
    }
};

struct Wave {
    Arena &A;
    Shared &S;
    uint64_t total;
    int force_spill;
    uint32_t start;
    uint32_t tick = 0;
    std::vector<int> &done;

    // copy ready link v to the global arena; true on success
    bool spill(int v)
    {
        uint32_t a = A.pop(A.qempty, start);
        for (Arena::Wait w; a == NIL && A.wait_on(w);) {
            std::this_thread::yield();
            a = A.pop(A.qempty, start);
        }
        if (a == NIL) return false;
        A.data[a] = S.link[v];
        A.hdr[a].store(S.ev[v].load(std::memory_order_relaxed) | (64u << 8), std::memory_order_relaxed);
        std::atomic_thread_fence(std::memory_order_release);
        if (!A.push(A.qfull, start, a)) return false;
        A.fill.fetch_add(1);
        A.spills.fetch_add(1);
        return true;
    }

    // a link of our own: a free one, else a ready one spilled to the arena
    int alloc()
    {
        for (;;) {
            int l = Shared::claim(S.freem);
            if (l >= 0) return l;
            int v = Shared::claim(S.readym);
            if (v >= 0) {
                if (spill(v)) return v;
                A.fail();
                return -1;
            }
            // every link is a partial or in another wavefront's hands for a
            // moment; the run has failed if that persists
            if (A.failed.load()) return -1;
            std::this_thread::yield();
        }
    }

    // deposit particles of event k
    void deposit(int k, std::vector<Particle> ps)
    {
        size_t off = 0;
        Arena::Wait w;
        while (off < ps.size()) {
            uint32_t n = (uint32_t)(ps.size() - off);
            uint32_t pk = S.part[k].load(std::memory_order_acquire);
            if (pk == NONE) {
                int l = alloc();
                if (l < 0) {
                    A.fail();
                    return;                          // particles dropped: the run fails
                }
                uint32_t tag = (S.resv[l].load(std::memory_order_relaxed) >> 16) + 1u;
                S.resv[l].store((tag & 0xFFFFu) << 16, std::memory_order_relaxed);
                S.wrt[l].store(0, std::memory_order_relaxed);
                S.ev[l].store((uint32_t)k, std::memory_order_relaxed);
                uint32_t want = ((tag & 0xFFFFu) << 8) | (uint32_t)l;
                uint32_t expect = NONE;
                if (!S.part[k].compare_exchange_strong(expect, want, std::memory_order_acq_rel)) {
                    S.freem.fetch_or(1u << l, std::memory_order_acq_rel);   // someone installed one first
                }
                continue;
            }
            int l = (int)(pk & 0xFFu);
            uint32_t tag = pk >> 8;
            uint32_t r = S.resv[l].load(std::memory_order_acquire);
            if ((r >> 16) != tag || (r & 0xFFFFu) >= SLOTS) {
                // recycled or full: the filler or a closer takes it out of part[k]
                if (!A.wait_on(w)) {
                    A.fail();
                    return;
                }
                std::this_thread::yield();
                continue;
            }
            uint32_t f = r & 0xFFFFu;
            uint32_t take = n < SLOTS - f ? n : SLOTS - f;
            if (!S.resv[l].compare_exchange_strong(r, r + take, std::memory_order_acq_rel)) continue;
            for (uint32_t i = 0; i < take; ++i) S.link[l][f + i] = ps[off + i];
            off += take;
            if (f + take == SLOTS) {
                uint32_t e2 = pk;
                S.part[k].compare_exchange_strong(e2, NONE, std::memory_order_acq_rel);
            }
            uint32_t wnow = S.wrt[l].fetch_add(take, std::memory_order_acq_rel) + take;
            if (wnow == SLOTS) {
                bool spill_now = force_spill > 0 && ++tick % (uint32_t)force_spill == 0;
                if (spill_now) {
                    if (spill(l)) S.freem.fetch_or(1u << l, std::memory_order_acq_rel);
                    else A.fail();
                } else {
                    S.readym.fetch_or(1u << l, std::memory_order_acq_rel);
                }
            }
        }
    }

    void run(std::vector<Particle> ps, int ev)
    {
        std::vector<Particle> out[E];
        for (auto &p : ps) {
            p.left -= 1;
            if (p.left <= 0) {
                if (done[p.id] != 0) A.err.fetch_add(1);
                done[p.id] += 1;
            } else {
                out[(ev + 1) % E].push_back(p);
            }
        }
        for (int k = 0; k < E; ++k)
            if (!out[k].empty()) deposit(k, out[k]);
    }

    // take a partial link of some event out of part[] and run what it holds
    bool steal()
    {
        for (int k = 0; k < E; ++k) {
            uint32_t pk = S.part[k].load(std::memory_order_acquire);
            if (pk == NONE) continue;
            uint32_t e2 = pk;
            if (!S.part[k].compare_exchange_strong(e2, NONE, std::memory_order_acq_rel)) continue;
            int l = (int)(pk & 0xFFu);
            uint32_t tag = pk >> 8;
            uint32_t r = S.resv[l].load(std::memory_order_acquire);
            uint32_t count;
            for (;;) {
                if ((r >> 16) != tag || (r & 0xFFFFu) >= SLOTS) {
                    count = SLOTS;                 // filled meanwhile: its last writer publishes it
                    break;
                }
                if (S.resv[l].compare_exchange_strong(r, r + SLOTS, std::memory_order_acq_rel)) {
                    count = r & 0xFFFFu;
                    break;
                }
            }
            if (count == SLOTS) continue;
            S.busy.fetch_add(1, std::memory_order_acq_rel);
            while (S.wrt[l].load(std::memory_order_acquire) != count) std::this_thread::yield();
            std::vector<Particle> ps(S.link[l].begin(), S.link[l].begin() + count);
            int ev = (int)S.ev[l].load(std::memory_order_relaxed);
            S.freem.fetch_or(1u << l, std::memory_order_acq_rel);
            if (count > 0) run(ps, ev);
            return true;
        }
        return false;
    }

    bool refill()
    {
        if (A.fill.load() == 0) return false;
        uint32_t a = A.pop(A.qfull, start);
        if (a == NIL) return false;
        A.fill.fetch_sub(1);
        std::atomic_thread_fence(std::memory_order_acquire);
        uint32_t h = A.hdr[a].load(std::memory_order_relaxed);
        int ev = (int)(h & 0xff), c = (int)(h >> 8);
        S.busy.fetch_add(1, std::memory_order_acq_rel);
        std::vector<Particle> ps(A.data[a].begin(), A.data[a].begin() + c);
        A.refills.fetch_add(1);
        if (!A.push(A.qempty, start, a)) A.fail();
        run(ps, ev);
        return true;
    }

    void main_loop()
    {
        bool src_done = false;
        Arena::Wait idle;
        for (;;) {
            // busy counts workers holding particles, raised once work is taken
            int l = Shared::claim(S.readym);
            if (l >= 0) {
                S.busy.fetch_add(1, std::memory_order_acq_rel);
                std::vector<Particle> ps(S.link[l].begin(), S.link[l].end());
                int ev = (int)S.ev[l].load(std::memory_order_relaxed);
                S.freem.fetch_or(1u << l, std::memory_order_acq_rel);
                run(ps, ev);
                S.busy.fetch_sub(1, std::memory_order_acq_rel);
                idle = Arena::Wait{};
                continue;
            }
            if (!src_done) {
                if (A.failed.load()) {
                    src_done = true;
                } else {
                    uint64_t b = A.cursor.fetch_add(SLOTS);
                    if (b >= total) {
                        src_done = true;
                    } else {
                        S.busy.fetch_add(1, std::memory_order_acq_rel);
                        std::vector<Particle> ps;
                        for (uint64_t g = b; g < b + SLOTS && g < total; ++g)
                            ps.push_back(Particle{(int32_t)g, (int32_t)(1 + (g * 2654435761u) % 37)});
                        deposit(0, ps);
                        S.busy.fetch_sub(1, std::memory_order_acq_rel);
                        idle = Arena::Wait{};
                        continue;
                    }
                }
            }
            if (refill() || steal()) {
                S.busy.fetch_sub(1, std::memory_order_acq_rel);
                idle = Arena::Wait{};
                continue;
            }
            // nothing to do: leave once the block holds nothing and no one
            // holds particles; wait (bounded) while the arena has links
            bool empty = S.readym.load() == 0 && S.busy.load() == 0;
            for (int k = 0; k < E; ++k)
                if (S.part[k].load() != NONE) empty = false;
            if (empty && A.fill.load() == 0) break;
            if (A.failed.load()) break;
            if (!A.wait_on(idle)) {
                if (A.fill.load() != 0) A.fail();
                break;
            }
            std::this_thread::yield();
        }
    }
};

}  // namespace

int main(int argc, char **argv)
{
    int blocks = argc > 1 ? atoi(argv[1]) : 2;
    int wpb = argc > 2 ? atoi(argv[2]) : 4;
    int links = argc > 3 ? atoi(argv[3]) : E + wpb + 2;
    uint64_t particles = argc > 4 ? strtoull(argv[4], nullptr, 10) : 20000;
    int force = argc > 5 ? atoi(argv[5]) : 0;
    int arena_links = argc > 6 ? atoi(argv[6]) : blocks * links + 1024;
    uint32_t seed = argc > 7 ? (uint32_t)atoi(argv[7]) : 1;
    if (links > MAXL || links < 1) return 2;
    Arena A(arena_links);
    std::vector<Shared *> sh;
    for (int b = 0; b < blocks; ++b) sh.push_back(new Shared(links));
    std::vector<int> done(particles, 0);
    std::vector<std::thread> th;
    std::vector<Wave *> ws;
    Clock::time_point t0 = Clock::now();
    for (int b = 0; b < blocks; ++b)
        for (int w = 0; w < wpb; ++w)
            ws.push_back(new Wave{A, *sh[b], particles, force, (uint32_t)(b * wpb + w + seed) * 2654435761u, 0u, done});
    for (auto *w : ws) th.emplace_back([w] { w->main_loop(); });
    for (auto &t : th) t.join();
    double ms = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
    uint64_t missing = 0, twice = 0;
    for (uint64_t i = 0; i < particles; ++i) {
        if (done[i] == 0) ++missing;
        if (done[i] > 1) ++twice;
    }
    uint32_t leftover = 0;
    for (auto *s : sh) {
        leftover += __builtin_popcount(s->readym.load());
        for (int k = 0; k < E; ++k)
            if (s->part[k].load() != NONE) ++leftover;
    }
    printf("blocks=%d wpb=%d links=%d particles=%llu force=%d spills=%llu refills=%llu fill=%u leftover=%u "
           "missing=%llu twice=%llu err=%llu failed=%u ms=%.1f\n",
           blocks, wpb, links, (unsigned long long)particles, force, (unsigned long long)A.spills.load(),
           (unsigned long long)A.refills.load(), A.fill.load(), leftover, (unsigned long long)missing,
           (unsigned long long)twice, (unsigned long long)A.err.load(), A.failed.load(), ms);
    for (auto *w : ws) delete w;
    for (auto *s : sh) delete s;
    return (missing || twice || A.err.load()) ? 1 : 0;
}
