// Asynchronous thread-data remapping (paper Sec. 3.2).
//
// One persistent launch.  Each wavefront (one per block) owns a stash of
// work links in LDS: a link holds up to 64 particles (one per lane) that all
// wait for the same event.  The stash keeps a free set, a ready set (links to
// run, normally full) and one partially filled link per event type; new
// particles of event k always go into the partial link of k, so packing
// stays optimal, and a link that fills up becomes ready.
//
// A wavefront repeats: run a ready link; else, while histories remain, call
// the source ("make_work") for 64 new particles; else refill a link from
// the global arena; else run its fullest partial link; else leave.
// When a deposit needs a link and the stash has none free, a ready link is
// spilled to the global arena.
//
// Global arena: links in HBM grouped into lock-free queues, one set holding
// empty links and one holding filled links.  A queue is a (head, tail) pair
// of link indices packed in one 64-bit word; a wavefront takes a queue by
// atomically exchanging it with a "claimed" marker, edits its list, and puts
// it back with another exchange.  Link data is published with an agent-scope
// release before the queue is put back and read after an acquire, so other
// XCDs see it.  No wavefront ever waits for another block's progress except
// for bounded retries when every queue is momentarily claimed.
#pragma once
#include <algorithm>

#include "bank.hpp"
#include "kernels.hpp"

namespace mcx {

struct AsyncArgs {
    const ProbDev *probs;
    int n_probs;
    const unsigned long long *prefix;
    unsigned long long total;
    RunCtl *ctl;
    Digest *digest;
    int links;                   // stash links per wavefront (<= 16)
    int link_bytes;              // bytes of one 64-slot link
    char *arena;                 // n_arena links
    uint32_t *hdr;               // per arena link: event | count << 8
    uint32_t *next;              // per arena link
    unsigned long long *qfull;   // queues of filled links [n_queues]
    unsigned long long *qempty;  // queues of empty links [n_queues]
    uint32_t *fill;              // number of filled links in the arena
    int n_arena, n_queues;
    int lacc_words;
    unsigned long long wait_ticks;   // budget of one bounded wait, in constant-rate clock ticks
    int force_spill;             // testing: spill every k-th filled link
    int consolidate;             // drained sparse stashes are handed to the arena and merged
    int tl_bytes;                // packed tables copied to LDS (single problem)
    int wpb;                     // wavefronts per block (each with its own stash)
    int drain_events;            // events per pass on a drained wavefront's partial link
    int bulk_events;             // fused: events per pass on a full link
};

constexpr uint32_t NIL = 0xFFFFFFFFu;
constexpr int DONATE_BELOW = 32;   // a drained stash with fewer particles is donated

// Whether a link's particles run another event in place (wave-uniform).  A
// drained wavefront's partial link goes on while any particle lives; a full
// link (fused events) while at most BULK_ENDED of its particles have
// ended, so few slots idle before it is repacked and refilled.  Every
// history draws from its own keyed streams and the tallies are integer
// sums, so how many events run in place never changes a result.
__device__ __forceinline__ bool goes_on(bool drained, bool act, bool live)
{
    if (drained) return __ballot(live) != 0;
    return __popcll(__ballot(act && !live)) <= BULK_ENDED;
}
constexpr unsigned long long Q_EMPTY = ~0ull;
constexpr unsigned long long Q_CLAIMED = 0xFFFFFFFEFFFFFFFEull;
__device__ __forceinline__ uint32_t q_head(unsigned long long q) { return (uint32_t)(q >> 32); }
__device__ __forceinline__ uint32_t q_tail(unsigned long long q) { return (uint32_t)q; }
__device__ __forceinline__ unsigned long long q_pack(uint32_t h, uint32_t t)
{
    return ((unsigned long long)h << 32) | (unsigned long long)t;
}

__device__ __forceinline__ unsigned long long q_exchange(unsigned long long *slot, unsigned long long v)
{
    unsigned long long old = 0;
    if (__lane_id() == 0)
        old = __hip_atomic_exchange(slot, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    return first_lane_u64(old);
}

__device__ __forceinline__ unsigned long long q_peek(unsigned long long *slot)
{
    unsigned long long v = 0;
    if (__lane_id() == 0) v = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return first_lane_u64(v);
}

__device__ __forceinline__ uint32_t lane0_load(uint32_t *p)
{
    uint32_t v = 0;
    if (__lane_id() == 0) v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return first_lane_u32(v);
}

__device__ __forceinline__ void lane0_store(uint32_t *p, uint32_t v)
{
    if (__lane_id() == 0) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded waits.  A wait (for an unclaimed queue, an empty arena link, or
// links in flight) gives up once the arena's count of filled links has not
// changed for A.wait_ticks of the constant-rate clock (no wavefront anywhere
// spilled or refilled, so nothing can free what the wait needs), or at once
// when the run has already failed for capacity: the wavefront that fails
// first publishes it in the run's error word, so an exhausted arena is
// reported within milliseconds while a slow but moving arena is waited for.
__device__ __forceinline__ bool run_failed(const AsyncArgs &A)
{
    uint32_t e = 0;
    if (__lane_id() == 0) e = __hip_atomic_load(&A.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (first_lane_u32(e) & ERR_CAPACITY) != 0u;
}

// One bounded wait: its clock start and the fill count last seen (wave-uniform).
struct Wait {
    unsigned long long t0 = 0;
    uint32_t seen = 0;
    bool started = false;
};

// keep waiting: the run has not failed and the fill count changed within the budget
__device__ __forceinline__ bool wait_on(const AsyncArgs &A, Wait &w)
{
    if (run_failed(A)) return false;
    const unsigned long long now = wall_clock64();
    const uint32_t f = lane0_load(A.fill);
    if (!w.started || f != w.seen) {
        w.started = true;
        w.t0 = now;
        w.seen = f;
        return true;
    }
    return now - w.t0 < A.wait_ticks;
}

// record a capacity failure and publish it to every wavefront at once
__device__ __forceinline__ void fail_capacity(const AsyncArgs &A, uint32_t &err)
{
    if (!(err & ERR_CAPACITY) && __lane_id() == 0) atomicOr(&A.ctl->error, ERR_CAPACITY);
    err |= ERR_CAPACITY;
}

// Pop one link from one of the 64 queues in `slots` (one queue per lane, so a
// single vector load inspects all of them).  Returns NIL if none had a link.
__device__ __forceinline__ uint32_t arena_pop(const AsyncArgs &A, unsigned long long *slots, uint32_t start)
{
    const int lane = __lane_id();
    unsigned long long mine = __hip_atomic_load(&slots[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t cand = __ballot(mine != Q_CLAIMED && q_head(mine) != NIL);
    // rotate so that wavefronts start at different queues
    uint32_t rot = start & 63u;
    cand = (cand >> rot) | (rot ? (cand << (64 - rot)) : 0ull);
    while (cand) {
        int j = __ffsll((unsigned long long)cand) - 1;
        cand &= cand - 1;
        int s = (int)((uint32_t)(j + (int)rot) & 63u);
        unsigned long long v = q_exchange(&slots[s], Q_CLAIMED);
        if (v == Q_CLAIMED) continue;                 // someone else holds it
        if (q_head(v) == NIL) {
            q_exchange(&slots[s], v);
            continue;
        }
        __threadfence();                              // acquire: see the list and link data
        uint32_t a = q_head(v);
        uint32_t nh = lane0_load(&A.next[a]);
        unsigned long long nv = (nh == NIL) ? Q_EMPTY : q_pack(nh, q_tail(v));
        q_exchange(&slots[s], nv);
        return a;
    }
    return NIL;
}

// Append link a to one of the 64 queues of `slots`; a bounded wait while
// all are claimed (the clock is read only once a pass has failed).
__device__ __forceinline__ bool arena_push(const AsyncArgs &A, unsigned long long *slots, uint32_t start, uint32_t a)
{
    lane0_store(&A.next[a], NIL);
    for (Wait w;;) {
        for (int i = 0; i < 64; ++i) {
            int s = (int)((start + (uint32_t)i) & 63u);
            unsigned long long v = q_exchange(&slots[s], Q_CLAIMED);
            if (v == Q_CLAIMED) continue;
            __threadfence();
            unsigned long long nv;
            if (q_head(v) == NIL) {
                nv = q_pack(a, a);
            } else {
                lane0_store(&A.next[q_tail(v)], a);
                nv = q_pack(q_head(v), a);
            }
            __threadfence();                          // release the link and list edits
            q_exchange(&slots[s], nv);
            return true;
        }
        if (!wait_on(A, w)) return false;
        __builtin_amdgcn_s_sleep(4);
    }
}

// filled links currently in the arena (may lag a push in flight; the
// wavefront doing that push re-checks before it leaves)
__device__ __forceinline__ unsigned int arena_fill(const AsyncArgs &A)
{
    return lane0_load(A.fill);
}

// Wave-uniform stash bookkeeping (all values live in scalar registers).
struct Stash {
    uint32_t freem, readym;
    unsigned long long clo, chi;   // 8-bit counts of links 0-7 and 8-15
    uint32_t evw;                  // 2-bit event of each link
    uint32_t part;                 // 8-bit partial link per event (0xff none)
    __device__ __forceinline__ int cnt(int l) const
    {
        return (int)(((l < 8) ? (clo >> (8 * l)) : (chi >> (8 * (l - 8)))) & 0xffull);
    }
    __device__ __forceinline__ void set_cnt(int l, int c)
    {
        if (l < 8) clo = (clo & ~(0xffull << (8 * l))) | ((unsigned long long)c << (8 * l));
        else chi = (chi & ~(0xffull << (8 * (l - 8)))) | ((unsigned long long)c << (8 * (l - 8)));
    }
    __device__ __forceinline__ int ev(int l) const { return (int)((evw >> (2 * l)) & 3u); }
    __device__ __forceinline__ void set_ev(int l, int e) { evw = (evw & ~(3u << (2 * l))) | ((uint32_t)e << (2 * l)); }
    __device__ __forceinline__ int partial(int k) const
    {
        int v = (int)((part >> (8 * k)) & 0xffu);
        return v == 0xff ? -1 : v;
    }
    __device__ __forceinline__ void set_partial(int k, int l) { part = (part & ~(0xffu << (8 * k))) | ((uint32_t)(l & 0xff) << (8 * k)); }
};

struct AsyncWave {
    const AsyncArgs &A;
    char *lds;
    int nd, nu;
    uint32_t qstart;
    Stash S;
    uint32_t tick;               // filled links so far (forced spills)
    __device__ SoA link(int l) const { return SoA{lds + (long)l * A.link_bytes, 64, nd}; }
    __device__ SoA alink(uint32_t a) const { return SoA{A.arena + (long)a * A.link_bytes, 64, nd}; }

    // move ready link v to the global arena
    __device__ __forceinline__ bool spill(int v)
    {
        uint32_t a = arena_pop(A, A.qempty, qstart);
        for (Wait w; a == NIL && wait_on(A, w);) {
            __builtin_amdgcn_s_sleep(4);
            a = arena_pop(A, A.qempty, qstart);
        }
        if (a == NIL) return false;
        copy_slot(alink(a), __lane_id(), link(v), __lane_id(), nd, nu);
        lane0_store(&A.hdr[a], (uint32_t)S.ev(v) | ((uint32_t)S.cnt(v) << 8));
        __threadfence();                              // release the link data
        if (!arena_push(A, A.qfull, qstart, a)) return false;
        if (__lane_id() == 0) atomicAdd(A.fill, 1u);
        return true;
    }

    // a free stash link, spilling a ready one if none is free; -1 on failure
    __device__ __forceinline__ int alloc(WaveCount &wc, uint32_t &err)
    {
        if (S.freem == 0) {
            if (S.readym == 0) {
                fail_capacity(A, err);
                return -1;
            }
            int v = __ffs(S.readym) - 1;
            if (!spill(v)) {
                fail_capacity(A, err);
                return -1;
            }
            S.readym &= ~(1u << v);
            S.freem |= 1u << v;
            wc.c[C_SPILLS] += 1;
        }
        int l = __ffs(S.freem) - 1;
        S.freem &= ~(1u << l);
        return l;
    }

    // pack this wavefront's particles into the partial links of their next events
    template <class LAY, int E>
    __device__ __forceinline__ void deposit(bool act, int ne, const Part &p, bool dig, WaveCount &wc, uint32_t &err)
    {
#pragma unroll
        for (int k = 0; k < E; ++k) {
            bool mine = act && ne == k;
            uint64_t mask = __ballot(mine);
            if (mask == 0) continue;
            int n = __popcll(mask);
            int r = (int)lane_rank(mask);
            int pl = S.partial(k);
            int f = 0;
            if (pl < 0) {
                pl = alloc(wc, err);
                if (pl < 0) continue;
                S.set_ev(pl, k);
                S.set_cnt(pl, 0);
                S.set_partial(k, pl);
            } else {
                f = S.cnt(pl);
            }
            int take = n < 64 - f ? n : 64 - f;
            if (mine && r < take) put<LAY>(link(pl), f + r, p, dig);
            if (f + take < 64) {
                S.set_cnt(pl, f + take);
                continue;
            }
            S.set_cnt(pl, 64);
            S.readym |= 1u << pl;
            S.set_partial(k, 0xff);
            if (A.force_spill > 0 && ++tick % (uint32_t)A.force_spill == 0) {
                if (spill(pl)) {
                    S.readym &= ~(1u << pl);
                    S.freem |= 1u << pl;
                    wc.c[C_SPILLS] += 1;
                } else {
                    fail_capacity(A, err);
                }
            }
            if (n > take) {
                int p2 = alloc(wc, err);
                if (p2 < 0) continue;
                S.set_ev(p2, k);
                S.set_cnt(p2, n - take);
                S.set_partial(k, p2);
                if (mine && r >= take) put<LAY>(link(p2), r - take, p, dig);
            }
        }
    }

    // bring one link back from the global arena; false if the arena had
    // none.  A full link is run as it is; with consolidation a partial one
    // (a donated remnant) is packed into the partial link of its event, so
    // remnants of many wavefronts merge into full links.
    template <class LAY, int E>
    __device__ __forceinline__ bool refill(bool dig, WaveCount &wc, uint32_t &err)
    {
        if (S.freem == 0 || arena_fill(A) == 0) return false;
        uint32_t a = arena_pop(A, A.qfull, qstart);
        if (a == NIL) return false;
        if (__lane_id() == 0) atomicSub(A.fill, 1u);
        int l = __ffs(S.freem) - 1;
        S.freem &= ~(1u << l);
        uint32_t h = lane0_load(&A.hdr[a]);
        copy_slot(link(l), __lane_id(), alink(a), __lane_id(), nd, nu);
        wc.c[C_REFILLS] += 1;
        if (!arena_push(A, A.qempty, qstart, a)) fail_capacity(A, err);
        int ev = (int)(h & 0xffu), c = (int)(h >> 8);
        if (!A.consolidate || c == 64) {
            S.set_ev(l, ev);
            S.set_cnt(l, c);
            S.readym |= 1u << l;
            return true;
        }
        bool act = __lane_id() < c;
        Part p;
        if (act) get<LAY>(link(l), __lane_id(), p, dig);
        S.freem |= 1u << l;
        deposit<LAY, E>(act, ev, p, dig, wc, err);
        return true;
    }

    // leave: one less live wavefront.  Donors publish their links before
    // they count themselves out, so when the last one finds the arena
    // non-empty those links are all visible; it stays (returns true) and
    // counts itself back in.
    __device__ __forceinline__ bool last_with_work(RunCtl *ctl)
    {
        unsigned int old = 0;
        if (__lane_id() == 0) old = __hip_atomic_fetch_sub(&ctl->active, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        old = first_lane_u32(old);
        if (old != 1u) return false;
        if (arena_fill(A) == 0) return false;
        if (__lane_id() == 0) __hip_atomic_fetch_add(&ctl->active, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        return true;
    }
};

// A block holds A.wpb wavefronts.  Each runs independently with its own
// stash; the block shares one LDS copy of the tables and one set of LDS
// tally sums, which one-wavefront blocks would each hold (the occupancy cost
// the paper attributes to per-warp stashes, Sec. 5.2).
// Occupancy caps (waves per SIMD), measured on MI355X: single problems 2
// (the event code keeps 160-175 registers live); batches 4, except split
// batches 3 (a 256-problem batch: fused 10.9 ms at 4 against 11.7 at 3, split
// 20.3 at 3 against 21.8 at 4).
// The problem table is also passed as a read-only, unaliased kernel argument:
// loads from it can then be scalar loads, which do not queue behind the
// wavefront's outstanding tally atomics (vector loads retire in order on
// gfx9, so a field read after a flight's adds would wait for all of them).
template <int GEOM, int EMODE, int MODE, int SPLIT, bool BATCH, int EXT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BATCH ? (SPLIT ? 3 : 4) : 2)))
async_kernel(AsyncArgs A, const ProbDev *__restrict__ probs)
{
    using LAY = Layout<EMODE, MODE, SPLIT, EXT>;
    constexpr int E = SPLIT ? 4 : 1;
    extern __shared__ __attribute__((aligned(16))) char lds[];
    const bool dig = A.digest != nullptr;
    const int L = A.links;
    const int wib = (int)(threadIdx.x >> 6);                       // wavefront in block
    const unsigned int gw = blockIdx.x * (unsigned int)A.wpb + (unsigned int)wib;   // global wavefront
    const size_t stash_bytes = (size_t)A.wpb * L * A.link_bytes;
    unsigned long long *lacc = (unsigned long long *)(lds + stash_bytes);
    char *tl = lds + tabs_lds_offset(stash_bytes + (size_t)A.lacc_words * 8);
    if constexpr (!BATCH) tabs_to_lds(probs[0], tl);
    // LDS block sums: pass B's per-(material, group) sums, or the bins of a small
    // energy-bin tally (single-problem launches)
    EvCtx cx{probs, A.digest, (MODE == MODE_REPLAY_B && A.lacc_words > 0) ? lacc : nullptr, BATCH ? 0 : 1,
             (MODE == MODE_FWD && A.lacc_words > 0) ? lacc : nullptr};
    if (A.lacc_words > 0) {
        lacc_zero(lacc, A.lacc_words);
        __syncthreads();
    }
    Lane ln{0, 0, 0, 0, (uint32_t)(gw % TREP)};
    WaveCount wc;
    wc.zero();
    const int lane = __lane_id();
    AsyncWave W{A, lds + (size_t)wib * L * A.link_bytes, LAY::nd(dig), LAY::nu(dig), gw * 2654435761u, Stash{}, 0u};
    W.S.freem = (L >= 32) ? 0xFFFFFFFFu : ((1u << L) - 1u);
    W.S.readym = 0;
    W.S.clo = 0;
    W.S.chi = 0;
    W.S.evw = 0;
    W.S.part = 0xFFFFFFFFu;
    bool src_done = false;
    bool may_donate = true;
    Wait idle;                                      // the current idle spell's wait
    bool drained = false;                           // link l is a partial one of a drained stash
    unsigned long long res_next = 0, res_end = 0;   // reserved source ids
    for (;;) {
        int l = -1;
        drained = false;
        if (W.S.readym) {
            l = __ffs(W.S.readym) - 1;
            W.S.readym &= ~(1u << l);
        } else if (!src_done) {
            // make_work: 64 new histories, reserved 256 at a time from the
            // shared source counter (one atomic per four calls)
            if (res_next >= res_end) {
                if (run_failed(A)) {                // a failed run sources nothing more
                    src_done = true;
                    continue;
                }
                unsigned long long b = 0;
                if (lane == 0) b = atomicAdd(&A.ctl->src_cursor, 256ull);
                b = first_lane_u64(b);
                if (b >= A.total) {
                    src_done = true;
                    continue;
                }
                res_next = b;
                res_end = b + 256ull < A.total ? b + 256ull : A.total;
            }
            unsigned long long b = res_next;
            res_next += 64ull;
            unsigned long long gid = b + lane;
            bool act = gid < res_end;
            Part p;
            if (act) {
                int pi = BATCH ? find_problem(A.prefix, A.n_probs, gid) : 0;
                const ProbDev &P = probs[pi];
                source<GEOM, MODE>(P, tabs_for<BATCH>(P, tl), p, (uint32_t)(P.first + (gid - P.gbase)), (uint32_t)pi);
            }
            wc.outcomes(act, O_SOURCE);
            wc.c[C_MAKE_WORK] += 1;
            W.template deposit<LAY, E>(act, EV_STEP, p, dig, wc, ln.err);
            continue;
        } else if (W.template refill<LAY, E>(dig, wc, ln.err)) {
            idle = Wait{};
            continue;
        } else {
            // drained: run the fullest partial link; a sparse stash is donated
            // to the arena instead so that the particles of many wavefronts
            // are packed into few full links
            int best = -1, bc = 0, tot = 0;
#pragma unroll
            for (int k = 0; k < E; ++k) {
                int pl = W.S.partial(k);
                if (pl >= 0) {
                    int c = W.S.cnt(pl);
                    tot += c;
                    if (c > bc) {
                        bc = c;
                        best = k;
                    }
                }
            }
            if (!A.consolidate) {
                if (tot > 0) {
                    l = W.S.partial(best);
                    W.S.set_partial(best, 0xff);
                    drained = true;
                } else {
                    // links may still be in flight to the arena; wait a bounded time
                    if (arena_fill(A) != 0 && !(ln.err & ERR_CAPACITY) && wait_on(A, idle)) {
                        __builtin_amdgcn_s_sleep(8);
                        continue;
                    }
                    break;
                }
            } else if (tot > 0 && (tot >= DONATE_BELOW || !may_donate)) {
                l = W.S.partial(best);
                W.S.set_partial(best, 0xff);
                drained = true;
            } else {
                if (tot > 0) {
#pragma unroll
                    for (int k = 0; k < E; ++k) {
                        int pl = W.S.partial(k);
                        if (pl < 0) continue;
                        if (W.spill(pl)) {
                            W.S.set_partial(k, 0xff);
                            W.S.freem |= 1u << pl;
                            wc.c[C_SPILLS] += 1;
                        } else {
                            fail_capacity(A, ln.err);
                        }
                    }
                    if (ln.err & ERR_CAPACITY) may_donate = false;   // keep what could not be donated
                    if (!may_donate) continue;
                }
                if (W.last_with_work(A.ctl)) {
                    may_donate = false;
                    if (wait_on(A, idle)) continue;
                    fail_capacity(A, ln.err);   // arena count never drained: report, do not spin
                }
                break;
            }
        }
        // run the event of link l on its particles.  A drained wavefront's
        // partial link has no full link to be packed with: its particles
        // run up to drain_events events in place (their histories draw from
        // their own keyed streams, so results do not change), which saves
        // the unpack and pack of every event on the longest histories.  A
        // full link of fused events runs up to bulk_events events in place
        // while few of its particles have ended (see bulk_goes_on).
        idle = Wait{};                              // the wait budget is per idle spell
        int ev = W.S.ev(l);
        int c = W.S.cnt(l);
        bool act = lane < c;
        Part p;
        if (act) get<LAY>(W.link(l), lane, p, dig);
        W.S.freem |= 1u << l;
        int ne = EV_DEAD;
        const int K = drained ? A.drain_events : (SPLIT ? 1 : A.bulk_events);
        int cur = ev;
        bool live = act;
        for (int i = 0;;) {
            uint32_t out = 0;
            if (live) ne = run_event_in<GEOM, EMODE, MODE, SPLIT, EXT, BATCH>(cur, probs, tl, cx, ln, p, out);
            wc.dispatch(live);
            wc.outcomes(live, out);
            if (++i >= K) break;
            live = live && ne != EV_DEAD;
            if (!goes_on(drained, act, live)) break;
            cur = ne;
        }
        W.template deposit<LAY, E>(act, ne, p, dig, wc, ln.err);
    }
    flush_wave(A.ctl, wc, ln, probs, BATCH ? 0 : 1, MODE);
    if (A.lacc_words > 0) {
        __syncthreads();
        if (cx.lacc) lacc_flush(lacc, probs[0]);
        if (cx.ltally) ltally_flush(lacc, probs[0], A.lacc_words);
    }
}

// ---------------------------------------------------------------------------
// Block-shared stash (the paper's Sec. 5.2 remedy for the stash's occupancy
// cost: lock-free stash transactions let several warps use one stash).  The
// wavefronts of a block share one pool of work links in LDS:
//  free, ready   bit masks of links; a wavefront claims a bit with an atomic
//                AND whose returned old value shows it was still set;
//  part[k]       the link being filled with particles of event k, tagged
//                (tag << 8 | link), or SH_NONE;
//  resv[l]       (tag << 16) | slots reserved: a depositor reserves slots with
//                a compare-and-swap that requires the tag it read in part[k]
//                and fewer than 64 reserved, so a reservation can never land
//                on a link that has since been recycled;
//  wrt[l]        slots written; the writer that completes the 64th slot
//                publishes the link as ready, the one that reserves it takes
//                the link out of part[k];
//  busy          wavefronts of the block holding particles outside the pool.
// A drained wavefront closes a partial link (takes it out of part[k], then
// adds 64 to its reservation), waits for the reserved slots to be written and
// runs it: the partial links of all the block's wavefronts merge.  A block's
// wavefronts leave once its pool is empty, none of them holds particles and
// the arena has nothing left.  The pool needs no per-wavefront slack (one
// partial link per event plus a few), so a block of several wavefronts takes
// far less LDS than as many private stashes.
constexpr uint32_t SH_NONE = 0xFFFFFFFFu;
constexpr int SH_MAX_LINKS = 32;

struct SharedCtl {
    uint32_t freem, readym, busy, pad;
    uint32_t part[4];
    uint32_t resv[SH_MAX_LINKS], wrt[SH_MAX_LINKS], ev[SH_MAX_LINKS];
};

typedef __attribute__((address_space(3))) uint32_t lu32;

__device__ __forceinline__ uint32_t sh_load(uint32_t *p)
{
    uint32_t v = 0;
    if (__lane_id() == 0) v = __hip_atomic_load((lu32 *)p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
    return first_lane_u32(v);
}

__device__ __forceinline__ void sh_store(uint32_t *p, uint32_t v)
{
    if (__lane_id() == 0) __hip_atomic_store((lu32 *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t sh_add(uint32_t *p, uint32_t v)
{
    // all lanes' earlier LDS writes (link slots) complete before the count moves
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    uint32_t old = 0;
    if (__lane_id() == 0) old = __hip_atomic_fetch_add((lu32 *)p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
    return first_lane_u32(old);
}

__device__ __forceinline__ void sh_or(uint32_t *p, uint32_t v)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (__lane_id() == 0) __hip_atomic_fetch_or((lu32 *)p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ bool sh_cas(uint32_t *p, uint32_t expect, uint32_t want)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    uint32_t ok = 0;
    if (__lane_id() == 0)
        ok = __hip_atomic_compare_exchange_strong((lu32 *)p, &expect, want, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE,
                                                  __HIP_MEMORY_SCOPE_WORKGROUP)
                 ? 1u
                 : 0u;
    return first_lane_u32(ok) != 0u;
}

// claim one set bit of a mask; -1 if none
__device__ __forceinline__ int sh_claim(uint32_t *mask)
{
    int r = -1;
    if (__lane_id() == 0) {
        for (;;) {
            uint32_t v = __hip_atomic_load((lu32 *)mask, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (v == 0u) break;
            int l = __ffs(v) - 1;
            uint32_t old = __hip_atomic_fetch_and((lu32 *)mask, ~(1u << l), __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old & (1u << l)) {
                r = l;
                break;
            }
        }
    }
    r = (int)first_lane_u32((uint32_t)r);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");   // every lane then reads the link
    return r;
}

struct SharedWave {
    const AsyncArgs &A;
    char *links;                 // the block's pool
    SharedCtl *C;
    int nd, nu;
    uint32_t qstart;
    uint32_t tick;               // published links so far (forced spills)
    __device__ SoA link(int l) const { return SoA{links + (long)l * A.link_bytes, 64, nd}; }
    __device__ SoA alink(uint32_t a) const { return SoA{A.arena + (long)a * A.link_bytes, 64, nd}; }

    // copy full link v of the pool to the global arena
    __device__ __forceinline__ bool spill(int v)
    {
        uint32_t a = arena_pop(A, A.qempty, qstart);
        for (Wait w; a == NIL && wait_on(A, w);) {
            __builtin_amdgcn_s_sleep(4);
            a = arena_pop(A, A.qempty, qstart);
        }
        if (a == NIL) return false;
        copy_slot(alink(a), __lane_id(), link(v), __lane_id(), nd, nu);
        lane0_store(&A.hdr[a], sh_load(&C->ev[v]) | (64u << 8));
        __threadfence();                              // release the link data
        if (!arena_push(A, A.qfull, qstart, a)) return false;
        if (__lane_id() == 0) atomicAdd(A.fill, 1u);
        return true;
    }

    // a link of the pool for this wavefront: a free one, else a ready one
    // spilled to the arena; -1 on failure (recorded)
    __device__ __forceinline__ int alloc(WaveCount &wc, uint32_t &err)
    {
        for (Wait w;;) {
            int l = sh_claim(&C->freem);
            if (l >= 0) return l;
            int v = sh_claim(&C->readym);
            if (v >= 0) {
                if (spill(v)) {
                    wc.c[C_SPILLS] += 1;
                    return v;
                }
                fail_capacity(A, err);
                return -1;
            }
            // every link is a partial or held by another wavefront for a moment
            if (!wait_on(A, w)) {
                fail_capacity(A, err);
                return -1;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }

    // the link of event k is complete: publish it (or, forced, spill it)
    __device__ __forceinline__ void publish(int l, WaveCount &wc, uint32_t &err)
    {
        if (A.force_spill > 0 && ++tick % (uint32_t)A.force_spill == 0) {
            if (spill(l)) {
                wc.c[C_SPILLS] += 1;
                sh_or(&C->freem, 1u << l);
            } else {
                fail_capacity(A, err);
            }
            return;
        }
        sh_or(&C->readym, 1u << l);
    }

    // add this wavefront's particles to the shared partial links of their next events
    template <class LAY, int E>
    __device__ __forceinline__ void deposit(bool act, int ne, const Part &p, bool dig, WaveCount &wc, uint32_t &err)
    {
#pragma unroll
        for (int k = 0; k < E; ++k) {
            bool mine = act && ne == k;
            Wait w;
            for (;;) {
                uint64_t mask = __ballot(mine);
                if (mask == 0) break;
                const uint32_t n = (uint32_t)__popcll(mask);
                const uint32_t pk = sh_load(&C->part[k]);
                if (pk == SH_NONE) {
                    int l = alloc(wc, err);
                    if (l < 0) break;                 // particles dropped: the run has failed
                    const uint32_t tag = ((sh_load(&C->resv[l]) >> 16) + 1u) & 0xFFFFu;
                    sh_store(&C->resv[l], tag << 16);
                    sh_store(&C->wrt[l], 0u);
                    sh_store(&C->ev[l], (uint32_t)k);
                    if (!sh_cas(&C->part[k], SH_NONE, (tag << 8) | (uint32_t)l)) sh_or(&C->freem, 1u << l);
                    continue;
                }
                const int l = (int)(pk & 0xFFu);
                const uint32_t tag = pk >> 8;
                const uint32_t r = sh_load(&C->resv[l]);
                if ((r >> 16) != tag || (r & 0xFFFFu) >= 64u) {
                    // recycled or full: its filler or a closer takes it out of part[k]
                    if (!wait_on(A, w)) {
                        fail_capacity(A, err);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                const uint32_t f = r & 0xFFFFu;
                const uint32_t take = n < 64u - f ? n : 64u - f;
                if (!sh_cas(&C->resv[l], r, r + take)) continue;
                const uint32_t rank = lane_rank(mask);
                const bool put_now = mine && rank < take;
                if (put_now) put<LAY>(link(l), (long)(f + rank), p, dig);
                mine = mine && !put_now;
                if (f + take == 64u) sh_cas(&C->part[k], pk, SH_NONE);
                if (sh_add(&C->wrt[l], take) + take == 64u) publish(l, wc, err);
            }
        }
    }

    // close a partial link of some event and return it (its particle count
    // in c), or -1 if none
    __device__ __forceinline__ int steal(int E, uint32_t &c)
    {
        for (int k = 0; k < E; ++k) {
            const uint32_t pk = sh_load(&C->part[k]);
            if (pk == SH_NONE) continue;
            if (!sh_cas(&C->part[k], pk, SH_NONE)) continue;
            const int l = (int)(pk & 0xFFu);
            const uint32_t tag = pk >> 8;
            uint32_t count = 64u;
            for (;;) {
                const uint32_t r = sh_load(&C->resv[l]);
                if ((r >> 16) != tag || (r & 0xFFFFu) >= 64u) break;   // filled meanwhile: published by its writer
                if (sh_cas(&C->resv[l], r, r + 64u)) {
                    count = r & 0xFFFFu;
                    break;
                }
            }
            if (count >= 64u) continue;
            // reservations are written without waiting on anything
            while (sh_load(&C->wrt[l]) != count) __builtin_amdgcn_s_sleep(1);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            c = count;
            return l;
        }
        return -1;
    }
};

template <int GEOM, int EMODE, int MODE, int SPLIT, bool BATCH, int EXT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BATCH ? (SPLIT ? 3 : 4) : 2)))
async_shared_kernel(AsyncArgs A, const ProbDev *__restrict__ probs)
{
    using LAY = Layout<EMODE, MODE, SPLIT, EXT>;
    constexpr int E = SPLIT ? 4 : 1;
    extern __shared__ __attribute__((aligned(16))) char lds[];
    const bool dig = A.digest != nullptr;
    const int NL = A.links;                                        // links in the block's pool
    const int wib = (int)(threadIdx.x >> 6);
    const unsigned int gw = blockIdx.x * (unsigned int)A.wpb + (unsigned int)wib;
    const size_t pool_bytes = (size_t)NL * A.link_bytes;
    SharedCtl *C = (SharedCtl *)(lds + pool_bytes);
    const size_t head = pool_bytes + sizeof(SharedCtl);
    unsigned long long *lacc = (unsigned long long *)(lds + head);
    char *tl = lds + tabs_lds_offset(head + (size_t)A.lacc_words * 8);
    if constexpr (!BATCH) tabs_to_lds(probs[0], tl);
    EvCtx cx{probs, A.digest, (MODE == MODE_REPLAY_B && A.lacc_words > 0) ? lacc : nullptr, BATCH ? 0 : 1,
             (MODE == MODE_FWD && A.lacc_words > 0) ? lacc : nullptr};
    if (A.lacc_words > 0) lacc_zero(lacc, A.lacc_words);
    if (threadIdx.x == 0) {
        C->freem = NL >= 32 ? 0xFFFFFFFFu : ((1u << NL) - 1u);
        C->readym = 0u;
        C->busy = 0u;
        for (int k = 0; k < 4; ++k) C->part[k] = SH_NONE;
        for (int l = 0; l < SH_MAX_LINKS; ++l) {
            C->resv[l] = 0u;
            C->wrt[l] = 0u;
            C->ev[l] = 0u;
        }
    }
    __syncthreads();
    Lane ln{0, 0, 0, 0, (uint32_t)(gw % TREP)};
    WaveCount wc;
    wc.zero();
    const int lane = __lane_id();
    SharedWave W{A, lds, C, LAY::nd(dig), LAY::nu(dig), gw * 2654435761u, 0u};
    bool src_done = false;
    Wait idle;
    unsigned long long res_next = 0, res_end = 0;   // reserved source ids
    for (;;) {
        // what to run: a ready link, new histories, an arena link, a closed
        // partial.  busy counts the wavefronts holding particles, raised once
        // work is taken: an idle wavefront looking for work must not keep the
        // others from seeing the block drained (a wavefront holding particles
        // re-checks the pool before it leaves, so the count only keeps idle
        // wavefronts waiting while new work may still appear).
        bool have = false, fresh = false, drained = false;
        int ev = 0, cnt = 0;
        Part p;
        bool act = false;
        const int l = sh_claim(&C->readym);
        if (l >= 0) {
            ev = (int)sh_load(&C->ev[l]);
            act = true;
            get<LAY>(W.link(l), lane, p, dig);
            sh_or(&C->freem, 1u << l);
            have = true;
        } else if (!src_done) {
            if (res_next >= res_end) {
                if (run_failed(A)) {
                    src_done = true;
                } else {
                    unsigned long long b = 0;
                    if (lane == 0) b = atomicAdd(&A.ctl->src_cursor, 256ull);
                    b = first_lane_u64(b);
                    if (b >= A.total) {
                        src_done = true;
                    } else {
                        res_next = b;
                        res_end = b + 256ull < A.total ? b + 256ull : A.total;
                    }
                }
            }
            if (!src_done) {
                unsigned long long b = res_next;
                res_next += 64ull;
                unsigned long long gid = b + lane;
                act = gid < res_end;
                if (act) {
                    int pi = BATCH ? find_problem(A.prefix, A.n_probs, gid) : 0;
                    const ProbDev &P = probs[pi];
                    source<GEOM, MODE>(P, tabs_for<BATCH>(P, tl), p, (uint32_t)(P.first + (gid - P.gbase)), (uint32_t)pi);
                }
                wc.outcomes(act, O_SOURCE);
                wc.c[C_MAKE_WORK] += 1;
                fresh = true;
                have = true;
            }
        }
        if (!have && arena_fill(A) != 0) {
            uint32_t a = arena_pop(A, A.qfull, W.qstart);
            if (a != NIL) {
                if (lane == 0) atomicSub(A.fill, 1u);
                uint32_t h = lane0_load(&A.hdr[a]);
                ev = (int)(h & 0xFFu);
                cnt = (int)(h >> 8);
                act = lane < cnt;
                if (act) get<LAY>(W.alink(a), lane, p, dig);
                wc.c[C_REFILLS] += 1;
                if (!arena_push(A, A.qempty, W.qstart, a)) fail_capacity(A, ln.err);
                have = true;
            }
        }
        if (!have) {
            uint32_t c = 0;
            const int sl = W.steal(E, c);
            if (sl >= 0) {
                ev = (int)sh_load(&C->ev[sl]);
                act = lane < (int)c;
                if (act) get<LAY>(W.link(sl), lane, p, dig);
                sh_or(&C->freem, 1u << sl);
                have = true;
                drained = true;
            }
        }
        if (!have) {
            // leave once the pool is empty, no wavefront of the block holds
            // particles and the arena has nothing left; wait a bounded time
            // while it does
            bool empty = sh_load(&C->readym) == 0u && sh_load(&C->busy) == 0u;
#pragma unroll
            for (int k = 0; k < E; ++k)
                if (sh_load(&C->part[k]) != SH_NONE) empty = false;
            if (empty && arena_fill(A) == 0) break;
            if (run_failed(A)) break;
            if (!wait_on(A, idle)) {
                if (arena_fill(A) != 0) fail_capacity(A, ln.err);
                break;
            }
            __builtin_amdgcn_s_sleep(8);
            continue;
        }
        idle = Wait{};
        sh_add(&C->busy, 1u);
        int ne = EV_STEP;
        if (!fresh) {
            // run the event on the particles; a drained wavefront's closed
            // partial link runs up to drain_events events in place, a full
            // link of fused events up to bulk_events
            ne = EV_DEAD;
            const int K = drained ? A.drain_events : (SPLIT ? 1 : A.bulk_events);
            int cur = ev;
            bool live = act;
            for (int i = 0;;) {
                uint32_t out = 0;
                if (live) ne = run_event_in<GEOM, EMODE, MODE, SPLIT, EXT, BATCH>(cur, probs, tl, cx, ln, p, out);
                wc.dispatch(live);
                wc.outcomes(live, out);
                if (++i >= K) break;
                live = live && ne != EV_DEAD;
                if (!goes_on(drained, act, live)) break;
                cur = ne;
            }
        }
        W.template deposit<LAY, E>(act, ne, p, dig, wc, ln.err);
        sh_add(&C->busy, 0xFFFFFFFFu);
    }
    flush_wave(A.ctl, wc, ln, probs, BATCH ? 0 : 1, MODE);
    if (A.lacc_words > 0) {
        __syncthreads();
        if (cx.lacc) lacc_flush(lacc, probs[0]);
        if (cx.ltally) ltally_flush(lacc, probs[0], A.lacc_words);
    }
}

static __global__ void arena_init(AsyncArgs A, unsigned int waves)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) A.ctl->active = waves;
    const int Q = A.n_queues, N = A.n_arena;
    if (i < N) A.next[i] = (i + Q < N) ? (uint32_t)(i + Q) : NIL;
    if (i == 0) A.fill[0] = 0;
    if (i < Q) {
        A.qfull[i] = Q_EMPTY;
        if (i < N) {
            uint32_t tail = (uint32_t)(i + Q * ((N - 1 - i) / Q));
            A.qempty[i] = q_pack((uint32_t)i, tail);
        } else {
            A.qempty[i] = Q_EMPTY;
        }
    }
}

// Launch shape of the block-shared stash: wpb wavefronts per block (default
// 4) sharing a pool of NL links (default one partial link per event, one per
// wavefront and two more, at most 32).
struct SharedShape {
    int wpb, links, per_cu;
    size_t lds;
};

template <int GEOM, int EMODE, int MODE, int SPLIT, bool BATCH, int EXT>
static hipError_t shared_shape(const LaunchArgs &a, SharedShape &sh)
{
    using LAY = Layout<EMODE, MODE, SPLIT, EXT>;
    constexpr int E = SPLIT ? 4 : 1;
    const int link_bytes = 64 * LAY::bytes(a.digest != nullptr);
    const int tl_bytes = BATCH ? 0 : a.tl_bytes;
    int wpb = a.async_block_waves > 0 ? a.async_block_waves : ASYNC_BLOCK_WAVES;
    if (wpb != 1 && wpb != 2 && wpb != 4) return hipErrorInvalidValue;
    auto kern = async_shared_kernel<GEOM, EMODE, MODE, SPLIT, BATCH, EXT>;
    for (;;) {
        int nl = a.stash_links > 0 ? a.stash_links : E + wpb + 2;
        nl = std::max(E + 1, std::min(nl, SH_MAX_LINKS));
        const size_t lds = tabs_lds_offset((size_t)nl * link_bytes + sizeof(SharedCtl) + (size_t)a.lacc_words * 8) +
                           (size_t)tl_bytes;
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * wpb, lds);
        if (e != hipSuccess) return e;
        if (per_cu >= 1 || wpb == 1) {
            if (per_cu < 1) return hipErrorInvalidConfiguration;
            sh = SharedShape{wpb, nl, per_cu, lds};
            return hipSuccess;
        }
        wpb >>= 1;
    }
}

template <int GEOM, int EMODE, int MODE, int SPLIT, bool BATCH, int EXT>
static hipError_t async_t(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm)
{
    using LAY = Layout<EMODE, MODE, SPLIT, EXT>;
    constexpr int E = SPLIT ? 4 : 1;
    const bool dig = a.digest != nullptr;
    // the block-shared stash: asked for, or by default for split events on
    // large runs (see ASYNC_SHARED_MIN_HISTORIES) unless a per-wavefront
    // stash size or stash donation is asked for
    const bool shared = a.async_shared == 1 ||
                        (a.async_shared == 0 && SPLIT && a.stash_links == 0 && a.consolidate != 1 &&
                         a.total >= ASYNC_SHARED_MIN_HISTORIES);
    // one partial link per event plus one: a stash with no free link then
    // always holds a ready link to spill.  Split events default to one more,
    // which keeps spills rare.
    int L = a.stash_links > 0 ? a.stash_links : (SPLIT ? E + 2 : E + 1);
    if (L < E + 1) L = E + 1;
    if (L > 16) L = 16;
    int link_bytes = 64 * LAY::bytes(dig);
    const int tl_bytes = BATCH ? 0 : a.tl_bytes;
    int wpb = a.async_block_waves > 0 ? a.async_block_waves : ASYNC_BLOCK_WAVES;
    if (wpb != 1 && wpb != 2 && wpb != 4) return hipErrorInvalidValue;
    auto kern = shared ? async_shared_kernel<GEOM, EMODE, MODE, SPLIT, BATCH, EXT>
                       : async_kernel<GEOM, EMODE, MODE, SPLIT, BATCH, EXT>;
    // when the block's LDS would not fit: first the smallest default stash
    // (one link per event plus one), then fewer wavefronts per block
    size_t lds = 0;
    int per_cu = 0;
    hipError_t e = hipSuccess;
    if (shared) {
        SharedShape sh{};
        e = shared_shape<GEOM, EMODE, MODE, SPLIT, BATCH, EXT>(a, sh);
        if (e != hipSuccess) return e;
        wpb = sh.wpb;
        L = sh.links;
        lds = sh.lds;
        per_cu = sh.per_cu;
    }
    for (; !shared;) {
        lds = tabs_lds_offset((size_t)wpb * L * link_bytes + (size_t)a.lacc_words * 8) + (size_t)tl_bytes;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * wpb, lds);
        if (e != hipSuccess) return e;
        if (per_cu >= 1) break;
        if (a.stash_links == 0 && L > E + 1) {
            L = E + 1;
        } else if (wpb > 1) {
            wpb >>= 1;
        } else {
            break;
        }
    }
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    // Default shape: two wavefronts per block with the smallest stash, when
    // that keeps more wavefronts resident per CU than the default four (split
    // events, whose stashes are large: 6 against 4 waves per CU on the
    // lattice and the pin cell).  With large LDS tally sums four per block
    // sharing them stay ahead, and fused events are register limited, so
    // there the default stands.
    auto capped = [&](int w) { return (a.waves_per_cu > 0 && a.waves_per_cu < w) ? a.waves_per_cu : w; };
    if (!shared && a.async_block_waves == 0 && a.stash_links == 0 && wpb == 4) {
        const int L2 = E + 1;
        const size_t lds2 = tabs_lds_offset((size_t)2 * L2 * link_bytes + (size_t)a.lacc_words * 8) + (size_t)tl_bytes;
        int per_cu2 = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu2, kern, 128, lds2);
        if (e != hipSuccess) return e;
        if (capped(2 * per_cu2) > capped(4 * per_cu)) {
            wpb = 2;
            L = L2;
            lds = lds2;
            per_cu = per_cu2;
        }
    }
    int wpc = per_cu * wpb;           // resident wavefronts per CU
    if (a.waves_per_cu > 0 && a.waves_per_cu < wpc) wpc = std::max(wpb, a.waves_per_cu / wpb * wpb);
    long blocks = (long)a.num_cus * (wpc / wpb);
    long waves = blocks * wpb;
    const int Q = 64;                 // one queue per lane of a wavefront
    int n_arena = a.arena_links > 0 ? a.arena_links : (int)(waves * (E + 2) + 1024);
    size_t arena_bytes = (size_t)n_arena * link_bytes;
    size_t need = arena_bytes + (size_t)n_arena * 8 + (size_t)Q * 16 + 1024;
    if (a.ws_query) {
        *a.ws_query = need;
        return hipSuccess;
    }
    e = ws_reserve(ws, need);
    if (e != hipSuccess) return e;
    AsyncArgs A;
    A.probs = a.probs;
    A.n_probs = a.n_probs;
    A.prefix = a.prefix;
    A.total = a.total;
    A.ctl = a.ctl;
    A.digest = (Digest *)a.digest;
    A.links = L;
    A.link_bytes = link_bytes;
    A.arena = (char *)ws.ptr;
    char *meta = (char *)ws.ptr + (arena_bytes + 255) / 256 * 256;
    A.hdr = (uint32_t *)meta;
    A.next = A.hdr + n_arena;
    A.qfull = (unsigned long long *)(((uintptr_t)(A.next + n_arena) + 255) / 256 * 256);
    A.qempty = A.qfull + Q;
    A.fill = (uint32_t *)(A.qempty + Q);
    A.n_arena = n_arena;
    A.n_queues = Q;
    A.lacc_words = a.lacc_words;
    A.wait_ticks = (unsigned long long)(a.wall_clock_khz > 0 ? a.wall_clock_khz : 100000) * ASYNC_WAIT_MS;
    A.force_spill = a.force_spill;
    A.consolidate = a.consolidate == 1 ? 1 : 0;   // off unless asked for
    A.tl_bytes = tl_bytes;
    A.wpb = wpb;
    A.drain_events = a.async_drain_events > 0 ? a.async_drain_events : ASYNC_DRAIN_EVENTS;
    A.bulk_events = a.async_bulk_events > 0 ? a.async_bulk_events : ASYNC_BULK_EVENTS;
    int ib = (std::max(n_arena, Q) + 255) / 256;
    hipLaunchKernelGGL(arena_init, dim3(ib), dim3(256), 0, a.stream, A, (unsigned int)waves);
    st.grid_blocks = (int)blocks;
    st.block_threads = 64 * wpb;
    st.lds_bytes = (int)lds;
    tm.begin();
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * wpb), lds, a.stream, A, a.probs);
    tm.end();
    st.launches += 2;
    st.rounds = 1;
    return hipGetLastError();
}

template <int GEOM, int EMODE, int MODE, int SPLIT, int EXT>
static hipError_t async_b(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm)
{
    return (a.n_probs > 1 || a.tl_bytes == 0) ? async_t<GEOM, EMODE, MODE, SPLIT, true, EXT>(a, ws, st, tm)
                                              : async_t<GEOM, EMODE, MODE, SPLIT, false, EXT>(a, ws, st, tm);
}

template <int GEOM, int EMODE, int MODE, int EXT>
static hipError_t async_s(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm)
{
    return a.split ? async_b<GEOM, EMODE, MODE, 1, EXT>(a, ws, st, tm)
                   : async_b<GEOM, EMODE, MODE, 0, EXT>(a, ws, st, tm);
}

// every event program of one particle-state mode (without or with time and weight)
template <int EXT>
static hipError_t launch_async_tm(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm)
{
    if (a.emode == EMODE_CE) {
        if (a.geom != GEOM_LATTICE || a.mode != MODE_FWD) return hipErrorInvalidValue;
        return async_s<GEOM_LATTICE, EMODE_CE, MODE_FWD, EXT>(a, ws, st, tm);
    }
    if (a.geom == GEOM_BOX) {
        if (a.mode == MODE_FWD) return async_s<GEOM_BOX, EMODE_MG, MODE_FWD, EXT>(a, ws, st, tm);
        if (a.mode == MODE_REPLAY_A) return async_s<GEOM_BOX, EMODE_MG, MODE_REPLAY_A, EXT>(a, ws, st, tm);
        return async_s<GEOM_BOX, EMODE_MG, MODE_REPLAY_B, EXT>(a, ws, st, tm);
    }
    if (a.mode == MODE_FWD) return async_s<GEOM_LATTICE, EMODE_MG, MODE_FWD, EXT>(a, ws, st, tm);
    if (a.mode == MODE_REPLAY_A) return async_s<GEOM_LATTICE, EMODE_MG, MODE_REPLAY_A, EXT>(a, ws, st, tm);
    return async_s<GEOM_LATTICE, EMODE_MG, MODE_REPLAY_B, EXT>(a, ws, st, tm);
}

}  // namespace mcx
