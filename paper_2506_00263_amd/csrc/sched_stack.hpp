// Stack-based thread-data remapping (paper Sec. 3.1).
//
// Every event type has one global input and one global output stack (a
// structure-of-arrays region in HBM).  A kernel launch is one remapping
// round: wavefronts pop 64 particles at a time from an input stack with one
// atomic per wavefront, run that event on them, and push each survivor onto
// the output stack of its next event -- per destination one ballot, one
// prefix count (mbcnt) and one atomic per wavefront.  A wavefront that finds
// every input stack drained calls the source ("make_work") until the
// fullest output stack passes a threshold, then leaves.  Between rounds the
// input and output stacks swap roles.
//
// Round r reads bank r&1 and writes bank (r+1)&1.  Stack sizes rotate over
// three counter sets so that consecutive launches can be queued without a
// host round trip: round r reads sizes[r%3], pushes with sizes[(r+1)%3], and
// clears sizes[(r+2)%3] for round r+1.  The host polls a done flag (first
// round that finds no input and no source left) every few rounds.
//
// MI355X layout: each stack is cut into stripes with separate counters (see
// NSTRIPE); the input chunks of a round are dealt to wavefronts in a fixed
// order because the input stacks do not change during the round.
#pragma once
#include <algorithm>

#include "bank.hpp"
#include "kernels.hpp"

namespace mcx {

// Stripes per event stack.  Stripe s < NSTRIPE-1 holds up to `scap`
// particles; the last stripe is the overflow stripe with room for every live
// particle, so a push never fails.  Each stripe has its own counter on its
// own 128-byte line: on MI355X a device-scope atomic on one hot address
// serialises every wavefront of all eight XCDs, striping spreads them.
constexpr int NSTRIPE = 64;
// Events a popped particle runs in place in the tail, at most (default).
// Measured on MI355X (lattice 1e6, one event per pop in the bulk): 8 2.56 ms,
// 16 2.48, 32 2.42, 64 2.40, 256 2.40 (fused); split 4.73, 4.41, 4.39, 4.37,
// 4.34.
constexpr int STACK_TAIL_EVENTS = 64;
constexpr int CTR_STRIDE = 32;   // 32 x 4 bytes = one counter per 128-byte line

struct StackArgs {
    const ProbDev *probs;
    int n_probs;
    const unsigned long long *prefix;
    unsigned long long total;
    RunCtl *ctl;
    Digest *digest;
    char *bank[2];              // [event][stripe] regions
    long scap;                  // particles per ordinary stripe
    long ocap;                  // particles in the overflow stripe
    long stripe_bytes;          // bytes of one ordinary stripe region
    long tile_bytes;            // bytes of one 64-particle tile
    long event_bytes;           // bytes of one event (all stripes)
    unsigned int *sizes;        // [3][E][NSTRIPE] counters, CTR_STRIDE apart
    unsigned long long threshold;
    int lacc_words;
    int tail_events;            // most events a popped particle runs in place in the tail
    int min_events;             // events a popped particle runs at least
    int bulk_events;            // fused: most events a popped chunk runs while few of its particles end
    int tl_bytes;               // packed tables copied to LDS (single problem)
    unsigned long long static_share;   // > 0: round 0 sources wavefront w's ids [w s, (w+1) s)
};

__device__ __forceinline__ unsigned int *stripe_ctr(const StackArgs &A, int set, int E, int e, int s)
{
    return A.sizes + ((long)(set * E + e) * NSTRIPE + s) * CTR_STRIDE;
}

// stripe s of event e's stack: a run of 64-particle tiles
__device__ __forceinline__ Tiles stripe_soa(const StackArgs &A, char *bank, int e, int s, int nd)
{
    return Tiles{bank + (long)e * A.event_bytes + (long)s * A.stripe_bytes, A.tile_bytes, nd};
}

// push the wavefront's survivors onto the output stacks of their next
// events: per destination one ballot, one prefix count and one atomic on the
// wavefront's home stripe (a second one on the overflow stripe if full)
template <class LAY, int E>
__device__ __forceinline__ void push(const StackArgs &A, char *bank, int set, int home, bool act, int ne,
                                     const Part &p, bool dig, uint32_t &err)
{
#pragma unroll
    for (int k = 0; k < E; ++k) {
        bool mine = act && ne == k;
        uint64_t mask = __ballot(mine);
        if (mask == 0) continue;
        unsigned int cnt = (unsigned int)__popcll(mask);
        unsigned int b = 0;
        if (__lane_id() == 0) b = atomicAdd(stripe_ctr(A, set, E, k, home), cnt);
        b = first_lane_u32(b);
        unsigned long slot = (unsigned long)b + lane_rank(mask);
        bool spill = (unsigned long)b + cnt > (unsigned long)A.scap;
        unsigned int ob = 0;
        if (spill) {
            unsigned long first_over = (unsigned long)b > (unsigned long)A.scap ? (unsigned long)b
                                                                                : (unsigned long)A.scap;
            unsigned int n_over = (unsigned int)((unsigned long)b + cnt - first_over);
            if (__lane_id() == 0) ob = atomicAdd(stripe_ctr(A, set, E, k, NSTRIPE - 1), n_over);
            ob = first_lane_u32(ob);
            if (mine && slot >= (unsigned long)A.scap) {
                unsigned long o = (unsigned long)ob + (slot - first_over);
                if (o < (unsigned long)A.ocap) put<LAY>(stripe_soa(A, bank, k, NSTRIPE - 1, LAY::nd(dig)), (long)o, p, dig);
                else err |= ERR_CAPACITY;
            }
        }
        if (mine && slot < (unsigned long)A.scap)
            put<LAY>(stripe_soa(A, bank, k, home, LAY::nd(dig)), (long)slot, p, dig);
    }
}

// wave-uniform view of one event's input stripes: chunk counts and prefixes
// for chunks of 2^cs_log2 particles (a divisor of the 64-particle tile)
struct StripeView {
    unsigned int n_lane;         // this lane's stripe size (clamped)
    unsigned int excl, incl;     // exclusive / inclusive chunk prefix of this lane's stripe
    unsigned int chunks;         // total chunks of the event
};

__device__ __forceinline__ StripeView stripe_view(const StackArgs &A, int set, int E, int e, int cs_log2)
{
    const int lane = __lane_id();
    unsigned int n = __hip_atomic_load(stripe_ctr(A, set, E, e, lane), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned int cap = (lane == NSTRIPE - 1) ? (unsigned int)A.ocap : (unsigned int)A.scap;
    n = n < cap ? n : cap;
    unsigned int c = (n + (1u << cs_log2) - 1u) >> cs_log2;
    unsigned int incl = c;
    for (int off = 1; off < 64; off <<= 1) {
        unsigned int o = __shfl_up(incl, off);
        if (lane >= off) incl += o;
    }
    StripeView v;
    v.n_lane = n;
    v.incl = incl;
    v.excl = incl - c;
    v.chunks = __shfl(incl, 63);
    return v;
}

// total 64-particle input chunks of one event, and its particles (wave-uniform)
__device__ __forceinline__ unsigned int event_chunks(const StackArgs &A, int set, int E, int e, unsigned int &parts)
{
    const int lane = __lane_id();
    unsigned int n = __hip_atomic_load(stripe_ctr(A, set, E, e, lane), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned int cap = (lane == NSTRIPE - 1) ? (unsigned int)A.ocap : (unsigned int)A.scap;
    n = n < cap ? n : cap;
    unsigned int c = (n + 63u) >> 6;
    for (int off = 32; off > 0; off >>= 1) {
        c += __shfl_xor(c, off);
        n += __shfl_xor(n, off);
    }
    parts = n;
    return c;
}

// The problem table is also passed as a read-only, unaliased kernel argument
// so that loads from it can be scalar loads, which do not queue behind the
// wavefront's outstanding tally atomics (vector loads retire in order).
template <int GEOM, int EMODE, int MODE, int SPLIT, bool BATCH, int EXT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((BATCH || EMODE == EMODE_CE) ? 3 : 2)))
stack_round(StackArgs A, int round, const ProbDev *__restrict__ probs)
{
    using LAY = Layout<EMODE, MODE, SPLIT, EXT>;
    constexpr int E = SPLIT ? 4 : 1;
    extern __shared__ __attribute__((aligned(16))) unsigned long long lacc[];
    char *tl = (char *)lacc + tabs_lds_offset((size_t)A.lacc_words * 8);
    const bool dig = A.digest != nullptr;
    const int set_in = round % 3, set_out = (round + 1) % 3;
    char *bin = A.bank[round & 1];
    char *bout = A.bank[(round + 1) & 1];
    if (blockIdx.x == 0 && threadIdx.x < E * NSTRIPE)
        __hip_atomic_store(&A.sizes[((long)((round + 2) % 3) * E * NSTRIPE + threadIdx.x) * CTR_STRIDE], 0u,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int lane = __lane_id();
    const unsigned int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const unsigned int n_waves = (gridDim.x * blockDim.x) >> 6;
    const int home = (int)(wave % (NSTRIPE - 1));
    // every history has ended (wavefronts add their ended histories once, at
    // the end of a round, so this count can only reach the total when no
    // particle is left anywhere): the run is over
    unsigned long long ended = __hip_atomic_load(&A.ctl->stripe[lane].c[C_COMPLETED], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    for (int off = 32; off > 0; off >>= 1) ended += __shfl_xor(ended, off);
    if (ended >= A.total) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && A.ctl->done_round == 0) A.ctl->done_round = (unsigned)round + 1;
        return;
    }
    // (a wavefront that returned above no longer takes part in block barriers)
    if constexpr (!BATCH) tabs_to_lds(probs[0], tl);
    // LDS block sums: pass B's per-(material, group) sums, or the bins of a small
    // energy-bin tally (single-problem launches)
    EvCtx cx{probs, A.digest, (MODE == MODE_REPLAY_B && A.lacc_words > 0) ? lacc : nullptr, BATCH ? 0 : 1,
             (MODE == MODE_FWD && A.lacc_words > 0) ? lacc : nullptr};
    if (A.lacc_words > 0) {
        lacc_zero(lacc, A.lacc_words);
        __syncthreads();
    }
    Lane ln{0, 0, 0, 0, (uint32_t)(wave % TREP)};
    WaveCount wc;
    wc.zero();
    // A popped particle runs K events in place before it is pushed: at least
    // min_events (1: remap after every event).  Tail: when the round's input
    // chunks no longer give every wavefront one, remapping cannot fill the
    // device and each round costs a launch plus one event's latency, so K
    // grows as the population shrinks (up to tail_events).  Fused events go
    // on past K, up to bulk_events, while at least 64 - BULK_ENDED of the
    // chunk's lanes hold live particles: a full chunk has nothing to gain
    // from being pushed and popped again (a partly filled one would hold the
    // round for its few particles).  Every history draws from its own keyed
    // streams, so results do not change.
    int K = A.min_events;
    int cs_log2 = 6;                 // particles per popped chunk: 64, fewer in the tail
    {
        unsigned int all = 0, parts = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            unsigned int pe = 0;
            all += event_chunks(A, set_in, E, e, pe);
            parts += pe;
        }
        // the round's input population, kept for the first rounds
        if (blockIdx.x == 0 && threadIdx.x == 0 && round < STACK_ROUND_LOG) A.ctl->round_in[round] = parts;
        if (all < n_waves) {
            unsigned int q = n_waves / (all ? all : 1u);
            int kt = (int)(q < (unsigned int)A.tail_events ? q : (unsigned int)A.tail_events);
            K = kt > K ? kt : K;
        }
        // Tail: fewer live particles than 64 per wavefront.  Whole tiles would
        // leave most wavefronts idle while each busy one runs its events over
        // 64 diverging lanes; chunks of the smallest power of two that spreads
        // the particles over all wavefronts shorten each event (every
        // wavefront derives the same size from the same read-only inputs, so
        // the chunks still partition the stacks).
        if (parts < 64u * n_waves) {
            const unsigned int per = (parts + n_waves - 1u) / n_waves;
            cs_log2 = 0;
            while ((1u << cs_log2) < per) ++cs_log2;
        }
    }
    // pop: the input stacks are read-only during a round, so the 64-particle
    // chunks are dealt to wavefronts in a fixed order (no pop atomics)
#pragma unroll 1
    for (int e = 0; e < E; ++e) {
        StripeView v = stripe_view(A, set_in, E, e, cs_log2);
        for (unsigned int c = wave; c < v.chunks; c += n_waves) {
            uint64_t in_stripe = __ballot(c < v.incl);
            int s = __ffsll((unsigned long long)in_stripe) - 1;
            unsigned int excl = __shfl(v.excl, s);
            unsigned int ns = __shfl(v.n_lane, s);
            unsigned int base = (c - excl) << cs_log2;
            bool act = (unsigned int)lane < (1u << cs_log2) && base + (unsigned int)lane < ns;
            Part p;
            if (act) get<LAY>(stripe_soa(A, bin, e, s, LAY::nd(dig)), (long)(base + lane), p, dig);
            int ne = EV_DEAD, cur = e;
            bool live = act;
            for (int i = 0;;) {
                uint32_t out = 0;
                if (live) ne = run_event_in<GEOM, EMODE, MODE, SPLIT, EXT, BATCH>(cur, probs, tl, cx, ln, p, out);
                wc.dispatch(live);
                wc.outcomes(live, out);
                ++i;
                live = live && ne != EV_DEAD;
                if (i >= K && (SPLIT || i >= A.bulk_events || __popcll(__ballot(live)) < 64 - BULK_ENDED))
                    break;
                if (__ballot(live) == 0) break;
                cur = ne;
            }
            push<LAY, E>(A, bout, set_out, home, act, ne, p, dig, ln.err);
        }
    }
    // make_work.  When the stacks hold every history and the threshold cannot
    // stop the source, round 0 sources all of them: wavefront w takes its own
    // contiguous share of the ids, with no claims on the shared cursor (a few
    // thousand claims on one word serialise at the memory-side atomic unit).
    if (A.static_share > 0) {
        if (round == 0) {
            const unsigned long long b0 = (unsigned long long)wave * A.static_share;
            const unsigned long long e0 = b0 + A.static_share < A.total ? b0 + A.static_share : A.total;
            for (unsigned long long b = b0; b < e0; b += 64ull) {
                unsigned long long gid = b + lane;
                bool act = gid < e0;
                Part p;
                if (act) {
                    int pi = BATCH ? find_problem(A.prefix, A.n_probs, gid) : 0;
                    const ProbDev &P = probs[pi];
                    source<GEOM, MODE>(P, tabs_for<BATCH>(P, tl), p, (uint32_t)(P.first + (gid - P.gbase)),
                                       (uint32_t)pi);
                }
                wc.outcomes(act, O_SOURCE);
                wc.c[C_MAKE_WORK] += 1;
                push<LAY, E>(A, bout, set_out, home, act, EV_STEP, p, dig, ln.err);
            }
        }
    }
    // otherwise: source new histories (256 per claim) until the fullest
    // output stack passes the threshold or the source is exhausted
    for (; A.static_share == 0;) {
        unsigned long long cur = __hip_atomic_load(&A.ctl->src_cursor, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur >= A.total) break;
        unsigned long long fullest = 0;
#pragma unroll
        for (int k = 0; k < E; ++k) {
            unsigned long long t = __hip_atomic_load(stripe_ctr(A, set_out, E, k, lane), __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
            for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
            fullest = t > fullest ? t : fullest;
        }
        if (fullest >= A.threshold) break;
        unsigned long long b = 0;
        if (lane == 0) b = atomicAdd(&A.ctl->src_cursor, 256ull);
        b = first_lane_u64(b);
        if (b >= A.total) break;
        for (int j = 0; j < 4; ++j) {
            unsigned long long gid = b + 64ull * j + lane;
            bool act = gid < A.total;
            if (b + 64ull * j >= A.total) break;
            Part p;
            if (act) {
                int pi = BATCH ? find_problem(A.prefix, A.n_probs, gid) : 0;
                const ProbDev &P = probs[pi];
                source<GEOM, MODE>(P, tabs_for<BATCH>(P, tl), p, (uint32_t)(P.first + (gid - P.gbase)), (uint32_t)pi);
            }
            wc.outcomes(act, O_SOURCE);
            wc.c[C_MAKE_WORK] += 1;
            push<LAY, E>(A, bout, set_out, home, act, EV_STEP, p, dig, ln.err);
        }
    }
    flush_wave(A.ctl, wc, ln, probs, BATCH ? 0 : 1, MODE);
    if (A.lacc_words > 0) {
        __syncthreads();
        if (cx.lacc) lacc_flush(lacc, probs[0]);
        if (cx.ltally) ltally_flush(lacc, probs[0], A.lacc_words);
    }
}

template <int GEOM, int EMODE, int MODE, int SPLIT, bool BATCH, int EXT>
static hipError_t stack_t(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm, unsigned int *flag)
{
    using LAY = Layout<EMODE, MODE, SPLIT, EXT>;
    constexpr int E = SPLIT ? 4 : 1;
    const bool dig = a.digest != nullptr;
    const int block = 256;
    // every block of a round is resident at once: the grid is the resident
    // capacity (or the requested waves per CU, if fewer)
    auto kern = stack_round<GEOM, EMODE, MODE, SPLIT, BATCH, EXT>;
    const size_t lds_need = tabs_lds_offset((size_t)a.lacc_words * 8) + (size_t)(BATCH ? 0 : a.tl_bytes);
    int per_cu = 0;
    hipError_t oe = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, lds_need);
    if (oe != hipSuccess) return oe;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    int wpc = per_cu * (block / 64);
    if (a.waves_per_cu > 0 && a.waves_per_cu < wpc) wpc = a.waves_per_cu;
    long blocks = std::max(1L, (long)a.num_cus * wpc / (block / 64));
    long waves = blocks * (block / 64);
    long slack = 2 * (waves * 256 + 64);          // particles sourced past the threshold
    long cap = a.stack_capacity > 0 ? (long)a.stack_capacity : (long)a.total + slack;
    const long cap_max = 1L << 24;
    if (cap > cap_max + slack) cap = cap_max + slack;
    cap = (cap + 63) / 64 * 64;
    long thr;
    if (a.stack_threshold > 0) thr = (long)a.stack_threshold;
    else if (cap >= (long)a.total + slack) thr = cap;
    else thr = std::max(256L, (cap - slack) / E);
    long scap = ((2 * cap) / (NSTRIPE - 1) + 63) / 64 * 64 + 64;
    long ocap = cap;
    long bytes = LAY::bytes(dig);
    // scap and ocap are multiples of 64: stripes are whole tiles
    long tile_bytes = 64 * bytes;
    long stripe_bytes = scap / 64 * tile_bytes;
    long event_bytes = stripe_bytes * (NSTRIPE - 1) + ocap / 64 * tile_bytes;
    size_t ctr_bytes = (size_t)3 * E * NSTRIPE * CTR_STRIDE * 4;
    size_t need = (size_t)event_bytes * E * 2 + ctr_bytes;
    if (a.ws_query) {
        *a.ws_query = need;
        return hipSuccess;
    }
    hipError_t e = ws_reserve(ws, need);
    if (e != hipSuccess) return e;
    StackArgs A;
    A.probs = a.probs;
    A.n_probs = a.n_probs;
    A.prefix = a.prefix;
    A.total = a.total;
    A.ctl = a.ctl;
    A.digest = (Digest *)a.digest;
    A.bank[0] = (char *)ws.ptr;
    A.bank[1] = (char *)ws.ptr + (size_t)event_bytes * E;
    A.scap = scap;
    A.ocap = ocap;
    A.stripe_bytes = stripe_bytes;
    A.tile_bytes = tile_bytes;
    A.event_bytes = event_bytes;
    A.sizes = (unsigned int *)((char *)ws.ptr + (size_t)event_bytes * E * 2);
    A.threshold = (unsigned long long)thr;
    A.lacc_words = a.lacc_words;
    A.tail_events = a.stack_tail_events > 0 ? a.stack_tail_events : STACK_TAIL_EVENTS;
    A.min_events = a.stack_min_events > 0 ? a.stack_min_events : 1;
    A.bulk_events = a.stack_bulk_events > 0 ? a.stack_bulk_events : (a.emode == EMODE_CE ? STACK_BULK_EVENTS : 1);
    A.tl_bytes = BATCH ? 0 : a.tl_bytes;
    // every history fits and the threshold would not stop the source: round 0
    // sources them all, each wavefront its own share (a multiple of 64)
    A.static_share = 0;
    if (thr >= (long)a.total && cap >= (long)a.total + slack)
        A.static_share = ((a.total + (unsigned long long)waves - 1) / (unsigned long long)waves + 63) / 64 * 64;
    e = hipMemsetAsync(A.sizes, 0, ctr_bytes, a.stream);
    if (e != hipSuccess) return e;
    size_t lds = lds_need;
    st.grid_blocks = (int)blocks;
    st.block_threads = block;
    st.lds_bytes = (int)lds;
    // Rounds are queued in batches.  After each batch the control block's
    // error and done words are copied to pinned host memory behind an
    // event; the host queues the next batch before it waits for the
    // previous batch's words, so the device never idles on a poll.  A batch
    // queued past the last round costs only its early exits.
    const hipEvent_t *polled = a.poll;
    int round = 0;
    const int batch = 8;
    auto queue_batch = [&](int slot) -> hipError_t {
        for (int i = 0; i < batch; ++i) {
            tm.begin();
            hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(block), lds, a.stream, A, round, a.probs);
            tm.end();
            ++round;
            st.launches += 1;
        }
        hipError_t r = hipGetLastError();
        if (r != hipSuccess) return r;
        // error and done_round are adjacent words of the control block
        r = hipMemcpyAsync(flag + 2 * slot, &a.ctl->error, 8, hipMemcpyDeviceToHost, a.stream);
        if (r != hipSuccess) return r;
        return hipEventRecord(polled[slot], a.stream);
    };
    e = queue_batch(0);
    for (int b = 0; e == hipSuccess; ++b) {
        if (round > (1 << 26)) {
            e = hipErrorLaunchTimeOut;
            break;
        }
        e = queue_batch((b + 1) & 1);
        if (e != hipSuccess) break;
        e = hipEventSynchronize(polled[b & 1]);
        if (e != hipSuccess) break;
        const unsigned int *f = flag + 2 * (b & 1);
        if (f[1] != 0) {
            st.rounds = f[1];
            break;
        }
        if (f[0] & ERR_CAPACITY) {
            st.rounds = (unsigned long long)round;
            break;
        }
    }
    hipError_t e2 = hipStreamSynchronize(a.stream);
    if (e != hipSuccess) return e;
    if (e2 != hipSuccess) return e2;
    return hipSuccess;
}

template <int GEOM, int EMODE, int MODE, int SPLIT, int EXT>
static hipError_t stack_b(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm, unsigned int *flag)
{
    return (a.n_probs > 1 || a.tl_bytes == 0) ? stack_t<GEOM, EMODE, MODE, SPLIT, true, EXT>(a, ws, st, tm, flag)
                                              : stack_t<GEOM, EMODE, MODE, SPLIT, false, EXT>(a, ws, st, tm, flag);
}

template <int GEOM, int EMODE, int MODE, int EXT>
static hipError_t stack_s(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm, unsigned int *flag)
{
    return a.split ? stack_b<GEOM, EMODE, MODE, 1, EXT>(a, ws, st, tm, flag)
                   : stack_b<GEOM, EMODE, MODE, 0, EXT>(a, ws, st, tm, flag);
}

// every event program of one particle-state mode (without or with time and weight)
template <int EXT>
static hipError_t launch_stack_tm(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm,
                                  unsigned int *flag)
{
    if (a.emode == EMODE_CE) {
        if (a.geom != GEOM_LATTICE || a.mode != MODE_FWD) return hipErrorInvalidValue;
        return stack_s<GEOM_LATTICE, EMODE_CE, MODE_FWD, EXT>(a, ws, st, tm, flag);
    }
    if (a.geom == GEOM_BOX) {
        if (a.mode == MODE_FWD) return stack_s<GEOM_BOX, EMODE_MG, MODE_FWD, EXT>(a, ws, st, tm, flag);
        if (a.mode == MODE_REPLAY_A) return stack_s<GEOM_BOX, EMODE_MG, MODE_REPLAY_A, EXT>(a, ws, st, tm, flag);
        return stack_s<GEOM_BOX, EMODE_MG, MODE_REPLAY_B, EXT>(a, ws, st, tm, flag);
    }
    if (a.mode == MODE_FWD) return stack_s<GEOM_LATTICE, EMODE_MG, MODE_FWD, EXT>(a, ws, st, tm, flag);
    if (a.mode == MODE_REPLAY_A) return stack_s<GEOM_LATTICE, EMODE_MG, MODE_REPLAY_A, EXT>(a, ws, st, tm, flag);
    return stack_s<GEOM_LATTICE, EMODE_MG, MODE_REPLAY_B, EXT>(a, ws, st, tm, flag);
}

}  // namespace mcx
