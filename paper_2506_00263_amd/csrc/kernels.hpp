// Host-visible launch interface of the scheduler kernels (kernels in
// sched_naive.hpp, sched_stack.hpp and sched_async.hpp; each is built once
// for particles without extended state, sched_*.hip, and once for particles
// that carry time and weight, sched_*_ext.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>
#include <vector>

#include "problem.hpp"

namespace mcx {

// Per-launch HIP-event timing on the run's stream (optional).  Events come
// from a pool owned by the problem handle and are reused across runs, so
// timing adds two event records per launch and no event creation.
struct LaunchTimer {
    bool on = false;
    hipStream_t stream = nullptr;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> *pool = nullptr;
    size_t used = 0;
    void begin()
    {
        if (!on || !pool) return;
        if (used == pool->size()) {
            hipEvent_t a, b;
            if (hipEventCreate(&a) != hipSuccess) return;
            if (hipEventCreate(&b) != hipSuccess) {
                (void)hipEventDestroy(a);
                return;
            }
            pool->emplace_back(a, b);
        }
        (void)hipEventRecord((*pool)[used].first, stream);
    }
    void end()
    {
        if (!on || !pool || used == pool->size()) return;
        (void)hipEventRecord((*pool)[used].second, stream);
        ++used;
    }
    // after the stream has been synchronised
    double total_ms()
    {
        double t = 0.0;
        for (size_t i = 0; pool && i < used; ++i) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, (*pool)[i].first, (*pool)[i].second) == hipSuccess) t += ms;
        }
        used = 0;
        return t;
    }
};

// What a launcher needs to know about the run.
struct LaunchArgs {
    const ProbDev *probs;                  // device array [n_probs]
    int n_probs;
    const unsigned long long *prefix;      // device [n_probs + 1] flattened id offsets
    unsigned long long total;              // flattened histories of the run
    RunCtl *ctl;                           // device control block
    void *digest;                          // device Digest array or null
    int geom, emode, mode, split;
    int ext;                               // 1: particles carry time and weight (time bins or
                                           //    implicit capture in some problem)
    int lacc_words;                        // pass B per-block sums in LDS (single problem), 0 = none
    int tl_bytes;                          // single problem: packed tables copied to LDS; 0 = read globally
    hipStream_t stream;
    int num_cus;
    // tuning (0 = default)
    int block_size;                        // naive
    int waves_per_cu;                      // stack / async
    long long stack_capacity, stack_threshold;
    int stash_links, arena_links;
    int force_spill;                       // async, testing
    int consolidate;                       // async: 0 default, 1 on, 2 off
    int stack_tail_events;                 // stack: events per pop in the tail (0 = default)
    int stack_min_events;                  // stack: events per pop at least (0 = default 1)
    int async_block_waves;                 // async: wavefronts per block, 1, 2 or 4 (0 = ASYNC_BLOCK_WAVES)
    int async_drain_events;                // async: events per pass on a drained wavefront's partial link (0 = default)
    int async_bulk_events;                 // async fused: events per pass on a full link (0 = default)
    int stack_bulk_events;                 // stack fused: events per pop while few particles end (0 = default)
    int async_shared;                      // async: 1 = the block's wavefronts share one stash (0, 2: one each)
    size_t *ws_query;                      // non-null: only report the workspace bytes the launch
                                           // needs (nothing is allocated or launched)
    hipEvent_t poll[2];                    // stack: two events (timing off) owned by the handle,
                                           // recorded behind each batch of rounds
    int wall_clock_khz;                    // rate of the device's constant-rate clock
};

// Default wavefronts per asynchronous block.  Measured on MI355X (1e6
// histories unless noted): sharing the block's LDS tables and tally sums
// among 4 wavefronts made the continuous-energy pin cell with 3200 LDS bins
// 1.7x (fused) and 1.9x (split) faster, the box 1.2x and the 1e7 lattice 1.1x,
// and changed the rest by a few percent either way.
constexpr int ASYNC_BLOCK_WAVES = 4;
constexpr int ASYNC_DRAIN_EVENTS = 8;
// Fused events on a full link (async) or a full popped chunk (stack): its
// particles run up to ASYNC_BULK_EVENTS / STACK_BULK_EVENTS events in place,
// until more than BULK_ENDED of them have ended, before they are repacked
// and refilled.  Measured on MI355X at 1e6 histories: the continuous-energy
// pin cell (670 flights per history, about one lane in ten ends within ten
// events) 3.5 % faster with async and 15 % with the stack scheme; the
// multigroup lattice (11 flights per history) unchanged with async and 3 %
// slower with the stack scheme, whose rounds wait for the chunks that go
// on, so there the stack default is off for multigroup problems.
constexpr int ASYNC_BULK_EVENTS = 64;
constexpr int STACK_BULK_EVENTS = 64;
constexpr int BULK_ENDED = 4;
// Budget of one bounded wait in the asynchronous scheduler (a queue claimed
// by others, no empty arena link, links in flight): far beyond any transient
// contention (a queue is held for well under a microsecond), short enough
// that an exhausted arena is reported promptly.
constexpr int ASYNC_WAIT_MS = 20;
// Split events use the block-shared stash by default from this many histories
// per launch.  Measured on MI355X (private stash of 2 wavefronts per block
// against a shared one of 4): lattice 1e6 2.39 -> 2.22 ms, 1e7 14.7 -> 12.4,
// box 1e6 0.77 -> 0.66, continuous-energy pin cell 1e6 120 -> 107, the
// 256-problem batch 15.5 -> 12.1; slower at 1e5 (1.42 -> 1.65); fused events,
// register-bound, gain no wavefronts and run a few percent slower.
constexpr unsigned long long ASYNC_SHARED_MIN_HISTORIES = 500000;

struct LaunchStats {
    unsigned long long launches = 0, rounds = 0;
    int grid_blocks = 0, block_threads = 0, lds_bytes = 0;
};

// Device scratch of a run: owned by the problem handle and grown on demand,
// or, when `fixed`, memory of a given size that is never reallocated (a
// caller's workspace or the library's static scratch).
struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
    bool fixed = false;
};

hipError_t ws_reserve(Workspace &ws, size_t bytes);

hipError_t launch_naive(const LaunchArgs &a, LaunchStats &st, LaunchTimer &tm);
hipError_t launch_stack(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm,
                        unsigned int *host_flag_pinned);
hipError_t launch_async(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm);
hipError_t launch_naive_ext(const LaunchArgs &a, LaunchStats &st, LaunchTimer &tm);
hipError_t launch_stack_ext(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm,
                             unsigned int *host_flag_pinned);
hipError_t launch_async_ext(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm);

// k-eigenvalue banking between cycles (eigen.hip).  tsum holds
// eigen_tiles(n) words; totals are written to device memory.
uint64_t eigen_tiles(uint64_t n);
hipError_t eigen_count_sites(const uint32_t *fn, uint64_t n, uint64_t *tsum, uint64_t *total, hipStream_t s);
hipError_t eigen_gather_sites(const uint32_t *fn, const double *fpos, uint64_t n, const uint64_t *tsum,
                              double *sites, hipStream_t s);
hipError_t eigen_count_copies(uint32_t key0, uint32_t key1, uint32_t stream, uint64_t fl, double fr, uint64_t m,
                              uint64_t *tsum, uint64_t *total, hipStream_t s);
hipError_t eigen_scatter_copies(uint32_t key0, uint32_t key1, uint32_t stream, uint64_t fl, double fr, uint64_t m,
                                const uint64_t *tsum, const double *sites, double *next, uint64_t cap,
                                hipStream_t s);

// Weight-window generations (eigen.hip): order the m copies staged by a
// generation's n histories (first: the generation's first history id;
// gn[i]: copies of history first + i) into next, by (parent, ordinal).
// tsum holds eigen_tiles(n) words, off n words; *total receives m.
hipError_t ww_order_copies(const uint32_t *gn, uint64_t n, uint32_t first, const SiteRec *stage, uint64_t m,
                           uint64_t *tsum, uint64_t *total, uint64_t *off, SiteRec *next, hipStream_t s);

}  // namespace mcx
