/*
 * mcx -- event-based Monte Carlo particle transport with thread-data
 * remapping (TDR) on AMD Instinct MI355X (gfx950).  C ABI.
 *
 * The transport method: independent particle histories (source, flights,
 * collisions, surface crossings, track-length tallies) processed as events.
 * Thread-data remapping (Sec. 2 of the paper) regroups particles between
 * events so that the lanes of a wavefront run the same event; it reorders
 * work but never changes what a history computes.  Three schedulers run the
 * same events:
 *   MCX_SCHED_NAIVE  one lane runs one whole history (the history-based
 *                    baseline the remapping methods are measured against);
 *   MCX_SCHED_STACK  stack-based remapping (Sec. 3.1): one global input and
 *                    one global output stack per event type, wavefront-
 *                    aggregated push/pop, on-demand source ("make_work")
 *                    only once all input stacks are drained and only until
 *                    the fullest output stack passes a threshold; one kernel
 *                    launch per remapping round;
 *   MCX_SCHED_ASYNC  asynchronous remapping (Sec. 3.2): one persistent
 *                    launch; each wavefront keeps a stash of work links
 *                    (64-particle arrays of one event type) in LDS, spills
 *                    to and refills from a global link arena through
 *                    lock-free queues, with no inter-block synchronisation.
 * Event decomposition (Sec. 4): MCX_DECOMP_FUSED is the monolithic "step"
 * event (one transport segment); MCX_DECOMP_SPLIT uses separate lookup,
 * move(+tally), surface-crossing and collision events.
 *
 * Results are exact integers: tallies are int64 fixed point (track length
 * times 2^tally_scale_log2, round half to even) and every scheduler, event
 * decomposition, lookup method and launch shape yields the same integers.
 *
 * Conventions
 *  - Every call returns mcx_status; nothing throws across the ABI.
 *  - "where" arguments: MCX_HOST (pointer is host memory) or MCX_DEVICE
 *    (pointer is device memory on the problem's device).
 *  - Calls on one handle are not thread-safe; distinct handles are.
 *  - Device memory passed in (tallies out, digests, dL/dT, gradients) is
 *    owned by the caller; the library never frees caller memory.
 *  - On MCX_E_CAPACITY or MCX_E_OVERFLOW the run's tallies are invalid and
 *    reading them returns MCX_E_STATE until the next successful run.
 */
#ifndef MCX_H
#define MCX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mcx_problem_s *mcx_problem_t;

typedef enum {
    MCX_OK = 0,
    MCX_E_INVALID_ARG = 1,   /* bad descriptor, option or pointer            */
    MCX_E_OOM = 2,           /* device allocation failed                     */
    MCX_E_DEVICE = 3,        /* HIP runtime error (see mcx_last_error)       */
    MCX_E_CAPACITY = 4,      /* stack / link arena capacity exhausted        */
    MCX_E_OVERFLOW = 5,      /* fixed-point total reached 2^63               */
    MCX_E_STATE = 6          /* call not valid in the handle's state         */
} mcx_status;

enum { MCX_HOST = 0, MCX_DEVICE = 1 };
enum { MCX_GEOM_BOX = 0, MCX_GEOM_LATTICE = 1 };
enum { MCX_MG = 0, MCX_CE = 1 };
enum { MCX_BC_VACUUM = 0, MCX_BC_REFLECT = 1 };
enum { MCX_SRC_POINT = 0, MCX_SRC_BOX = 1, MCX_SRC_DISC = 2 };
enum { MCX_TALLY_MESH = 0, MCX_TALLY_ENERGY = 1 };
typedef enum { MCX_SCHED_NAIVE = 0, MCX_SCHED_STACK = 1, MCX_SCHED_ASYNC = 2 } mcx_sched;
typedef enum { MCX_DECOMP_FUSED = 0, MCX_DECOMP_SPLIT = 1 } mcx_decomp;
typedef enum { MCX_LOOKUP_BINARY = 0, MCX_LOOKUP_HASH = 1 } mcx_lookup;
enum { MCX_FATE_LEAK = 0, MCX_FATE_ABSORB = 1, MCX_FATE_CUTOFF = 2, MCX_FATE_KILLED = 3, MCX_FATE_ROULETTE = 4 };

/* One fixed-source problem.  All arrays are host memory; mcx_create_problem
 * deep-copies them, so the caller may free them afterwards.
 *
 * Geometry (all coordinates in cm):
 *  BOX      box [box_lo, box_hi] cut by x-planes slab_planes[0..n_slabs]
 *           (slab_planes[0] = box_lo[0], slab_planes[n_slabs] = box_hi[0]);
 *           slab i has material slab_mat[i].
 *  LATTICE  nx*ny rectangular cells bounded by xplanes[0..nx], yplanes[0..ny]
 *           (outer planes = box faces), z in [box_lo[2], box_hi[2]] (may be
 *           +-inf); cell (i,j) holds a full-height cylinder of radius
 *           `radius` centred (cx[i], cy[j]) of material pin_mat[j*nx+i];
 *           the rest is material mod_mat.
 *  bc[6]    boundary condition of faces x-, x+, y-, y+, z-, z+.
 * Physics:
 *  MG       sigma_t, sigma_s [n_mat*n_grp] (1/cm), transfer_cdf
 *           [n_mat*n_grp*n_grp]: cumulative outgoing-group probabilities per
 *           (material, incoming group); the last entry of a row is 1.0.
 *  CE       n_species pointwise tables on sorted grids e_grid[s*grid_len..],
 *           sig_a, sig_s (same layout), target mass ratios awr[s], number
 *           densities density[m*n_species+s]; histories end below e_min;
 *           source energy e_source.  hash_bins > 0 sizes the hashed-grid
 *           index (uniform in ln E); 0 picks a default.
 * Source (sampled per history from its own random numbers):
 *  POINT at src_pos; BOX uniform in [src_lo, src_hi]; DISC uniform in the
 *  disc of radius src_radius about (src_pos x, y) at z = src_pos z.
 *  Direction isotropic if src_isotropic, else src_dir.  Group src_group
 *  (MG) or energy e_source (CE).
 * Tally: MESH track length on the tensor mesh mesh_x/y/z (edges, mesh_n[a]+1
 *  each, containing the box), bins [g][iz][iy][ix]; ENERGY track length per
 *  flight into the bin [e_edges[k], e_edges[k+1]) holding the particle energy
 *  (the last bin holds its upper edge; continuous energy: the edges contain
 *  [e_min, e_source]).  Raw values are int64 sum of rint(length *
 *  2^tally_scale_log2).  A mesh or energy edges not containing these are
 *  rejected (MCX_E_INVALID_ARG).
 * Random numbers: Philox4x32-10 keyed by (seed, problem_id), indexed by
 *  (history, flight, slot); identical on every scheduler.
 */
typedef struct {
    int32_t geometry;
    double box_lo[3], box_hi[3];
    int32_t bc[6];
    int32_t n_slabs;
    const double *slab_planes;
    const int32_t *slab_mat;
    int32_t nx, ny;
    const double *xplanes, *yplanes, *cx, *cy;
    double radius;
    const int32_t *pin_mat;
    int32_t mod_mat;
    int32_t energy_mode;
    int32_t n_mat, n_grp;
    const double *sigma_t, *sigma_s, *transfer_cdf;
    int32_t n_species, grid_len;
    const double *e_grid, *sig_a, *sig_s, *awr, *density;
    double e_min, e_source;
    int32_t hash_bins;
    int32_t src_kind, src_isotropic, src_group;
    double src_pos[3], src_lo[3], src_hi[3], src_dir[3];
    double src_radius;
    int32_t tally_kind;
    int32_t mesh_n[3];
    const double *mesh_x, *mesh_y, *mesh_z;
    int32_t n_ebins;
    const double *e_edges;
    int32_t tally_scale_log2;
    uint32_t problem_id;
    uint64_t seed;
    uint64_t n_histories;
    int64_t max_steps;
    /* Time-binned tally (the temporal tally resolution of Sec. 4 of the
     * paper).  n_tbins > 0 adds a time dimension of n_tbins equal bins over
     * [0, t_max): a particle starts at time 0 and moves at speed[g] (MG,
     * n_grp entries, cm per unit time) or speed_coef * sqrt(E) (CE); a
     * flight that would reach t_max stops there and its history ends (fate
     * CUTOFF, counted in cutoffs); a track piece is split where the
     * particle's time passes a bin edge.  Bins are laid out [time bin][bins
     * without time].  n_tbins = 0: no time dimension (the other three
     * fields are ignored). */
    int32_t n_tbins;
    double t_max;
    const double *speed;
    double speed_coef;
    /* Fission, for k-eigenvalue runs (mcx_run_eigen; multigroup).  sigma_f,
     * nu [n_mat*n_grp]: an absorption in (m, g) is a fission with probability
     * sigma_f / (sigma_t - sigma_s) and banks floor(nu + xi) neutrons at the
     * collision site (0 <= sigma_f <= sigma_t - sigma_s, 0 <= nu < 15);
     * chi [n_mat*n_grp]: cumulative fission spectrum of each material (rows
     * non-decreasing, ending at 1.0).  NULL sigma_f: no fission data.  Other
     * runs treat a fission as an absorption. */
    const double *sigma_f, *nu, *chi;
    /* Non-analog weights (the closeout of the paper's decomposed transport
     * loop, Sec. 4: weights and weight windows).  implicit_capture = 1: a
     * collision never absorbs; the particle scatters with its weight times
     * the scattering probability (sigma_s / sigma_t, or the chosen species'
     * sigma_s / (sigma_a + sigma_s)); then, if the weight is below w_cutoff,
     * Russian roulette (random-number slot 5) keeps it with probability
     * w / w_survival at weight w_survival, else the history ends (fate
     * ROULETTE).  Tally pieces score length times weight.  Needs
     * 0 <= w_cutoff <= w_survival, w_survival > 0.  Forward runs only (the
     * backward and k-eigenvalue runs take analog problems). */
    int32_t implicit_capture;
    double w_cutoff, w_survival;
    /* Spatial weight windows, applied by the closeout that ends every
     * collision leaving the particle alive and every surface crossing that
     * does not leak (the paper's closeout event, Sec. 4, "handles weights and
     * weight windows").  ww_n[0] > 0: a uniform grid of ww_n[0] x ww_n[1] x
     * ww_n[2] cells over the (finite) box; the cell of a point has ix = the
     * integer part of (x - box_lo) * (ww_n / (box_hi - box_lo)), clamped to
     * the grid, index (iz * ww_n[1] + iy) * ww_n[0] + ix.  ww_lo[cell] is the
     * window's lower bound (0: no window there), ww_ratio * ww_lo its upper
     * bound and ww_surv * ww_lo the survival weight (need ww_ratio > ww_surv
     * > 1).  A weight above the window splits into n = floor(w / survival)
     * copies, clamped to [2, ww_max_split], of weight w / n: the particle
     * continues as the first, the others become histories of the next
     * generation, ordered by (parent history, copy), drawing from
     * random-number stream = generation; the run goes on until a generation
     * splits nothing (at most 64).  A weight below the window plays roulette
     * (slot 5): survival weight with probability w / survival, else the
     * history ends (ROULETTE).  With windows, implicit capture's global
     * cutoff roulette is off.  Single-problem forward runs (not batches,
     * mcx_backward, mcx_run_eigen or mcx_run_noalloc). */
    int32_t ww_n[3];
    const double *ww_lo;
    double ww_ratio, ww_surv;
    int32_t ww_max_split;
} mcx_problem_desc;

/* Options of one run.  Zero-initialise and set what you need; zero means the
 * default for every tuning field.  Tuning fields never change results. */
typedef struct {
    int32_t sched;            /* mcx_sched                                      */
    int32_t decomp;           /* mcx_decomp                                     */
    int32_t lookup;           /* mcx_lookup (continuous energy)                 */
    int32_t accumulate;       /* 0: zero the tallies first; 1: add into them    */
    uint64_t first_history;   /* single-problem handles: run histories          */
    uint64_t n_histories;     /*   [first, first+n); n = 0 means all            */
    int64_t stack_capacity;   /* stack: particles per event stack               */
    int64_t stack_threshold;  /* stack: make_work stops above this fill         */
    int32_t stash_links;      /* async: work links per wavefront stash (0 =
                                 library default: one per event plus one,
                                 plus one more for split events unless a
                                 smaller stash keeps more wavefronts resident) */
    int32_t arena_links;      /* async: links in the global arena               */
    int32_t waves_per_cu;     /* stack/async: resident wavefronts per CU        */
    int32_t block_size;       /* naive: threads per block                       */
    void *hip_stream;         /* hipStream_t; NULL = the default stream         */
    void *digest;             /* optional device array of mcx_digest, one per
                                 history (all problems, in order)               */
    int32_t time_kernels;     /* 1: time every launch with HIP events           */
    int32_t force_spill;      /* async, testing: send every k-th filled link
                                 through the global arena (0 = never)           */
    int32_t consolidate;      /* async: a drained wavefront whose stash holds
                                 few particles hands them to the arena, where
                                 other wavefronts merge them into full links:
                                 0 = library default, 1 = on, 2 = off           */
    int32_t stack_tail_events;/* stack: when the live particles no longer fill
                                 the resident wavefronts, a popped particle
                                 runs up to this many events before it is
                                 pushed (0 = default 64, 1 = one per round)   */
    int32_t stack_min_events; /* stack: events a popped particle runs before it
                                 is pushed again, at least (0 = default 1:
                                 remap after every event)                     */
    int32_t tally_path;       /* single-problem forward runs: where tally adds
                                 go (mcx_tally_path; 0 = chosen by tally size
                                 and scheduler).  Batches and backward passes
                                 add into the tallies directly.               */
    int32_t async_block_waves;/* async: wavefronts per block, 1, 2 or 4; each
                                 keeps its own stash, the block shares one LDS
                                 copy of the tables and tally sums (0 =
                                 library default, 4; with stash_links 0, 2
                                 with the smallest stash when that keeps more
                                 wavefronts resident per CU; fewer when the
                                 block's LDS would not fit)                   */
    int32_t async_drain_events;/* async: once a wavefront has run out of full
                                 links (source done, arena empty) a partly
                                 filled link's particles run up to this many
                                 events in place before they are packed again
                                 (0 = library default, 8; 1 = one per pass)   */
    int32_t async_shared_stash;/* async: 1 = the wavefronts of a block share one
                                 stash of work links through lock-free
                                 transactions (paper Sec. 5.2: one stash used
                                 by several warps for higher occupancy);
                                 stash_links then sizes the block's pool
                                 (0 = one link per event, one per wavefront
                                 and two more; at most 32).  0 = library
                                 default: shared for split events on runs of
                                 at least 5e5 histories unless stash_links or
                                 consolidate is set, else one stash per
                                 wavefront; 2 = one stash per wavefront      */
    void *workspace;          /* optional caller-owned device memory (on the
                                 handle's device, 256-byte aligned) of ws_bytes
                                 bytes for the run's scheduler state and tally
                                 replicas (mcx_run, mcx_backward); the library
                                 then allocates no scratch of its own for it.
                                 Too small (see mcx_workspace_size):
                                 MCX_E_INVALID_ARG before anything runs.  NULL:
                                 the handle's own workspace, grown on demand. */
    size_t ws_bytes;
    int32_t async_bulk_events;/* async, fused events: a full link's particles
                                 run up to this many events in place, until
                                 more than 4 of them have ended, before the
                                 link is repacked and refilled (0 = library
                                 default, 64; 1 = one event per pass)         */
    int32_t stack_bulk_events;/* stack, fused events: a popped chunk's
                                 particles go on past their events per pop,
                                 up to this many events in place, while at
                                 least 60 of its 64 lanes hold live particles
                                 (0 = library default: 64 for continuous
                                 energy, 1 = off for multigroup problems,
                                 whose short histories make the rounds wait
                                 for the chunks that go on)                   */
} mcx_run_opts;

/* Tally paths (results are the same integers on every path):
 *  MCX_TALLY_PATH_LDS       each block sums its adds in LDS and adds the
 *                           sums once at its end (at most 4096 bins);
 *  MCX_TALLY_PATH_REPLICAS  adds go to one of 16 copies of the tally,
 *                           chosen by wavefront, summed after the launch
 *                           (at most 2^24 bins);
 *  MCX_TALLY_PATH_DIRECT    adds go to the tally itself. */
enum { MCX_TALLY_PATH_AUTO = 0, MCX_TALLY_PATH_LDS = 1, MCX_TALLY_PATH_REPLICAS = 2, MCX_TALLY_PATH_DIRECT = 3 };

/* one record per history, written by runs that pass opts.digest */
typedef struct {
    int64_t qsum;             /* sum of the history's tally contributions       */
    uint32_t flights;
    uint32_t collisions;
    uint32_t fate;            /* MCX_FATE_*                                     */
    uint32_t pad;
} mcx_digest;

/* totals of the last run.  After mcx_backward: the events of its second
 * replay (pass B), with launches, rounds and kernel_ms summed over both
 * replays. */
typedef struct {
    uint64_t sourced, flights, collisions, scatters, absorbs, crossings;
    uint64_t leaks, reflections, cutoffs, killed, pieces, qsum;
    uint64_t overflow;        /* 1 if the total of all contributions hit 2^63   */
    uint64_t events;          /* event executions (per particle)                */
    uint64_t lane_slots;      /* 64 x wavefront event dispatches                */
    uint64_t dispatches;      /* wavefront event dispatches                     */
    uint64_t spills, refills; /* async: links moved to / from the global arena  */
    uint64_t make_work;       /* wavefront source calls                         */
    uint64_t rounds;          /* stack: kernel launches (remapping rounds)      */
    uint64_t launches;        /* kernel launches of the run                     */
    double kernel_ms;         /* summed launch durations (time_kernels = 1)     */
    int32_t grid_blocks;      /* blocks of the main launch                      */
    int32_t block_threads;    /* threads per block of the main launch           */
    int32_t lds_bytes;        /* dynamic LDS per block of the main launch       */
    int32_t pad;
    uint64_t fissions;        /* k-eigenvalue runs: fissions (all cycles)       */
    uint64_t sites;           /*   and neutrons banked                          */
    uint64_t roulettes;       /* histories ended by weight roulette             */
    uint64_t cdf_scans;       /* multigroup scatters: transfer-CDF entries read
                                 to find the outgoing group (k + 1 for group k) */
    uint64_t splits;          /* weight windows: copies split off (all generations) */
    uint64_t generations;     /* weight windows: generations run (1 without)    */
} mcx_counters_t;

/* k-eigenvalue power iteration (the multigroup workload of Sec. 4 of the
 * paper).  Cycle c runs N_c histories on random-number stream c (the fourth
 * Philox counter word): cycle 0 from the problem's source (N_0 = N, the same
 * histories as mcx_run), later cycles from the source bank.  Every fission
 * banks its neutrons at its site; the bank is ordered by history.
 * Splitting-roulette brings the M_c banked neutrons back to about N: with
 * r = N / M_c each site is copied floor(r) times, plus once when
 * u_j < r - floor(r), u_j the first deviate of counter (j, 0xFFFFFFFF, 0, c);
 * the copies in site order are the next cycle's source.  A banked neutron
 * starts isotropic with a group drawn from chi of the material at its site
 * (slot 0).  Tallies are summed over cycles c >= n_inactive; counters over all
 * cycles.  Single-problem multigroup handles with fission data and no time
 * bins; the source bank holds at most 2 N + 1024 particles (MCX_E_CAPACITY
 * beyond); a cycle that banks nothing fails with MCX_E_STATE. */
typedef struct {
    uint64_t n_particles;     /* N: source particles per cycle (1 .. 2^30)       */
    int32_t n_cycles;         /* cycles (>= 1)                                   */
    int32_t n_inactive;       /* first cycles not tallied (0 .. n_cycles)        */
    double *k_cycle;          /* out, host [n_cycles]: M_c / N_c                 */
    uint64_t *n_source;       /* out, host [n_cycles]: N_c                       */
} mcx_eigen_opts;

/* Create a handle for n_problems independent problems (a batch runs all of
 * them in one launch).  The problems are those of the paper's Sec. 4 (a
 * multigroup lattice and a continuous-energy pin cell, with mesh, energy and
 * time tallies) and simpler boxes for checks.  All problems of a batch must share geometry kind,
 * energy mode and tally kind.  Invalid descriptors are rejected with no side
 * effect.  Uses the current HIP device. */
mcx_status mcx_create_problem(const mcx_problem_desc *descs, int32_t n_problems, mcx_problem_t *out);

/* Replace the multigroup Sigma_t, Sigma_s [n_mat*n_grp] of one problem
 * (transfer probabilities stay): the parameters of the differentiable run
 * (no passage of the paper; see mcx_backward).  Both must satisfy 0 <= Sigma_s <= Sigma_t,
 * Sigma_t > 0. */
mcx_status mcx_set_xs(mcx_problem_t p, int32_t problem, const double *sigma_t, const double *sigma_s,
                      int32_t where);

/* Run histories through the selected scheduler (forward transport with
 * tallies): the event loop of the paper's Sec. 4 (monolithic or decomposed
 * events) under thread-data remapping (Sec. 2), stack-based (Sec. 3.1) or
 * asynchronous (Sec. 3.2), with histories generated on demand from an atomic
 * counter and keyed random numbers (Sec. 3).  Synchronises the run's stream
 * before returning.  Errors: MCX_E_INVALID_ARG (bad options, history range
 * or workspace; nothing runs), MCX_E_CAPACITY (stack or link arena full),
 * MCX_E_OVERFLOW, MCX_E_DEVICE; on any error the tallies read MCX_E_STATE. */
mcx_status mcx_run(mcx_problem_t p, const mcx_run_opts *opts);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): mcx_run
 * with the run's scheduler state (stack banks and counters, or the async
 * link arena) and tally replicas in a fixed device array of the library,
 * MCX_NOALLOC_SCRATCH_BYTES per device, held from the first mcx_create_problem
 * on that device until the process ends.  It calls no hipMalloc, hipFree or
 * other allocating routine; the handle (mcx_create_problem) owns the
 * tallies and problem tables as for mcx_run.  Same results as mcx_run.
 * A run whose scratch exceeds the array returns MCX_E_INVALID_ARG before
 * anything runs.  The async link arena depends on the launch shape, not on
 * the history count (tens of MB at the default shape); the stack scheme's
 * banks scale with its capacity and resident wavefronts and by default do
 * not fit: give stack_capacity and waves_per_cu (e.g. 262144 and 1 for fused
 * events).  opts.workspace must be NULL and opts.time_kernels 0.  Every call on one device shares that device's array
 * (each run initialises what it reads): calls that overlap on one device,
 * from any handle or stream, race. */
#define MCX_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
mcx_status mcx_run_noalloc(mcx_problem_t p, const mcx_run_opts *opts);

/* Copy problem `problem`'s raw int64 tally (n = its bin count) to out: the
 * track-length tallies of the paper's Sec. 4 (mesh, or energy bins with an
 * optional time dimension).  MCX_E_STATE without a successful run. */
mcx_status mcx_tallies(mcx_problem_t p, int32_t problem, int64_t *out, int64_t n, int32_t where);

/* Score-function (likelihood-ratio) backward of the last forward run (the
 * paper has no derivatives; this is the differentiable extension): for
 * T_b = raw_b 2^-S / N (per problem, N = histories run), given dL/dT_b,
 * returns grad Sigma_t and grad Sigma_s [n_mat*n_grp] of
 * sum_b dL/dT_b dE[T_b]/d theta, estimated by replaying every history from
 * its random-number keys twice (pass A: G_h = sum over the history's tally
 * pieces of dL/dT_bin * length; pass B: G_h times track length, absorptions
 * and scatters per (material, group), in int64 fixed point at an adaptive
 * power-of-two scale).  problem = -1 covers all problems of a batch:
 * dL_dT is then the concatenation of every problem's bins and the gradients
 * the concatenation of every problem's n_mat*n_grp entries.  With implicit
 * capture the tally's weights are products of Sigma_s / Sigma_t over earlier
 * collisions: pass B also walks the tally for the running score F and adds,
 * at every collision, G_h and the score still to come, G_h - F, so that
 * grad Sigma_t = -SL + (SC - SR) / Sigma_t and grad Sigma_s = SR / Sigma_s
 * (times 2^-s / N); the roulette's survival probability is held at its value
 * (a fixed-probability roulette is unbiased for every Sigma).  Multigroup
 * problems without weight windows only (MCX_E_INVALID_ARG otherwise).
 * opts selects the scheduler and tuning for the replays (accumulate, range
 * and digest fields are ignored). */
mcx_status mcx_backward(mcx_problem_t p, int32_t problem, const double *dL_dT, double *grad_sigma_t,
                        double *grad_sigma_s, int32_t where, const mcx_run_opts *opts);

/* Run a k-eigenvalue calculation (see mcx_eigen_opts; the C5G7 power
 * iteration with splitting-roulette population control of the paper's
 * Sec. 4) through the scheduler and tuning of opts (its range, accumulate and digest fields are ignored).
 * On success the tallies hold the active cycles' sum and k_cycle, n_source
 * are filled; mcx_backward does not apply to it. */
mcx_status mcx_run_eigen(mcx_problem_t p, const mcx_run_opts *opts, const mcx_eigen_opts *eig);

/* Device scratch (bytes) that mcx_run, and mcx_backward after it, with
 * these options need for their scheduler state (stack banks and counters,
 * Sec. 3.1 of the paper; or the async scheduler's global link arena, its
 * reservoir for spilled work links, Sec. 3.2) and tally replicas: the smallest opts.workspace
 * they accept.  0 for the naive scheduler without replicas.  Without a
 * caller workspace the library grows its own to this size and keeps it.
 * Allocates and launches nothing. */
mcx_status mcx_workspace_size(mcx_problem_t p, const mcx_run_opts *opts, size_t *bytes);

/* Totals of the last run (see mcx_counters_t): events, lane slots and
 * launches measure the remapping itself (the paper's Sec. 5.1 calls for
 * profiling to find what limits it). */
mcx_status mcx_counters(mcx_problem_t p, mcx_counters_t *out);

/* Stack scheduler (paper Sec. 3.1: one launch per remapping round): the
 * input population (particles popped) of each round of the last pass, for
 * its first 512 rounds.  Writes min(max_rounds, *n_rounds) entries to
 * particles (host memory) and the number of recorded rounds to *n_rounds
 * (0 after a run of another scheduler). */
mcx_status mcx_stack_rounds(mcx_problem_t p, uint32_t *particles, int32_t max_rounds, int32_t *n_rounds);

/* Sizes of problem `problem`: tally bins, materials, groups, histories
 * (bookkeeping, no passage). */
mcx_status mcx_problem_info(mcx_problem_t p, int32_t problem, int64_t *n_bins, int32_t *n_mat, int32_t *n_grp,
                            uint64_t *n_histories);

/* Free the handle and everything the library allocated for it (never caller
 * memory).  NULL is a no-op. */
void mcx_destroy_problem(mcx_problem_t p);
/* Static text of a status; the handle's last error message (owned by the
 * handle, valid until its next call). */
const char *mcx_status_str(mcx_status s);
const char *mcx_last_error(mcx_problem_t p);

#ifdef __cplusplus
}
#endif
#endif
