/*
 * CPU oracle for event-based Monte Carlo transport -- TEST INFRASTRUCTURE.
 *
 * This is the plain, slow, history-based definition of what the transport
 * hot path computes.  Thread-data remapping (paper Sec. 2) only reorders
 * independent histories and the events inside them; it never changes what
 * a history computes.  So the result of every scheduler (naive, stack-based,
 * asynchronous, batched) must equal the loop
 *
 *     for each history h: run h to completion, add each fixed-point
 *                         track-length contribution into an int64 tally
 *
 * which is what this file implements, one history at a time.
 *
 * Only the tests, the package smoke check and the benchmark's CPU baseline
 * may load this library.  It shares no code, header, table or constant with
 * the GPU library.
 *
 * "parity unpinned" against the paper itself: the paper prints no worked
 * example or table of values for this workload; pins are closed forms,
 * library routines and brute force (see tests/test_oracle_*.py).
 */
#ifndef MCX_ORACLE_H
#define MCX_ORACLE_H
#include <stdint.h>

typedef struct {
    int32_t geometry;          /* 0 box of x-slabs, 1 pin lattice            */
    double box_lo[3], box_hi[3];
    int32_t bc[6];             /* x-,x+,y-,y+,z-,z+ : 0 vacuum, 1 reflective */
    int32_t n_slabs;           /* box: slab planes [n_slabs+1], materials    */
    const double *slab_planes;
    const int32_t *slab_mat;
    int32_t nx, ny;            /* lattice                                    */
    const double *xplanes, *yplanes, *cx, *cy;
    double radius;
    const int32_t *pin_mat;
    int32_t mod_mat;
    int32_t energy_mode;       /* 0 multigroup, 1 continuous energy          */
    int32_t n_mat, n_grp;
    const double *sigma_t, *sigma_s, *cdf;   /* [M*G], [M*G], [M*G*G]        */
    int32_t n_species, grid_len;
    const double *e_grid, *sig_a, *sig_s;    /* [S*grid_len]                 */
    const double *awr, *density;             /* [S], [M*S]                   */
    double e_min, e_source;
    int32_t src_kind;          /* 0 point, 1 box volume, 2 disc              */
    int32_t src_isotropic;
    int32_t src_group;
    int32_t tally_kind;        /* 0 mesh, 1 energy bins                      */
    double src_pos[3], src_lo[3], src_hi[3], src_dir[3];
    double src_radius;
    int32_t mesh_n[3];
    const double *mesh_x, *mesh_y, *mesh_z;
    int32_t n_ebins;
    const double *e_edges;
    int32_t tally_scale_log2;
    uint32_t problem_id;
    uint64_t seed;
    int64_t max_steps;
    /* time-binned tallies (0 bins: no time dimension).  A particle starts at
       time 0 and moves at speed v: speed[g] (multigroup) or
       speed_coef * sqrt(E) (continuous energy).  A flight that would reach
       t_max ends there and the history ends (a cutoff).  Bins are
       [k dt, (k+1) dt), dt = t_max / n_tbins; the tally is laid out
       [time bin][bins without time]. */
    int32_t n_tbins;
    double t_max;
    const double *speed;       /* [G], multigroup                            */
    double speed_coef;         /* continuous energy                          */
    /* fission (multigroup k-eigenvalue runs; NULL sigma_f: none).  An
       absorption in (m, g) is a fission with probability
       sigma_f / (sigma_t - sigma_s); it emits floor(nu + xi) neutrons at the
       collision site.  chi [M*G]: cumulative fission spectrum per material.
       Fixed-source runs ignore fission (it is one kind of absorption). */
    const double *sigma_f, *nu, *chi;
    /* non-analog weights (the closeout of a collision): with implicit
       capture a collision never absorbs, the particle scatters with its
       weight times the scattering probability (Sigma_s / Sigma_t, or the
       chosen species' sigma_s / (sigma_a + sigma_s)); then, if the weight is
       below w_cutoff, Russian roulette (slot 5) keeps it with probability
       w / w_survival at weight w_survival, else the history ends (fate
       ROULETTE).  Every tally piece scores length times weight. */
    int32_t implicit_capture;
    double w_cutoff, w_survival;
    /* spatial weight windows, applied by the closeout that ends every
       collision leaving the particle alive and every surface crossing that
       does not leak (weights and weight windows for the next flight).
       ww_n[0] > 0: a uniform grid of ww_n[0] x ww_n[1] x ww_n[2] cells over
       the box; the cell of a point has ix = the integer part of
       (x - box_lo) * (ww_n / (box_hi - box_lo)), clamped to the grid, and
       index c = (iz * ww_n[1] + iy) * ww_n[0] + ix.  ww_lo[c] is the lower
       bound of the window of cell c (0: no window there), ww_ratio * ww_lo
       the upper bound, ww_surv * ww_lo the survival weight.  A weight above
       the upper bound is split into n = floor(w / survival), clamped to
       [2, ww_max_split], copies of weight w / n: the particle continues as
       the first and the others are banked, in order, as histories of the
       next generation; a weight below the lower bound plays roulette (slot 5):
       it survives with probability w / survival at the survival weight, else
       the history ends (ROULETTE).  With windows, implicit capture's global
       cutoff roulette is off.  Needs a finite box, ww_ratio > ww_surv > 1 and
       ww_max_split >= 2 (checked by the Python marshalling); forward runs
       only (orc_run_gen). */
    int32_t ww_n[3];
    const double *ww_lo;
    double ww_ratio, ww_surv;
    int32_t ww_max_split;
} orc_problem;

/* a banked split copy: a history of the next generation starts from it */
typedef struct {
    double pos[3], dir[3], e, w, t;
    int32_t g, cell[3];
} orc_site;

/* what a history ended with */
enum { ORC_FATE_LEAK = 0, ORC_FATE_ABSORB = 1, ORC_FATE_CUTOFF = 2, ORC_FATE_KILLED = 3, ORC_FATE_ROULETTE = 4 };

typedef struct {              /* one record per history                    */
    int64_t qsum;             /* sum of its fixed-point tally contributions */
    uint32_t flights;
    uint32_t collisions;
    uint32_t fate;
    uint32_t pad;
} orc_digest;

typedef struct {              /* totals over a run (scheduler invariant)   */
    uint64_t sourced, flights, collisions, scatters, absorbs, crossings;
    uint64_t leaks, reflections, cutoffs, killed, pieces, qsum;
    uint64_t overflow;        /* 1 if the total of all q reached 2^63       */
    uint64_t fissions, sites; /* k-eigenvalue runs: fissions, neutrons banked */
    uint64_t roulettes;       /* histories ended by weight roulette          */
    uint64_t cdf_scans;       /* multigroup scatters: transfer-CDF entries read
                                 to find the outgoing group (k + 1 for group k) */
    uint64_t splits;          /* weight windows: copies banked for the next generation */
} orc_counts;

/* primitives, exposed for tests */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_uniform(uint64_t seed, uint32_t problem_id, uint32_t particle, uint32_t step,
                   uint32_t slot, uint32_t stream);
double orc_nlog(double x);
double orc_sqrt(double x);
void orc_cos_sin_turn(double t, double *c, double *s);
int64_t orc_fixed(double x, int32_t scale_log2);

/* geometry hooks for tests: distance to the next surface from a located state */
int32_t orc_locate(const orc_problem *p, const double pos[3], const double dir[3], int32_t cell[3]);
double orc_distance(const orc_problem *p, const double pos[3], const double dir[3],
                    const int32_t cell[3], int32_t *surface);
int32_t orc_ce_index(const double *grid, int32_t n, double e);        /* linear scan  */
int32_t orc_ce_index_fast(const double *grid, int32_t n, double e);   /* bisection    */
int32_t orc_edge_index(const double *edges, int32_t n, double x, double dir, int32_t fast);

double orc_elastic(double A, double e, double xi_mu, double xi_phi, double dir[3]);
void orc_tally_segment(const orc_problem *p, const double pos[3], const double dir[3], double d,
                       int32_t g, double *out);
double orc_ce_xs_hook(const orc_problem *p, int32_t m, double e, double *sa, double *ss);

/* forward: histories [h0, h1) added into tally; digest (optional) indexed h-h0;
   returns 0, 1 (overflow) or 4 (a problem with weight windows: see orc_run_gen) */
int orc_run(const orc_problem *p, uint64_t h0, uint64_t h1, int64_t *tally,
            orc_digest *digest, orc_counts *counts);

/* one generation of a run with weight windows: histories [h0, h1) of
   generation gen (0: the problem's source; gen > 0: history h starts from
   src[h] and draws from random-number stream gen), tallies added into
   tally; the copies split off are appended to bank (capacity bank_cap) in
   history order, *bank_n counting them.  Returns 0, 1 (overflow) or 3
   (bank full). */
int orc_run_gen(const orc_problem *p, int32_t gen, const orc_site *src, uint64_t h0, uint64_t h1, int64_t *tally,
                orc_digest *digest, orc_counts *counts, orc_site *bank, uint64_t bank_cap, uint64_t *bank_n);

/* score-function backward, pass A: G_h = sum over tally pieces of w[bin]*len
   (len times the weight in weighted runs), with L_h (track length) and n_h
   (flights); U += ceil(|G_h| * (L_h + n_h)), or with implicit capture
   U += ceil((|G_h| + A_h) * (L_h + n_h)), A_h = sum of |w[bin]*len| */
int orc_replay_a(const orc_problem *p, uint64_t h0, uint64_t h1, const double *w,
                 double *G, uint64_t *U);

/* pass B at scale 2^s, q(x) = rint(x * 2^s): SL[m*G+g] += q(G_h*len) per
   flight.  Analog runs: SA += q(G_h) per absorption, SS += q(G_h) per
   scatter (w unused, may be NULL).  Implicit capture: at every collision
   SA += q(G_h) and SS += q(G_h - F), F the score w[bin]*len of the pieces
   flown so far (w required; returns 2 without it). */
int orc_replay_b(const orc_problem *p, uint64_t h0, uint64_t h1, const double *w, const double *G, int32_t s,
                 int64_t *SL, int64_t *SA, int64_t *SS);

/* k-eigenvalue power iteration (multigroup, fission data required).
   Cycle c runs N_c histories with random-number stream c: cycle 0 from the
   problem's source (N_0 = N), later cycles from the source bank.  Every
   fission banks its neutrons at the collision site, in history order.
   Splitting-roulette brings the M_c banked neutrons back to about N: with
   r = N / M_c each site is copied floor(r) times plus once more when
   u_j < r - floor(r), u_j = orc_uniform(seed, id, j, 0xFFFFFFFF, 0, c); the
   copies in site order are the next source.  A banked neutron starts with
   an isotropic direction (slots 3, 4) and a group drawn from chi of the
   material at its site (slot 0).  k_c = M_c / N_c; n_source[c] = N_c.
   Cycles c >= n_inactive add into tally; counts are totals over all cycles.
   bank (optional, 3 doubles per particle, capacity bank_cap) receives the
   source of the cycle after the last, *bank_n its size.
   Returns 0, 1 (overflow), 2 (no neutron banked in a cycle), 3 (bank full). */
int orc_eigen(const orc_problem *p, uint64_t N, int32_t n_cycles, int32_t n_inactive, int64_t *tally,
              double *k_cycle, uint64_t *n_source, orc_counts *counts, double *bank, uint64_t bank_cap,
              uint64_t *bank_n);

#endif
