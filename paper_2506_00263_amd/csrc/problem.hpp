// Device-resident description of one problem of a run, filled by the host
// side of the library (api.cpp) and read by every kernel.  Pointers are
// device addresses.  Run-specific fields (history range, backward buffers)
// are refreshed before every launch sequence.
#pragma once
#include <stdint.h>

namespace mcx {

enum : int { GEOM_BOX = 0, GEOM_LATTICE = 1 };
enum : int { EMODE_MG = 0, EMODE_CE = 1 };
enum : int { MODE_FWD = 0, MODE_REPLAY_A = 1, MODE_REPLAY_B = 2 };
enum : int { MAX_SPECIES = 4 };

// A copy split off by a weight window: a history of the next generation
// starts from it.  parent: the history that split it off (index in its
// generation); seq: the copy's ordinal among that history's copies.
struct SiteRec {
    double pos[3], dir[3], e, w, t;
    uint32_t gc, parent, seq, pad;
};

struct ProbDev {
    // geometry
    int32_t geometry, n_slabs, nx, ny;
    int32_t mod_mat, refl_mask;      // bit f: face f (x-,x+,y-,y+,z-,z+) reflects
    double box_lo[3], box_hi[3];
    double radius, r2;               // r2 = radius * radius
    const double *xpl;               // slab planes (box) or lattice x planes
    const double *ypl, *cxs, *cys;
    const int32_t *cmat;             // slab materials or pin materials
    // multigroup
    int32_t n_mat, n_grp;
    const double *sig_t, *sig_s, *cdf;
    // continuous energy
    int32_t n_species, grid_len;
    const double *egrid, *siga, *sigs, *awr, *dens;
    double e_min, e_src;
    int32_t hash_bins, lookup_hash;
    double hash_ln_lo, hash_inv;
    const int32_t *hash_lo, *hash_hi;   // [species][bin]
    // source
    int32_t src_kind, src_iso, src_group, tally_kind;
    double src_pos[3], src_lo[3], src_ext[3], src_dir[3];
    double src_radius;
    // tally
    int32_t mesh_n[3], n_ebins;
    const double *mx, *my, *mz, *eedges;
    // index guesses for (nearly) uniform edges: cell ~ (x - lo) * inv, then
    // corrected against the edges; inv = 0 means search instead
    double mesh_lo[3], mesh_inv[3];
    double ebin_lnlo, ebin_inv;      // energy bins uniform in ln E
    double tscale;                   // 2^tally_scale_log2
    unsigned long long *tally;       // this problem's bins
    unsigned long long *trep;        // [TREP][n_bins] replicas of a large energy-bin tally
                                     // (summed into tally after the run), or null
    // random numbers and histories of the current run
    uint32_t key0, key1;
    uint64_t first, count;           // histories [first, first + count)
    uint64_t gbase;                  // offset in the run's flattened id space
    int64_t max_steps;
    // score-function backward of the current run
    const double *w;                 // dL/dT over this problem's bins
    double *G;                       // per history, indexed gbase + (h - first)
    double gscale;                   // 2^s of pass B
    unsigned long long *U;           // pass A bound (uint64)
    unsigned long long *SL, *SA, *SS;  // pass B sums [n_mat*n_grp] (int64 bits)
    int32_t acc_off, pad;            // offset of this problem in per-wave LDS sums
    // The small tables every event reads (Sigma_t, Sigma_s, transfer CDF,
    // planes, pin centres, mesh edges, group speeds, then the int32 cell
    // materials) sit packed at tl_src; single-problem launches copy them
    // into LDS.
    // tl_off[t]: offset of table t in 8-byte words (TL_CMAT: in 4-byte words).
    const double *tl_src;
    int32_t tl_bytes;                // packed size, a multiple of 16
    int32_t tl_off[15];
    // time-binned tally (temporal tally resolution, paper Sec. 4): n_tbins
    // equal bins of width tw = t_max / n_tbins; 0 = no time dimension.  A
    // particle moves at speed[g] (multigroup, a packed table) or
    // speed_coef * sqrt(E); bins are laid out [time bin][nbase bins].
    int32_t n_tbins, pad1;
    double t_max, tw, speed_coef;
    long long nbase;                 // bins of the tally without time
    long long n_bins;                // all bins of this problem's tally
    const double *speed;
    // fission (k-eigenvalue cycles, multigroup): Sigma_f, nu per (material,
    // group) and the cumulative fission spectrum chi per material (packed
    // tables).  Cycle state, null outside k-eigenvalue cycles: the cycle's
    // source positions (3 per history) and, per history, the neutrons it
    // banks and its fission site (3 doubles).
    const double *sigf, *nu, *chi;
    const double *sbank;
    uint32_t *fn;
    double *fpos;
    uint32_t stream;                 // random-number stream: the cycle (0 otherwise)
    // non-analog weights: implicit capture, and weight roulette below w_cut
    // to weight w_surv (the closeout of a collision)
    int32_t implicit;
    double w_cut, w_surv;
    // spatial weight windows (the closeout of a collision or crossing): a
    // uniform grid of ww_n cells over the box, ww_inv = ww_n / (box_hi -
    // box_lo), lower bound ww_lo per cell (0: none), upper ww_ratio * lo,
    // survival ww_surv * lo, at most ww_max_split copies; ww_n[0] = 0: none
    int32_t ww_n[3], ww_max_split;
    double ww_inv[3];
    const double *ww_lo;
    double ww_ratio, ww_surv;
    // generations of split copies: this generation's source sites (null in
    // generation 0), the staging area for the copies it splits off (gcap
    // records, gcount filled), and per history the copies it banked
    const SiteRec *gsrc;
    SiteRec *gout;
    unsigned long long *gcount;
    uint64_t gcap;
    uint32_t *gn;
};

enum : int {
    TL_SIG_T = 0, TL_SIG_S, TL_CDF, TL_XPL, TL_YPL, TL_CXS, TL_CYS, TL_MX, TL_MY, TL_MZ, TL_SPEED,
    TL_SIGF, TL_NU, TL_CHI, TL_CMAT
};
constexpr int TL_NDBL = TL_CMAT;      // tables of doubles in front of the int32 materials
constexpr int TL_MAX_BYTES = 32768;   // larger tables stay in global memory
constexpr int LT_MAX_BINS = 4096;     // tallies up to this size can be summed in LDS per block
constexpr int TREP = 16;              // or go to TREP replicas chosen by wavefront
constexpr long long TREP_MAX_BINS = 1ll << 24;

enum Counter : int {
    C_SOURCED = 0, C_FLIGHTS, C_COLLISIONS, C_SCATTERS, C_ABSORBS, C_CROSSINGS, C_LEAKS, C_REFLECTIONS,
    C_CUTOFFS, C_KILLED, C_PIECES, C_EVENTS, C_LANE_SLOTS, C_DISPATCHES, C_SPILLS, C_REFILLS, C_MAKE_WORK,
    C_FISSIONS, C_ROULETTES, C_COMPLETED, C_QSUM, C_PASSA_U, C_CDF, C_SPLITS, C_NUM
};
constexpr int C_WAVE = C_COMPLETED;   // entries counted per wavefront (32-bit)

// Run totals are kept in CTL_STRIPES copies, one 256-byte block each; a
// wavefront adds into copy (wave id mod CTL_STRIPES) and the host sums the
// copies.  One shared copy would serialise every wavefront's atomics.
constexpr int CTL_STRIPES = 64;
struct CtlStripe {
    unsigned long long c[32];        // Counter entries, padded to 256 bytes
};

constexpr int STACK_ROUND_LOG = 512;   // stack rounds whose input population is recorded

// Per-run control block in device memory.
struct RunCtl {
    unsigned long long src_cursor;   // next flattened history id to source
    unsigned long long total;        // flattened histories of the run
    unsigned int error;              // bit 0 capacity, bit 1 overflow, bit 2 pass-A bound
    unsigned int done_round;         // stack: round that found every history ended (+1)
    unsigned int active;             // async: wavefronts still running
    unsigned int pad0;
    unsigned long long pad[12];
    CtlStripe stripe[CTL_STRIPES];
    unsigned int round_in[STACK_ROUND_LOG];   // stack: input particles of each round (first rounds)
};

enum : unsigned int { ERR_CAPACITY = 1u, ERR_OVERFLOW = 2u, ERR_BOUND = 4u };

}  // namespace mcx
