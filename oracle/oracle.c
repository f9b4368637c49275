/*
 * CPU oracle for event-based Monte Carlo transport -- TEST INFRASTRUCTURE.
 * Plain, single-threaded, one history at a time.  See oracle.h.
 *
 * Floating point: IEEE binary64, round to nearest even, no contraction
 * (built with -ffp-contract=off), every expression evaluated exactly as
 * parenthesised below.  Comparisons are explicit; no fmin/fmax.
 *
 * The paper (Sec. 3) generates particles on demand with atomic counters and
 * a hash-based (counter-based) random number scheme, so that any particle's
 * random numbers can be produced on any processor.  Here that scheme is
 * Philox4x32-10 keyed by (seed, problem) and indexed by (particle, flight,
 * slot).  One history is the history-based loop whose single iteration
 * is the paper's monolithic "step" event (Sec. 4): sample a flight, move
 * to the next collision or surface with its tally, then collide or cross.
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ RNG */

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
   easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies with the
   round keys advanced by the Weyl increments between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* One uniform deviate in [2^-53, 1 - 2^-53].  Key = (lo32(seed), hi32(seed)
   xor problem); counter = (particle, step, slot/2, stream); slot parity picks
   words (0,1) or (2,3); 53 bits with the lowest forced to one. */
double orc_uniform(uint64_t seed, uint32_t problem_id, uint32_t particle, uint32_t step,
                   uint32_t slot, uint32_t stream)
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) ^ problem_id };
    uint32_t ctr[4] = { particle, step, slot >> 1, stream };
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    uint32_t a = r[2 * (slot & 1)], b = r[2 * (slot & 1) + 1];
    uint64_t v = ((uint64_t)a << 32) | (uint64_t)b;
    uint64_t k = (v >> 11) | 1u;
    return (double)k * 0x1p-53;
}

/* ------------------------------------------------------- deterministic math */

/* -ln(x) for positive normal x.  x = m 2^e exactly from the bits; m folded
   into [sqrt(2)/2, sqrt(2)]; ln m = 2 atanh(s), s = (m-1)/(m+1), as the odd
   series s * sum_k 2/(2k+1) s^(2k), k = 0..10 (Horner); ln 2 split in a
   head with trailing zero bits (so e*head is exact) and a tail. */
static double orc_series_coef[11];
static double orc_cos_coef[11], orc_sin_coef[11];
static int orc_tables_ready = 0;

static void orc_init_tables(void)
{
    if (orc_tables_ready) return;
    for (int k = 0; k <= 10; ++k) orc_series_coef[k] = 2.0 / (double)(2 * k + 1);
    double fact[22];
    fact[0] = 1.0;
    for (int n = 1; n < 22; ++n) fact[n] = fact[n - 1] * (double)n;   /* exact up to 22! */
    for (int k = 0; k <= 10; ++k) {
        double sg = (k & 1) ? -1.0 : 1.0;
        orc_cos_coef[k] = sg / fact[2 * k];
        orc_sin_coef[k] = sg / fact[2 * k + 1];
    }
    orc_tables_ready = 1;
}

static const double ORC_LN2_HI = 0x1.62e42fefa38p-1;    /* 42 significant bits */
static const double ORC_LN2_LO = 0x1.ef35793c7673p-45;  /* ln 2 - LN2_HI       */
static const double ORC_SQRT2 = 0x1.6a09e667f3bcdp+0;
static const double ORC_PI_2 = 0x1.921fb54442d18p+0;

double orc_nlog(double x)
{
    orc_init_tables();
    uint64_t bits;
    memcpy(&bits, &x, 8);
    int e = (int)((bits >> 52) & 0x7ff) - 1023;
    uint64_t mbits = (bits & 0x000fffffffffffffull) | 0x3ff0000000000000ull;
    double m;
    memcpy(&m, &mbits, 8);
    if (m > ORC_SQRT2) {
        m = m * 0.5;
        e = e + 1;
    }
    double s = (m - 1.0) / (m + 1.0);
    double z = s * s;
    double poly = orc_series_coef[10];
    for (int k = 9; k >= 0; --k) poly = (poly * z) + orc_series_coef[k];
    double lnm = s * poly;
    double de = (double)e;
    double lnx = (de * ORC_LN2_HI) + ((de * ORC_LN2_LO) + lnm);
    return -lnx;
}

/* sqrt by Newton iteration on 1/sqrt(x): bit-level initial guess
   0x5FE6EB50C7B537A9 - (bits >> 1) (the published fast inverse square root
   for binary64), four iterations y <- y (1.5 - (x/2) y y), then s = x y and
   one correction s <- s + ((x - s s)/2) y.  x <= 0 (and NaN) give 0; tiny x
   is scaled by an exact power of two. */
double orc_sqrt(double x)
{
    if (!(x > 0.0)) return 0.0;
    if (x < 0x1p-1000) return orc_sqrt(x * 0x1p+1000) * 0x1p-500;
    uint64_t bits;
    memcpy(&bits, &x, 8);
    uint64_t ybits = 0x5FE6EB50C7B537A9ull - (bits >> 1);
    double y;
    memcpy(&y, &ybits, 8);
    double hx = 0.5 * x;
    for (int it = 0; it < 4; ++it) y = y * (1.5 - ((hx * y) * y));
    double s = x * y;
    s = s + ((0.5 * (x - (s * s))) * y);
    return s;
}

/* (cos 2 pi t, sin 2 pi t): quarter-turn reduction q = floor(4t), r = 4t - q
   (both exact), centred to |r| <= 1/2, x = r * (pi/2); Taylor series in x^2
   to x^20 (cos) and x^21 (sin); exact rotation by q mod 4. */
void orc_cos_sin_turn(double t, double *cp, double *sp)
{
    orc_init_tables();
    double t4 = 4.0 * t;
    double qd = floor(t4);
    double r = t4 - qd;
    long q = (long)qd;
    if (r > 0.5) {
        r = r - 1.0;
        q = q + 1;
    }
    double x = r * ORC_PI_2;
    double x2 = x * x;
    double c = orc_cos_coef[10];
    for (int k = 9; k >= 0; --k) c = (c * x2) + orc_cos_coef[k];
    double s = orc_sin_coef[10];
    for (int k = 9; k >= 0; --k) s = (s * x2) + orc_sin_coef[k];
    s = x * s;
    switch ((int)(((q % 4) + 4) % 4)) {
    case 0: *cp = c;  *sp = s;  break;
    case 1: *cp = -s; *sp = c;  break;
    case 2: *cp = -c; *sp = -s; break;
    default: *cp = s; *sp = -c; break;
    }
}

/* fixed point: rint(x * 2^S) with round-half-even (default rounding mode) */
int64_t orc_fixed(double x, int32_t scale_log2)
{
    return (int64_t)nearbyint(x * ldexp(1.0, scale_log2));
}

/* --------------------------------------------------------------- geometry */

/* largest i in [0, n-1] with edges[i] <= x (edges has n+1 entries); a point
   exactly on edge i moving in the negative direction belongs to cell i-1 */
static int32_t orc_cell_index(const double *edges, int32_t n, double x, double dir)
{
    int32_t i = 0;
    for (int32_t k = 0; k <= n; ++k)
        if (edges[k] <= x) i = k;
    if (i > n - 1) i = n - 1;
    if (x == edges[i] && dir < 0.0 && i > 0) i = i - 1;
    return i;
}

/* the same definition by bisection, used in the history loop for speed;
   tests pin it to the linear scan above */
static int32_t orc_cell_index_fast(const double *edges, int32_t n, double x, double dir)
{
    int32_t i = 0;
    if (edges[0] <= x) {
        int32_t lo = 0, hi = n;               /* edges[lo] <= x */
        while (lo < hi) {
            int32_t mid = lo + (hi - lo + 1) / 2;
            if (edges[mid] <= x) lo = mid; else hi = mid - 1;
        }
        i = lo;
    }
    if (i > n - 1) i = n - 1;
    if (x == edges[i] && dir < 0.0 && i > 0) i = i - 1;
    return i;
}

int32_t orc_edge_index(const double *edges, int32_t n, double x, double dir, int32_t fast)
{
    return fast ? orc_cell_index_fast(edges, n, x, dir) : orc_cell_index(edges, n, x, dir);
}

static double orc_plane_dist(double lo, double hi, double x, double u)
{
    double d = INFINITY;
    if (u > 0.0) d = (hi - x) / u;
    else if (u < 0.0) d = (lo - x) / u;
    if (d < 0.0) d = 0.0;
    return d;
}

/* surfaces: 0 x-plane, 1 y-plane, 2 z-plane, 3 cylinder */
int32_t orc_locate(const orc_problem *p, const double pos[3], const double dir[3], int32_t cell[3])
{
    if (p->geometry == 0) {
        cell[0] = orc_cell_index(p->slab_planes, p->n_slabs, pos[0], dir[0]);
        cell[1] = 0;
        cell[2] = 0;
    } else {
        cell[0] = orc_cell_index(p->xplanes, p->nx, pos[0], dir[0]);
        cell[1] = orc_cell_index(p->yplanes, p->ny, pos[1], dir[1]);
        double dx = pos[0] - p->cx[cell[0]];
        double dy = pos[1] - p->cy[cell[1]];
        cell[2] = (((dx * dx) + (dy * dy)) < (p->radius * p->radius)) ? 1 : 0;
    }
    return 0;
}

static int32_t orc_material(const orc_problem *p, const int32_t cell[3])
{
    if (p->geometry == 0) return p->slab_mat[cell[0]];
    if (cell[2]) return p->pin_mat[cell[1] * p->nx + cell[0]];
    return p->mod_mat;
}

double orc_distance(const orc_problem *p, const double pos[3], const double dir[3],
                    const int32_t cell[3], int32_t *surface)
{
    double x = pos[0], y = pos[1], z = pos[2], u = dir[0], v = dir[1], w = dir[2];
    double dx = INFINITY, dy = INFINITY, dz, dc = INFINITY;
    if (p->geometry == 0) {
        int32_t i = cell[0];
        dx = orc_plane_dist(p->slab_planes[i], p->slab_planes[i + 1], x, u);
        dy = orc_plane_dist(p->box_lo[1], p->box_hi[1], y, v);
        dz = orc_plane_dist(p->box_lo[2], p->box_hi[2], z, w);
    } else {
        int32_t i = cell[0], j = cell[1], inside = cell[2];
        dz = orc_plane_dist(p->box_lo[2], p->box_hi[2], z, w);
        double ddx = x - p->cx[i], ddy = y - p->cy[j];
        double a = (u * u) + (v * v);
        double k = (ddx * u) + (ddy * v);
        double c = ((ddx * ddx) + (ddy * ddy)) - (p->radius * p->radius);
        double disc = (k * k) - (a * c);
        if (inside) {
            if (a > 0.0) {
                if (disc < 0.0) disc = 0.0;
                dc = (orc_sqrt(disc) - k) / a;
            }
        } else {
            dx = orc_plane_dist(p->xplanes[i], p->xplanes[i + 1], x, u);
            dy = orc_plane_dist(p->yplanes[j], p->yplanes[j + 1], y, v);
            if (a > 0.0 && k < 0.0 && disc >= 0.0) dc = c / (orc_sqrt(disc) - k);
        }
        if (dc < 0.0) dc = 0.0;
    }
    int32_t s = 0;
    double d = dx;
    if (dy < d) { d = dy; s = 1; }
    if (dz < d) { d = dz; s = 2; }
    if (dc < d) { d = dc; s = 3; }
    *surface = s;
    return d;
}

/* ---------------------------------------------------------- cross sections */

/* largest i with grid[i] <= e, at most n-2 (e already clamped to the grid);
   plain linear scan from the bottom */
int32_t orc_ce_index(const double *grid, int32_t n, double e)
{
    int32_t i = 0;
    while (i + 1 < n - 1 && grid[i + 1] <= e) i = i + 1;
    return i;
}

/* binary search with the same definition, used for speed in the history
   loop; tests pin it to the linear scan above */
static int32_t orc_ce_index_bisect(const double *grid, int32_t n, double e)
{
    int32_t lo = 0, hi = n - 1;                 /* grid[lo] <= e holds */
    while (hi - lo > 1) {
        int32_t mid = lo + (hi - lo) / 2;
        if (grid[mid] <= e) lo = mid; else hi = mid;
    }
    if (lo > n - 2) lo = n - 2;
    return lo;
}

int32_t orc_ce_index_fast(const double *grid, int32_t n, double e)
{
    return orc_ce_index_bisect(grid, n, e);
}

typedef struct { double sa[8], ss[8], tot[8], cum[8], sigma_t; } orc_ce_xs;

/* per species: clamp E to the grid, bracket, lin-lin interpolation of the
   absorption and scattering cross sections; macroscopic total in ascending
   species order */
static void orc_ce_lookup(const orc_problem *p, int32_t m, double e, orc_ce_xs *xs)
{
    double cum = 0.0;
    int32_t n = p->grid_len;
    for (int32_t s = 0; s < p->n_species; ++s) {
        const double *g = p->e_grid + (int64_t)s * n;
        const double *sa = p->sig_a + (int64_t)s * n;
        const double *ss = p->sig_s + (int64_t)s * n;
        double ec = e;
        if (ec < g[0]) ec = g[0];
        if (ec > g[n - 1]) ec = g[n - 1];
        int32_t i = orc_ce_index_bisect(g, n, ec);
        double f = (ec - g[i]) / (g[i + 1] - g[i]);
        xs->sa[s] = sa[i] + (f * (sa[i + 1] - sa[i]));
        xs->ss[s] = ss[i] + (f * (ss[i + 1] - ss[i]));
        double dens = p->density[m * p->n_species + s];
        xs->tot[s] = dens * (xs->sa[s] + xs->ss[s]);
        cum = cum + xs->tot[s];
        xs->cum[s] = cum;
    }
    xs->sigma_t = cum;
}

/* ------------------------------------------------------------------ tallies */

typedef struct {
    int mode;                 /* 0 forward tally, 1 pass A, 2 pass B, 3 hook    */
    double *dtally;           /* mode 3: lengths in double                      */
    int64_t *tally;
    const double *w;
    double G, L;              /* pass A accumulators (path order); in pass B of
                                 a weighted run G is the running score F      */
    double A;                 /* pass A, weighted runs: sum of |w[bin] * len|  */
    uint64_t nfl;
    int64_t hq;               /* this history's q sum                           */
    orc_counts *cnt;
    uint64_t qsum_total;      /* running exact sum of q                         */
    int overflow;
    /* time split of the current flight (n_tbins > 0): flight start time, speed,
       bin width, current bin, bins without time */
    double t0, v, tw;
    int32_t tk;
    int64_t nbase;
    double wt;                /* the particle's weight (1 in analog runs)      */
} orc_acc;

static void orc_score_bin(const orc_problem *p, orc_acc *acc, int64_t bin, double len)
{
    if (acc->mode == 1) {
        acc->G = acc->G + (acc->w[bin] * len);
        if (p->implicit_capture) acc->A = acc->A + fabs(acc->w[bin] * len);
        return;
    }
    if (acc->mode == 2) {
        /* weighted pass B: the score of the pieces flown so far */
        acc->G = acc->G + (acc->w[bin] * len);
        return;
    }
    if (acc->mode == 3) {
        acc->dtally[bin] += len;
        return;
    }
    if (acc->mode != 0) return;
    int64_t q = orc_fixed(len, p->tally_scale_log2);
    if (q == 0) return;
    acc->tally[bin] += q;
    acc->hq += q;
    acc->cnt->pieces += 1;
    uint64_t before = acc->qsum_total;
    acc->qsum_total = before + (uint64_t)q;
    if (acc->qsum_total < before || acc->qsum_total >= 0x8000000000000000ull) acc->overflow = 1;
}

/* Largest k in [0, n-1] with k dt <= t: a first guess from t / dt, then
   corrected against the edges k dt (the edges are exactly these products). */
static int32_t orc_time_bin(double t, double dt, int32_t n)
{
    double g = t / dt;
    int32_t k = 0;
    if (g > 0.0) k = (g < (double)n) ? (int32_t)g : n - 1;
    while (k + 1 < n && ((double)(k + 1) * dt) <= t) k = k + 1;
    while (k > 0 && ((double)k * dt) > t) k = k - 1;
    return k;
}

/* Score the piece [a, b] of the current flight (lengths from its start) into
   bin `bin` of the time-free tally.  With time bins the piece is cut where
   the particle's time t0 + s / v crosses a bin edge: the edge after bin k
   lies at length ((k+1) dt - t0) v; the last bin takes the rest. */
static void orc_score_piece(const orc_problem *p, orc_acc *acc, int64_t bin, double a, double b)
{
    if (p->n_tbins <= 0) {
        orc_score_bin(p, acc, bin, (b - a) * acc->wt);
        return;
    }
    for (;;) {
        int32_t k = acc->tk;
        if (k + 1 >= p->n_tbins) {
            orc_score_bin(p, acc, (int64_t)k * acc->nbase + bin, (b - a) * acc->wt);
            return;
        }
        double se = (((double)(k + 1) * acc->tw) - acc->t0) * acc->v;
        if (se >= b) {
            orc_score_bin(p, acc, (int64_t)k * acc->nbase + bin, (b - a) * acc->wt);
            return;
        }
        orc_score_bin(p, acc, (int64_t)k * acc->nbase + bin, (se - a) * acc->wt);
        a = se;
        acc->tk = k + 1;
    }
}

/* Track-length mesh tally over one flight from pos (direction dir, length d):
   walk the mesh cells the segment crosses, each crossing parameter measured
   from the flight start, ties broken x, y, z; score each piece's length. */
static void orc_tally_mesh(const orc_problem *p, orc_acc *acc, const double pos[3],
                           const double dir[3], double d, int32_t g)
{
    const double *edge[3] = { p->mesh_x, p->mesh_y, p->mesh_z };
    int32_t n[3] = { p->mesh_n[0], p->mesh_n[1], p->mesh_n[2] };
    int32_t idx[3];
    double t[3];
    for (int a = 0; a < 3; ++a) {
        idx[a] = orc_cell_index_fast(edge[a], n[a], pos[a], dir[a]);
        double ta = INFINITY;
        if (dir[a] > 0.0) ta = (edge[a][idx[a] + 1] - pos[a]) / dir[a];
        else if (dir[a] < 0.0) ta = (edge[a][idx[a]] - pos[a]) / dir[a];
        if (ta < 0.0) ta = 0.0;
        t[a] = ta;
    }
    double t0 = 0.0;
    for (;;) {
        int a = 0;
        double tm = t[0];
        if (t[1] < tm) { tm = t[1]; a = 1; }
        if (t[2] < tm) { tm = t[2]; a = 2; }
        double t1 = (tm < d) ? tm : d;
        int64_t bin = (((int64_t)g * n[2] + idx[2]) * n[1] + idx[1]) * n[0] + idx[0];
        orc_score_piece(p, acc, bin, t0, t1);
        if (tm >= d) break;
        idx[a] = idx[a] + ((dir[a] > 0.0) ? 1 : -1);
        if (idx[a] < 0 || idx[a] >= n[a]) break;
        double ta = (edge[a][idx[a] + ((dir[a] > 0.0) ? 1 : 0)] - pos[a]) / dir[a];
        if (ta < 0.0) ta = 0.0;
        t[a] = ta;
        t0 = t1;
    }
}

/* energy-bin tally: the whole flight into the bin holding E */
static void orc_tally_energy(const orc_problem *p, orc_acc *acc, double e, double d)
{
    int32_t k = orc_cell_index_fast(p->e_edges, p->n_ebins, e, 1.0);
    orc_score_piece(p, acc, k, 0.0, d);
}

/* ------------------------------------------------------ elastic kinematics */

/* Elastic scattering off a target of mass ratio A at rest: isotropic in the
   centre-of-mass frame, mu_c = 2 xi - 1; outgoing energy
   E' = E (A^2 + 2 A mu_c + 1)/(A + 1)^2; lab-frame cosine
   mu_L = (1 + A mu_c)/sqrt(A^2 + 2 A mu_c + 1); the direction is rotated by
   mu_L about the old one at azimuth 2 pi xi_phi (no renormalisation).
   Returns E' and overwrites dir. */
double orc_elastic(double A, double e, double xi_mu, double xi_phi, double dir[3])
{
    double muc = (2.0 * xi_mu) - 1.0;
    double D = ((A * A) + ((2.0 * A) * muc)) + 1.0;
    double enew = (e * D) / ((A + 1.0) * (A + 1.0));
    double mul = (1.0 + (A * muc)) / orc_sqrt(D);
    double cp, sphi;
    orc_cos_sin_turn(xi_phi, &cp, &sphi);
    double aa = orc_sqrt((1.0 - mul) * (1.0 + mul));
    double u = dir[0], v = dir[1], w = dir[2];
    double bb = orc_sqrt((1.0 - w) * (1.0 + w));
    if (bb > 1e-10) {
        dir[0] = (mul * u) + ((aa * (((u * w) * cp) - (v * sphi))) / bb);
        dir[1] = (mul * v) + ((aa * (((v * w) * cp) + (u * sphi))) / bb);
        dir[2] = (mul * w) - ((aa * bb) * cp);
    } else {
        dir[0] = aa * cp;
        dir[1] = aa * sphi;
        dir[2] = (w >= 0.0) ? mul : -mul;
    }
    return enew;
}

/* ------------------------------------------------------------------ history */

typedef struct {
    const double *G;          /* pass B: per-history G_h, indexed h - h0        */
    uint64_t h0;
    double scale;             /* pass B: 2^s                                    */
    int64_t *SL, *SA, *SS;
} orc_grad;

static int64_t orc_qs(double x, double scale) { return (int64_t)nearbyint(x * scale); }

static void orc_isotropic(double xi_mu, double xi_phi, double dir[3])
{
    double mu = (2.0 * xi_mu) - 1.0;
    double c, s;
    orc_cos_sin_turn(xi_phi, &c, &s);
    double st = orc_sqrt((1.0 - mu) * (1.0 + mu));
    dir[0] = st * c;
    dir[1] = st * s;
    dir[2] = mu;
}

/* State of one k-eigenvalue cycle (NULL in fixed-source runs). */
typedef struct {
    uint32_t stream;          /* random-number stream: the cycle number      */
    const double *bank;       /* source positions, 3 per history (NULL: the
                                 problem's own source)                       */
    uint32_t *fn;             /* out: neutrons banked by each history        */
    double *fpos;             /* out: its fission site, 3 per history        */
} orc_cycle;

/* a generation of a weight-window run: where its histories start and where
   the copies they split off go */
typedef struct {
    int32_t gen;
    const orc_site *src;      /* NULL in generation 0                          */
    orc_site *bank;
    uint64_t cap, n;
    int full;
} orc_gen;

/* cell of a point on the uniform weight-window grid */
static int64_t orc_ww_cell(const orc_problem *p, const double pos[3])
{
    int64_t c = 0;
    for (int a = 2; a >= 0; --a) {
        int32_t n = p->ww_n[a];
        double tt = (pos[a] - p->box_lo[a]) * ((double)n / (p->box_hi[a] - p->box_lo[a]));
        int32_t i = 0;
        if (tt > 0.0) i = (tt < (double)n) ? (int32_t)tt : n - 1;
        c = c * n + i;
    }
    return c;
}

/* the weight-window closeout; returns 1 if the history ends (roulette) */
static int orc_ww_closeout(const orc_problem *p, orc_acc *acc, orc_gen *gn, double xi5, const double pos[3],
                           const double dir[3], double e, double t, int32_t g, const int32_t cell[3])
{
    double lo = p->ww_lo[orc_ww_cell(p, pos)];
    if (!(lo > 0.0)) return 0;
    double surv = p->ww_surv * lo;
    double w = acc->wt;
    if (w > p->ww_ratio * lo) {
        double q = w / surv;
        int32_t n = (q < (double)p->ww_max_split) ? (int32_t)q : p->ww_max_split;
        if (n < 2) n = 2;
        double wn = w / (double)n;
        acc->wt = wn;
        for (int32_t k = 1; k < n; ++k) {
            if (!gn || gn->n >= gn->cap) {
                if (gn) gn->full = 1;
                continue;
            }
            orc_site *st = &gn->bank[gn->n++];
            for (int a = 0; a < 3; ++a) {
                st->pos[a] = pos[a];
                st->dir[a] = dir[a];
                st->cell[a] = cell[a];
            }
            st->e = e;
            st->w = wn;
            st->t = t;
            st->g = g;
            acc->cnt->splits += 1;
        }
        return 0;
    }
    if (w < lo) {
        if ((xi5 * surv) < w) {
            acc->wt = surv;
            return 0;
        }
        return 1;
    }
    return 0;
}

static void orc_history(const orc_problem *p, uint32_t h, orc_acc *acc, orc_grad *gr,
                        orc_digest *dig, const orc_cycle *cy, orc_gen *gn)
{
    orc_counts *cnt = acc->cnt;
    uint64_t seed = p->seed;
    uint32_t pid = p->problem_id;
    uint32_t stream = gn ? (uint32_t)gn->gen : (cy ? cy->stream : 0);
    const int ww = p->ww_n[0] > 0;
    const orc_site *from = (gn && gn->src) ? &gn->src[h] : NULL;
    double pos[3], dir[3];
    int32_t cell[3];
    int32_t g = p->src_group;
    double e = p->e_source;
    double Gh = 0.0;
    if (acc->mode == 2) Gh = gr->G[h - gr->h0];

    /* source event: flight counter 0, slots 0-2 position, 3-4 direction */
    double xi0 = orc_uniform(seed, pid, h, 0, 0, stream);
    double xi1 = orc_uniform(seed, pid, h, 0, 1, stream);
    double xi2 = orc_uniform(seed, pid, h, 0, 2, stream);
    double xi3 = orc_uniform(seed, pid, h, 0, 3, stream);
    double xi4 = orc_uniform(seed, pid, h, 0, 4, stream);
    if (cy && cy->bank) {
        /* a banked fission neutron: its site, an isotropic direction, and a
           group from the fission spectrum of the material found there */
        pos[0] = cy->bank[3 * (uint64_t)h];
        pos[1] = cy->bank[3 * (uint64_t)h + 1];
        pos[2] = cy->bank[3 * (uint64_t)h + 2];
    } else if (p->src_kind == 0) {
        pos[0] = p->src_pos[0]; pos[1] = p->src_pos[1]; pos[2] = p->src_pos[2];
    } else if (p->src_kind == 1) {
        pos[0] = p->src_lo[0] + (xi0 * (p->src_hi[0] - p->src_lo[0]));
        pos[1] = p->src_lo[1] + (xi1 * (p->src_hi[1] - p->src_lo[1]));
        pos[2] = p->src_lo[2] + (xi2 * (p->src_hi[2] - p->src_lo[2]));
    } else {
        double r = p->src_radius * orc_sqrt(xi0);
        double c, s;
        orc_cos_sin_turn(xi1, &c, &s);
        pos[0] = p->src_pos[0] + (r * c);
        pos[1] = p->src_pos[1] + (r * s);
        pos[2] = p->src_pos[2];
    }
    if (p->src_isotropic || (cy && cy->bank)) {
        orc_isotropic(xi3, xi4, dir);
    } else {
        dir[0] = p->src_dir[0]; dir[1] = p->src_dir[1]; dir[2] = p->src_dir[2];
    }
    orc_locate(p, pos, dir, cell);
    if (from) {
        /* a split copy: the state it was banked with (no source draws used) */
        for (int a = 0; a < 3; ++a) {
            pos[a] = from->pos[a];
            dir[a] = from->dir[a];
            cell[a] = from->cell[a];
        }
        g = from->g;
        e = from->e;
    }
    if (cy && cy->bank) {
        const double *row = p->chi + (int64_t)orc_material(p, cell) * p->n_grp;
        g = p->n_grp - 1;
        for (int32_t k = 0; k < p->n_grp; ++k) {
            if (xi0 < row[k]) { g = k; break; }
        }
    }
    if (cy && cy->fn) cy->fn[h] = 0;
    cnt->sourced += 1;

    uint32_t flights = 0, collisions = 0, fate = ORC_FATE_LEAK;
    double t = 0.0;                      /* particle time (time-binned tallies) */
    if (p->n_tbins > 0) {
        acc->tw = p->t_max / (double)p->n_tbins;
        acc->nbase = (p->tally_kind == 0)
                         ? (int64_t)p->mesh_n[0] * p->mesh_n[1] * p->mesh_n[2] * (p->energy_mode == 0 ? p->n_grp : 1)
                         : (int64_t)p->n_ebins;
    }
    acc->hq = 0;
    acc->wt = from ? from->w : 1.0;
    if (from) t = from->t;
    acc->G = 0.0;
    acc->L = 0.0;
    acc->A = 0.0;
    acc->nfl = 0;
    int64_t step = 1;
    for (;;) {
        if (step > p->max_steps) { fate = ORC_FATE_KILLED; cnt->killed += 1; break; }
        uint32_t st32 = (uint32_t)step;
        int32_t m = orc_material(p, cell);
        /* lookup */
        double sigma_t;
        orc_ce_xs xs;
        if (p->energy_mode == 0) {
            sigma_t = p->sigma_t[m * p->n_grp + g];
        } else {
            orc_ce_lookup(p, m, e, &xs);
            sigma_t = xs.sigma_t;
        }
        /* flight: distance to collision, nearest surface, the shorter wins
           (a collision only if strictly shorter) */
        double dcol = orc_nlog(orc_uniform(seed, pid, h, st32, 0, stream)) / sigma_t;
        int32_t surf;
        double dsurf = orc_distance(p, pos, dir, cell, &surf);
        int collide = dcol < dsurf;
        double d = collide ? dcol : dsurf;
        /* time: a flight that would reach t_max ends there (ties go to the
           time boundary); the tally pieces are split at time-bin edges.  The
           sum t + d / v of an earlier flight can round to just past t_max:
           the remaining length is then zero, never negative. */
        int timecut = 0;
        double v = 0.0;
        if (p->n_tbins > 0) {
            v = (p->energy_mode == 0) ? p->speed[g] : p->speed_coef * orc_sqrt(e);
            double dtime = (p->t_max - t) * v;
            if (!(d < dtime)) {
                d = (dtime > 0.0) ? dtime : 0.0;
                timecut = 1;
                collide = 0;
            }
            acc->t0 = t;
            acc->v = v;
            acc->tk = orc_time_bin(t, acc->tw, p->n_tbins);
        }
        /* track-length tally along the flight */
        if (acc->mode != 2 || p->implicit_capture) {
            if (p->tally_kind == 0) orc_tally_mesh(p, acc, pos, dir, d, g);
            else orc_tally_energy(p, acc, e, d);
        }
        if (acc->mode == 2) gr->SL[m * p->n_grp + g] += orc_qs(Gh * d, gr->scale);
        acc->L = acc->L + d;
        acc->nfl += 1;
        /* move */
        pos[0] = pos[0] + (d * dir[0]);
        pos[1] = pos[1] + (d * dir[1]);
        pos[2] = pos[2] + (d * dir[2]);
        flights += 1;
        cnt->flights += 1;
        if (timecut) {
            fate = ORC_FATE_CUTOFF;
            cnt->cutoffs += 1;
            break;
        }
        if (p->n_tbins > 0) t = t + (d / v);
        if (collide) {
            collisions += 1;
            cnt->collisions += 1;
            double c1 = orc_uniform(seed, pid, h, st32, 1, stream);
            double c2 = orc_uniform(seed, pid, h, st32, 2, stream);
            double c3 = orc_uniform(seed, pid, h, st32, 3, stream);
            double c4 = orc_uniform(seed, pid, h, st32, 4, stream);
            if (p->energy_mode == 0) {
                double ss = p->sigma_s[m * p->n_grp + g];
                if (p->implicit_capture) {
                    /* implicit capture: no absorption, the weight carries it.
                       Pass B: G_h for the collision density Sigma_t, and the
                       score still to come, G_h - F, for the weight factor
                       Sigma_s / Sigma_t that every later piece carries */
                    acc->wt = acc->wt * (ss / sigma_t);
                    if (acc->mode == 2) {
                        gr->SA[m * p->n_grp + g] += orc_qs(Gh, gr->scale);
                        gr->SS[m * p->n_grp + g] += orc_qs(Gh - acc->G, gr->scale);
                    }
                } else if (!((c1 * sigma_t) < ss)) {
                    fate = ORC_FATE_ABSORB;
                    cnt->absorbs += 1;
                    if (acc->mode == 2) gr->SA[m * p->n_grp + g] += orc_qs(Gh, gr->scale);
                    /* k-eigenvalue cycle: the absorption is a fission with
                       probability Sigma_f / Sigma_a and banks floor(nu + xi)
                       neutrons at the collision site */
                    if (cy && cy->fn && ((c2 * (sigma_t - ss)) < p->sigma_f[m * p->n_grp + g])) {
                        uint32_t n = (uint32_t)(p->nu[m * p->n_grp + g] + c3);
                        cy->fn[h] = n;
                        cy->fpos[3 * (uint64_t)h] = pos[0];
                        cy->fpos[3 * (uint64_t)h + 1] = pos[1];
                        cy->fpos[3 * (uint64_t)h + 2] = pos[2];
                        cnt->fissions += 1;
                        cnt->sites += n;
                    }
                    break;
                }
                cnt->scatters += 1;
                if (acc->mode == 2 && !p->implicit_capture) gr->SS[m * p->n_grp + g] += orc_qs(Gh, gr->scale);
                const double *row = p->cdf + ((int64_t)m * p->n_grp + g) * p->n_grp;
                int32_t gn = p->n_grp - 1;
                for (int32_t k = 0; k < p->n_grp; ++k) {
                    if (c2 < row[k]) { gn = k; break; }
                }
                cnt->cdf_scans += (uint64_t)gn + 1;
                g = gn;
                orc_isotropic(c3, c4, dir);
            } else {
                /* species, then absorb/scatter, then elastic kinematics in
                   the centre-of-mass frame with target mass ratio A */
                int32_t sp = p->n_species - 1;
                double target = c1 * sigma_t;
                for (int32_t s = 0; s < p->n_species; ++s) {
                    if (target < xs.cum[s]) { sp = s; break; }
                }
                double sa = xs.sa[sp], ss = xs.ss[sp];
                if (p->implicit_capture) {
                    acc->wt = acc->wt * (ss / (sa + ss));
                } else if (!((c2 * (sa + ss)) < ss)) {
                    fate = ORC_FATE_ABSORB;
                    cnt->absorbs += 1;
                    break;
                }
                cnt->scatters += 1;
                double enew = orc_elastic(p->awr[sp], e, c3, c4, dir);
                if (enew < p->e_min) {
                    fate = ORC_FATE_CUTOFF;
                    cnt->cutoffs += 1;
                    break;
                }
                e = enew;
            }
            /* closeout: weight windows, or without them the weight roulette
               below the cutoff (slot 5) */
            if (ww) {
                double c5 = orc_uniform(seed, pid, h, st32, 5, stream);
                if (orc_ww_closeout(p, acc, gn, c5, pos, dir, e, t, g, cell)) {
                    fate = ORC_FATE_ROULETTE;
                    cnt->roulettes += 1;
                    break;
                }
            } else if (p->implicit_capture && acc->wt < p->w_cutoff) {
                double c5 = orc_uniform(seed, pid, h, st32, 5, stream);
                if ((c5 * p->w_survival) < acc->wt) {
                    acc->wt = p->w_survival;
                } else {
                    fate = ORC_FATE_ROULETTE;
                    cnt->roulettes += 1;
                    break;
                }
            }
        } else {
            /* surface crossing: snap to the plane, then leak, reflect or
               enter the neighbouring cell */
            cnt->crossings += 1;
            int face = -1;          /* boundary face crossed, if any */
            if (surf == 3) {
                cell[2] = 1 - cell[2];
            } else if (surf == 0) {
                const double *pl = (p->geometry == 0) ? p->slab_planes : p->xplanes;
                int32_t n = (p->geometry == 0) ? p->n_slabs : p->nx;
                if (dir[0] > 0.0) {
                    pos[0] = pl[cell[0] + 1];
                    if (cell[0] + 1 == n) face = 1; else cell[0] += 1;
                } else {
                    pos[0] = pl[cell[0]];
                    if (cell[0] == 0) face = 0; else cell[0] -= 1;
                }
            } else if (surf == 1) {
                if (p->geometry == 0) {
                    pos[1] = (dir[1] > 0.0) ? p->box_hi[1] : p->box_lo[1];
                    face = (dir[1] > 0.0) ? 3 : 2;
                } else if (dir[1] > 0.0) {
                    pos[1] = p->yplanes[cell[1] + 1];
                    if (cell[1] + 1 == p->ny) face = 3; else cell[1] += 1;
                } else {
                    pos[1] = p->yplanes[cell[1]];
                    if (cell[1] == 0) face = 2; else cell[1] -= 1;
                }
            } else {
                pos[2] = (dir[2] > 0.0) ? p->box_hi[2] : p->box_lo[2];
                face = (dir[2] > 0.0) ? 5 : 4;
            }
            if (face >= 0) {
                if (p->bc[face] == 0) {
                    fate = ORC_FATE_LEAK;
                    cnt->leaks += 1;
                    break;
                }
                cnt->reflections += 1;
                dir[face >> 1] = -dir[face >> 1];
            }
            /* closeout of the crossing: weight windows (slot 5) */
            if (ww) {
                double c5 = orc_uniform(seed, pid, h, st32, 5, stream);
                if (orc_ww_closeout(p, acc, gn, c5, pos, dir, e, t, g, cell)) {
                    fate = ORC_FATE_ROULETTE;
                    cnt->roulettes += 1;
                    break;
                }
            }
        }
        step = step + 1;
    }
    if (dig) {
        dig->qsum = acc->hq;
        dig->flights = flights;
        dig->collisions = collisions;
        dig->fate = fate;
        dig->pad = 0;
    }
}

int orc_run(const orc_problem *p, uint64_t h0, uint64_t h1, int64_t *tally,
            orc_digest *digest, orc_counts *counts)
{
    if (p->ww_n[0] > 0) return 4;        /* weight windows: generations (orc_run_gen) */
    orc_counts local;
    memset(&local, 0, sizeof local);
    orc_acc acc;
    memset(&acc, 0, sizeof acc);
    acc.mode = 0;
    acc.tally = tally;
    acc.cnt = &local;
    for (uint64_t h = h0; h < h1; ++h)
        orc_history(p, (uint32_t)h, &acc, NULL, digest ? &digest[h - h0] : NULL, NULL, NULL);
    local.qsum = acc.qsum_total;
    local.overflow = (uint64_t)acc.overflow;
    if (counts) *counts = local;
    return acc.overflow ? 1 : 0;
}

int orc_run_gen(const orc_problem *p, int32_t gen, const orc_site *src, uint64_t h0, uint64_t h1, int64_t *tally,
                orc_digest *digest, orc_counts *counts, orc_site *bank, uint64_t bank_cap, uint64_t *bank_n)
{
    orc_counts local;
    memset(&local, 0, sizeof local);
    orc_acc acc;
    memset(&acc, 0, sizeof acc);
    acc.mode = 0;
    acc.tally = tally;
    acc.cnt = &local;
    orc_gen gn = {gen, gen > 0 ? src : NULL, bank, bank_cap, 0, 0};
    for (uint64_t h = h0; h < h1; ++h)
        orc_history(p, (uint32_t)h, &acc, NULL, digest ? &digest[h - h0] : NULL, NULL, &gn);
    local.qsum = acc.qsum_total;
    local.overflow = (uint64_t)acc.overflow;
    if (counts) *counts = local;
    *bank_n = gn.n;
    if (gn.full) return 3;
    return acc.overflow ? 1 : 0;
}

int orc_replay_a(const orc_problem *p, uint64_t h0, uint64_t h1, const double *w,
                 double *G, uint64_t *U)
{
    orc_counts local;
    memset(&local, 0, sizeof local);
    orc_acc acc;
    memset(&acc, 0, sizeof acc);
    acc.mode = 1;
    acc.w = w;
    acc.cnt = &local;
    uint64_t u = 0;
    int bad = 0;
    for (uint64_t h = h0; h < h1; ++h) {
        orc_history(p, (uint32_t)h, &acc, NULL, NULL, NULL, NULL);
        G[h - h0] = acc.G;
        /* every pass B sum of the history is at most this in magnitude (the
           score still to come at a collision is at most A_h) */
        double bound = p->implicit_capture ? ceil((fabs(acc.G) + acc.A) * (acc.L + (double)acc.nfl))
                                           : ceil(fabs(acc.G) * (acc.L + (double)acc.nfl));
        if (!(bound < 0x1p63)) { bad = 1; continue; }
        uint64_t before = u;
        u = u + (uint64_t)bound;
        if (u < before) bad = 1;
    }
    *U = u;
    return bad;
}

int orc_replay_b(const orc_problem *p, uint64_t h0, uint64_t h1, const double *w, const double *G, int32_t s,
                 int64_t *SL, int64_t *SA, int64_t *SS)
{
    orc_counts local;
    memset(&local, 0, sizeof local);
    orc_acc acc;
    memset(&acc, 0, sizeof acc);
    acc.mode = 2;
    acc.w = w;
    acc.cnt = &local;
    if (p->implicit_capture && !w) return 2;
    orc_grad gr;
    gr.G = G;
    gr.h0 = h0;
    gr.scale = ldexp(1.0, s);
    gr.SL = SL; gr.SA = SA; gr.SS = SS;
    for (uint64_t h = h0; h < h1; ++h) orc_history(p, (uint32_t)h, &acc, &gr, NULL, NULL, NULL);
    return 0;
}

/* ------------------------------------------------------------ k-eigenvalue */

int orc_eigen(const orc_problem *p, uint64_t N, int32_t n_cycles, int32_t n_inactive, int64_t *tally,
              double *k_cycle, uint64_t *n_source, orc_counts *counts, double *bank, uint64_t bank_cap,
              uint64_t *bank_n)
{
    int64_t nbins = (p->tally_kind == 0)
                        ? (int64_t)p->mesh_n[0] * p->mesh_n[1] * p->mesh_n[2] * (p->energy_mode == 0 ? p->n_grp : 1)
                        : (int64_t)p->n_ebins;
    if (p->n_tbins > 0) nbins *= p->n_tbins;
    int64_t *scratch = calloc((size_t)nbins, sizeof(int64_t));   /* inactive cycles score here */
    orc_counts total;
    memset(&total, 0, sizeof total);
    double *src = NULL;          /* source of the current cycle (NULL: cycle 0) */
    uint64_t Nc = N;
    int status = 0;
    for (int32_t c = 0; c < n_cycles && status == 0; ++c) {
        uint32_t *fn = malloc((size_t)(Nc ? Nc : 1) * sizeof(uint32_t));
        double *fpos = malloc((size_t)(Nc ? Nc : 1) * 3 * sizeof(double));
        orc_cycle cy = { (uint32_t)c, src, fn, fpos };
        orc_counts local;
        memset(&local, 0, sizeof local);
        orc_acc acc;
        memset(&acc, 0, sizeof acc);
        acc.mode = 0;
        acc.tally = (c >= n_inactive) ? tally : scratch;
        acc.cnt = &local;
        for (uint64_t h = 0; h < Nc; ++h) orc_history(p, (uint32_t)h, &acc, NULL, NULL, &cy, NULL);
        /* totals over cycles; the overflow rule applies to the sum over all of them */
        uint64_t q_before = total.qsum;
        total.sourced += local.sourced; total.flights += local.flights;
        total.collisions += local.collisions; total.scatters += local.scatters;
        total.absorbs += local.absorbs; total.crossings += local.crossings; total.leaks += local.leaks;
        total.reflections += local.reflections; total.cutoffs += local.cutoffs; total.killed += local.killed;
        total.pieces += local.pieces; total.fissions += local.fissions; total.sites += local.sites;
        total.roulettes += local.roulettes; total.cdf_scans += local.cdf_scans; total.splits += local.splits;
        total.qsum = q_before + acc.qsum_total;
        if (acc.overflow || total.qsum < q_before || total.qsum >= 0x8000000000000000ull) total.overflow = 1;
        /* the bank: each history's neutrons in history order */
        uint64_t M = 0;
        for (uint64_t h = 0; h < Nc; ++h) M += fn[h];
        n_source[c] = Nc;
        k_cycle[c] = (double)M / (double)Nc;
        if (M == 0) {
            status = 2;
        } else {
            double *sites = malloc((size_t)M * 3 * sizeof(double));
            uint64_t s = 0;
            for (uint64_t h = 0; h < Nc; ++h)
                for (uint32_t j = 0; j < fn[h]; ++j, ++s) {
                    sites[3 * s] = fpos[3 * h];
                    sites[3 * s + 1] = fpos[3 * h + 1];
                    sites[3 * s + 2] = fpos[3 * h + 2];
                }
            /* splitting-roulette back to about N particles */
            double r = (double)N / (double)M;
            double fl = floor(r);
            double fr = r - fl;
            uint64_t Nn = 0;
            for (uint64_t j = 0; j < M; ++j) {
                double u = orc_uniform(p->seed, p->problem_id, (uint32_t)j, 0xFFFFFFFFu, 0, (uint32_t)c);
                Nn += (uint64_t)fl + ((u < fr) ? 1u : 0u);
            }
            double *next = malloc((size_t)(Nn ? Nn : 1) * 3 * sizeof(double));
            uint64_t o = 0;
            for (uint64_t j = 0; j < M; ++j) {
                double u = orc_uniform(p->seed, p->problem_id, (uint32_t)j, 0xFFFFFFFFu, 0, (uint32_t)c);
                uint64_t copies = (uint64_t)fl + ((u < fr) ? 1u : 0u);
                for (uint64_t i = 0; i < copies; ++i, ++o) {
                    next[3 * o] = sites[3 * j];
                    next[3 * o + 1] = sites[3 * j + 1];
                    next[3 * o + 2] = sites[3 * j + 2];
                }
            }
            free(sites);
            free(src);
            src = next;
            Nc = Nn;
            if (Nc == 0) status = 2;
        }
        free(fn);
        free(fpos);
    }
    if (bank_n) *bank_n = Nc;
    if (bank && src) {
        if (Nc > bank_cap) status = status ? status : 3;
        else memcpy(bank, src, (size_t)Nc * 3 * sizeof(double));
    }
    free(src);
    free(scratch);
    if (counts) *counts = total;
    if (status == 0 && total.overflow) status = 1;
    return status;
}

/* ------------------------------------------------------------- test hooks */

void orc_tally_segment(const orc_problem *p, const double pos[3], const double dir[3], double d,
                       int32_t g, double *out)
{
    orc_counts local;
    memset(&local, 0, sizeof local);
    orc_acc acc;
    memset(&acc, 0, sizeof acc);
    acc.mode = 3;
    acc.wt = 1.0;
    acc.dtally = out;
    acc.cnt = &local;
    orc_problem q = *p;           /* the mesh walk alone, without time bins */
    q.n_tbins = 0;
    orc_tally_mesh(&q, &acc, pos, dir, d, g);
}

double orc_ce_xs_hook(const orc_problem *p, int32_t m, double e, double *sa, double *ss)
{
    orc_ce_xs xs;
    orc_ce_lookup(p, m, e, &xs);
    for (int32_t s = 0; s < p->n_species; ++s) { sa[s] = xs.sa[s]; ss[s] = xs.ss[s]; }
    return xs.sigma_t;
}
