// Event programs of Monte Carlo particle transport: analog fixed-source
// histories, with optional time bins, non-analog weights (implicit capture
// with a roulette closeout) and k-eigenvalue fission banking.
//
// A history is: a source event (position, direction, group or energy from
// the history's own random numbers), then flights.  One flight samples a
// distance to collision, finds the nearest surface, moves the particle to
// whichever is closer (a collision only if strictly closer) while scoring
// the track length into the tally, and then either collides (absorb or
// scatter) or crosses the surface (leak, reflect or enter the next cell).
//
// The paper (Sec. 4) runs this loop either as one monolithic "step" event
// per flight or decomposed into separate events at the points where lanes
// diverge.  Both forms are here: ev_step (fused) and ev_move (the step),
// ev_surface, ev_collide, ev_closeout (split).  Random numbers are keyed by (history,
// flight, slot), never by event, so the two forms and every scheduler give
// identical bits.
//
// Random-number slots per flight k >= 1: 0 distance; 1 absorb/scatter (MG)
// or species (CE); 2 outgoing group (MG) or absorb/scatter (CE); 3 polar
// cosine (MG) or centre-of-mass cosine (CE); 4 azimuth; 5 weight roulette.
// At an absorption (k-eigenvalue cycles) 2 decides fission and 3 rounds nu.
// Source (k = 0): 0-2 position, 3 polar cosine, 4 azimuth; a banked fission
// neutron uses 0 for its group.  The fourth counter word is the k-eigenvalue
// cycle (0 otherwise).
//
// The extended kernels (template flag EXT) carry each particle's time and
// weight; the others carry neither and score plain track lengths.
#pragma once
#include "problem.hpp"
#include "rng_math.hpp"

#pragma clang fp contract(off)

namespace mcx {

// A pointer to global memory with its address space stated: buffers named by
// the problem record (packed tables, source bank, fission records, digests)
// would otherwise be accessed with flat instructions, which on gfx9 count on
// the LDS counter as well and so hold up later LDS reads.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gmem(T *p)
{
    return (__attribute__((address_space(1))) T *)p;
}

// the same pointer as a plain one, for code that takes plain pointers: after
// inlining the compiler still sees that it points to global memory
template <class T>
__device__ __forceinline__ T *gptr(T *p)
{
    return (T *)gmem(p);
}

enum : int { EV_STEP = 0, EV_SURFACE = 1, EV_COLLIDE = 2, EV_CLOSEOUT = 3, EV_DEAD = 7 };
enum : uint32_t {
    O_SOURCE = 1u << 0, O_FLIGHT = 1u << 1, O_COLL = 1u << 2, O_SCAT = 1u << 3, O_ABS = 1u << 4,
    O_CROSS = 1u << 5, O_LEAK = 1u << 6, O_REFL = 1u << 7, O_CUT = 1u << 8, O_KILL = 1u << 9,
    O_FISS = 1u << 10, O_ROUL = 1u << 11
};
enum : uint32_t { FATE_LEAK = 0, FATE_ABSORB = 1, FATE_CUTOFF = 2, FATE_KILLED = 3, FATE_ROULETTE = 4 };

struct Digest {   // same layout as mcx_digest
    long long qsum;
    uint32_t flights, collisions, fate, pad;
};

// A particle in registers while an event runs.
struct Part {
    double x, y, z, u, v, w;
    double e;         // energy (continuous energy)
    double sigt;      // total cross section of the current flight (split events)
    double G, L, A;   // backward: pass A score, track length and (weighted
                      // runs) absolute score; pass B G_h and (weighted runs)
                      // the running score in L
    double t;         // particle time (time-binned tallies)
    double wgt;       // statistical weight (non-analog runs; 1 otherwise)
    long long hq;     // this history's tally sum (digest)
    uint32_t hid;     // history index within its problem
    uint32_t step;    // flight counter (0 = source)
    uint32_t gc;      // packed group | cell | inside | surface
    uint32_t prob;    // problem index in the batch
    uint32_t ncoll;   // collisions so far (digest)
    uint32_t nsplit;  // copies split off so far (weight windows)
};

// gc: bits 0-7 group, 8-17 cell x / slab, 18-27 cell y, 28 inside pin,
// 29-30 surface to cross (split events)
__device__ __forceinline__ int gc_group(uint32_t gc) { return (int)(gc & 0xffu); }
__device__ __forceinline__ int gc_c0(uint32_t gc) { return (int)((gc >> 8) & 0x3ffu); }
__device__ __forceinline__ int gc_c1(uint32_t gc) { return (int)((gc >> 18) & 0x3ffu); }
__device__ __forceinline__ int gc_in(uint32_t gc) { return (int)((gc >> 28) & 1u); }
__device__ __forceinline__ int gc_surf(uint32_t gc) { return (int)((gc >> 29) & 3u); }
__device__ __forceinline__ uint32_t gc_pack(int g, int c0, int c1, int in, int surf)
{
    return (uint32_t)g | ((uint32_t)c0 << 8) | ((uint32_t)c1 << 18) | ((uint32_t)in << 28) | ((uint32_t)surf << 29);
}

// Per-lane accumulators of a run.
struct Lane {
    unsigned long long q;    // exact sum of contributions
    unsigned long long u;    // pass A bound (single-problem runs)
    uint32_t pieces;
    uint32_t err;
    uint32_t rep;            // this wavefront's tally replica (wavefront id mod TREP)
    uint32_t cdf;            // transfer-CDF entries read by multigroup scatters
    uint32_t splits;         // copies split off by weight windows
};

// Everything an event needs besides the particle.
struct EvCtx {
    const ProbDev *probs;
    Digest *digest;                  // optional per-history records
    unsigned long long *lacc;        // pass B per-block sums (LDS) or null
    int single;                      // one problem in the run
    unsigned long long *ltally;      // energy-bin tally per-block sums (LDS) or null
};

// The small tables an event reads.  TabsG reads them from the problem's
// arrays in global memory (batched launches, where the problem differs per
// lane); TabsL holds pointers into this block's LDS copy (single-problem
// launches).  LDS reads are waited for on their own counter, so they never
// wait behind the wavefront's outstanding tally atomics, which go to memory.
struct TabsG {
    const ProbDev &P;
    __device__ __forceinline__ const double *sig_t() const { return gptr(P.sig_t); }
    __device__ __forceinline__ const double *sig_s() const { return gptr(P.sig_s); }
    __device__ __forceinline__ const double *cdf() const { return gptr(P.cdf); }
    __device__ __forceinline__ const double *xpl() const { return gptr(P.xpl); }
    __device__ __forceinline__ const double *ypl() const { return gptr(P.ypl); }
    __device__ __forceinline__ const double *cxs() const { return gptr(P.cxs); }
    __device__ __forceinline__ const double *cys() const { return gptr(P.cys); }
    __device__ __forceinline__ const double *mx() const { return gptr(P.mx); }
    __device__ __forceinline__ const double *my() const { return gptr(P.my); }
    __device__ __forceinline__ const double *mz() const { return gptr(P.mz); }
    __device__ __forceinline__ const double *speed() const { return gptr(P.speed); }
    __device__ __forceinline__ const double *sigf() const { return gptr(P.sigf); }
    __device__ __forceinline__ const double *nu() const { return gptr(P.nu); }
    __device__ __forceinline__ const double *chi() const { return gptr(P.chi); }
    __device__ __forceinline__ const int32_t *cmat() const { return gptr(P.cmat); }
};

struct TabsL {
    const double *d;                 // LDS copy of the packed tables
    const ProbDev &P;
    __device__ __forceinline__ const double *sig_t() const { return d + P.tl_off[TL_SIG_T]; }
    __device__ __forceinline__ const double *sig_s() const { return d + P.tl_off[TL_SIG_S]; }
    __device__ __forceinline__ const double *cdf() const { return d + P.tl_off[TL_CDF]; }
    __device__ __forceinline__ const double *xpl() const { return d + P.tl_off[TL_XPL]; }
    __device__ __forceinline__ const double *ypl() const { return d + P.tl_off[TL_YPL]; }
    __device__ __forceinline__ const double *cxs() const { return d + P.tl_off[TL_CXS]; }
    __device__ __forceinline__ const double *cys() const { return d + P.tl_off[TL_CYS]; }
    __device__ __forceinline__ const double *mx() const { return d + P.tl_off[TL_MX]; }
    __device__ __forceinline__ const double *my() const { return d + P.tl_off[TL_MY]; }
    __device__ __forceinline__ const double *mz() const { return d + P.tl_off[TL_MZ]; }
    __device__ __forceinline__ const double *speed() const { return d + P.tl_off[TL_SPEED]; }
    __device__ __forceinline__ const double *sigf() const { return d + P.tl_off[TL_SIGF]; }
    __device__ __forceinline__ const double *nu() const { return d + P.tl_off[TL_NU]; }
    __device__ __forceinline__ const double *chi() const { return d + P.tl_off[TL_CHI]; }
    __device__ __forceinline__ const int32_t *cmat() const { return (const int32_t *)d + P.tl_off[TL_CMAT]; }
};

// Copy problem P's packed tables into LDS at dst (every thread of the block
// takes part; ends with a block barrier).
__device__ __forceinline__ void tabs_to_lds(const ProbDev &P, char *dst)
{
    const auto *src = gmem((const unsigned long long *)P.tl_src);
    unsigned long long *d = (unsigned long long *)dst;
    const int n = P.tl_bytes >> 3;
    for (int i = (int)threadIdx.x; i < n; i += (int)blockDim.x) d[i] = src[i];
    __syncthreads();
}

// Table accessor of a launch: per-lane problem tables in batched launches,
// the block's LDS copy otherwise.
template <bool BATCH>
__device__ __forceinline__ auto tabs_for(const ProbDev &P, const char *lds)
{
    if constexpr (BATCH) return TabsG{P};
    else return TabsL{(const double *)lds, P};
}

// LDS bytes in front of the table copy (16-byte aligned)
__host__ __device__ __forceinline__ size_t tabs_lds_offset(size_t before) { return (before + 15) / 16 * 16; }

__device__ __forceinline__ double inf() { return __builtin_huge_val(); }

// largest i in [0, n-1] with e[i] <= x; a point on edge i moving in the
// negative direction belongs to cell i-1
__device__ __forceinline__ int edge_index(const double *__restrict__ e, int n, double x, double dir)
{
    int i = 0;
    if (e[0] <= x) {
        int lo = 0, hi = n;
        while (lo < hi) {
            int mid = lo + ((hi - lo + 1) >> 1);
            if (e[mid] <= x) lo = mid;
            else hi = mid - 1;
        }
        i = lo;
    }
    if (i > n - 1) i = n - 1;
    if (x == e[i] && dir < 0.0 && i > 0) i = i - 1;
    return i;
}

// The same index from a guess g (any value in [0, n-1]): walk up while the
// next edge is <= x, down while this edge is > x; the result is the largest
// i in [0, n-1] with e[i] <= x (0 if none), whatever the guess.
__device__ __forceinline__ int edge_index_from(const double *__restrict__ e, int n, double x, double dir, int g)
{
    int i = g < 0 ? 0 : (g > n - 1 ? n - 1 : g);
    while (i < n - 1 && e[i + 1] <= x) i = i + 1;
    while (i > 0 && e[i] > x) i = i - 1;
    if (x == e[i] && dir < 0.0 && i > 0) i = i - 1;
    return i;
}

// cell index on an axis whose edges are (nearly) uniform: one multiply for
// the guess, usually no correction step
__device__ __forceinline__ int edge_index_guess(const double *__restrict__ e, int n, double x, double dir, double lo,
                                                double inv)
{
    if (inv == 0.0) return edge_index(e, n, x, dir);
    double t = (x - lo) * inv;
    int g = 0;
    if (t > 0.0) g = (t < (double)n) ? (int)t : n - 1;
    return edge_index_from(e, n, x, dir, g);
}

// (one division whatever the sign of u: lanes moving either way share it)
__device__ __forceinline__ double plane_dist(double lo, double hi, double x, double u)
{
    const double q = ((u > 0.0) ? (hi - x) : (lo - x)) / u;
    double d = (u > 0.0 || u < 0.0) ? q : inf();
    if (d < 0.0) d = 0.0;
    return d;
}

template <int GEOM, class TB>
__device__ __forceinline__ int material(const ProbDev &P, const TB &T, uint32_t gc)
{
    if (GEOM == GEOM_BOX) return T.cmat()[gc_c0(gc)];
    // read the pin's material unconditionally (the index is always valid) and
    // select afterwards: a load through a pointer chosen between LDS and the
    // problem record would have to be a flat load
    int pin = T.cmat()[gc_c1(gc) * P.nx + gc_c0(gc)];
    return gc_in(gc) ? pin : P.mod_mat;
}

template <int GEOM, class TB>
__device__ __forceinline__ uint32_t locate(const ProbDev &P, const TB &T, double x, double y, double u, double v, int g)
{
    if (GEOM == GEOM_BOX) return gc_pack(g, edge_index(T.xpl(), P.n_slabs, x, u), 0, 0, 0);
    int i = edge_index(T.xpl(), P.nx, x, u);
    int j = edge_index(T.ypl(), P.ny, y, v);
    double ddx = x - T.cxs()[i], ddy = y - T.cys()[j];
    int in = (((ddx * ddx) + (ddy * ddy)) < P.r2) ? 1 : 0;
    return gc_pack(g, i, j, in, 0);
}

// Distance to the nearest bounding surface of the particle's cell; surf:
// 0 x-plane, 1 y-plane, 2 z-plane, 3 cylinder; ties go to the lower number.
template <int GEOM, class TB>
__device__ __forceinline__ double surface_distance(const ProbDev &P, const TB &T, const Part &p, int &surf)
{
    double dx = inf(), dy = inf(), dz, dc = inf();
    int c0 = gc_c0(p.gc);
    if (GEOM == GEOM_BOX) {
        dx = plane_dist(T.xpl()[c0], T.xpl()[c0 + 1], p.x, p.u);
        dy = plane_dist(P.box_lo[1], P.box_hi[1], p.y, p.v);
        dz = plane_dist(P.box_lo[2], P.box_hi[2], p.z, p.w);
    } else {
        int c1 = gc_c1(p.gc);
        dz = plane_dist(P.box_lo[2], P.box_hi[2], p.z, p.w);
        double ddx = p.x - T.cxs()[c0], ddy = p.y - T.cys()[c1];
        double a = (p.u * p.u) + (p.v * p.v);
        double k = (ddx * p.u) + (ddy * p.v);
        double c = ((ddx * ddx) + (ddy * ddy)) - P.r2;
        double disc = (k * k) - (a * c);
        // inside the pin the cylinder is left at (sqrt(disc) - k) / a; outside
        // it is met (if at all) at c / (sqrt(disc) - k) and the cell planes
        // bound the flight too.  Both sides are evaluated with the same root
        // and one division, operands chosen per lane, so a wavefront with
        // lanes on both sides runs each once
        const bool in = gc_in(p.gc) != 0;
        const double px = plane_dist(T.xpl()[c0], T.xpl()[c0 + 1], p.x, p.u);
        const double py = plane_dist(T.ypl()[c1], T.ypl()[c1 + 1], p.y, p.v);
        dx = in ? inf() : px;
        dy = in ? inf() : py;
        const double r = root((disc < 0.0) ? 0.0 : disc);
        const bool hit = in ? (a > 0.0) : (a > 0.0 && k < 0.0 && disc >= 0.0);
        const double q = (in ? (r - k) : c) / (in ? a : (r - k));
        dc = hit ? q : inf();
        if (dc < 0.0) dc = 0.0;
    }
    int s = 0;
    double d = dx;
    if (dy < d) { d = dy; s = 1; }
    if (dz < d) { d = dz; s = 2; }
    if (dc < d) { d = dc; s = 3; }
    surf = s;
    return d;
}

// ------------------------------------------------------ continuous energy

struct CEXS {
    double sa[MAX_SPECIES], ss[MAX_SPECIES], cum[MAX_SPECIES];
};

// largest i <= n-2 with g[i] <= e (e within [g[0], g[n-1]]), starting from a
// bracket lo <= answer that ends with g[hi] > e or hi = n-1
__device__ __forceinline__ int bisect(const double *__restrict__ g, int lo, int hi, double e)
{
    while (hi - lo > 1) {
        int mid = lo + ((hi - lo) >> 1);
        if (g[mid] <= e) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int ce_bracket(const ProbDev &P, int s, const double *__restrict__ g, double e, double lnE)
{
    int n = P.grid_len;
    int lo = 0, hi = n - 1;
    if (P.lookup_hash) {
        // hashed grid: uniform bins in ln E give a starting bracket that is
        // widened until it provably contains the answer
        double t = (lnE - P.hash_ln_lo) * P.hash_inv;
        int b = 0;
        if (t > 0.0) b = (t < (double)P.hash_bins) ? (int)t : P.hash_bins - 1;
        lo = gptr(P.hash_lo)[s * P.hash_bins + b];
        hi = gptr(P.hash_hi)[s * P.hash_bins + b];
        while (lo > 0 && g[lo] > e) lo = lo - 1;
        while (hi < n - 1 && g[hi] <= e) hi = hi + 1;
    }
    int i = bisect(g, lo, hi, e);
    if (i > n - 2) i = n - 2;
    return i;
}

// Per species: clamp E to the grid, bracket it, interpolate sigma_a and
// sigma_s linearly in E; macroscopic total in ascending species order.
__device__ __forceinline__ double ce_lookup(const ProbDev &P, int m, double e, CEXS &X)
{
    double lnE = 0.0;
    if (P.lookup_hash) lnE = -neg_log(e);
    double cum = 0.0;
    const int n = P.grid_len;
#pragma unroll
    for (int s = 0; s < MAX_SPECIES; ++s) {
        X.sa[s] = 0.0;
        X.ss[s] = 0.0;
        X.cum[s] = cum;
        if (s < P.n_species) {
            const double *g = gptr(P.egrid) + (long)s * n;
            const double *a = gptr(P.siga) + (long)s * n;
            const double *b = gptr(P.sigs) + (long)s * n;
            double ec = e;
            if (ec < g[0]) ec = g[0];
            if (ec > g[n - 1]) ec = g[n - 1];
            int i = ce_bracket(P, s, g, ec, lnE);
            double f = (ec - g[i]) / (g[i + 1] - g[i]);
            double sa = a[i] + (f * (a[i + 1] - a[i]));
            double ss = b[i] + (f * (b[i + 1] - b[i]));
            X.sa[s] = sa;
            X.ss[s] = ss;
            cum = cum + (gptr(P.dens)[m * P.n_species + s] * (sa + ss));
            X.cum[s] = cum;
        }
    }
    return cum;
}

// elastic scattering off a target at rest with mass ratio A, isotropic in the
// centre-of-mass frame; returns E' and rotates the direction by the lab
// cosine about the old direction at azimuth 2 pi xi_phi
__device__ __forceinline__ double elastic(double A, double e, double xi_mu, double xi_phi, Part &p)
{
    double muc = (2.0 * xi_mu) - 1.0;
    double D = ((A * A) + ((2.0 * A) * muc)) + 1.0;
    double enew = (e * D) / ((A + 1.0) * (A + 1.0));
    double mul = (1.0 + (A * muc)) / root(D);
    double cp, sphi;
    turn_cos_sin(xi_phi, cp, sphi);
    double aa = root((1.0 - mul) * (1.0 + mul));
    double u = p.u, v = p.v, w = p.w;
    double bb = root((1.0 - w) * (1.0 + w));
    if (bb > 1e-10) {
        p.u = (mul * u) + ((aa * (((u * w) * cp) - (v * sphi))) / bb);
        p.v = (mul * v) + ((aa * (((v * w) * cp) + (u * sphi))) / bb);
        p.w = (mul * w) - ((aa * bb) * cp);
    } else {
        p.u = aa * cp;
        p.v = aa * sphi;
        p.w = (w >= 0.0) ? mul : -mul;
    }
    return enew;
}

__device__ __forceinline__ void isotropic(double xi_mu, double xi_phi, Part &p)
{
    double mu = (2.0 * xi_mu) - 1.0;
    double c, s;
    turn_cos_sin(xi_phi, c, s);
    double st = root((1.0 - mu) * (1.0 + mu));
    p.u = st * c;
    p.v = st * s;
    p.w = mu;
}

// ---------------------------------------------------------------- tallies

// Integer adds with the address space stated.  Tally and sum pointers come
// out of the problem record, so the compiler cannot tell global memory from
// LDS and would issue flat atomics; on gfx9 a flat access counts on both
// the vector-memory and the LDS counters, so every later LDS table read
// would wait for the atomic's round trip to memory.
typedef __attribute__((address_space(1))) unsigned long long gu64;
typedef __attribute__((address_space(3))) unsigned long long lu64;

__device__ __forceinline__ void add_global(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_fetch_add((gu64 *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void add_lds(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_fetch_add((lu64 *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Where a flight's tally pieces go, read from the problem record once per
// flight rather than per piece (inside the mesh walk every such read is a
// scalar load the piece would wait for): this block's LDS copy of the bins
// (a small tally: every flight would hit the same few global words, and the
// device serialises atomics per address), or the global tally, or for a
// large energy-bin tally this wavefront's replica (particles of a round or
// wavefront have similar energies and hit the same few bins, so the adds are
// spread over replicas); the fixed-point scale; the replays' dL/dT (pass B
// reads it only in weighted runs), and whether pass A also sums |w len|.
struct Sink {
    unsigned long long *lt;
    unsigned long long *g;
    double tscale;
    const double *w;
    bool wabs;
};

template <int MODE>
__device__ __forceinline__ Sink sink_of(const ProbDev &P, const Lane &ln, unsigned long long *lt)
{
    Sink k;
    k.lt = lt;
    k.g = nullptr;
    k.tscale = 0.0;
    k.w = nullptr;
    k.wabs = false;
    if (MODE == MODE_FWD) {
        k.g = P.trep ? P.trep + (size_t)ln.rep * (size_t)P.n_bins : P.tally;
        k.tscale = P.tscale;
    } else {
        k.w = gptr(P.w);
        k.wabs = MODE == MODE_REPLAY_A && P.implicit;
    }
    return k;
}

template <int MODE>
__device__ __forceinline__ void score(const Sink &k, Lane &ln, Part &p, long bin, double len)
{
    if (MODE == MODE_FWD) {
        // rint(len 2^S) as an integer: for 0 <= v < 2^52 the sum v + 2^52,
        // rounded to nearest even, is 2^52 + rint(v) exactly, whose bit
        // pattern less that of 2^52 is the integer (no float-to-int64
        // conversion sequence)
        const double v = len * k.tscale;
        long long q;
        if (v >= 0.0 && v < 0x1p52) q = (long long)(__double_as_longlong(v + 0x1p52) - 0x4330000000000000ll);
        else q = (long long)to_fixed(len, k.tscale);
        if (q != 0) {
            if (k.lt) add_lds(k.lt + bin, (unsigned long long)q);
            else add_global(k.g + bin, (unsigned long long)q);
            p.hq += q;
            unsigned long long before = ln.q;
            ln.q = before + (unsigned long long)q;
            if (ln.q < before) ln.err |= ERR_OVERFLOW;
            ln.pieces += 1;
        }
    } else if (MODE == MODE_REPLAY_A) {
        p.G = p.G + (k.w[bin] * len);
        if (k.wabs) p.A = p.A + fabs(k.w[bin] * len);
    } else {
        // weighted pass B: the score of the pieces flown so far
        p.L = p.L + (k.w[bin] * len);
    }
}

// Time split of the current flight (time-binned tallies): the flight starts
// at time t0 in time bin k and moves at speed v.
struct TSplit {
    double t0, v;
    int k;
};

// largest k in [0, n-1] with k dt <= t (0 if none): a guess from t / dt,
// corrected against the edges k dt themselves
__device__ __forceinline__ int time_bin(double t, double dt, int n)
{
    double g = t / dt;
    int k = 0;
    if (g > 0.0) k = (g < (double)n) ? (int)g : n - 1;
    while (k + 1 < n && ((double)(k + 1) * dt) <= t) k = k + 1;
    while (k > 0 && ((double)k * dt) > t) k = k - 1;
    return k;
}

// Score the piece [a, b] of the current flight (distances from its start)
// into bin `bin` of the tally without time; a piece scores its length times
// the particle's weight (extended state; the weight is 1 unless the problem
// uses implicit capture).  With time bins the piece is cut where the
// particle's time t0 + s / v passes a bin edge: the edge closing bin k lies
// at s = ((k + 1) tw - t0) v; the last time bin takes the rest.
template <int MODE, int EXT>
__device__ __forceinline__ void score_piece(const ProbDev &P, const Sink &sk, Lane &ln, Part &p, TSplit &ts, long bin,
                                            double a, double b)
{
    if (!EXT) {
        score<MODE>(sk, ln, p, bin, b - a);
        return;
    }
    if (P.n_tbins <= 0) {
        score<MODE>(sk, ln, p, bin, (b - a) * p.wgt);
        return;
    }
    for (;;) {
        const int k = ts.k;
        const long kb = (long)k * P.nbase + bin;
        if (k + 1 >= P.n_tbins) {
            score<MODE>(sk, ln, p, kb, (b - a) * p.wgt);
            return;
        }
        double se = (((double)(k + 1) * P.tw) - ts.t0) * ts.v;
        if (se >= b) {
            score<MODE>(sk, ln, p, kb, (b - a) * p.wgt);
            return;
        }
        score<MODE>(sk, ln, p, kb, (se - a) * p.wgt);
        a = se;
        ts.k = k + 1;
    }
}

__device__ __forceinline__ double axis_t(const double *__restrict__ e, int i, double x0, double u)
{
    const double q = (e[(u > 0.0) ? i + 1 : i] - x0) / u;
    double t = (u > 0.0 || u < 0.0) ? q : inf();
    if (t < 0.0) t = 0.0;
    return t;
}

// Track-length mesh tally of one flight of length d from the current
// position: visit the mesh cells the segment crosses; every crossing
// parameter is measured from the flight start; ties go x, y, z.
template <int MODE, int EXT, class TB>
__device__ __forceinline__ void walk_mesh(const ProbDev &P, const TB &T, const Sink &sk, Lane &ln, Part &p, double d,
                                          int g, TSplit &ts)
{
    const int n0 = P.mesh_n[0], n1 = P.mesh_n[1], n2 = P.mesh_n[2];
    const double *mx = T.mx(), *my = T.my(), *mz = T.mz();
    int i0 = edge_index_guess(mx, n0, p.x, p.u, P.mesh_lo[0], P.mesh_inv[0]);
    int i1 = edge_index_guess(my, n1, p.y, p.v, P.mesh_lo[1], P.mesh_inv[1]);
    int i2 = edge_index_guess(mz, n2, p.z, p.w, P.mesh_lo[2], P.mesh_inv[2]);
    double t0 = axis_t(mx, i0, p.x, p.u);
    double t1 = axis_t(my, i1, p.y, p.v);
    double t2 = axis_t(mz, i2, p.z, p.w);
    double tprev = 0.0;
    // the bin of cell (i0, i1, i2) in group g; a crossing moves it by the
    // axis stride 1, n0 or n0 n1
    long bin = (((long)g * n2 + i2) * n1 + i1) * n0 + i0;
    const long sy = n0, sz = (long)n0 * n1;
    for (;;) {
        int a = 0;
        double tm = t0;
        if (t1 < tm) { tm = t1; a = 1; }
        if (t2 < tm) { tm = t2; a = 2; }
        double tend = (tm < d) ? tm : d;
        score_piece<MODE, EXT>(P, sk, ln, p, ts, bin, tprev, tend);
        if (tm >= d) break;
        // advance along the crossed axis: its edges, position, direction and
        // index are selected, so every lane makes one edge read and one
        // division whichever axis it crosses (a branch per axis would make a
        // wavefront whose lanes cross different axes pay for all three)
        const double ua = (a == 0) ? p.u : (a == 1) ? p.v : p.w;
        const double xa = (a == 0) ? p.x : (a == 1) ? p.y : p.z;
        const double *ea = (a == 0) ? mx : (a == 1) ? my : mz;
        const int na = (a == 0) ? n0 : (a == 1) ? n1 : n2;
        int ia = ((a == 0) ? i0 : (a == 1) ? i1 : i2) + ((ua > 0.0) ? 1 : -1);
        if (ia < 0 || ia >= na) break;
        double ta = (ea[ia + ((ua > 0.0) ? 1 : 0)] - xa) / ua;
        if (ta < 0.0) ta = 0.0;
        const long sa = (a == 0) ? 1l : (a == 1) ? sy : sz;
        bin += (ua > 0.0) ? sa : -sa;
        i0 = (a == 0) ? ia : i0;
        i1 = (a == 1) ? ia : i1;
        i2 = (a == 2) ? ia : i2;
        t0 = (a == 0) ? ta : t0;
        t1 = (a == 1) ? ta : t1;
        t2 = (a == 2) ? ta : t2;
        tprev = tend;
    }
}

template <int MODE>
__device__ __forceinline__ void pass_b_add(const ProbDev &P, const EvCtx &cx, int which, int mg, long long q)
{
    if (q == 0) return;
    if (cx.lacc) {
        add_lds(cx.lacc + (which * P.n_mat * P.n_grp + mg), (unsigned long long)q);
    } else {
        unsigned long long *dst = (which == 0) ? P.SL : (which == 1) ? P.SA : P.SS;
        add_global(dst + mg, (unsigned long long)q);
    }
}

// Score a flight of length d that started at the particle's position.
template <int EMODE, int MODE, int EXT, class TB>
__device__ __forceinline__ void score_flight(const ProbDev &P, const TB &T, const EvCtx &cx, Lane &ln, Part &p, double d,
                                             int m, TSplit &ts)
{
    int g = gc_group(p.gc);
    if (MODE == MODE_REPLAY_B) {
        pass_b_add<MODE>(P, cx, 0, m * P.n_grp + g, (long long)to_fixed(p.G * d, P.gscale));
        // weighted runs walk the tally as well, for the running score
        if (!(EXT && P.implicit)) return;
    }
    const Sink sk = sink_of<MODE>(P, ln, cx.ltally);
    if (P.tally_kind == 0) {
        walk_mesh<MODE, EXT>(P, T, sk, ln, p, d, g, ts);
    } else {
        int k;
        if (P.ebin_inv != 0.0) {
            double t = ((-neg_log(p.e)) - P.ebin_lnlo) * P.ebin_inv;
            int g = 0;
            if (t > 0.0) g = (t < (double)P.n_ebins) ? (int)t : P.n_ebins - 1;
            k = edge_index_from(gptr(P.eedges), P.n_ebins, p.e, 1.0, g);
        } else {
            k = edge_index(gptr(P.eedges), P.n_ebins, p.e, 1.0);
        }
        score_piece<MODE, EXT>(P, sk, ln, p, ts, k, 0.0, d);
    }
    if (MODE == MODE_REPLAY_A) p.L = p.L + d;
}

// First k in [0, n) with xi < row[k], else n - 1 (the outgoing group of a
// scatter).  Entries are read four at a time as independent loads, so the
// scan waits for one LDS round trip per four entries rather than per entry.
__device__ __forceinline__ int cdf_first_above(const double *row, int n, double xi)
{
    for (int k = 0; k < n; k += 4) {
        const int last = n - 1;
        const double r0 = row[k];
        const double r1 = row[(k + 1 < n) ? k + 1 : last];
        const double r2 = row[(k + 2 < n) ? k + 2 : last];
        const double r3 = row[(k + 3 < n) ? k + 3 : last];
        if (xi < r0) return k;
        if (k + 1 < n && xi < r1) return k + 1;
        if (k + 2 < n && xi < r2) return k + 2;
        if (k + 3 < n && xi < r3) return k + 3;
    }
    return n - 1;
}

// ---------------------------------------------------------------- events

template <int MODE>
__device__ __forceinline__ void finish(const ProbDev &P, const EvCtx &cx, Lane &ln, Part &p, uint32_t fate)
{
    uint32_t flights = (fate == FATE_KILLED) ? p.step - 1 : p.step;
    uint64_t idx = P.gbase + (uint64_t)(p.hid - P.first);
    if (MODE == MODE_FWD && P.gn) *gmem(P.gn + idx) = p.nsplit;   // copies this history split off
    if (MODE == MODE_FWD) {
        if (cx.digest) {
            auto *dg = gmem(cx.digest + idx);
            dg->qsum = p.hq;
            dg->flights = flights;
            dg->collisions = p.ncoll;
            dg->fate = fate;
            dg->pad = 0;
        }
    } else if (MODE == MODE_REPLAY_A) {
        *gmem(P.G + idx) = p.G;
        // every pass B sum of the history is at most this in magnitude (in a
        // weighted run the score still to come at a collision is at most A)
        double bound = P.implicit ? ceil((fabs(p.G) + p.A) * (p.L + (double)flights))
                                  : ceil(fabs(p.G) * (p.L + (double)flights));
        if (!(bound < 0x1p63)) {
            ln.err |= ERR_BOUND;
        } else if (cx.single) {
            unsigned long long before = ln.u;
            ln.u = before + (unsigned long long)bound;
            if (ln.u < before) ln.err |= ERR_BOUND;
        } else {
            unsigned long long old = __hip_atomic_fetch_add(gmem(P.U), (unsigned long long)bound, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT);
            if (old + (unsigned long long)bound < old) ln.err |= ERR_BOUND;
        }
    }
}

// Source event ("make_work" output): the history's start state.
template <int GEOM, int MODE, class TB>
__device__ __forceinline__ void source(const ProbDev &P, const TB &T, Part &p, uint32_t hid, uint32_t prob)
{
    Key k{P.key0, P.key1};
    double x0, x1, x2, x3, x4, x5;
    uniform_pair(k, hid, 0, 0, x0, x1, P.stream);
    uniform_pair(k, hid, 0, 1, x2, x3, P.stream);
    uniform_pair(k, hid, 0, 2, x4, x5, P.stream);
    const uint64_t idx = P.gbase + (uint64_t)(hid - P.first);
    const bool banked = P.sbank != nullptr;   // a k-eigenvalue cycle after the first
    if (banked) {
        const auto *sb = gmem(P.sbank + 3 * idx);
        p.x = sb[0];
        p.y = sb[1];
        p.z = sb[2];
    } else if (P.src_kind == 0) {
        p.x = P.src_pos[0]; p.y = P.src_pos[1]; p.z = P.src_pos[2];
    } else if (P.src_kind == 1) {
        p.x = P.src_lo[0] + (x0 * P.src_ext[0]);
        p.y = P.src_lo[1] + (x1 * P.src_ext[1]);
        p.z = P.src_lo[2] + (x2 * P.src_ext[2]);
    } else {
        double r = P.src_radius * root(x0);
        double c, s;
        turn_cos_sin(x1, c, s);
        p.x = P.src_pos[0] + (r * c);
        p.y = P.src_pos[1] + (r * s);
        p.z = P.src_pos[2];
    }
    if (P.src_iso || banked) {
        isotropic(x3, x4, p);
    } else {
        p.u = P.src_dir[0]; p.v = P.src_dir[1]; p.w = P.src_dir[2];
    }
    p.e = P.e_src;
    p.gc = locate<GEOM>(P, T, p.x, p.y, p.u, p.v, P.src_group);
    if (banked) {
        // a banked fission neutron: group from the fission spectrum of the
        // material at its site (slot 0)
        const double *row = T.chi() + (long)material<GEOM>(P, T, p.gc) * P.n_grp;
        int g = P.n_grp - 1;
        for (int k2 = 0; k2 < P.n_grp; ++k2) {
            if (x0 < row[k2]) {
                g = k2;
                break;
            }
        }
        p.gc = (p.gc & ~0xffu) | (uint32_t)g;
    }
    if (P.fn) *gmem(P.fn + idx) = 0u;
    p.hid = hid;
    p.prob = prob;
    p.step = 1;
    p.ncoll = 0;
    p.nsplit = 0;
    p.hq = 0;
    p.sigt = 0.0;
    p.L = 0.0;
    p.G = 0.0;
    p.A = 0.0;
    p.t = 0.0;
    p.wgt = 1.0;
    if (P.gsrc) {
        // a history of a later generation: the state its copy was split off
        // with (no source draws are used)
        const auto *r = gmem(P.gsrc + idx);
        p.x = r->pos[0];
        p.y = r->pos[1];
        p.z = r->pos[2];
        p.u = r->dir[0];
        p.v = r->dir[1];
        p.w = r->dir[2];
        p.e = r->e;
        p.wgt = r->w;
        p.t = r->t;
        p.gc = r->gc;
    }
    if (MODE == MODE_REPLAY_B) p.G = *gmem(P.G + (P.gbase + (uint64_t)(hid - P.first)));
}

// flight cap; true if the history was killed
template <int MODE>
__device__ __forceinline__ bool kill_check(const ProbDev &P, const EvCtx &cx, Lane &ln, Part &p, uint32_t &out)
{
    if ((long long)p.step > P.max_steps) {
        out |= O_KILL;
        finish<MODE>(P, cx, ln, p, FATE_KILLED);
        return true;
    }
    return false;
}

enum : int { FLY_SURFACE = 0, FLY_COLLIDE = 1, FLY_TIME = 2 };

// Move to the next collision site or surface, scoring the track on the way.
// With time bins a flight that would reach t_max stops there (a tie goes to
// the time boundary) and the history ends; otherwise the particle's time
// advances by d / v.  That sum can round to just past t_max; the remaining
// length is then zero, never negative.
template <int GEOM, int EMODE, int MODE, int EXT, class TB>
__device__ __forceinline__ int fly(const ProbDev &P, const TB &T, const EvCtx &cx, Lane &ln, Part &p, double sigt,
                                   double xi0, int m, int &surf)
{
    double dcol = neg_log(xi0) / sigt;
    double dsurf = surface_distance<GEOM>(P, T, p, surf);
    int res = (dcol < dsurf) ? FLY_COLLIDE : FLY_SURFACE;
    double d = (res == FLY_COLLIDE) ? dcol : dsurf;
    TSplit ts{0.0, 0.0, 0};
    const bool timed = EXT && P.n_tbins > 0;
    if (timed) {
        const double v = (EMODE == EMODE_MG) ? T.speed()[gc_group(p.gc)] : P.speed_coef * root(p.e);
        const double dtime = (P.t_max - p.t) * v;
        if (!(d < dtime)) {
            d = (dtime > 0.0) ? dtime : 0.0;
            res = FLY_TIME;
        }
        ts.t0 = p.t;
        ts.v = v;
        ts.k = time_bin(p.t, P.tw, P.n_tbins);
    }
    score_flight<EMODE, MODE, EXT>(P, T, cx, ln, p, d, m, ts);
    p.x = p.x + (d * p.u);
    p.y = p.y + (d * p.v);
    p.z = p.z + (d * p.w);
    if (timed && res != FLY_TIME) p.t = p.t + (d / ts.v);
    return res;
}

// Cross the surface `surf`: snap to the plane, then leak, reflect or enter
// the neighbouring cell.  Returns false if the particle leaked.
template <int GEOM, class TB>
__device__ __forceinline__ bool cross(const ProbDev &P, const TB &T, Part &p, int surf, uint32_t &out)
{
    // new values are formed in scalars and stored unconditionally, so no
    // field of the particle is ever addressed through a computed index
    out |= O_CROSS;
    int g = gc_group(p.gc), c0 = gc_c0(p.gc), c1 = gc_c1(p.gc), in = gc_in(p.gc);
    double x = p.x, y = p.y, z = p.z;
    int face = -1;
    if (surf == 3) {
        in = 1 - in;
    } else if (surf == 0) {
        int n = (GEOM == GEOM_BOX) ? P.n_slabs : P.nx;
        if (p.u > 0.0) {
            x = T.xpl()[c0 + 1];
            if (c0 + 1 == n) face = 1; else c0 = c0 + 1;
        } else {
            x = T.xpl()[c0];
            if (c0 == 0) face = 0; else c0 = c0 - 1;
        }
    } else if (surf == 1) {
        if (GEOM == GEOM_BOX) {
            y = (p.v > 0.0) ? P.box_hi[1] : P.box_lo[1];
            face = (p.v > 0.0) ? 3 : 2;
        } else if (p.v > 0.0) {
            y = T.ypl()[c1 + 1];
            if (c1 + 1 == P.ny) face = 3; else c1 = c1 + 1;
        } else {
            y = T.ypl()[c1];
            if (c1 == 0) face = 2; else c1 = c1 - 1;
        }
    } else {
        z = (p.w > 0.0) ? P.box_hi[2] : P.box_lo[2];
        face = (p.w > 0.0) ? 5 : 4;
    }
    p.x = x;
    p.y = y;
    p.z = z;
    if (face >= 0) {
        if (!((P.refl_mask >> face) & 1)) {
            out |= O_LEAK;
            return false;
        }
        out |= O_REFL;
        int axis = face >> 1;
        double u = p.u, v = p.v, w = p.w;
        p.u = (axis == 0) ? -u : u;
        p.v = (axis == 1) ? -v : v;
        p.w = (axis == 2) ? -w : w;
    }
    p.gc = gc_pack(g, c0, c1, in, 0);
    return true;
}

// Collision at the current site with the flight's random numbers xi1..xi5.
// Returns false if the history ends (absorption, energy cutoff, roulette).
// Weight-window closeout (extended particles; after a collision that leaves
// the particle alive, or a surface crossing that does not leak).  The cell of
// the position on the window grid gives the window [lo, ratio lo] and the
// survival weight surv lo.  Above the window the particle splits into
// n = floor(w / (surv lo)) copies, clamped to [2, max_split], of weight w / n:
// it continues as the first, the other n - 1 are staged for the next
// generation with their parent and ordinal (the next generation orders them
// by those, whatever wavefront staged them).  Below the window it plays
// roulette with xi5: survival weight with probability w / (surv lo), else the
// history ends.  Returns false if it ended.
template <int MODE>
__device__ __forceinline__ bool ww_closeout(const ProbDev &P, const EvCtx &cx, Lane &ln, Part &p, double xi5,
                                            uint32_t &out)
{
    const double pos[3] = {p.x, p.y, p.z};
    long c = 0;
#pragma unroll
    for (int a = 2; a >= 0; --a) {
        const int n = P.ww_n[a];
        const double tt = (pos[a] - P.box_lo[a]) * P.ww_inv[a];
        int i = 0;
        if (tt > 0.0) i = (tt < (double)n) ? (int)tt : n - 1;
        c = c * n + i;
    }
    const double lo = gptr(P.ww_lo)[c];
    if (!(lo > 0.0)) return true;
    const double surv = P.ww_surv * lo;
    const double w = p.wgt;
    if (w > P.ww_ratio * lo) {
        const double q = w / surv;
        int n = (q < (double)P.ww_max_split) ? (int)q : P.ww_max_split;
        if (n < 2) n = 2;
        const double wn = w / (double)n;
        p.wgt = wn;
        if (MODE == MODE_FWD) {
            const unsigned long long at = __hip_atomic_fetch_add((gu64 *)P.gcount, (unsigned long long)(n - 1),
                                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int k = 1; k < n; ++k) {
                const unsigned long long i = at + (unsigned long long)(k - 1);
                if (i >= P.gcap) {
                    ln.err |= ERR_CAPACITY;
                    continue;
                }
                auto *r = gmem(P.gout + i);
                r->pos[0] = p.x;
                r->pos[1] = p.y;
                r->pos[2] = p.z;
                r->dir[0] = p.u;
                r->dir[1] = p.v;
                r->dir[2] = p.w;
                r->e = p.e;
                r->w = wn;
                r->t = p.t;
                r->gc = p.gc & ~(3u << 29);      // no surface pending
                r->parent = p.hid;
                r->seq = p.nsplit + (uint32_t)(k - 1);
                r->pad = 0;
            }
            p.nsplit += (uint32_t)(n - 1);
            ln.splits += (uint32_t)(n - 1);
        }
        return true;
    }
    if (w < lo) {
        if ((xi5 * surv) < w) {
            p.wgt = surv;
            return true;
        }
        out |= O_ROUL;
        finish<MODE>(P, cx, ln, p, FATE_ROULETTE);
        return false;
    }
    return true;
}

// With implicit capture (extended state) a collision never absorbs: the
// particle scatters with its weight times the scattering probability, and
// the closeout then plays weight roulette below the cutoff (xi5).
template <int EMODE, int MODE, int EXT, bool CLOSE, class TB>
__device__ __forceinline__ bool collide(const ProbDev &P, const TB &T, const EvCtx &cx, Lane &ln, Part &p, int m,
                                        double sigt, const CEXS &X, double xi1, double xi2, double xi3, double xi4,
                                        double xi5, uint32_t &out)
{
    out |= O_COLL;
    p.ncoll += 1;
    const bool implicit = EXT && P.implicit;
    if (EMODE == EMODE_MG) {
        int g = gc_group(p.gc);
        int mg = m * P.n_grp + g;
        double ss = T.sig_s()[mg];
        if (implicit) {
            p.wgt = p.wgt * (ss / sigt);
            // pass B: G_h for the collision density, and the score still to
            // come, G_h - F, for the factor Sigma_s / Sigma_t in every later
            // piece's weight
            if (MODE == MODE_REPLAY_B) {
                pass_b_add<MODE>(P, cx, 1, mg, (long long)to_fixed(p.G, P.gscale));
                pass_b_add<MODE>(P, cx, 2, mg, (long long)to_fixed(p.G - p.L, P.gscale));
            }
        } else if (!((xi1 * sigt) < ss)) {
            out |= O_ABS;
            if (MODE == MODE_REPLAY_B) pass_b_add<MODE>(P, cx, 1, mg, (long long)to_fixed(p.G, P.gscale));
            // k-eigenvalue cycle: the absorption is a fission with probability
            // Sigma_f / Sigma_a and banks floor(nu + xi) neutrons at the site
            if (MODE == MODE_FWD && P.fn && ((xi2 * (sigt - ss)) < T.sigf()[mg])) {
                const uint64_t idx = P.gbase + (uint64_t)(p.hid - P.first);
                *gmem(P.fn + idx) = (uint32_t)(T.nu()[mg] + xi3);
                auto *fp = gmem(P.fpos + 3 * idx);
                fp[0] = p.x;
                fp[1] = p.y;
                fp[2] = p.z;
                out |= O_FISS;
            }
            finish<MODE>(P, cx, ln, p, FATE_ABSORB);
            return false;
        }
        out |= O_SCAT;
        if (MODE == MODE_REPLAY_B && !implicit) pass_b_add<MODE>(P, cx, 2, mg, (long long)to_fixed(p.G, P.gscale));
        const int gn = cdf_first_above(T.cdf() + (long)mg * P.n_grp, P.n_grp, xi2);
        ln.cdf += (uint32_t)gn + 1u;
        p.gc = (p.gc & ~0xffu) | (uint32_t)gn;
        isotropic(xi3, xi4, p);
    } else {
        double target = xi1 * sigt;
        int sp = P.n_species - 1;
#pragma unroll
        for (int s = MAX_SPECIES - 1; s >= 0; --s)
            if (s < P.n_species && target < X.cum[s]) sp = s;
        double sa = 0.0, ss = 0.0;
#pragma unroll
        for (int s = 0; s < MAX_SPECIES; ++s)
            if (s == sp) { sa = X.sa[s]; ss = X.ss[s]; }
        if (implicit) {
            p.wgt = p.wgt * (ss / (sa + ss));
        } else if (!((xi2 * (sa + ss)) < ss)) {
            out |= O_ABS;
            finish<MODE>(P, cx, ln, p, FATE_ABSORB);
            return false;
        }
        out |= O_SCAT;
        double enew = elastic(gptr(P.awr)[sp], p.e, xi3, xi4, p);
        if (enew < P.e_min) {
            out |= O_CUT;
            finish<MODE>(P, cx, ln, p, FATE_CUTOFF);
            return false;
        }
        p.e = enew;
    }
    // closeout (split events: an event of its own): weight windows, or
    // without them weight roulette below the cutoff
    if (!CLOSE) return true;
    if (EXT && P.ww_n[0] > 0) return ww_closeout<MODE>(P, cx, ln, p, xi5, out);
    if (implicit && p.wgt < P.w_cut) {
        if ((xi5 * P.w_surv) < p.wgt) {
            p.wgt = P.w_surv;
        } else {
            out |= O_ROUL;
            finish<MODE>(P, cx, ln, p, FATE_ROULETTE);
            return false;
        }
    }
    return true;
}

// Monolithic event: one whole flight (lookup, move with tally, collide or cross).
template <int GEOM, int EMODE, int MODE, int EXT, class TB>
__device__ __forceinline__ int ev_step(const ProbDev &P, const TB &T, const EvCtx &cx, Lane &ln, Part &p, uint32_t &out)
{
    if (kill_check<MODE>(P, cx, ln, p, out)) return EV_DEAD;
    int m = material<GEOM>(P, T, p.gc);
    CEXS X;
    double sigt;
    if (EMODE == EMODE_MG) sigt = T.sig_t()[m * P.n_grp + gc_group(p.gc)];
    else sigt = ce_lookup(P, m, p.e, X);
    Key k{P.key0, P.key1};
    double xi0, xi1;
    uniform_pair(k, p.hid, p.step, 0, xi0, xi1, P.stream);
    int surf;
    const int res = fly<GEOM, EMODE, MODE, EXT>(P, T, cx, ln, p, sigt, xi0, m, surf);
    out |= O_FLIGHT;
    if (EXT && res == FLY_TIME) {
        out |= O_CUT;
        finish<MODE>(P, cx, ln, p, FATE_CUTOFF);
        return EV_DEAD;
    }
    if (res == FLY_COLLIDE) {
        double xi2, xi3, xi4, xi5;
        uniform_pair(k, p.hid, p.step, 1, xi2, xi3, P.stream);
        uniform_pair(k, p.hid, p.step, 2, xi4, xi5, P.stream);
        if (!collide<EMODE, MODE, EXT, true>(P, T, cx, ln, p, m, sigt, X, xi1, xi2, xi3, xi4, xi5, out)) return EV_DEAD;
    } else {
        if (!cross<GEOM>(P, T, p, surf, out)) {
            finish<MODE>(P, cx, ln, p, FATE_LEAK);
            return EV_DEAD;
        }
        if (EXT && P.ww_n[0] > 0) {
            double xi4, xi5;
            uniform_pair(k, p.hid, p.step, 2, xi4, xi5, P.stream);
            if (!ww_closeout<MODE>(P, cx, ln, p, xi5, out)) return EV_DEAD;
        }
    }
    p.step += 1;
    return EV_STEP;
}

// Decomposed events: the paper's decomposed scheme (Sec. 4) without domain
// crossing.  STEP looks up the total cross section, moves the particle to
// its next collision site or surface and scores the track on the way;
// SURFACE crosses; COLLIDE collides; CLOSEOUT (extended particles with
// weight windows, or implicit capture after a collision) applies weights
// and weight windows before the next flight.  The flight counter advances
// when the particle goes back to STEP, so every event of a flight draws
// from that flight's slots.

template <int EXT>
__device__ __forceinline__ bool closeout_after_collision(const ProbDev &P)
{
    return EXT && (P.ww_n[0] > 0 || P.implicit);
}

template <int EXT>
__device__ __forceinline__ bool closeout_after_crossing(const ProbDev &P)
{
    return EXT && P.ww_n[0] > 0;
}

template <int GEOM, int EMODE, int MODE, int EXT, class TB>
__device__ __forceinline__ int ev_move(const ProbDev &P, const TB &T, const EvCtx &cx, Lane &ln, Part &p, uint32_t &out)
{
    if (kill_check<MODE>(P, cx, ln, p, out)) return EV_DEAD;
    int m = material<GEOM>(P, T, p.gc);
    double sigt;
    if (EMODE == EMODE_MG) {
        sigt = T.sig_t()[m * P.n_grp + gc_group(p.gc)];
    } else {
        CEXS X;
        sigt = ce_lookup(P, m, p.e, X);
    }
    Key k{P.key0, P.key1};
    double xi0, xi1;
    uniform_pair(k, p.hid, p.step, 0, xi0, xi1, P.stream);
    int surf;
    const int res = fly<GEOM, EMODE, MODE, EXT>(P, T, cx, ln, p, sigt, xi0, m, surf);
    out |= O_FLIGHT;
    if (EXT && res == FLY_TIME) {
        out |= O_CUT;
        finish<MODE>(P, cx, ln, p, FATE_CUTOFF);
        return EV_DEAD;
    }
    p.gc = (p.gc & ~(3u << 29)) | ((uint32_t)surf << 29);
    return (res == FLY_COLLIDE) ? EV_COLLIDE : EV_SURFACE;
}

template <int GEOM, int EMODE, int MODE, int EXT, class TB>
__device__ __forceinline__ int ev_surface(const ProbDev &P, const TB &T, const EvCtx &cx, Lane &ln, Part &p,
                                          uint32_t &out)
{
    if (!cross<GEOM>(P, T, p, gc_surf(p.gc), out)) {
        finish<MODE>(P, cx, ln, p, FATE_LEAK);
        return EV_DEAD;
    }
    if (closeout_after_crossing<EXT>(P)) return EV_CLOSEOUT;
    p.step += 1;
    return EV_STEP;
}

template <int GEOM, int EMODE, int MODE, int EXT, class TB>
__device__ __forceinline__ int ev_collide(const ProbDev &P, const TB &T, const EvCtx &cx, Lane &ln, Part &p,
                                          uint32_t &out)
{
    int m = material<GEOM>(P, T, p.gc);
    CEXS X;
    // the flight's total cross section, as its STEP found it
    double sigt;
    if (EMODE == EMODE_MG) sigt = T.sig_t()[m * P.n_grp + gc_group(p.gc)];
    else sigt = ce_lookup(P, m, p.e, X);
    Key k{P.key0, P.key1};
    double xi0, xi1, xi2, xi3, xi4, xi5;
    uniform_pair(k, p.hid, p.step, 0, xi0, xi1, P.stream);
    uniform_pair(k, p.hid, p.step, 1, xi2, xi3, P.stream);
    xi4 = 0.0;
    xi5 = 0.0;
    uniform_pair(k, p.hid, p.step, 2, xi4, xi5, P.stream);
    if (!collide<EMODE, MODE, EXT, false>(P, T, cx, ln, p, m, sigt, X, xi1, xi2, xi3, xi4, xi5, out)) return EV_DEAD;
    if (closeout_after_collision<EXT>(P)) return EV_CLOSEOUT;
    p.step += 1;
    return EV_STEP;
}

// Closeout of a collision or crossing (slot 5 of the flight): weight
// windows, or without them implicit capture's roulette below the cutoff.
template <int GEOM, int EMODE, int MODE, int EXT, class TB>
__device__ __forceinline__ int ev_closeout(const ProbDev &P, const TB &T, const EvCtx &cx, Lane &ln, Part &p,
                                           uint32_t &out)
{
    Key k{P.key0, P.key1};
    double xi4, xi5;
    uniform_pair(k, p.hid, p.step, 2, xi4, xi5, P.stream);
    if (EXT && P.ww_n[0] > 0) {
        if (!ww_closeout<MODE>(P, cx, ln, p, xi5, out)) return EV_DEAD;
    } else if (EXT && P.implicit && p.wgt < P.w_cut) {
        if ((xi5 * P.w_surv) < p.wgt) {
            p.wgt = P.w_surv;
        } else {
            out |= O_ROUL;
            finish<MODE>(P, cx, ln, p, FATE_ROULETTE);
            return EV_DEAD;
        }
    }
    p.step += 1;
    return EV_STEP;
}

template <int GEOM, int EMODE, int MODE, int SPLIT, int EXT, class TB>
__device__ __forceinline__ int run_event(int ev, const ProbDev &P, const TB &T, const EvCtx &cx, Lane &ln, Part &p,
                                         uint32_t &out)
{
    if (!SPLIT) return ev_step<GEOM, EMODE, MODE, EXT>(P, T, cx, ln, p, out);
    if (ev == EV_STEP) return ev_move<GEOM, EMODE, MODE, EXT>(P, T, cx, ln, p, out);
    if (ev == EV_SURFACE) return ev_surface<GEOM, EMODE, MODE, EXT>(P, T, cx, ln, p, out);
    if (ev == EV_COLLIDE) return ev_collide<GEOM, EMODE, MODE, EXT>(P, T, cx, ln, p, out);
    return ev_closeout<GEOM, EMODE, MODE, EXT>(P, T, cx, ln, p, out);
}

// ------------------------------------------------------- wavefront helpers

// Value of the first active lane.  The builtin returns a signed int, so the
// 64-bit form must zero-extend the low half: a sign extension would smear
// bit 31 over the high half.
__device__ __forceinline__ uint32_t first_lane_u32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ __forceinline__ unsigned long long first_lane_u64(unsigned long long v)
{
    return ((unsigned long long)first_lane_u32((uint32_t)(v >> 32)) << 32) |
           (unsigned long long)first_lane_u32((uint32_t)v);
}

// Run one event for the active lanes with the problem record of each
// particle.  Batched launches: when every active lane holds a particle of
// the same problem (the common case: histories are sourced in consecutive
// runs of ids) the record is read at a wave-uniform index, with scalar
// loads that do not queue behind the wavefront's tally atomics; otherwise
// per lane.  Call with only the active lanes executing.
template <int GEOM, int EMODE, int MODE, int SPLIT, int EXT, bool BATCH>
__device__ __forceinline__ int run_event_in(int ev, const ProbDev *__restrict__ probs, const char *tl,
                                            const EvCtx &cx, Lane &ln, Part &p, uint32_t &out)
{
    if constexpr (!BATCH) {
        const ProbDev &P = probs[0];
        return run_event<GEOM, EMODE, MODE, SPLIT, EXT>(ev, P, tabs_for<false>(P, tl), cx, ln, p, out);
    } else {
        const uint32_t p0 = first_lane_u32(p.prob);
        if (__ballot(p.prob != p0) == 0) {
            const ProbDev &P = probs[p0];
            return run_event<GEOM, EMODE, MODE, SPLIT, EXT>(ev, P, TabsG{P}, cx, ln, p, out);
        }
        const ProbDev &P = probs[p.prob];
        return run_event<GEOM, EMODE, MODE, SPLIT, EXT>(ev, P, TabsG{P}, cx, ln, p, out);
    }
}

__device__ __forceinline__ uint32_t lane_rank(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// wave-uniform event counters (32-bit per wavefront; flushed once into the
// 64-bit run totals)
struct WaveCount {
    uint32_t c[C_WAVE];
    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int i = 0; i < C_WAVE; ++i) c[i] = 0;
    }
    __device__ __forceinline__ void outcomes(bool act, uint32_t out)
    {
        c[C_SOURCED] += (uint32_t)__popcll(__ballot(act && (out & O_SOURCE)));
        c[C_FLIGHTS] += (uint32_t)__popcll(__ballot(act && (out & O_FLIGHT)));
        c[C_COLLISIONS] += (uint32_t)__popcll(__ballot(act && (out & O_COLL)));
        c[C_SCATTERS] += (uint32_t)__popcll(__ballot(act && (out & O_SCAT)));
        c[C_ABSORBS] += (uint32_t)__popcll(__ballot(act && (out & O_ABS)));
        c[C_CROSSINGS] += (uint32_t)__popcll(__ballot(act && (out & O_CROSS)));
        c[C_LEAKS] += (uint32_t)__popcll(__ballot(act && (out & O_LEAK)));
        c[C_REFLECTIONS] += (uint32_t)__popcll(__ballot(act && (out & O_REFL)));
        c[C_CUTOFFS] += (uint32_t)__popcll(__ballot(act && (out & O_CUT)));
        c[C_KILLED] += (uint32_t)__popcll(__ballot(act && (out & O_KILL)));
        c[C_FISSIONS] += (uint32_t)__popcll(__ballot(act && (out & O_FISS)));
        c[C_ROULETTES] += (uint32_t)__popcll(__ballot(act && (out & O_ROUL)));
    }
    __device__ __forceinline__ void dispatch(bool act)
    {
        c[C_EVENTS] += (uint32_t)__popcll(__ballot(act));
        c[C_LANE_SLOTS] += 64;
        c[C_DISPATCHES] += 1;
    }
};

// Flush wave counters and lane accumulators into this wavefront's stripe of
// the run control block (only non-zero entries: one atomic each).
__device__ __forceinline__ void flush_wave(RunCtl *ctl, const WaveCount &wc, const Lane &ln, const ProbDev *probs,
                                           int single, int mode)
{
    // exact wave sum of the lanes' contribution totals, with wrap detection
    unsigned long long q = ln.q;
    uint32_t err = ln.err;
    unsigned long long pieces = ln.pieces;
    unsigned long long cdf = ln.cdf;
    unsigned long long spl = ln.splits;
    unsigned long long u = ln.u;
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long oq = __shfl_xor(q, off);
        unsigned long long ou = __shfl_xor(u, off);
        uint32_t oe = __shfl_xor(err, off);
        unsigned long long op = __shfl_xor(pieces, off);
        unsigned long long oc = __shfl_xor(cdf, off);
        unsigned long long os = __shfl_xor(spl, off);
        unsigned long long nq = q + oq;
        if (nq < q) err |= ERR_OVERFLOW;
        q = nq;
        unsigned long long nu = u + ou;
        if (nu < u) err |= ERR_BOUND;
        u = nu;
        err |= oe;
        pieces += op;
        cdf += oc;
        spl += os;
    }
    if (__lane_id() == 0) {
        const unsigned int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
        unsigned long long *S = ctl->stripe[wave % CTL_STRIPES].c;
        if (mode == MODE_FWD && q) {
            unsigned long long old = atomicAdd(&S[C_QSUM], q);
            if (old + q < old) err |= ERR_OVERFLOW;
        }
        if (mode == MODE_REPLAY_A && single && u) {
            unsigned long long old = atomicAdd(&S[C_PASSA_U], u);
            if (old + u < old) err |= ERR_BOUND;
        }
        if (err) atomicOr(&ctl->error, err);
        unsigned long long ended = (unsigned long long)wc.c[C_LEAKS] + wc.c[C_ABSORBS] + wc.c[C_CUTOFFS] +
                                   wc.c[C_KILLED] + wc.c[C_ROULETTES];
        if (ended) atomicAdd(&S[C_COMPLETED], ended);
#pragma unroll
        for (int i = 0; i < C_WAVE; ++i)
            if (wc.c[i]) atomicAdd(&S[i], (unsigned long long)wc.c[i]);
        if (pieces) atomicAdd(&S[C_PIECES], pieces);
        if (cdf) atomicAdd(&S[C_CDF], cdf);
        if (spl) atomicAdd(&S[C_SPLITS], spl);
    }
}

// Flattened history id -> problem (prefix[p] <= gid < prefix[p+1]).
__device__ __forceinline__ int find_problem(const unsigned long long *__restrict__ prefix, int n, unsigned long long gid)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= gid) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Pass B per-block sums: zero at block start, add to global at block end.
__device__ __forceinline__ void lacc_zero(unsigned long long *lacc, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) lacc[i] = 0;
}

// add a block's LDS energy-bin sums into the problem's tally
__device__ __forceinline__ void ltally_flush(const unsigned long long *lt, const ProbDev &P, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        unsigned long long v = lt[i];
        if (v) add_global(P.tally + i, v);
    }
}

__device__ __forceinline__ void lacc_flush(unsigned long long *lacc, const ProbDev &P)
{
    int mg = P.n_mat * P.n_grp;
    for (int i = threadIdx.x; i < 3 * mg; i += blockDim.x) {
        unsigned long long v = lacc[i];
        if (v) {
            unsigned long long *dst = (i < mg) ? P.SL : (i < 2 * mg) ? P.SA : P.SS;
            add_global(dst + (i % mg), v);
        }
    }
}

}  // namespace mcx
