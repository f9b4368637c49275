// C ABI of the transport library: problem upload, validation, run
// orchestration, tallies and the score-function backward (host side).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mcx.h"
#include "kernels.hpp"

using namespace mcx;

static_assert(sizeof(mcx_digest) == 24, "digest layout");

// Device scratch of mcx_run_noalloc: a fixed array in this code object, so
// runs through that entry point need no device allocation.  Every device the
// library runs on holds its own copy until the process ends.  In host code
// the array's name is not a device address: kernels and copies use the
// per-device address that hipGetSymbolAddress returns (scratch_setup).
static __device__ __align__(256) unsigned char scratch[MCX_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_addr[SCRATCH_MAX_DEVICES];   // device address of `scratch`, per device
}  // namespace

namespace {

// host copy of one problem's arrays, owned by the handle
struct HostProblem {
    mcx_problem_desc d;
    std::vector<double> xpl, ypl, cxs, cys, sig_t, sig_s, cdf, egrid, siga, sigs, awr, dens, mx, my, mz, eedges;
    std::vector<double> speed;            // group speeds (time bins, multigroup)
    std::vector<double> sigf, nu, chi;    // fission (k-eigenvalue runs)
    std::vector<double> wwlo;             // weight-window lower bounds (or {0})
    bool ww = false;
    bool fission = false;
    std::vector<int32_t> cmat, hash_lo, hash_hi;
    double hash_ln_lo = 0.0, hash_inv = 0.0;
    int32_t hash_bins = 0;
    int64_t n_bins = 0;                   // all bins (time bins included)
    int64_t nbase = 0;                    // bins without time
};

}  // namespace

struct mcx_problem_s {
    int device = 0;
    int num_cus = 256;
    int wall_clock_khz = 0;
    int n = 0;
    int geom = 0, emode = 0, tally_kind = 0;
    std::vector<HostProblem> hp;
    std::vector<ProbDev> pd;              // host image of the device table
    std::vector<size_t> tally_off;        // bin offset of each problem
    size_t total_bins = 0;
    // device memory
    void *blob = nullptr;                 // static arrays of every problem
    ProbDev *d_probs = nullptr;
    unsigned long long *d_prefix = nullptr;
    unsigned long long *d_tally = nullptr;
    unsigned long long *d_trep = nullptr;  // replicas of a large energy-bin tally
    size_t trep_words = 0;
    RunCtl *d_ctl = nullptr;
    // backward buffers
    double *d_G = nullptr;
    size_t G_cap = 0;
    double *d_w = nullptr;
    size_t w_cap = 0;
    unsigned long long *d_gacc = nullptr; // per problem: U, then SL, SA, SS
    std::vector<size_t> gacc_off;
    size_t gacc_words = 0;
    unsigned int *h_flag = nullptr;       // pinned
    RunCtl *h_ctl = nullptr;              // pinned
    Workspace ws;
    hipEvent_t poll[2] = {nullptr, nullptr};   // stack scheduler: batch-of-rounds events
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timer_events;   // reused by LaunchTimer
    std::vector<unsigned long long> run_prefix;   // [n + 1], reused by every pass
    std::vector<uint64_t> run_first, run_count;   // [n], reused by mcx_run
    // k-eigenvalue buffers (grown on demand): source banks (ping-pong), per
    // history banked count and fission site, the cycle's sites, scan tiles,
    // a tally for the inactive cycles, device and pinned host totals
    double *d_sbank[2] = {nullptr, nullptr};
    uint32_t *d_fn = nullptr;
    double *d_fpos = nullptr;
    size_t eig_cap = 0;                   // particles per source bank
    double *d_sites = nullptr;
    size_t sites_cap = 0;
    uint64_t *d_tsum = nullptr;
    size_t tsum_cap = 0;
    unsigned long long *d_scratch = nullptr;
    // weight-window generations (grown on demand): staged copies, the next
    // generation's ordered sources, per history copy counts and offsets, the
    // staging fill counter
    SiteRec *d_gstage = nullptr, *d_gsrc = nullptr;
    size_t g_cap = 0;
    uint32_t *d_gn = nullptr;
    size_t gn_cap = 0;
    uint64_t *d_goff = nullptr;
    size_t goff_cap = 0;
    unsigned long long *d_gcount = nullptr;
    uint64_t *d_tot = nullptr;
    uint64_t *h_tot = nullptr;            // pinned
    // state
    bool tallies_valid = false;
    bool have_forward = false;
    std::vector<uint64_t> last_first, last_count;
    unsigned long long passa_u = 0;       // single-problem pass A bound (summed stripes)
    std::vector<uint32_t> round_in;       // stack: input particles of each round of the last pass
    void *scratch = nullptr;              // this device's copy of the static scratch
    mcx_counters_t counters{};
    std::string err;
};

static mcx_status fail(mcx_problem_t p, mcx_status s, const char *fmt, ...)
{
    if (p) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        p->err = buf;
    }
    return s;
}

static mcx_status hip_fail(mcx_problem_t p, hipError_t e, const char *where)
{
    return fail(p, e == hipErrorOutOfMemory ? MCX_E_OOM : MCX_E_DEVICE, "%s: %s", where, hipGetErrorString(e));
}

#define HIP_TRY(p, call)                                    \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail(p, e_, #call); \
    } while (0)

// Default tally paths, from measurements on MI355X (1e6 histories: box with
// 2000 mesh bins, continuous-energy pin cell with 100 energy x 1..64 time
// bins, lattice with 364140 mesh bins): LDS sums are fastest up to 4096 bins,
// except for asynchronous launches with one-wavefront blocks, where each
// wavefront holds a copy (fused: faster up to about 2048 bins, split, with
// its larger stash: up to about 1024); replicas beat direct adds by 2-15x
// below 65536 bins and tie at 364140.
constexpr long long ASYNC_LDS_TALLY_BINS_FUSED = 2048;
constexpr long long ASYNC_LDS_TALLY_BINS_SPLIT = 1024;
constexpr long long AUTO_REPLICA_MAX_BINS = 1 << 16;

static bool sorted_strict(const double *a, int64_t n)
{
    for (int64_t i = 0; i + 1 < n; ++i)
        if (!(a[i] < a[i + 1])) return false;
    return true;
}

template <class T>
static std::vector<T> copy_of(const T *a, int64_t n)
{
    return std::vector<T>(a, a + n);
}

static int bit_length(unsigned long long u)
{
    int b = 0;
    while (u) {
        ++b;
        u >>= 1;
    }
    return b;
}

// largest i <= n-2 with g[i] <= e
static int host_bracket(const double *g, int n, double e)
{
    int i = (int)(std::upper_bound(g, g + n, e) - g) - 1;
    if (i < 0) i = 0;
    if (i > n - 2) i = n - 2;
    return i;
}

// n / (e[n] - e[0]) if the n+1 edges are uniform (in ln e when logscale) to
// within a tenth of a cell, else 0.
static double uniform_inverse(const double *e, int n, bool logscale)
{
    if (n < 1) return 0.0;
    if (logscale && !(e[0] > 0.0)) return 0.0;
    auto f = [&](int i) { return logscale ? std::log(e[i]) : e[i]; };
    double lo = f(0), hi = f(n);
    double w = (hi - lo) / n;
    if (!(w > 0.0)) return 0.0;
    for (int i = 1; i < n; ++i)
        if (std::fabs(f(i) - (lo + w * i)) > 0.1 * w) return 0.0;
    return (double)n / (hi - lo);
}

// Validate one descriptor and deep-copy its arrays.
static mcx_status import_problem(mcx_problem_t h, const mcx_problem_desc &d, int k, HostProblem &hp)
{
    hp.d = d;
    if (d.geometry != MCX_GEOM_BOX && d.geometry != MCX_GEOM_LATTICE)
        return fail(h, MCX_E_INVALID_ARG, "problem %d: bad geometry %d", k, d.geometry);
    if (d.energy_mode != MCX_MG && d.energy_mode != MCX_CE)
        return fail(h, MCX_E_INVALID_ARG, "problem %d: bad energy_mode", k);
    if (d.n_mat < 1) return fail(h, MCX_E_INVALID_ARG, "problem %d: n_mat < 1", k);
    for (int f = 0; f < 6; ++f)
        if (d.bc[f] != MCX_BC_VACUUM && d.bc[f] != MCX_BC_REFLECT)
            return fail(h, MCX_E_INVALID_ARG, "problem %d: bad boundary condition", k);
    for (int a = 0; a < 3; ++a)
        if (!(d.box_lo[a] < d.box_hi[a])) return fail(h, MCX_E_INVALID_ARG, "problem %d: empty box", k);
    if (d.geometry == MCX_GEOM_BOX) {
        if (d.n_slabs < 1 || d.n_slabs > 1023 || !d.slab_planes || !d.slab_mat)
            return fail(h, MCX_E_INVALID_ARG, "problem %d: n_slabs must be 1..1023", k);
        hp.xpl = copy_of(d.slab_planes, d.n_slabs + 1);
        if (!sorted_strict(hp.xpl.data(), d.n_slabs + 1) || hp.xpl[0] != d.box_lo[0] || hp.xpl[d.n_slabs] != d.box_hi[0])
            return fail(h, MCX_E_INVALID_ARG, "problem %d: slab planes must increase from box_lo.x to box_hi.x", k);
        if (!std::isfinite(d.box_lo[1]) || !std::isfinite(d.box_hi[1]) || !std::isfinite(d.box_lo[2]) ||
            !std::isfinite(d.box_hi[2]))
            return fail(h, MCX_E_INVALID_ARG, "problem %d: box faces must be finite", k);
        hp.cmat = copy_of(d.slab_mat, d.n_slabs);
        hp.ypl = {0.0};
        hp.cxs = {0.0};
        hp.cys = {0.0};
    } else {
        if (d.nx < 1 || d.ny < 1 || d.nx > 1023 || d.ny > 1023 || !d.xplanes || !d.yplanes || !d.cx || !d.cy ||
            !d.pin_mat)
            return fail(h, MCX_E_INVALID_ARG, "problem %d: lattice needs nx, ny in 1..1023 and its arrays", k);
        hp.xpl = copy_of(d.xplanes, d.nx + 1);
        hp.ypl = copy_of(d.yplanes, d.ny + 1);
        if (!sorted_strict(hp.xpl.data(), d.nx + 1) || !sorted_strict(hp.ypl.data(), d.ny + 1) ||
            hp.xpl[0] != d.box_lo[0] || hp.xpl[d.nx] != d.box_hi[0] || hp.ypl[0] != d.box_lo[1] ||
            hp.ypl[d.ny] != d.box_hi[1])
            return fail(h, MCX_E_INVALID_ARG, "problem %d: lattice planes must increase and span the box", k);
        hp.cxs = copy_of(d.cx, d.nx);
        hp.cys = copy_of(d.cy, d.ny);
        if (!(d.radius > 0.0)) return fail(h, MCX_E_INVALID_ARG, "problem %d: radius must be > 0", k);
        for (int i = 0; i < d.nx; ++i)
            if (!(hp.cxs[i] - d.radius > hp.xpl[i] && hp.cxs[i] + d.radius < hp.xpl[i + 1]))
                return fail(h, MCX_E_INVALID_ARG, "problem %d: pin %d crosses its cell in x", k, i);
        for (int j = 0; j < d.ny; ++j)
            if (!(hp.cys[j] - d.radius > hp.ypl[j] && hp.cys[j] + d.radius < hp.ypl[j + 1]))
                return fail(h, MCX_E_INVALID_ARG, "problem %d: pin %d crosses its cell in y", k, j);
        hp.cmat = copy_of(d.pin_mat, (int64_t)d.nx * d.ny);
        if (d.mod_mat < 0 || d.mod_mat >= d.n_mat) return fail(h, MCX_E_INVALID_ARG, "problem %d: bad mod_mat", k);
    }
    for (int32_t m : hp.cmat)
        if (m < 0 || m >= d.n_mat) return fail(h, MCX_E_INVALID_ARG, "problem %d: material index out of range", k);
    const int64_t MG = (int64_t)d.n_mat * d.n_grp;
    if (d.energy_mode == MCX_MG) {
        if (d.n_grp < 1 || d.n_grp > 255) return fail(h, MCX_E_INVALID_ARG, "problem %d: n_grp must be 1..255", k);
        if (!d.sigma_t || !d.sigma_s || !d.transfer_cdf)
            return fail(h, MCX_E_INVALID_ARG, "problem %d: missing multigroup tables", k);
        hp.sig_t = copy_of(d.sigma_t, MG);
        hp.sig_s = copy_of(d.sigma_s, MG);
        hp.cdf = copy_of(d.transfer_cdf, MG * d.n_grp);
        for (int64_t i = 0; i < MG; ++i)
            if (!(hp.sig_t[i] > 0.0 && hp.sig_s[i] >= 0.0 && hp.sig_s[i] <= hp.sig_t[i] && std::isfinite(hp.sig_t[i])))
                return fail(h, MCX_E_INVALID_ARG, "problem %d: need 0 <= sigma_s <= sigma_t, sigma_t > 0", k);
        for (int64_t r = 0; r < MG; ++r) {
            const double *row = hp.cdf.data() + r * d.n_grp;
            for (int g = 0; g + 1 < d.n_grp; ++g)
                if (!(row[g] >= 0.0 && row[g] <= row[g + 1]))
                    return fail(h, MCX_E_INVALID_ARG, "problem %d: transfer cdf rows must be non-decreasing", k);
            if (row[d.n_grp - 1] != 1.0)
                return fail(h, MCX_E_INVALID_ARG, "problem %d: transfer cdf rows must end at 1.0", k);
        }
        if (d.src_group < 0 || d.src_group >= d.n_grp) return fail(h, MCX_E_INVALID_ARG, "problem %d: bad src_group", k);
        hp.egrid = hp.siga = hp.sigs = hp.awr = hp.dens = {0.0};
        hp.hash_lo = hp.hash_hi = {0};
    } else {
        if (d.geometry != MCX_GEOM_LATTICE)
            return fail(h, MCX_E_INVALID_ARG, "problem %d: continuous energy needs the lattice geometry", k);
        if (d.n_species < 1 || d.n_species > MAX_SPECIES)
            return fail(h, MCX_E_INVALID_ARG, "problem %d: n_species must be 1..%d", k, (int)MAX_SPECIES);
        if (d.grid_len < 2 || !d.e_grid || !d.sig_a || !d.sig_s || !d.awr || !d.density)
            return fail(h, MCX_E_INVALID_ARG, "problem %d: missing continuous-energy tables", k);
        const int64_t SN = (int64_t)d.n_species * d.grid_len;
        hp.egrid = copy_of(d.e_grid, SN);
        hp.siga = copy_of(d.sig_a, SN);
        hp.sigs = copy_of(d.sig_s, SN);
        hp.awr = copy_of(d.awr, d.n_species);
        hp.dens = copy_of(d.density, (int64_t)d.n_mat * d.n_species);
        for (int s = 0; s < d.n_species; ++s) {
            if (!sorted_strict(hp.egrid.data() + (int64_t)s * d.grid_len, d.grid_len) || !(hp.egrid[(int64_t)s * d.grid_len] > 0.0))
                return fail(h, MCX_E_INVALID_ARG, "problem %d: energy grid %d must be positive and increasing", k, s);
            if (!(hp.awr[s] > 0.0)) return fail(h, MCX_E_INVALID_ARG, "problem %d: awr must be > 0", k);
        }
        for (int64_t i = 0; i < SN; ++i)
            if (!(hp.siga[i] >= 0.0 && hp.sigs[i] >= 0.0))
                return fail(h, MCX_E_INVALID_ARG, "problem %d: cross sections must be >= 0", k);
        for (double v : hp.dens)
            if (!(v >= 0.0)) return fail(h, MCX_E_INVALID_ARG, "problem %d: densities must be >= 0", k);
        if (!(d.e_min > 0.0) || !(d.e_source > 0.0))
            return fail(h, MCX_E_INVALID_ARG, "problem %d: e_min and e_source must be > 0", k);
        hp.sig_t = hp.sig_s = hp.cdf = {1.0};
        // hashed grid: uniform bins in ln E over the union of the grids
        double lo = hp.egrid[0], hi = hp.egrid[d.grid_len - 1];
        for (int s = 1; s < d.n_species; ++s) {
            lo = std::min(lo, hp.egrid[(int64_t)s * d.grid_len]);
            hi = std::max(hi, hp.egrid[(int64_t)s * d.grid_len + d.grid_len - 1]);
        }
        int M = d.hash_bins > 0 ? d.hash_bins : std::max(64, d.grid_len / 8);
        hp.hash_bins = M;
        hp.hash_ln_lo = std::log(lo);
        hp.hash_inv = (double)M / (std::log(hi) - std::log(lo));
        hp.hash_lo.resize((size_t)d.n_species * M);
        hp.hash_hi.resize((size_t)d.n_species * M);
        for (int s = 0; s < d.n_species; ++s) {
            const double *g = hp.egrid.data() + (int64_t)s * d.grid_len;
            for (int b = 0; b < M; ++b) {
                double e0 = std::exp(hp.hash_ln_lo + (double)b / hp.hash_inv);
                double e1 = std::exp(hp.hash_ln_lo + (double)(b + 1) / hp.hash_inv);
                int l = host_bracket(g, d.grid_len, e0) - 1;
                int u = host_bracket(g, d.grid_len, e1) + 2;
                hp.hash_lo[(size_t)s * M + b] = std::max(l, 0);
                hp.hash_hi[(size_t)s * M + b] = std::min(u, d.grid_len - 1);
            }
        }
    }
    if (d.src_kind < MCX_SRC_POINT || d.src_kind > MCX_SRC_DISC)
        return fail(h, MCX_E_INVALID_ARG, "problem %d: bad src_kind", k);
    if (d.tally_kind == MCX_TALLY_MESH) {
        for (int a = 0; a < 3; ++a)
            if (d.mesh_n[a] < 1) return fail(h, MCX_E_INVALID_ARG, "problem %d: mesh_n must be >= 1", k);
        if (!d.mesh_x || !d.mesh_y || !d.mesh_z) return fail(h, MCX_E_INVALID_ARG, "problem %d: missing mesh edges", k);
        hp.mx = copy_of(d.mesh_x, d.mesh_n[0] + 1);
        hp.my = copy_of(d.mesh_y, d.mesh_n[1] + 1);
        hp.mz = copy_of(d.mesh_z, d.mesh_n[2] + 1);
        if (!sorted_strict(hp.mx.data(), d.mesh_n[0] + 1) || !sorted_strict(hp.my.data(), d.mesh_n[1] + 1) ||
            !sorted_strict(hp.mz.data(), d.mesh_n[2] + 1))
            return fail(h, MCX_E_INVALID_ARG, "problem %d: mesh edges must increase", k);
        // the mesh must contain the box: track outside it would have no bin
        const std::vector<double> *edges[3] = {&hp.mx, &hp.my, &hp.mz};
        for (int a = 0; a < 3; ++a)
            if (!(edges[a]->front() <= d.box_lo[a] && edges[a]->back() >= d.box_hi[a]))
                return fail(h, MCX_E_INVALID_ARG, "problem %d: mesh edges must contain the box", k);
        hp.n_bins = (int64_t)d.mesh_n[0] * d.mesh_n[1] * d.mesh_n[2] * (d.energy_mode == MCX_MG ? d.n_grp : 1);
        hp.eedges = {0.0, 1.0};
    } else if (d.tally_kind == MCX_TALLY_ENERGY) {
        if (d.n_ebins < 1 || !d.e_edges) return fail(h, MCX_E_INVALID_ARG, "problem %d: n_ebins must be >= 1", k);
        hp.eedges = copy_of(d.e_edges, d.n_ebins + 1);
        if (!sorted_strict(hp.eedges.data(), d.n_ebins + 1))
            return fail(h, MCX_E_INVALID_ARG, "problem %d: energy edges must increase", k);
        // energies stay in [e_min, e_source] (elastic scattering only loses
        // energy; histories end below e_min): the edges must contain them
        // (the last bin holds its upper edge)
        if (d.energy_mode == MCX_CE && !(hp.eedges.front() <= d.e_min && d.e_source <= hp.eedges.back()))
            return fail(h, MCX_E_INVALID_ARG, "problem %d: energy edges must contain [e_min, e_source]", k);
        hp.n_bins = d.n_ebins;
        hp.mx = hp.my = hp.mz = {0.0, 1.0};
    } else {
        return fail(h, MCX_E_INVALID_ARG, "problem %d: bad tally_kind", k);
    }
    hp.sigf = hp.nu = hp.chi = {0.0};
    if (d.sigma_f) {
        if (d.energy_mode != MCX_MG)
            return fail(h, MCX_E_INVALID_ARG, "problem %d: fission data needs a multigroup problem", k);
        if (!d.nu || !d.chi) return fail(h, MCX_E_INVALID_ARG, "problem %d: fission needs nu and chi", k);
        hp.sigf = copy_of(d.sigma_f, MG);
        hp.nu = copy_of(d.nu, MG);
        hp.chi = copy_of(d.chi, MG);
        for (int64_t i = 0; i < MG; ++i) {
            if (!(hp.sigf[i] >= 0.0 && hp.sigf[i] <= hp.sig_t[i] - hp.sig_s[i]))
                return fail(h, MCX_E_INVALID_ARG, "problem %d: need 0 <= sigma_f <= sigma_t - sigma_s", k);
            if (!(hp.nu[i] >= 0.0 && hp.nu[i] < 15.0))
                return fail(h, MCX_E_INVALID_ARG, "problem %d: need 0 <= nu < 15", k);
        }
        for (int m = 0; m < d.n_mat; ++m) {
            const double *row = hp.chi.data() + (int64_t)m * d.n_grp;
            for (int g = 0; g < d.n_grp; ++g)
                if (!(row[g] >= 0.0 && row[g] <= 1.0 && (g == 0 || row[g - 1] <= row[g])))
                    return fail(h, MCX_E_INVALID_ARG, "problem %d: chi rows must be non-decreasing in [0, 1]", k);
            if (row[d.n_grp - 1] != 1.0) return fail(h, MCX_E_INVALID_ARG, "problem %d: chi rows must end at 1.0", k);
        }
        hp.fission = true;
    }
    if (d.implicit_capture != 0 && d.implicit_capture != 1)
        return fail(h, MCX_E_INVALID_ARG, "problem %d: implicit_capture must be 0 or 1", k);
    if (d.implicit_capture &&
        !(d.w_cutoff >= 0.0 && d.w_survival > 0.0 && d.w_cutoff <= d.w_survival && std::isfinite(d.w_survival)))
        return fail(h, MCX_E_INVALID_ARG, "problem %d: need 0 <= w_cutoff <= w_survival, w_survival > 0", k);
    hp.wwlo = {0.0};
    if (d.ww_n[0] > 0) {
        for (int a = 0; a < 3; ++a)
            if (d.ww_n[a] < 1 || d.ww_n[a] > 4096 || !std::isfinite(d.box_lo[a]) || !std::isfinite(d.box_hi[a]))
                return fail(h, MCX_E_INVALID_ARG, "problem %d: weight windows need 1..4096 cells per axis and a finite box", k);
        if (!d.ww_lo) return fail(h, MCX_E_INVALID_ARG, "problem %d: weight windows need ww_lo", k);
        if (!(d.ww_ratio > d.ww_surv && d.ww_surv > 1.0 && std::isfinite(d.ww_ratio)) || d.ww_max_split < 2)
            return fail(h, MCX_E_INVALID_ARG, "problem %d: weight windows need ww_ratio > ww_surv > 1, ww_max_split >= 2", k);
        const int64_t nw = (int64_t)d.ww_n[0] * d.ww_n[1] * d.ww_n[2];
        if (nw > (1 << 24)) return fail(h, MCX_E_INVALID_ARG, "problem %d: at most 2^24 weight-window cells", k);
        hp.wwlo = copy_of(d.ww_lo, nw);
        for (double v : hp.wwlo)
            if (!(v >= 0.0 && std::isfinite(v)))
                return fail(h, MCX_E_INVALID_ARG, "problem %d: weight-window bounds must be finite and >= 0", k);
        hp.ww = true;
    }
    hp.nbase = hp.n_bins;
    hp.speed = {1.0};
    if (d.n_tbins < 0 || d.n_tbins > (1 << 20))
        return fail(h, MCX_E_INVALID_ARG, "problem %d: n_tbins must be 0..%d", k, 1 << 20);
    if (d.n_tbins > 0) {
        if (!(d.t_max > 0.0) || !std::isfinite(d.t_max))
            return fail(h, MCX_E_INVALID_ARG, "problem %d: t_max must be finite and > 0", k);
        if (d.energy_mode == MCX_MG) {
            if (!d.speed) return fail(h, MCX_E_INVALID_ARG, "problem %d: time bins need group speeds", k);
            hp.speed = copy_of(d.speed, d.n_grp);
            for (double v : hp.speed)
                if (!(v > 0.0) || !std::isfinite(v))
                    return fail(h, MCX_E_INVALID_ARG, "problem %d: speeds must be finite and > 0", k);
        } else if (!(d.speed_coef > 0.0) || !std::isfinite(d.speed_coef)) {
            return fail(h, MCX_E_INVALID_ARG, "problem %d: speed_coef must be finite and > 0", k);
        }
        hp.n_bins *= d.n_tbins;
    }
    if (d.tally_scale_log2 < 0 || d.tally_scale_log2 > 62)
        return fail(h, MCX_E_INVALID_ARG, "problem %d: tally_scale_log2 must be 0..62", k);
    if (d.n_histories >= (1ull << 32)) return fail(h, MCX_E_INVALID_ARG, "problem %d: at most 2^32-1 histories", k);
    if (d.max_steps < 0) return fail(h, MCX_E_INVALID_ARG, "problem %d: max_steps must be >= 0", k);
    hp.d.max_steps = d.max_steps == 0 ? 1000000 : d.max_steps;
    if (hp.d.max_steps >= (int64_t)0xFFFFFFFFll) hp.d.max_steps = 0xFFFFFFFEll;
    return MCX_OK;
}

// Device blob layout: every array 256-byte aligned.
struct BlobBuilder {
    std::vector<char> bytes;
    template <class T>
    size_t add(const std::vector<T> &v)
    {
        size_t off = (bytes.size() + 255) / 256 * 256;
        bytes.resize(off + v.size() * sizeof(T));
        std::memcpy(bytes.data() + off, v.data(), v.size() * sizeof(T));
        return off;
    }
};

static mcx_status upload(mcx_problem_t h)
{
    BlobBuilder bb;
    struct Offs {
        size_t xpl, ypl, cxs, cys, cmat, sig_t, sig_s, cdf, egrid, siga, sigs, awr, dens, hlo, hhi, mx, my, mz, ee;
        size_t speed, sigf, nu, chi, wwlo;
    };
    std::vector<Offs> off(h->n);
    std::vector<size_t> tl_base(h->n), tl_bytes(h->n);
    std::vector<std::array<int32_t, 15>> tl_off(h->n);
    for (int k = 0; k < h->n; ++k) {
        HostProblem &p = h->hp[k];
        Offs &o = off[k];
        // the small per-event tables, packed: doubles, then the int32 materials
        const std::vector<double> *dt[TL_NDBL] = {&p.sig_t, &p.sig_s, &p.cdf,   &p.xpl, &p.ypl,
                                                  &p.cxs,   &p.cys,   &p.mx,    &p.my,  &p.mz,
                                                  &p.speed, &p.sigf,  &p.nu,    &p.chi};
        std::vector<double> packed;
        for (int t = 0; t < TL_NDBL; ++t) {
            tl_off[k][t] = (int32_t)packed.size();
            packed.insert(packed.end(), dt[t]->begin(), dt[t]->end());
        }
        tl_off[k][TL_CMAT] = (int32_t)(2 * packed.size());
        size_t nd = packed.size();
        packed.resize(nd + (p.cmat.size() + 1) / 2);
        if (!p.cmat.empty()) std::memcpy(packed.data() + nd, p.cmat.data(), p.cmat.size() * 4);
        if (packed.size() % 2) packed.push_back(0.0);   // 16-byte multiple
        tl_base[k] = bb.add(packed);
        tl_bytes[k] = packed.size() * 8;
        size_t b = tl_base[k];
        o.sig_t = b + 8 * (size_t)tl_off[k][TL_SIG_T]; o.sig_s = b + 8 * (size_t)tl_off[k][TL_SIG_S];
        o.cdf = b + 8 * (size_t)tl_off[k][TL_CDF]; o.xpl = b + 8 * (size_t)tl_off[k][TL_XPL];
        o.ypl = b + 8 * (size_t)tl_off[k][TL_YPL]; o.cxs = b + 8 * (size_t)tl_off[k][TL_CXS];
        o.cys = b + 8 * (size_t)tl_off[k][TL_CYS]; o.mx = b + 8 * (size_t)tl_off[k][TL_MX];
        o.my = b + 8 * (size_t)tl_off[k][TL_MY]; o.mz = b + 8 * (size_t)tl_off[k][TL_MZ];
        o.speed = b + 8 * (size_t)tl_off[k][TL_SPEED];
        o.sigf = b + 8 * (size_t)tl_off[k][TL_SIGF];
        o.nu = b + 8 * (size_t)tl_off[k][TL_NU];
        o.chi = b + 8 * (size_t)tl_off[k][TL_CHI];
        o.cmat = b + 4 * (size_t)tl_off[k][TL_CMAT];
        o.egrid = bb.add(p.egrid); o.siga = bb.add(p.siga); o.sigs = bb.add(p.sigs); o.awr = bb.add(p.awr);
        o.dens = bb.add(p.dens); o.hlo = bb.add(p.hash_lo); o.hhi = bb.add(p.hash_hi);
        o.ee = bb.add(p.eedges);
        o.wwlo = bb.add(p.wwlo);
    }
    HIP_TRY(h, hipMalloc(&h->blob, std::max<size_t>(bb.bytes.size(), 256)));
    HIP_TRY(h, hipMemcpy(h->blob, bb.bytes.data(), bb.bytes.size(), hipMemcpyHostToDevice));
    // tallies
    h->tally_off.resize(h->n);
    size_t tb = 0;
    for (int k = 0; k < h->n; ++k) {
        h->tally_off[k] = tb;
        tb += (size_t)h->hp[k].n_bins;
    }
    h->total_bins = tb;
    HIP_TRY(h, hipMalloc(&h->d_tally, std::max<size_t>(tb, 1) * 8));
    HIP_TRY(h, hipMemset(h->d_tally, 0, std::max<size_t>(tb, 1) * 8));
    // gradient accumulators: per problem U (1 word) + SL, SA, SS (3 MG words)
    h->gacc_off.resize(h->n);
    size_t gw = 0;
    for (int k = 0; k < h->n; ++k) {
        h->gacc_off[k] = gw;
        gw += 1 + 3 * (size_t)h->hp[k].d.n_mat * h->hp[k].d.n_grp;
    }
    h->gacc_words = gw;
    HIP_TRY(h, hipMalloc(&h->d_gacc, gw * 8));
    HIP_TRY(h, hipMalloc(&h->d_probs, sizeof(ProbDev) * h->n));
    HIP_TRY(h, hipMalloc(&h->d_prefix, sizeof(unsigned long long) * (h->n + 1)));
    HIP_TRY(h, hipMalloc(&h->d_ctl, sizeof(RunCtl)));
    HIP_TRY(h, hipHostMalloc((void **)&h->h_flag, 64, hipHostMallocDefault));
    HIP_TRY(h, hipHostMalloc((void **)&h->h_ctl, sizeof(RunCtl), hipHostMallocDefault));
    for (hipEvent_t &ev : h->poll) HIP_TRY(h, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    h->run_prefix.assign(h->n + 1, 0);
    h->round_in.reserve(STACK_ROUND_LOG);
    h->run_first.assign(h->n, 0);
    h->run_count.assign(h->n, 0);
    // host image of the problem table (static part)
    char *base = (char *)h->blob;
    h->pd.resize(h->n);
    for (int k = 0; k < h->n; ++k) {
        HostProblem &hp = h->hp[k];
        const mcx_problem_desc &d = hp.d;
        Offs &o = off[k];
        ProbDev &P = h->pd[k];
        std::memset(&P, 0, sizeof P);
        P.geometry = d.geometry;
        P.n_slabs = d.geometry == MCX_GEOM_BOX ? d.n_slabs : 0;
        P.nx = d.geometry == MCX_GEOM_LATTICE ? d.nx : 0;
        P.ny = d.geometry == MCX_GEOM_LATTICE ? d.ny : 0;
        P.mod_mat = d.mod_mat;
        P.refl_mask = 0;
        for (int f = 0; f < 6; ++f)
            if (d.bc[f] == MCX_BC_REFLECT) P.refl_mask |= 1 << f;
        for (int a = 0; a < 3; ++a) {
            P.box_lo[a] = d.box_lo[a];
            P.box_hi[a] = d.box_hi[a];
        }
        P.radius = d.radius;
        P.r2 = d.radius * d.radius;
        P.xpl = (const double *)(base + o.xpl);
        P.ypl = (const double *)(base + o.ypl);
        P.cxs = (const double *)(base + o.cxs);
        P.cys = (const double *)(base + o.cys);
        P.cmat = (const int32_t *)(base + o.cmat);
        P.n_mat = d.n_mat;
        P.n_grp = d.energy_mode == MCX_MG ? d.n_grp : 1;
        P.sig_t = (const double *)(base + o.sig_t);
        P.sig_s = (const double *)(base + o.sig_s);
        P.cdf = (const double *)(base + o.cdf);
        P.n_species = d.energy_mode == MCX_CE ? d.n_species : 0;
        P.grid_len = d.energy_mode == MCX_CE ? d.grid_len : 0;
        P.egrid = (const double *)(base + o.egrid);
        P.siga = (const double *)(base + o.siga);
        P.sigs = (const double *)(base + o.sigs);
        P.awr = (const double *)(base + o.awr);
        P.dens = (const double *)(base + o.dens);
        P.e_min = d.e_min;
        P.e_src = d.e_source;
        P.hash_bins = hp.hash_bins;
        P.hash_ln_lo = hp.hash_ln_lo;
        P.hash_inv = hp.hash_inv;
        P.hash_lo = (const int32_t *)(base + o.hlo);
        P.hash_hi = (const int32_t *)(base + o.hhi);
        P.src_kind = d.src_kind;
        P.src_iso = d.src_isotropic ? 1 : 0;
        P.src_group = d.energy_mode == MCX_MG ? d.src_group : 0;
        P.tally_kind = d.tally_kind;
        for (int a = 0; a < 3; ++a) {
            P.src_pos[a] = d.src_pos[a];
            P.src_lo[a] = d.src_lo[a];
            P.src_ext[a] = d.src_hi[a] - d.src_lo[a];
            P.src_dir[a] = d.src_dir[a];
            P.mesh_n[a] = d.tally_kind == MCX_TALLY_MESH ? d.mesh_n[a] : 1;
        }
        P.src_radius = d.src_radius;
        P.n_ebins = d.tally_kind == MCX_TALLY_ENERGY ? d.n_ebins : 1;
        P.mx = (const double *)(base + o.mx);
        P.my = (const double *)(base + o.my);
        P.mz = (const double *)(base + o.mz);
        P.eedges = (const double *)(base + o.ee);
        // guesses for uniform mesh axes and log-uniform energy bins (only a
        // starting point: the device corrects it against the edges)
        const std::vector<double> *axes[3] = {&hp.mx, &hp.my, &hp.mz};
        for (int a = 0; a < 3; ++a) {
            const std::vector<double> &e = *axes[a];
            int n = (int)e.size() - 1;
            P.mesh_lo[a] = e[0];
            P.mesh_inv[a] = uniform_inverse(e.data(), n, false);
        }
        P.ebin_lnlo = hp.eedges[0] > 0.0 ? std::log(hp.eedges[0]) : 0.0;
        P.ebin_inv = d.tally_kind == MCX_TALLY_ENERGY ? uniform_inverse(hp.eedges.data(), d.n_ebins, true) : 0.0;
        P.tscale = std::ldexp(1.0, d.tally_scale_log2);
        P.tally = h->d_tally + h->tally_off[k];
        P.key0 = (uint32_t)d.seed;
        P.key1 = (uint32_t)(d.seed >> 32) ^ d.problem_id;
        P.max_steps = hp.d.max_steps;
        unsigned long long *ga = h->d_gacc + h->gacc_off[k];
        size_t mg = (size_t)P.n_mat * P.n_grp;
        P.U = ga;
        P.SL = ga + 1;
        P.SA = ga + 1 + mg;
        P.SS = ga + 1 + 2 * mg;
        P.tl_src = (const double *)(base + tl_base[k]);
        P.tl_bytes = (int32_t)std::min<size_t>(tl_bytes[k], 1u << 30);
        for (int t = 0; t < 15; ++t) P.tl_off[t] = tl_off[k][t];
        P.sigf = (const double *)(base + o.sigf);
        P.nu = (const double *)(base + o.nu);
        P.chi = (const double *)(base + o.chi);
        P.n_tbins = d.n_tbins;
        P.t_max = d.n_tbins > 0 ? d.t_max : 0.0;
        P.tw = d.n_tbins > 0 ? d.t_max / (double)d.n_tbins : 0.0;
        P.speed_coef = d.speed_coef;
        P.nbase = hp.nbase;
        P.n_bins = hp.n_bins;
        P.speed = (const double *)(base + o.speed);
        P.implicit = d.implicit_capture ? 1 : 0;
        P.w_cut = d.implicit_capture ? d.w_cutoff : 0.0;
        P.w_surv = d.implicit_capture ? d.w_survival : 1.0;
        P.ww_lo = (const double *)(base + o.wwlo);
        for (int a = 0; a < 3; ++a) {
            P.ww_n[a] = hp.ww ? d.ww_n[a] : 0;
            P.ww_inv[a] = hp.ww ? (double)d.ww_n[a] / (d.box_hi[a] - d.box_lo[a]) : 0.0;
        }
        P.ww_ratio = hp.ww ? d.ww_ratio : 0.0;
        P.ww_surv = hp.ww ? d.ww_surv : 0.0;
        P.ww_max_split = hp.ww ? d.ww_max_split : 0;
    }
    return MCX_OK;
}

// Once per device, with that device current: the device address of the
// static scratch.
static mcx_status scratch_setup(mcx_problem_t h)
{
    if (h->device < 0 || h->device >= SCRATCH_MAX_DEVICES)
        return fail(h, MCX_E_DEVICE, "device %d: at most %d devices", h->device, SCRATCH_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_addr[h->device]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(h, e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(h, MCX_E_DEVICE, "hipGetSymbolAddress(scratch) gave a null address");
        scratch_addr[h->device] = ptr;
    }
    h->scratch = scratch_addr[h->device];
    return MCX_OK;
}

extern "C" mcx_status mcx_create_problem(const mcx_problem_desc *descs, int32_t n_problems, mcx_problem_t *out)
{
    if (!out) return MCX_E_INVALID_ARG;
    *out = nullptr;
    if (!descs || n_problems < 1) return MCX_E_INVALID_ARG;
    mcx_problem_t h = new mcx_problem_s();
    h->n = n_problems;
    h->hp.resize(n_problems);
    mcx_status s = MCX_OK;
    for (int k = 0; k < n_problems && s == MCX_OK; ++k) s = import_problem(h, descs[k], k, h->hp[k]);
    if (s == MCX_OK) {
        h->geom = descs[0].geometry;
        h->emode = descs[0].energy_mode;
        h->tally_kind = descs[0].tally_kind;
        for (int k = 1; k < n_problems; ++k)
            if (descs[k].geometry != h->geom || descs[k].energy_mode != h->emode || descs[k].tally_kind != h->tally_kind)
                s = fail(h, MCX_E_INVALID_ARG, "problems of one handle must share geometry, energy mode and tally kind");
        for (int k = 0; k < n_problems && s == MCX_OK && n_problems > 1; ++k)
            if (h->hp[k].ww) s = fail(h, MCX_E_INVALID_ARG, "weight windows run as single problems, not in batches");
    }
    if (s == MCX_OK) {
        hipError_t e = hipGetDevice(&h->device);
        hipDeviceProp_t prop;
        if (e == hipSuccess) e = hipGetDeviceProperties(&prop, h->device);
        if (e != hipSuccess) s = hip_fail(h, e, "hipGetDeviceProperties");
        else h->num_cus = prop.multiProcessorCount;
        if (e == hipSuccess && hipDeviceGetAttribute(&h->wall_clock_khz, hipDeviceAttributeWallClockRate, h->device) !=
                                   hipSuccess)
            h->wall_clock_khz = 0;   // launchers then assume 100 MHz
    }
    if (s == MCX_OK) s = scratch_setup(h);
    if (s == MCX_OK) s = upload(h);
    if (s != MCX_OK) {
        mcx_destroy_problem(h);
        return s;
    }
    *out = h;
    return MCX_OK;
}

extern "C" void mcx_destroy_problem(mcx_problem_t h)
{
    if (!h) return;
    if (h->blob) hipFree(h->blob);
    if (h->d_probs) hipFree(h->d_probs);
    if (h->d_prefix) hipFree(h->d_prefix);
    if (h->d_tally) hipFree(h->d_tally);
    if (h->d_trep) hipFree(h->d_trep);
    for (auto &ev : h->timer_events) {
        hipEventDestroy(ev.first);
        hipEventDestroy(ev.second);
    }
    for (hipEvent_t ev : h->poll)
        if (ev) hipEventDestroy(ev);
    if (h->d_ctl) hipFree(h->d_ctl);
    if (h->d_G) hipFree(h->d_G);
    if (h->d_w) hipFree(h->d_w);
    if (h->d_gacc) hipFree(h->d_gacc);
    if (h->h_flag) hipHostFree(h->h_flag);
    if (h->h_ctl) hipHostFree(h->h_ctl);
    if (h->ws.ptr) hipFree(h->ws.ptr);
    for (double *b : h->d_sbank)
        if (b) hipFree(b);
    if (h->d_fn) hipFree(h->d_fn);
    if (h->d_fpos) hipFree(h->d_fpos);
    if (h->d_sites) hipFree(h->d_sites);
    if (h->d_tsum) hipFree(h->d_tsum);
    if (h->d_scratch) hipFree(h->d_scratch);
    if (h->d_gstage) hipFree(h->d_gstage);
    if (h->d_gsrc) hipFree(h->d_gsrc);
    if (h->d_gn) hipFree(h->d_gn);
    if (h->d_goff) hipFree(h->d_goff);
    if (h->d_gcount) hipFree(h->d_gcount);
    if (h->d_tot) hipFree(h->d_tot);
    if (h->h_tot) hipHostFree(h->h_tot);
    delete h;
}

extern "C" mcx_status mcx_set_xs(mcx_problem_t h, int32_t problem, const double *sigma_t, const double *sigma_s,
                                 int32_t where)
{
    if (!h) return MCX_E_INVALID_ARG;
    if (problem < 0 || problem >= h->n) return fail(h, MCX_E_INVALID_ARG, "bad problem index");
    HostProblem &hp = h->hp[problem];
    if (hp.d.energy_mode != MCX_MG) return fail(h, MCX_E_INVALID_ARG, "mcx_set_xs needs a multigroup problem");
    size_t mg = (size_t)hp.d.n_mat * hp.d.n_grp;
    std::vector<double> st(mg), ss(mg);
    if (!sigma_t || !sigma_s) return fail(h, MCX_E_INVALID_ARG, "null cross-section pointer");
    if (where == MCX_DEVICE) {
        HIP_TRY(h, hipMemcpy(st.data(), sigma_t, mg * 8, hipMemcpyDeviceToHost));
        HIP_TRY(h, hipMemcpy(ss.data(), sigma_s, mg * 8, hipMemcpyDeviceToHost));
    } else {
        std::memcpy(st.data(), sigma_t, mg * 8);
        std::memcpy(ss.data(), sigma_s, mg * 8);
    }
    for (size_t i = 0; i < mg; ++i)
        if (!(st[i] > 0.0 && ss[i] >= 0.0 && ss[i] <= st[i] && std::isfinite(st[i])))
            return fail(h, MCX_E_INVALID_ARG, "need 0 <= sigma_s <= sigma_t, sigma_t > 0");
    if (hp.fission)
        for (size_t i = 0; i < mg; ++i)
            if (!(hp.sigf[i] <= st[i] - ss[i]))
                return fail(h, MCX_E_INVALID_ARG, "need sigma_f <= sigma_t - sigma_s");
    HIP_TRY(h, hipMemcpy((void *)h->pd[problem].sig_t, st.data(), mg * 8, hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy((void *)h->pd[problem].sig_s, ss.data(), mg * 8, hipMemcpyHostToDevice));
    hp.sig_t = st;
    hp.sig_s = ss;
    h->have_forward = false;
    return MCX_OK;
}

hipError_t mcx::ws_reserve(Workspace &ws, size_t bytes)
{
    if (ws.bytes >= bytes) return hipSuccess;
    if (ws.fixed) return hipErrorInvalidValue;   // never reallocated (sizes are checked before)
    if (ws.ptr) {
        hipError_t e = hipFree(ws.ptr);
        if (e != hipSuccess) return e;
        ws.ptr = nullptr;
        ws.bytes = 0;
    }
    hipError_t e = hipMalloc(&ws.ptr, bytes);
    if (e == hipSuccess) ws.bytes = bytes;
    return e;
}

static mcx_status check_opts(mcx_problem_t h, const mcx_run_opts &o)
{
    if (o.sched < MCX_SCHED_NAIVE || o.sched > MCX_SCHED_ASYNC) return fail(h, MCX_E_INVALID_ARG, "bad sched");
    if (o.decomp != MCX_DECOMP_FUSED && o.decomp != MCX_DECOMP_SPLIT) return fail(h, MCX_E_INVALID_ARG, "bad decomp");
    if (o.lookup != MCX_LOOKUP_BINARY && o.lookup != MCX_LOOKUP_HASH) return fail(h, MCX_E_INVALID_ARG, "bad lookup");
    if (o.sched == MCX_SCHED_NAIVE && o.decomp == MCX_DECOMP_SPLIT)
        return fail(h, MCX_E_INVALID_ARG, "the naive scheduler runs whole histories (fused only)");
    if (o.stack_capacity < 0 || o.stack_threshold < 0 || o.stash_links < 0 || o.arena_links < 0 ||
        o.waves_per_cu < 0 || o.block_size < 0 || o.force_spill < 0 || o.stack_tail_events < 0 ||
        o.stack_min_events < 0)
        return fail(h, MCX_E_INVALID_ARG, "negative tuning value");
    if (o.consolidate < 0 || o.consolidate > 2) return fail(h, MCX_E_INVALID_ARG, "bad consolidate");
    if (o.async_block_waves != 0 && o.async_block_waves != 1 && o.async_block_waves != 2 &&
        o.async_block_waves != 4)
        return fail(h, MCX_E_INVALID_ARG, "async_block_waves must be 0, 1, 2 or 4");
    if (o.async_shared_stash < 0 || o.async_shared_stash > 2)
        return fail(h, MCX_E_INVALID_ARG, "async_shared_stash must be 0, 1 or 2");
    if (o.async_drain_events < 0 || o.async_drain_events > 1024)
        return fail(h, MCX_E_INVALID_ARG, "async_drain_events must be in [0, 1024]");
    if (o.async_bulk_events < 0 || o.async_bulk_events > 1024)
        return fail(h, MCX_E_INVALID_ARG, "async_bulk_events must be in [0, 1024]");
    if (o.stack_bulk_events < 0 || o.stack_bulk_events > 1024)
        return fail(h, MCX_E_INVALID_ARG, "stack_bulk_events must be in [0, 1024]");
    if (o.workspace && ((uintptr_t)o.workspace % 256) != 0)
        return fail(h, MCX_E_INVALID_ARG, "workspace must be 256-byte aligned");
    if (o.workspace && o.ws_bytes == 0) return fail(h, MCX_E_INVALID_ARG, "workspace given with ws_bytes 0");
    if (o.tally_path < MCX_TALLY_PATH_AUTO || o.tally_path > MCX_TALLY_PATH_DIRECT)
        return fail(h, MCX_E_INVALID_ARG, "bad tally_path");
    if (o.tally_path == MCX_TALLY_PATH_LDS && h->hp[0].n_bins > LT_MAX_BINS)
        return fail(h, MCX_E_INVALID_ARG, "tally_path LDS needs at most %d bins", LT_MAX_BINS);
    if (o.tally_path == MCX_TALLY_PATH_REPLICAS && h->hp[0].n_bins > TREP_MAX_BINS)
        return fail(h, MCX_E_INVALID_ARG, "tally_path REPLICAS needs at most %lld bins", TREP_MAX_BINS);
    return MCX_OK;
}

// tally[b] += sum over replicas r of rep[r][b] (exact: int64 bits, wrapping)
__global__ void trep_reduce(unsigned long long *tally, const unsigned long long *rep, int n, int nrep)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    unsigned long long v = 0;
    for (int r = 0; r < nrep; ++r) v += rep[(size_t)r * n + b];
    tally[b] += v;
}

// Where a run's tally adds go.  Single-problem forward runs: a small tally is
// summed per block in LDS, a larger one spread over replicas (on MI355X every
// device-scope atomic is carried out at the memory side, so the adds of all
// wavefronts to a few hot words serialise there), a very large one, whose
// adds are spread anyway, is added directly.  Batches and backward passes add
// directly.
static int tally_path(mcx_problem_t h, const mcx_run_opts &o, int mode)
{
    if (h->n != 1 || mode != MODE_FWD) return MCX_TALLY_PATH_DIRECT;
    if (o.tally_path != MCX_TALLY_PATH_AUTO) return o.tally_path;
    const long long nb = h->hp[0].n_bins;
    long long lds_max = LT_MAX_BINS;
    const int wpb = o.async_block_waves > 0 ? o.async_block_waves : ASYNC_BLOCK_WAVES;
    if (o.sched == MCX_SCHED_ASYNC && wpb == 1)
        lds_max = o.decomp == MCX_DECOMP_SPLIT ? ASYNC_LDS_TALLY_BINS_SPLIT : ASYNC_LDS_TALLY_BINS_FUSED;
    if (nb <= lds_max) return MCX_TALLY_PATH_LDS;
    if (nb <= AUTO_REPLICA_MAX_BINS) return MCX_TALLY_PATH_REPLICAS;
    return MCX_TALLY_PATH_DIRECT;
}

// Launch description of one pass (scheduler-independent fields and tuning).
static LaunchArgs launch_args(mcx_problem_t h, const mcx_run_opts &o, int mode, unsigned long long total, int path,
                              void *digest)
{
    LaunchArgs a{};
    a.probs = h->d_probs;
    a.n_probs = h->n;
    a.prefix = h->d_prefix;
    a.total = total;
    a.ctl = h->d_ctl;
    a.digest = digest;
    a.geom = h->geom;
    a.emode = h->emode;
    a.mode = mode;
    a.split = o.decomp == MCX_DECOMP_SPLIT ? 1 : 0;
    a.ext = 0;
    for (int k = 0; k < h->n; ++k)
        if (h->pd[k].n_tbins > 0 || h->pd[k].implicit || h->pd[k].ww_n[0] > 0) a.ext = 1;
    a.lacc_words = 0;
    if (h->n == 1 && mode == MODE_REPLAY_B) a.lacc_words = 3 * h->pd[0].n_mat * h->pd[0].n_grp;
    if (path == MCX_TALLY_PATH_LDS) a.lacc_words = (int)h->hp[0].n_bins;
    a.tl_bytes = (h->n == 1 && h->pd[0].tl_bytes <= TL_MAX_BYTES) ? h->pd[0].tl_bytes : 0;
    a.stream = (hipStream_t)o.hip_stream;
    a.num_cus = h->num_cus;
    a.block_size = o.block_size;
    a.waves_per_cu = o.waves_per_cu;
    a.stack_capacity = o.stack_capacity;
    a.stack_threshold = o.stack_threshold;
    a.stash_links = o.stash_links;
    a.arena_links = o.arena_links;
    a.force_spill = o.force_spill;
    a.consolidate = o.consolidate;
    a.stack_tail_events = o.stack_tail_events;
    a.stack_min_events = o.stack_min_events;
    a.async_block_waves = o.async_block_waves;
    a.async_drain_events = o.async_drain_events;
    a.async_bulk_events = o.async_bulk_events;
    a.stack_bulk_events = o.stack_bulk_events;
    a.async_shared = o.async_shared_stash;
    a.ws_query = nullptr;
    a.poll[0] = h->poll[0];
    a.poll[1] = h->poll[1];
    a.wall_clock_khz = h->wall_clock_khz;
    return a;
}

static hipError_t launch_sched(const mcx_run_opts &o, const LaunchArgs &a, Workspace &ws, LaunchStats &st,
                               LaunchTimer &tm, unsigned int *host_flag)
{
    if (o.sched == MCX_SCHED_NAIVE) return launch_naive(a, st, tm);
    if (o.sched == MCX_SCHED_STACK) return launch_stack(a, ws, st, tm, host_flag);
    return launch_async(a, ws, st, tm);
}

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Device scratch of one pass: the scheduler's state (stack banks and
// counters, or the async link arena), then, 256-byte aligned, the tally
// replicas when the pass adds into them.
static mcx_status scratch_bytes(mcx_problem_t h, const mcx_run_opts &o, const LaunchArgs &a, int path,
                                size_t &sched_bytes, size_t &total_bytes)
{
    LaunchArgs q = a;
    size_t need = 0;
    q.ws_query = &need;
    LaunchStats st;
    LaunchTimer tm;
    Workspace none;
    hipError_t e = a.total > 0 ? launch_sched(o, q, none, st, tm, h->h_flag) : hipSuccess;
    if (e != hipSuccess) return hip_fail(h, e, "workspace query");
    sched_bytes = need;
    total_bytes = need;
    if (path == MCX_TALLY_PATH_REPLICAS) total_bytes = align256(need) + (size_t)TREP * (size_t)h->hp[0].n_bins * 8;
    return MCX_OK;
}

// One pass over the run's histories with the given mode.  `fixed` (or null)
// is device scratch that the pass must fit in and never reallocates: the
// caller's workspace or the library's static scratch; without it the handle's
// own workspace and replicas grow as needed.
static mcx_status run_pass(mcx_problem_t h, const mcx_run_opts &o, int mode, const std::vector<uint64_t> &first,
                           const std::vector<uint64_t> &count, void *digest, unsigned int *err_out,
                           Workspace *fixed = nullptr)
{
    hipStream_t stream = (hipStream_t)o.hip_stream;
    std::vector<unsigned long long> &prefix = h->run_prefix;
    prefix[0] = 0;
    for (int k = 0; k < h->n; ++k) {
        ProbDev &P = h->pd[k];
        P.first = first[k];
        P.count = count[k];
        P.gbase = prefix[k];
        P.lookup_hash = o.lookup == MCX_LOOKUP_HASH ? 1 : 0;
        P.trep = nullptr;
        prefix[k + 1] = prefix[k] + count[k];
    }
    unsigned long long total = prefix[h->n];
    const int path = tally_path(h, o, mode);
    const bool use_trep = path == MCX_TALLY_PATH_REPLICAS;
    LaunchArgs a = launch_args(h, o, mode, total, path, digest);
    Workspace *ws = &h->ws;
    unsigned long long *trep = nullptr;
    if (fixed) {
        size_t sched_b = 0, total_b = 0;
        mcx_status s = scratch_bytes(h, o, a, path, sched_b, total_b);
        if (s != MCX_OK) return s;
        if (total_b > fixed->bytes)
            return fail(h, MCX_E_INVALID_ARG, "the run needs %zu bytes of device scratch; the workspace holds %zu",
                        total_b, fixed->bytes);
        ws = fixed;
        if (use_trep) trep = (unsigned long long *)((char *)fixed->ptr + align256(sched_b));
    }
    if (use_trep && fixed) {
        HIP_TRY(h, hipMemsetAsync(trep, 0, (size_t)TREP * (size_t)h->hp[0].n_bins * 8, stream));
        h->pd[0].trep = trep;
    } else if (use_trep) {
        size_t words = (size_t)TREP * (size_t)h->hp[0].n_bins;
        if (h->trep_words < words) {
            if (h->d_trep) HIP_TRY(h, hipFree(h->d_trep));
            h->d_trep = nullptr;
            h->trep_words = 0;
            HIP_TRY(h, hipMalloc(&h->d_trep, words * 8));
            h->trep_words = words;
        }
        HIP_TRY(h, hipMemsetAsync(h->d_trep, 0, words * 8, stream));
        h->pd[0].trep = h->d_trep;
    }
    HIP_TRY(h, hipMemcpyAsync(h->d_probs, h->pd.data(), sizeof(ProbDev) * h->n, hipMemcpyHostToDevice, stream));
    HIP_TRY(h, hipMemcpyAsync(h->d_prefix, prefix.data(), sizeof(unsigned long long) * (h->n + 1),
                              hipMemcpyHostToDevice, stream));
    RunCtl &ctl = *h->h_ctl;   // pinned host image of the control block
    std::memset(&ctl, 0, sizeof ctl);
    ctl.total = total;
    HIP_TRY(h, hipMemcpyAsync(h->d_ctl, &ctl, sizeof ctl, hipMemcpyHostToDevice, stream));

    LaunchStats st;
    LaunchTimer tm;
    tm.on = o.time_kernels != 0;
    tm.stream = stream;
    tm.pool = &h->timer_events;
    hipError_t e = hipSuccess;
    if (total > 0) {
        e = launch_sched(o, a, *ws, st, tm, h->h_flag);
        if (e == hipSuccess && use_trep) {
            int n = (int)h->hp[0].n_bins;
            hipLaunchKernelGGL(trep_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                               h->pd[0].tally, (const unsigned long long *)h->pd[0].trep, n, TREP);
            e = hipGetLastError();
        }
    }
    if (e != hipSuccess) {
        tm.total_ms();
        return hip_fail(h, e, "kernel launch");
    }
    HIP_TRY(h, hipMemcpyAsync(&ctl, h->d_ctl, sizeof ctl, hipMemcpyDeviceToHost, stream));
    HIP_TRY(h, hipStreamSynchronize(stream));
    unsigned long long tot[C_NUM] = {0};
    unsigned __int128 qsum = 0;
    for (int s = 0; s < CTL_STRIPES; ++s) {
        for (int i = 0; i < C_NUM; ++i) tot[i] += ctl.stripe[s].c[i];
        qsum += ctl.stripe[s].c[C_QSUM];
    }
    // overflow rule: the exact total of all contributions reached 2^63
    if (qsum >= ((unsigned __int128)1 << 63)) ctl.error |= ERR_OVERFLOW;
    mcx_counters_t &c = h->counters;
    std::memset(&c, 0, sizeof c);
    c.sourced = tot[C_SOURCED];
    c.flights = tot[C_FLIGHTS];
    c.collisions = tot[C_COLLISIONS];
    c.scatters = tot[C_SCATTERS];
    c.absorbs = tot[C_ABSORBS];
    c.crossings = tot[C_CROSSINGS];
    c.leaks = tot[C_LEAKS];
    c.reflections = tot[C_REFLECTIONS];
    c.cutoffs = tot[C_CUTOFFS];
    c.killed = tot[C_KILLED];
    c.pieces = tot[C_PIECES];
    c.qsum = (uint64_t)qsum;
    c.overflow = (ctl.error & ERR_OVERFLOW) ? 1 : 0;
    c.events = tot[C_EVENTS];
    c.lane_slots = tot[C_LANE_SLOTS];
    c.dispatches = tot[C_DISPATCHES];
    c.spills = tot[C_SPILLS];
    c.refills = tot[C_REFILLS];
    c.make_work = tot[C_MAKE_WORK];
    c.fissions = tot[C_FISSIONS];
    c.roulettes = tot[C_ROULETTES];
    c.cdf_scans = tot[C_CDF];
    c.splits = tot[C_SPLITS];
    c.generations = 1;
    c.rounds = st.rounds;
    c.launches = st.launches;
    c.kernel_ms = tm.total_ms();
    c.grid_blocks = st.grid_blocks;
    c.block_threads = st.block_threads;
    c.lds_bytes = st.lds_bytes;
    h->passa_u = tot[C_PASSA_U];
    h->round_in.clear();
    if (o.sched == MCX_SCHED_STACK)
        h->round_in.assign(ctl.round_in, ctl.round_in + std::min<unsigned long long>(st.rounds, STACK_ROUND_LOG));
    *err_out = ctl.error;
    if (ctl.error & ERR_CAPACITY) return fail(h, MCX_E_CAPACITY, "scheduler capacity exhausted (stack or link arena)");
    if (tot[C_SOURCED] != total || tot[C_COMPLETED] != total)
        return fail(h, MCX_E_DEVICE, "internal: sourced %llu, ended %llu of %llu histories", tot[C_SOURCED],
                    tot[C_COMPLETED], total);
    return MCX_OK;
}

// The history range of a forward run: per problem [first, first + count).
static mcx_status run_range(mcx_problem_t h, const mcx_run_opts &o, std::vector<uint64_t> &first,
                            std::vector<uint64_t> &count)
{
    if (h->n == 1) {
        uint64_t N = h->hp[0].d.n_histories;
        if (o.first_history > N) return fail(h, MCX_E_INVALID_ARG, "first_history beyond n_histories");
        first[0] = o.first_history;
        count[0] = o.n_histories ? o.n_histories : N - o.first_history;
        if (count[0] > N - first[0]) return fail(h, MCX_E_INVALID_ARG, "history range beyond n_histories");
    } else {
        if (o.first_history || o.n_histories)
            return fail(h, MCX_E_INVALID_ARG, "history ranges apply to single-problem handles only");
        for (int k = 0; k < h->n; ++k) {
            first[k] = 0;
            count[k] = h->hp[k].d.n_histories;
        }
    }
    return MCX_OK;
}

// grow a device buffer to at least `count` elements (contents not kept)
template <class T>
static hipError_t grow(T *&ptr, size_t &cap, size_t count)
{
    if (cap >= count && ptr) return hipSuccess;
    if (ptr) {
        hipError_t e = hipFree(ptr);
        ptr = nullptr;
        cap = 0;
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipMalloc((void **)&ptr, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) cap = count;
    return e;
}

// device total -> host (on the run's stream)
static mcx_status read_total(mcx_problem_t h, hipStream_t stream, uint64_t &out)
{
    HIP_TRY(h, hipMemcpyAsync(h->h_tot, h->d_tot, 8, hipMemcpyDeviceToHost, stream));
    HIP_TRY(h, hipStreamSynchronize(stream));
    out = *h->h_tot;
    return MCX_OK;
}

// add one pass's counters into a run's totals
static void add_counters(mcx_counters_t &sum, const mcx_counters_t &pc)
{
    sum.sourced += pc.sourced; sum.flights += pc.flights; sum.collisions += pc.collisions;
    sum.scatters += pc.scatters; sum.absorbs += pc.absorbs; sum.crossings += pc.crossings;
    sum.leaks += pc.leaks; sum.reflections += pc.reflections; sum.cutoffs += pc.cutoffs;
    sum.killed += pc.killed; sum.pieces += pc.pieces; sum.events += pc.events;
    sum.lane_slots += pc.lane_slots; sum.dispatches += pc.dispatches; sum.spills += pc.spills;
    sum.refills += pc.refills; sum.make_work += pc.make_work; sum.rounds += pc.rounds;
    sum.launches += pc.launches; sum.kernel_ms += pc.kernel_ms; sum.fissions += pc.fissions;
    sum.roulettes += pc.roulettes; sum.cdf_scans += pc.cdf_scans; sum.splits += pc.splits;
    sum.grid_blocks = pc.grid_blocks; sum.block_threads = pc.block_threads; sum.lds_bytes = pc.lds_bytes;
}

constexpr int WW_MAX_GENERATIONS = 64;

// A forward run with weight windows, in generations: generation 0 runs
// histories [first, first + count) from the problem's source; the copies a
// generation splits off, in (parent, ordinal) order, are the histories of
// the next one, on random-number stream = generation; until a generation
// splits nothing.  Tallies add up over generations, counters too; digests
// cover generation 0.
static mcx_status forward_generations(mcx_problem_t h, const mcx_run_opts &o, Workspace *fixed, uint64_t first0,
                                      uint64_t count0)
{
    hipStream_t stream = (hipStream_t)o.hip_stream;
    ProbDev &P = h->pd[0];
    const size_t cap = std::max<size_t>(2 * (size_t)count0, 65536);
    if (h->g_cap < cap) {
        size_t c0 = 0;
        HIP_TRY(h, grow(h->d_gstage, c0, cap));
        c0 = 0;
        HIP_TRY(h, grow(h->d_gsrc, c0, cap));
        h->g_cap = cap;
    }
    const size_t maxn = std::max<size_t>((size_t)count0, cap);
    HIP_TRY(h, grow(h->d_gn, h->gn_cap, maxn));
    HIP_TRY(h, grow(h->d_goff, h->goff_cap, maxn));
    HIP_TRY(h, grow(h->d_tsum, h->tsum_cap, (size_t)eigen_tiles(maxn) + 1));
    if (!h->d_gcount) HIP_TRY(h, hipMalloc(&h->d_gcount, 64));
    if (!h->d_tot) HIP_TRY(h, hipMalloc(&h->d_tot, 64));
    if (!h->h_tot) HIP_TRY(h, hipHostMalloc((void **)&h->h_tot, 64, hipHostMallocDefault));
    auto restore = [&]() {
        P.gsrc = nullptr;
        P.gout = nullptr;
        P.gcount = nullptr;
        P.gcap = 0;
        P.gn = nullptr;
        P.stream = 0;
    };
    mcx_counters_t sum{};
    unsigned __int128 qsum = 0;
    uint64_t first = first0, n = count0;
    int gen = 0;
    for (;; ++gen) {
        if (gen >= WW_MAX_GENERATIONS) {
            restore();
            return fail(h, MCX_E_CAPACITY, "weight windows: copies still split off after %d generations",
                        WW_MAX_GENERATIONS);
        }
        HIP_TRY(h, hipMemsetAsync(h->d_gcount, 0, 8, stream));
        P.gsrc = gen > 0 ? h->d_gsrc : nullptr;
        P.gout = h->d_gstage;
        P.gcount = h->d_gcount;
        P.gcap = cap;
        P.gn = h->d_gn;
        P.stream = (uint32_t)gen;
        std::vector<uint64_t> f{first}, c{n};
        unsigned int err = 0;
        mcx_status s = run_pass(h, o, MODE_FWD, f, c, gen == 0 ? o.digest : nullptr, &err, fixed);
        if (s != MCX_OK) {
            restore();
            return s;
        }
        add_counters(sum, h->counters);
        qsum += h->counters.qsum;
        uint64_t m = 0;
        HIP_TRY(h, hipMemcpyAsync(h->h_tot, h->d_gcount, 8, hipMemcpyDeviceToHost, stream));
        HIP_TRY(h, hipStreamSynchronize(stream));
        m = *h->h_tot;
        if (m > cap) {
            restore();
            return fail(h, MCX_E_CAPACITY, "weight windows: generation %d split off %llu copies (room for %zu)", gen,
                        (unsigned long long)m, cap);
        }
        if (m == 0) break;
        // the next generation: the copies in (parent, ordinal) order
        hipError_t e = ww_order_copies(h->d_gn, n, (uint32_t)first, h->d_gstage, m, h->d_tsum, h->d_tot, h->d_goff,
                                       h->d_gsrc, stream);
        if (e != hipSuccess) {
            restore();
            return hip_fail(h, e, "weight-window copies");
        }
        uint64_t chk = 0;
        s = read_total(h, stream, chk);
        if (s != MCX_OK) {
            restore();
            return s;
        }
        if (chk != m) {
            restore();
            return fail(h, MCX_E_DEVICE, "internal: generation %d staged %llu copies, counted %llu", gen,
                        (unsigned long long)m, (unsigned long long)chk);
        }
        first = 0;
        n = m;
    }
    restore();
    sum.qsum = (uint64_t)qsum;
    sum.overflow = qsum >= ((unsigned __int128)1 << 63) ? 1 : 0;
    sum.generations = (uint64_t)gen + 1;
    h->counters = sum;
    if (sum.overflow) return fail(h, MCX_E_OVERFLOW, "fixed-point tally total reached 2^63");
    return MCX_OK;
}

// A forward run into the handle's tallies; `fixed`: device scratch the run
// must fit in (never reallocated), or null for the handle's own.
static mcx_status forward(mcx_problem_t h, const mcx_run_opts &o, Workspace *fixed)
{
    std::vector<uint64_t> &first = h->run_first, &count = h->run_count;
    mcx_status s = run_range(h, o, first, count);
    if (s != MCX_OK) return s;
    if (fixed) {
        // refuse a run that does not fit before anything changes
        unsigned long long total = 0;
        for (int k = 0; k < h->n; ++k) total += count[k];
        const int path = tally_path(h, o, MODE_FWD);
        size_t sched_b = 0, need = 0;
        s = scratch_bytes(h, o, launch_args(h, o, MODE_FWD, total, path, o.digest), path, sched_b, need);
        if (s != MCX_OK) return s;
        if (need > fixed->bytes)
            return fail(h, MCX_E_INVALID_ARG, "the run needs %zu bytes of device scratch; the workspace holds %zu",
                        need, fixed->bytes);
    }
    h->tallies_valid = false;
    h->have_forward = false;
    if (!o.accumulate)
        HIP_TRY(h, hipMemsetAsync(h->d_tally, 0, std::max<size_t>(h->total_bins, 1) * 8, (hipStream_t)o.hip_stream));
    unsigned int err = 0;
    if (h->n == 1 && h->hp[0].ww) {
        s = forward_generations(h, o, fixed, first[0], count[0]);
        if (s != MCX_OK) return s;
        h->tallies_valid = true;
        h->have_forward = true;
        h->last_first = first;
        h->last_count = count;
        return MCX_OK;
    }
    s = run_pass(h, o, MODE_FWD, first, count, o.digest, &err, fixed);
    if (s != MCX_OK) return s;
    if (err & ERR_OVERFLOW) return fail(h, MCX_E_OVERFLOW, "fixed-point tally total reached 2^63");
    h->tallies_valid = true;
    h->have_forward = true;
    h->last_first = first;
    h->last_count = count;
    return MCX_OK;
}

// the caller's workspace of a run's options, if it gave one
static Workspace *caller_ws(const mcx_run_opts &o, Workspace &w)
{
    if (!o.workspace) return nullptr;
    w.ptr = o.workspace;
    w.bytes = o.ws_bytes;
    w.fixed = true;
    return &w;
}

extern "C" mcx_status mcx_run(mcx_problem_t h, const mcx_run_opts *opts)
{
    if (!h || !opts) return MCX_E_INVALID_ARG;
    const mcx_run_opts &o = *opts;
    mcx_status s = check_opts(h, o);
    if (s != MCX_OK) return s;
    Workspace w;
    return forward(h, o, caller_ws(o, w));
}

extern "C" mcx_status mcx_run_noalloc(mcx_problem_t h, const mcx_run_opts *opts)
{
    if (!h || !opts) return MCX_E_INVALID_ARG;
    const mcx_run_opts &o = *opts;
    mcx_status s = check_opts(h, o);
    if (s != MCX_OK) return s;
    if (o.workspace) return fail(h, MCX_E_INVALID_ARG, "mcx_run_noalloc runs in the library's fixed scratch: workspace must be NULL");
    if (o.time_kernels) return fail(h, MCX_E_INVALID_ARG, "mcx_run_noalloc does not time launches (time_kernels must be 0)");
    if (h->hp[0].ww) return fail(h, MCX_E_INVALID_ARG, "mcx_run_noalloc takes no weight windows (their generations need device memory)");
    if (!h->scratch) return fail(h, MCX_E_DEVICE, "no device scratch on this device");
    Workspace w;
    w.ptr = h->scratch;
    w.bytes = MCX_NOALLOC_SCRATCH_BYTES;
    w.fixed = true;
    return forward(h, o, &w);
}

extern "C" mcx_status mcx_run_eigen(mcx_problem_t h, const mcx_run_opts *opts, const mcx_eigen_opts *eig)
{
    if (!h || !opts || !eig) return MCX_E_INVALID_ARG;
    mcx_run_opts o = *opts;
    mcx_status s = check_opts(h, o);
    if (s != MCX_OK) return s;
    if (h->n != 1) return fail(h, MCX_E_INVALID_ARG, "k-eigenvalue runs take a single problem");
    const HostProblem &hp = h->hp[0];
    if (!hp.fission) return fail(h, MCX_E_INVALID_ARG, "k-eigenvalue runs need fission data");
    if (hp.d.n_tbins > 0) return fail(h, MCX_E_INVALID_ARG, "k-eigenvalue runs take no time bins");
    if (hp.d.implicit_capture) return fail(h, MCX_E_INVALID_ARG, "k-eigenvalue runs are analog (no implicit capture)");
    if (hp.ww) return fail(h, MCX_E_INVALID_ARG, "k-eigenvalue runs take no weight windows");
    const uint64_t N = eig->n_particles;
    if (N < 1 || N > (1ull << 30)) return fail(h, MCX_E_INVALID_ARG, "n_particles must be 1..2^30");
    if (eig->n_cycles < 1 || eig->n_inactive < 0 || eig->n_inactive > eig->n_cycles)
        return fail(h, MCX_E_INVALID_ARG, "need n_cycles >= 1 and 0 <= n_inactive <= n_cycles");
    if (!eig->k_cycle || !eig->n_source) return fail(h, MCX_E_INVALID_ARG, "null k_cycle or n_source");
    if (o.workspace) return fail(h, MCX_E_INVALID_ARG, "k-eigenvalue runs use the library's own workspace");
    o.digest = nullptr;
    o.first_history = 0;
    o.n_histories = 0;
    hipStream_t stream = (hipStream_t)o.hip_stream;
    h->tallies_valid = false;
    h->have_forward = false;
    // buffers: source banks hold up to 2N + 1024 particles; a history banks
    // at most 15 neutrons
    const size_t cap = 2 * (size_t)N + 1024;
    if (h->eig_cap < cap) {
        size_t c0 = 0;
        for (double *&b : h->d_sbank) {
            c0 = 0;
            HIP_TRY(h, grow(b, c0, 3 * cap));
        }
        c0 = 0;
        HIP_TRY(h, grow(h->d_fn, c0, cap));
        c0 = 0;
        HIP_TRY(h, grow(h->d_fpos, c0, 3 * cap));
        h->eig_cap = cap;
    }
    HIP_TRY(h, grow(h->d_tsum, h->tsum_cap, (size_t)eigen_tiles(16 * (uint64_t)cap) + 1));
    if (!h->d_scratch) HIP_TRY(h, hipMalloc(&h->d_scratch, std::max<size_t>(h->total_bins, 1) * 8));
    if (!h->d_tot) HIP_TRY(h, hipMalloc(&h->d_tot, 64));
    if (!h->h_tot) HIP_TRY(h, hipHostMalloc((void **)&h->h_tot, 64, hipHostMallocDefault));
    HIP_TRY(h, hipMemsetAsync(h->d_tally, 0, std::max<size_t>(h->total_bins, 1) * 8, stream));

    mcx_counters_t sum{};
    unsigned __int128 qsum = 0;
    uint64_t Nc = N;
    const double *src = nullptr;      // cycle 0: the problem's own source
    int next = 0;
    ProbDev &P = h->pd[0];
    auto restore = [&]() {
        P.sbank = nullptr;
        P.fn = nullptr;
        P.fpos = nullptr;
        P.stream = 0;
        P.tally = h->d_tally;
    };
    for (int c = 0; c < eig->n_cycles; ++c) {
        P.sbank = src;
        P.fn = h->d_fn;
        P.fpos = h->d_fpos;
        P.stream = (uint32_t)c;
        P.tally = c >= eig->n_inactive ? h->d_tally : h->d_scratch;
        std::vector<uint64_t> first{0}, count{Nc};
        unsigned int err = 0;
        s = run_pass(h, o, MODE_FWD, first, count, nullptr, &err);
        restore();
        if (s != MCX_OK) return s;
        if (err & ERR_OVERFLOW) return fail(h, MCX_E_OVERFLOW, "fixed-point tally total reached 2^63");
        const mcx_counters_t &pc = h->counters;
        sum.sourced += pc.sourced; sum.flights += pc.flights; sum.collisions += pc.collisions;
        sum.scatters += pc.scatters; sum.absorbs += pc.absorbs; sum.crossings += pc.crossings;
        sum.leaks += pc.leaks; sum.reflections += pc.reflections; sum.cutoffs += pc.cutoffs;
        sum.killed += pc.killed; sum.pieces += pc.pieces; sum.events += pc.events;
        sum.lane_slots += pc.lane_slots; sum.dispatches += pc.dispatches; sum.spills += pc.spills;
        sum.refills += pc.refills; sum.make_work += pc.make_work; sum.rounds += pc.rounds;
        sum.launches += pc.launches; sum.kernel_ms += pc.kernel_ms; sum.fissions += pc.fissions;
        sum.roulettes += pc.roulettes;
        sum.cdf_scans += pc.cdf_scans;
        sum.grid_blocks = pc.grid_blocks; sum.block_threads = pc.block_threads; sum.lds_bytes = pc.lds_bytes;
        qsum += pc.qsum;
        // the bank: each history's neutrons, in history order
        uint64_t M = 0;
        hipError_t e = eigen_count_sites(h->d_fn, Nc, h->d_tsum, h->d_tot, stream);
        if (e != hipSuccess) return hip_fail(h, e, "fission bank count");
        s = read_total(h, stream, M);
        if (s != MCX_OK) return s;
        eig->n_source[c] = Nc;
        eig->k_cycle[c] = (double)M / (double)Nc;
        sum.sites += M;
        if (M == 0) return fail(h, MCX_E_STATE, "cycle %d banked no fission neutron", c);
        if (M >= (1ull << 32)) return fail(h, MCX_E_CAPACITY, "cycle %d banked 2^32 neutrons or more", c);
        HIP_TRY(h, grow(h->d_sites, h->sites_cap, 3 * (size_t)M));
        e = eigen_gather_sites(h->d_fn, h->d_fpos, Nc, h->d_tsum, h->d_sites, stream);
        if (e != hipSuccess) return hip_fail(h, e, "fission bank gather");
        // splitting-roulette back to about N
        const double r = (double)N / (double)M;
        const double fl = std::floor(r);
        const double fr = r - fl;
        uint64_t Nn = 0;
        e = eigen_count_copies(P.key0, P.key1, (uint32_t)c, (uint64_t)fl, fr, M, h->d_tsum, h->d_tot, stream);
        if (e != hipSuccess) return hip_fail(h, e, "population control count");
        s = read_total(h, stream, Nn);
        if (s != MCX_OK) return s;
        if (Nn == 0) return fail(h, MCX_E_STATE, "population control left no particle after cycle %d", c);
        if (Nn > cap) return fail(h, MCX_E_CAPACITY, "source bank overflow after cycle %d", c);
        e = eigen_scatter_copies(P.key0, P.key1, (uint32_t)c, (uint64_t)fl, fr, M, h->d_tsum, h->d_sites,
                                 h->d_sbank[next], cap, stream);
        if (e != hipSuccess) return hip_fail(h, e, "population control scatter");
        src = h->d_sbank[next];
        next ^= 1;
        Nc = Nn;
    }
    HIP_TRY(h, hipStreamSynchronize(stream));
    sum.qsum = (uint64_t)qsum;
    sum.overflow = qsum >= ((unsigned __int128)1 << 63) ? 1 : 0;
    sum.generations = 1;
    h->counters = sum;
    if (sum.overflow) return fail(h, MCX_E_OVERFLOW, "fixed-point tally total reached 2^63");
    h->tallies_valid = true;
    return MCX_OK;
}

extern "C" mcx_status mcx_tallies(mcx_problem_t h, int32_t problem, int64_t *out, int64_t n, int32_t where)
{
    if (!h || !out) return MCX_E_INVALID_ARG;
    if (problem < 0 || problem >= h->n) return fail(h, MCX_E_INVALID_ARG, "bad problem index");
    if (!h->tallies_valid) return fail(h, MCX_E_STATE, "no valid tallies (no successful run)");
    if (n != h->hp[problem].n_bins) return fail(h, MCX_E_INVALID_ARG, "tally size is %lld", (long long)h->hp[problem].n_bins);
    HIP_TRY(h, hipMemcpy(out, h->d_tally + h->tally_off[problem], (size_t)n * 8,
                         where == MCX_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    return MCX_OK;
}

extern "C" mcx_status mcx_backward(mcx_problem_t h, int32_t problem, const double *dL_dT, double *grad_sigma_t,
                                   double *grad_sigma_s, int32_t where, const mcx_run_opts *opts)
{
    if (!h || !opts || !dL_dT || !grad_sigma_t || !grad_sigma_s) return MCX_E_INVALID_ARG;
    if (h->emode != MCX_MG) return fail(h, MCX_E_INVALID_ARG, "the backward needs multigroup problems");
    for (int k = 0; k < h->n; ++k)
        if (h->hp[k].ww) return fail(h, MCX_E_INVALID_ARG, "the backward takes no weight windows");
    if (problem < -1 || problem >= h->n) return fail(h, MCX_E_INVALID_ARG, "bad problem index");
    if (!h->have_forward) return fail(h, MCX_E_STATE, "mcx_backward needs a successful forward run first");
    mcx_run_opts o = *opts;
    mcx_status s = check_opts(h, o);
    if (s != MCX_OK) return s;
    hipStream_t stream = (hipStream_t)o.hip_stream;
    // per-problem replay ranges: those of the last forward, selected problems only
    std::vector<uint64_t> first = h->last_first, count = h->last_count;
    size_t wtot = 0;
    std::vector<size_t> woff(h->n, 0);
    for (int k = 0; k < h->n; ++k) {
        if (problem >= 0 && k != problem) count[k] = 0;
        woff[k] = wtot;
        if (problem < 0 || k == problem) wtot += (size_t)h->hp[k].n_bins;
    }
    if (wtot * 8 > h->w_cap) {
        if (h->d_w) hipFree(h->d_w);
        h->d_w = nullptr;
        h->w_cap = 0;
        HIP_TRY(h, hipMalloc(&h->d_w, wtot * 8));
        h->w_cap = wtot * 8;
    }
    HIP_TRY(h, hipMemcpyAsync(h->d_w, dL_dT, wtot * 8, where == MCX_DEVICE ? hipMemcpyDeviceToDevice
                                                                          : hipMemcpyHostToDevice, stream));
    unsigned long long gtot = 0;
    for (int k = 0; k < h->n; ++k) gtot += count[k];
    if (gtot * 8 > h->G_cap) {
        if (h->d_G) hipFree(h->d_G);
        h->d_G = nullptr;
        h->G_cap = 0;
        HIP_TRY(h, hipMalloc(&h->d_G, std::max<unsigned long long>(gtot, 1) * 8));
        h->G_cap = std::max<unsigned long long>(gtot, 1) * 8;
    }
    HIP_TRY(h, hipMemsetAsync(h->d_gacc, 0, h->gacc_words * 8, stream));
    for (int k = 0; k < h->n; ++k) {
        h->pd[k].w = h->d_w + woff[k];
        h->pd[k].G = h->d_G;
        h->pd[k].gscale = 1.0;
    }
    unsigned int err = 0;
    Workspace w;
    Workspace *fixed = caller_ws(o, w);
    s = run_pass(h, o, MODE_REPLAY_A, first, count, nullptr, &err, fixed);
    if (s != MCX_OK) return s;
    if (err & ERR_BOUND) return fail(h, MCX_E_OVERFLOW, "score-function bound does not fit 64 bits");
    const double ms_a = h->counters.kernel_ms;
    const uint64_t launches_a = h->counters.launches, rounds_a = h->counters.rounds;
    std::vector<unsigned long long> acc(h->gacc_words);
    HIP_TRY(h, hipMemcpy(acc.data(), h->d_gacc, h->gacc_words * 8, hipMemcpyDeviceToHost));
    if (h->n == 1) acc[h->gacc_off[0]] += h->passa_u;   // single-problem runs sum U per wavefront
    std::vector<int> scale(h->n, 0);
    for (int k = 0; k < h->n; ++k) {
        scale[k] = 62 - bit_length(acc[h->gacc_off[k]]);
        h->pd[k].gscale = std::ldexp(1.0, scale[k]);
    }
    s = run_pass(h, o, MODE_REPLAY_B, first, count, nullptr, &err, fixed);
    if (s != MCX_OK) return s;
    h->counters.kernel_ms += ms_a;
    h->counters.launches += launches_a;
    h->counters.rounds += rounds_a;
    HIP_TRY(h, hipMemcpy(acc.data(), h->d_gacc, h->gacc_words * 8, hipMemcpyDeviceToHost));
    // gradients, analog: grad Sigma_t = (-SL + SA/Sigma_a) 2^-s / N and
    // grad Sigma_s = (SS/Sigma_s - SA/Sigma_a) 2^-s / N; implicit capture (SA
    // over collisions, SS the score still to come at them):
    // grad Sigma_t = (-SL + (SA/Sigma_t - SS/Sigma_t)) 2^-s / N and
    // grad Sigma_s = (SS/Sigma_s) 2^-s / N
    std::vector<double> gt, gs;
    for (int k = 0; k < h->n; ++k) {
        if (problem >= 0 && k != problem) continue;
        const HostProblem &hp = h->hp[k];
        size_t mg = (size_t)hp.d.n_mat * hp.d.n_grp;
        const long long *SL = (const long long *)&acc[h->gacc_off[k] + 1];
        const long long *SA = SL + mg;
        const long long *SS = SL + 2 * mg;
        double sc = std::ldexp(1.0, -scale[k]);
        double n = (double)h->last_count[k];
        const bool weighted = hp.d.implicit_capture != 0;
        for (size_t i = 0; i < mg; ++i) {
            const double st = hp.sig_t[i], ss = hp.sig_s[i];
            if (weighted) {
                gt.push_back(((-(double)SL[i]) + (((double)SA[i] / st) - ((double)SS[i] / st))) * sc / n);
                gs.push_back(((double)SS[i] / ss) * sc / n);
            } else {
                double sa = st - ss;
                gt.push_back(((-(double)SL[i]) + ((double)SA[i] / sa)) * sc / n);
                gs.push_back((((double)SS[i] / ss) - ((double)SA[i] / sa)) * sc / n);
            }
        }
    }
    size_t nb = gt.size() * 8;
    hipMemcpyKind kind = where == MCX_DEVICE ? hipMemcpyHostToDevice : hipMemcpyHostToHost;
    HIP_TRY(h, hipMemcpy(grad_sigma_t, gt.data(), nb, kind));
    HIP_TRY(h, hipMemcpy(grad_sigma_s, gs.data(), nb, kind));
    return MCX_OK;
}

extern "C" mcx_status mcx_workspace_size(mcx_problem_t h, const mcx_run_opts *opts, size_t *bytes)
{
    if (!h || !opts || !bytes) return MCX_E_INVALID_ARG;
    const mcx_run_opts &o = *opts;
    mcx_status s = check_opts(h, o);
    if (s != MCX_OK) return s;
    std::vector<uint64_t> first(h->n), count(h->n);
    s = run_range(h, o, first, count);
    if (s != MCX_OK) return s;
    unsigned long long total = 0;
    for (int k = 0; k < h->n; ++k) total += count[k];
    // forward, and the backward's two replays where the handle has them
    bool replays = h->emode == MCX_MG;
    for (int k = 0; k < h->n; ++k)
        if (h->hp[k].ww) replays = false;
    size_t need = 0;
    for (int mode : {MODE_FWD, MODE_REPLAY_A, MODE_REPLAY_B}) {
        if (mode != MODE_FWD && !replays) continue;
        const int path = tally_path(h, o, mode);
        LaunchArgs a = launch_args(h, o, mode, total, path, mode == MODE_FWD ? o.digest : nullptr);
        size_t sched_b = 0, b = 0;
        s = scratch_bytes(h, o, a, path, sched_b, b);
        if (s != MCX_OK) return s;
        need = std::max(need, b);
    }
    *bytes = need;
    return MCX_OK;
}

extern "C" mcx_status mcx_stack_rounds(mcx_problem_t h, uint32_t *particles, int32_t max_rounds, int32_t *n_rounds)
{
    if (!h || !n_rounds || max_rounds < 0 || (max_rounds > 0 && !particles)) return MCX_E_INVALID_ARG;
    const int32_t n = (int32_t)std::min<size_t>(h->round_in.size(), (size_t)max_rounds);
    for (int32_t r = 0; r < n; ++r) particles[r] = h->round_in[r];
    *n_rounds = (int32_t)h->round_in.size();
    return MCX_OK;
}

extern "C" mcx_status mcx_counters(mcx_problem_t h, mcx_counters_t *out)
{
    if (!h || !out) return MCX_E_INVALID_ARG;
    *out = h->counters;
    return MCX_OK;
}

extern "C" mcx_status mcx_problem_info(mcx_problem_t h, int32_t problem, int64_t *n_bins, int32_t *n_mat,
                                       int32_t *n_grp, uint64_t *n_histories)
{
    if (!h) return MCX_E_INVALID_ARG;
    if (problem < 0 || problem >= h->n) return fail(h, MCX_E_INVALID_ARG, "bad problem index");
    const HostProblem &hp = h->hp[problem];
    if (n_bins) *n_bins = hp.n_bins;
    if (n_mat) *n_mat = hp.d.n_mat;
    if (n_grp) *n_grp = hp.d.energy_mode == MCX_MG ? hp.d.n_grp : 1;
    if (n_histories) *n_histories = hp.d.n_histories;
    return MCX_OK;
}

extern "C" const char *mcx_status_str(mcx_status s)
{
    switch (s) {
    case MCX_OK: return "ok";
    case MCX_E_INVALID_ARG: return "invalid argument";
    case MCX_E_OOM: return "out of device memory";
    case MCX_E_DEVICE: return "device error";
    case MCX_E_CAPACITY: return "scheduler capacity exhausted";
    case MCX_E_OVERFLOW: return "fixed-point overflow";
    case MCX_E_STATE: return "invalid state";
    }
    return "unknown status";
}

extern "C" const char *mcx_last_error(mcx_problem_t h)
{
    return h ? h->err.c_str() : "null handle";
}
