// Fission banking and population control between k-eigenvalue cycles
// (the paper's multigroup workload, Sec. 4: power iteration with
// splitting-roulette population control).
//
// After a cycle every history h has banked fn[h] neutrons at its fission
// site fpos[h].  The bank is those neutrons in history order: site offsets
// are an exclusive prefix sum of fn, so the order does not depend on which
// wavefront ran which history.  Splitting-roulette then copies site j
// floor(r) times, plus once more when u_j < r - floor(r) (r = N / M, u_j the
// first deviate of counter (j, 0xFFFFFFFF, 0, cycle) -- a flight counter no
// history reaches), and a second prefix sum over the copy counts places the
// copies, in site order, into the next cycle's source bank.
//
// Prefix sums: tiles of 4096 items (256 threads x 16 consecutive items);
// one pass sums each tile, one single-block pass scans the tile sums (and
// writes the total), one pass rescans each tile from its offset and moves
// the data.
#include "kernels.hpp"
#include "rng_math.hpp"

namespace mcx {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

// neutrons banked by history i
struct SiteCount {
    const uint32_t *fn;
    __device__ __forceinline__ uint64_t operator()(uint64_t i) const { return fn[i]; }
};

// copies of site j made by splitting-roulette
struct CopyCount {
    Key key;
    uint32_t stream;
    uint64_t fl;      // floor(r)
    double fr;        // r - floor(r)
    __device__ __forceinline__ uint64_t operator()(uint64_t j) const
    {
        double a, b;
        uniform_pair(key, (uint32_t)j, 0xFFFFFFFFu, 0u, a, b, stream);
        return fl + ((a < fr) ? 1ull : 0ull);
    }
};

// block-wide exclusive scan of one value per thread; returns this thread's
// exclusive prefix, the block total in *total (LDS)
__device__ __forceinline__ uint64_t block_exclusive(uint64_t v, uint64_t *sh, uint64_t *total)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_THREADS; off <<= 1) {
        uint64_t o = (t >= off) ? sh[t - off] : 0ull;
        __syncthreads();
        sh[t] += o;
        __syncthreads();
    }
    uint64_t incl = sh[t];
    if (t == SCAN_THREADS - 1) *total = incl;
    __syncthreads();
    return incl - v;
}

template <class CNT>
__global__ void __launch_bounds__(SCAN_THREADS) tile_sums(CNT cnt, uint64_t n, uint64_t *tsum)
{
    __shared__ uint64_t sh[SCAN_THREADS];
    __shared__ uint64_t tot;
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint64_t s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k)
        if (base + k < n) s += cnt(base + k);
    (void)block_exclusive(s, sh, &tot);
    if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

// exclusive scan of the nt tile sums in place (one block); total to *total
__global__ void __launch_bounds__(SCAN_THREADS) scan_tile_sums(uint64_t *tsum, uint64_t nt, uint64_t *total)
{
    __shared__ uint64_t sh[SCAN_THREADS];
    __shared__ uint64_t tot;
    uint64_t carry = 0;
    for (uint64_t b = 0; b < nt; b += SCAN_THREADS) {
        const uint64_t i = b + threadIdx.x;
        uint64_t v = i < nt ? tsum[i] : 0ull;
        uint64_t ex = block_exclusive(v, sh, &tot);
        if (i < nt) tsum[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

// sites[o + j] = fpos[i] for j < fn[i], o = offset of history i
struct GatherSites {
    const double *fpos;
    double *sites;
    __device__ __forceinline__ void operator()(uint64_t i, uint64_t o, uint64_t c) const
    {
        const double x = fpos[3 * i], y = fpos[3 * i + 1], z = fpos[3 * i + 2];
        for (uint64_t j = 0; j < c; ++j) {
            sites[3 * (o + j)] = x;
            sites[3 * (o + j) + 1] = y;
            sites[3 * (o + j) + 2] = z;
        }
    }
};

// next[o + j] = sites[i] for j < copies(i); copies past cap are dropped (the
// host checks the total against cap before it uses the bank)
struct ScatterCopies {
    const double *sites;
    double *next;
    uint64_t cap;
    __device__ __forceinline__ void operator()(uint64_t i, uint64_t o, uint64_t c) const
    {
        const double x = sites[3 * i], y = sites[3 * i + 1], z = sites[3 * i + 2];
        for (uint64_t j = 0; j < c && o + j < cap; ++j) {
            next[3 * (o + j)] = x;
            next[3 * (o + j) + 1] = y;
            next[3 * (o + j) + 2] = z;
        }
    }
};

template <class CNT, class OUT>
__global__ void __launch_bounds__(SCAN_THREADS) tile_apply(CNT cnt, uint64_t n, const uint64_t *tsum, OUT out)
{
    __shared__ uint64_t sh[SCAN_THREADS];
    __shared__ uint64_t tot;
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint64_t c[SCAN_ITEMS];
    uint64_t s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        c[k] = (base + k < n) ? cnt(base + k) : 0ull;
        s += c[k];
    }
    uint64_t o = tsum[blockIdx.x] + block_exclusive(s, sh, &tot);
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < n && c[k] != 0) out(base + k, o, c[k]);
        o += c[k];
    }
}

static uint64_t n_tiles(uint64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE; }

template <class CNT>
static hipError_t count_total(CNT cnt, uint64_t n, uint64_t *tsum, uint64_t *total, hipStream_t s)
{
    const uint64_t nt = n_tiles(n);
    if (nt > 0) hipLaunchKernelGGL(tile_sums<CNT>, dim3((unsigned)nt), dim3(SCAN_THREADS), 0, s, cnt, n, tsum);
    hipLaunchKernelGGL(scan_tile_sums, dim3(1), dim3(SCAN_THREADS), 0, s, tsum, nt, total);
    return hipGetLastError();
}

hipError_t eigen_count_sites(const uint32_t *fn, uint64_t n, uint64_t *tsum, uint64_t *total, hipStream_t s)
{
    return count_total(SiteCount{fn}, n, tsum, total, s);
}

hipError_t eigen_gather_sites(const uint32_t *fn, const double *fpos, uint64_t n, const uint64_t *tsum,
                              double *sites, hipStream_t s)
{
    const uint64_t nt = n_tiles(n);
    if (nt == 0) return hipSuccess;
    hipLaunchKernelGGL((tile_apply<SiteCount, GatherSites>), dim3((unsigned)nt), dim3(SCAN_THREADS), 0, s,
                       SiteCount{fn}, n, tsum, GatherSites{fpos, sites});
    return hipGetLastError();
}

hipError_t eigen_count_copies(uint32_t key0, uint32_t key1, uint32_t stream, uint64_t fl, double fr, uint64_t m,
                              uint64_t *tsum, uint64_t *total, hipStream_t s)
{
    return count_total(CopyCount{Key{key0, key1}, stream, fl, fr}, m, tsum, total, s);
}

hipError_t eigen_scatter_copies(uint32_t key0, uint32_t key1, uint32_t stream, uint64_t fl, double fr, uint64_t m,
                                const uint64_t *tsum, const double *sites, double *next, uint64_t cap,
                                hipStream_t s)
{
    const uint64_t nt = n_tiles(m);
    if (nt == 0) return hipSuccess;
    hipLaunchKernelGGL((tile_apply<CopyCount, ScatterCopies>), dim3((unsigned)nt), dim3(SCAN_THREADS), 0, s,
                       CopyCount{Key{key0, key1}, stream, fl, fr}, m, tsum, ScatterCopies{sites, next, cap});
    return hipGetLastError();
}

uint64_t eigen_tiles(uint64_t n) { return n_tiles(n); }

// ---------------------------------------------------------------------------
// Generations of weight-window copies.  Every history of a generation staged
// its copies in any order (whichever wavefront ran it), each with its parent
// and ordinal, and counted them in gn.  The next generation is those copies
// in (parent, ordinal) order: parent offsets are an exclusive prefix sum of
// gn (the same tile scan as the fission bank), and copy (parent, k) lands at
// offset(parent) + k.

struct StoreOffset {
    uint64_t *off;
    __device__ __forceinline__ void operator()(uint64_t i, uint64_t o, uint64_t) const { off[i] = o; }
};

__global__ void __launch_bounds__(256) ww_scatter_kernel(const SiteRec *stage, uint64_t m, const uint64_t *off,
                                                         uint32_t first, SiteRec *next)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const SiteRec r = stage[i];
    next[off[r.parent - first] + r.seq] = r;
}

hipError_t ww_order_copies(const uint32_t *gn, uint64_t n, uint32_t first, const SiteRec *stage, uint64_t m,
                           uint64_t *tsum, uint64_t *total, uint64_t *off, SiteRec *next, hipStream_t s)
{
    hipError_t e = count_total(SiteCount{gn}, n, tsum, total, s);
    if (e != hipSuccess) return e;
    const uint64_t nt = n_tiles(n);
    if (nt > 0)
        hipLaunchKernelGGL((tile_apply<SiteCount, StoreOffset>), dim3((unsigned)nt), dim3(SCAN_THREADS), 0, s,
                           SiteCount{gn}, n, (const uint64_t *)tsum, StoreOffset{off});
    if (m > 0)
        hipLaunchKernelGGL(ww_scatter_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, stage, m,
                           (const uint64_t *)off, first, next);
    return hipGetLastError();
}

}  // namespace mcx
