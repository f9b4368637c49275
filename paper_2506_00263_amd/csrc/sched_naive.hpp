// History-based baseline: one lane runs one whole history, flight after
// flight, until it ends.  Lanes of a wavefront diverge as soon as their
// histories take different paths or lengths (the divergence thread-data
// remapping removes, paper Sec. 2); the wavefront runs until its longest
// history ends.
#pragma once
#include "kernels.hpp"
#include "transport.hpp"

namespace mcx {

template <int GEOM, int EMODE, int MODE, bool BATCH, int EXT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) naive_kernel(const ProbDev *__restrict__ probs, int n_probs,
                                                    const unsigned long long *__restrict__ prefix,
                                                    unsigned long long total, RunCtl *ctl, Digest *digest,
                                                    int lacc_words)
{
    extern __shared__ __attribute__((aligned(16))) unsigned long long lacc[];
    char *tl = (char *)lacc + tabs_lds_offset((size_t)lacc_words * 8);
    if constexpr (!BATCH) tabs_to_lds(probs[0], tl);
    // LDS block sums: pass B's per-(material, group) sums, or the bins of a small
    // energy-bin tally (single-problem launches)
    EvCtx cx{probs, digest, (MODE == MODE_REPLAY_B && lacc_words > 0) ? lacc : nullptr, BATCH ? 0 : 1,
             (MODE == MODE_FWD && lacc_words > 0) ? lacc : nullptr};
    if (lacc_words > 0) {
        lacc_zero(lacc, lacc_words);
        __syncthreads();
    }
    Lane ln{0, 0, 0, 0, (uint32_t)(((blockIdx.x * blockDim.x + threadIdx.x) >> 6) % TREP)};
    WaveCount wc;
    wc.zero();
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long base = (unsigned long long)blockIdx.x * blockDim.x; base < total; base += stride) {
        unsigned long long gid = base + threadIdx.x;
        bool act = gid < total;
        Part p;
        int ev = EV_DEAD;
        if (act) {
            int pi = BATCH ? find_problem(prefix, n_probs, gid) : 0;
            const ProbDev &P = probs[pi];
            source<GEOM, MODE>(P, tabs_for<BATCH>(P, tl), p, (uint32_t)(P.first + (gid - P.gbase)), (uint32_t)pi);
            ev = EV_STEP;
        }
        wc.outcomes(act, O_SOURCE);
        while (__ballot(ev != EV_DEAD)) {
            bool alive = ev != EV_DEAD;
            uint32_t out = 0;
            if (alive) ev = run_event_in<GEOM, EMODE, MODE, 0, EXT, BATCH>(EV_STEP, probs, tl, cx, ln, p, out);
            wc.dispatch(alive);
            wc.outcomes(alive, out);
        }
    }
    flush_wave(ctl, wc, ln, probs, BATCH ? 0 : 1, MODE);
    if (lacc_words > 0) {
        __syncthreads();
        if (cx.lacc) lacc_flush(lacc, probs[0]);
        if (cx.ltally) ltally_flush(lacc, probs[0], lacc_words);
    }
}

template <int GEOM, int EMODE, int MODE, bool BATCH, int EXT>
static hipError_t launch_naive_t(const LaunchArgs &a, LaunchStats &st, LaunchTimer &tm)
{
    int bs = a.block_size > 0 ? a.block_size : 256;
    if (bs > 256) bs = 256;
    bs = (bs + 63) / 64 * 64;
    unsigned long long blocks = (a.total + bs - 1) / bs;
    unsigned long long cap = (unsigned long long)a.num_cus * 64;   // grid-stride beyond this
    if (blocks > cap) blocks = cap;
    if (blocks == 0) blocks = 1;
    size_t lds = tabs_lds_offset((size_t)a.lacc_words * 8) + (BATCH ? 0 : (size_t)a.tl_bytes);
    if (a.ws_query) {
        *a.ws_query = 0;      // the naive kernel keeps particles in registers only
        return hipSuccess;
    }
    st.grid_blocks = (int)blocks;
    st.block_threads = bs;
    st.lds_bytes = (int)lds;
    tm.begin();
    hipLaunchKernelGGL((naive_kernel<GEOM, EMODE, MODE, BATCH, EXT>), dim3((unsigned)blocks), dim3(bs), lds, a.stream,
                       a.probs, a.n_probs, a.prefix, a.total, a.ctl, (Digest *)a.digest, a.lacc_words);
    tm.end();
    st.launches += 1;
    return hipGetLastError();
}

template <int GEOM, int EMODE, int MODE, int EXT>
static hipError_t naive_b(const LaunchArgs &a, LaunchStats &st, LaunchTimer &tm)
{
    return (a.n_probs > 1 || a.tl_bytes == 0) ? launch_naive_t<GEOM, EMODE, MODE, true, EXT>(a, st, tm)
                                              : launch_naive_t<GEOM, EMODE, MODE, false, EXT>(a, st, tm);
}

// every event program of one particle-state mode (without or with time and weight)
template <int EXT>
static hipError_t launch_naive_tm(const LaunchArgs &a, LaunchStats &st, LaunchTimer &tm)
{
    if (a.emode == EMODE_CE) {
        if (a.geom != GEOM_LATTICE || a.mode != MODE_FWD) return hipErrorInvalidValue;
        return naive_b<GEOM_LATTICE, EMODE_CE, MODE_FWD, EXT>(a, st, tm);
    }
    if (a.geom == GEOM_BOX) {
        if (a.mode == MODE_FWD) return naive_b<GEOM_BOX, EMODE_MG, MODE_FWD, EXT>(a, st, tm);
        if (a.mode == MODE_REPLAY_A) return naive_b<GEOM_BOX, EMODE_MG, MODE_REPLAY_A, EXT>(a, st, tm);
        return naive_b<GEOM_BOX, EMODE_MG, MODE_REPLAY_B, EXT>(a, st, tm);
    }
    if (a.mode == MODE_FWD) return naive_b<GEOM_LATTICE, EMODE_MG, MODE_FWD, EXT>(a, st, tm);
    if (a.mode == MODE_REPLAY_A) return naive_b<GEOM_LATTICE, EMODE_MG, MODE_REPLAY_A, EXT>(a, st, tm);
    return naive_b<GEOM_LATTICE, EMODE_MG, MODE_REPLAY_B, EXT>(a, st, tm);
}

}  // namespace mcx
