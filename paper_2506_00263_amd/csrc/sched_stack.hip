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
// host round trip: round r reads sizes[r%3], pops with heads[r%3], pushes
// with sizes[(r+1)%3], and clears the sets round r+1 will need
// (sizes[(r+2)%3], heads[(r+1)%3]).  The host polls a done flag (first round
// that finds no input and no source left) every few rounds.
#include <algorithm>

#include "bank.hpp"
#include "kernels.hpp"

namespace mcx {

struct StackArgs {
    const ProbDev *probs;
    int n_probs;
    const unsigned long long *prefix;
    unsigned long long total;
    RunCtl *ctl;
    Digest *digest;
    char *bank[2];              // [event][nd doubles, nu words] x cap
    long cap;
    long region_bytes;          // bytes of one event stack
    unsigned int *sizes;        // [3][E]
    unsigned int *heads;        // [3][E]
    unsigned int threshold;
    int lacc_words;
};

__device__ __forceinline__ unsigned int wave_claim(unsigned int *ctr, unsigned int n)
{
    unsigned int b = 0;
    if (__lane_id() == 0) b = atomicAdd(ctr, n);
    return __builtin_amdgcn_readfirstlane(b);
}

template <class LAY, int E>
__device__ __forceinline__ void push(const StackArgs &A, char *bank, unsigned int *size_out, bool act, int ne,
                                     const Part &p, bool dig, uint32_t &err)
{
#pragma unroll
    for (int k = 0; k < E; ++k) {
        bool mine = act && ne == k;
        uint64_t mask = __ballot(mine);
        if (mask == 0) continue;
        unsigned int cnt = (unsigned int)__popcll(mask);
        unsigned int b = 0;
        if (__lane_id() == 0) b = atomicAdd(&size_out[k], cnt);
        b = __builtin_amdgcn_readfirstlane(b);
        if (mine) {
            unsigned long slot = (unsigned long)b + lane_rank(mask);
            if (slot < (unsigned long)A.cap) {
                SoA s{bank + (long)k * A.region_bytes, A.cap, LAY::nd(dig)};
                put<LAY>(s, (long)slot, p, dig);
            } else {
                err |= ERR_CAPACITY;
            }
        }
    }
}

template <int GEOM, int EMODE, int MODE, int SPLIT, bool BATCH>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) stack_round(StackArgs A, int round)
{
    using LAY = Layout<EMODE, MODE, SPLIT>;
    constexpr int E = SPLIT ? 4 : 1;
    extern __shared__ unsigned long long lacc[];
    const bool dig = A.digest != nullptr;
    unsigned int *size_in = A.sizes + (round % 3) * E;
    unsigned int *head = A.heads + (round % 3) * E;
    unsigned int *size_out = A.sizes + ((round + 1) % 3) * E;
    char *bin = A.bank[round & 1];
    char *bout = A.bank[(round + 1) & 1];
    if (blockIdx.x == 0 && threadIdx.x < E) {
        A.sizes[((round + 2) % 3) * E + threadIdx.x] = 0;
        A.heads[((round + 1) % 3) * E + threadIdx.x] = 0;
    }
    // no input and no source left: the previous round finished the run
    unsigned int n_any = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) n_any |= size_in[e];
    unsigned long long cursor = __hip_atomic_load(&A.ctl->src_cursor, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (n_any == 0 && cursor >= A.total) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && A.ctl->done_round == 0) A.ctl->done_round = (unsigned)round + 1;
        return;
    }
    EvCtx cx{A.probs, A.digest, (MODE == MODE_REPLAY_B && A.lacc_words > 0) ? lacc : nullptr, BATCH ? 0 : 1};
    if (cx.lacc) {
        lacc_zero(lacc, A.lacc_words);
        __syncthreads();
    }
    Lane ln{0, 0, 0, 0};
    WaveCount wc;
    wc.zero();
    const int lane = __lane_id();
    // drain the input stacks
#pragma unroll 1
    for (int e = 0; e < E; ++e) {
        unsigned int n_in = size_in[e];
        if (n_in > (unsigned int)A.cap) n_in = (unsigned int)A.cap;
        SoA sin{bin + (long)e * A.region_bytes, A.cap, LAY::nd(dig)};
        for (;;) {
            unsigned int base = wave_claim(&head[e], 64);
            if (base >= n_in) break;
            bool act = base + lane < n_in;
            Part p;
            int ne = EV_DEAD;
            uint32_t out = 0;
            if (act) {
                get<LAY>(sin, (long)(base + lane), p, dig);
                const ProbDev &P = A.probs[BATCH ? (int)p.prob : 0];
                ne = run_event<GEOM, EMODE, MODE, SPLIT>(e, P, cx, ln, p, out);
            }
            wc.dispatch(act);
            wc.outcomes(act, out);
            push<LAY, E>(A, bout, size_out, act, ne, p, dig, ln.err);
        }
    }
    // make_work: source new histories until the fullest output stack passes
    // the threshold or the source is exhausted
    for (;;) {
        unsigned long long cur = __hip_atomic_load(&A.ctl->src_cursor, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur >= A.total) break;
        unsigned int fullest = 0;
#pragma unroll
        for (int k = 0; k < E; ++k) {
            unsigned int s = __hip_atomic_load(&size_out[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            fullest = s > fullest ? s : fullest;
        }
        if (fullest >= A.threshold) break;
        unsigned long long b = 0;
        if (lane == 0) b = atomicAdd(&A.ctl->src_cursor, 64ull);
        b = ((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(b >> 32)) << 32) |
            (unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)b);
        if (b >= A.total) break;
        unsigned long long gid = b + lane;
        bool act = gid < A.total;
        Part p;
        if (act) {
            int pi = BATCH ? find_problem(A.prefix, A.n_probs, gid) : 0;
            const ProbDev &P = A.probs[pi];
            source<GEOM, MODE>(P, p, (uint32_t)(P.first + (gid - P.gbase)), (uint32_t)pi);
        }
        wc.outcomes(act, O_SOURCE);
        wc.c[C_MAKE_WORK] += 1;
        push<LAY, E>(A, bout, size_out, act, EV_STEP, p, dig, ln.err);
    }
    flush_wave(A.ctl, wc, ln, A.probs, BATCH ? 0 : 1, MODE);
    if (cx.lacc) {
        __syncthreads();
        lacc_flush(lacc, A.probs[0]);
    }
}

template <int GEOM, int EMODE, int MODE, int SPLIT, bool BATCH>
static hipError_t stack_t(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm, unsigned int *flag)
{
    using LAY = Layout<EMODE, MODE, SPLIT>;
    constexpr int E = SPLIT ? 4 : 1;
    const bool dig = a.digest != nullptr;
    const int block = 256;
    int wpc = a.waves_per_cu > 0 ? a.waves_per_cu : 16;
    long blocks = std::max(1L, (long)a.num_cus * wpc / (block / 64));
    long slack = 2 * (blocks * (block / 64) * 64 + 64);
    long cap = a.stack_capacity > 0 ? (long)a.stack_capacity : (long)a.total + slack;
    const long cap_max = 1L << 24;
    if (cap > cap_max + slack) cap = cap_max + slack;
    cap = (cap + 63) / 64 * 64;
    long thr;
    if (a.stack_threshold > 0) thr = (long)a.stack_threshold;
    else if (cap >= (long)a.total + slack) thr = cap;
    else thr = std::max(64L, (cap - slack) / E);
    if (thr > 0xFFFFFFFFL) thr = 0xFFFFFFFFL;
    long region = (long)LAY::bytes(dig) * cap;
    region = (region + 255) / 256 * 256;
    size_t need = (size_t)region * E * 2 + 256 * 2;
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
    A.bank[1] = (char *)ws.ptr + (size_t)region * E;
    A.cap = cap;
    A.region_bytes = region;
    A.sizes = (unsigned int *)((char *)ws.ptr + (size_t)region * E * 2);
    A.heads = A.sizes + 32;
    A.threshold = (unsigned int)thr;
    A.lacc_words = a.lacc_words;
    e = hipMemsetAsync(A.sizes, 0, 512, a.stream);
    if (e != hipSuccess) return e;
    size_t lds = (size_t)a.lacc_words * 8;
    st.grid_blocks = (int)blocks;
    st.block_threads = block;
    st.lds_bytes = (int)lds;
    int round = 0;
    int batch = 4;
    for (;;) {
        for (int i = 0; i < batch; ++i) {
            tm.begin();
            hipLaunchKernelGGL((stack_round<GEOM, EMODE, MODE, SPLIT, BATCH>), dim3((unsigned)blocks), dim3(block), lds,
                               a.stream, A, round);
            tm.end();
            ++round;
            st.launches += 1;
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        // error and done_round are adjacent words of the control block
        e = hipMemcpyAsync(flag, &a.ctl->error, 8, hipMemcpyDeviceToHost, a.stream);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(a.stream);
        if (e != hipSuccess) return e;
        if (flag[1] != 0) {
            st.rounds = flag[1];
            break;
        }
        if (flag[0] & ERR_CAPACITY) {
            st.rounds = (unsigned long long)round;
            break;
        }
        if (batch < 64) batch *= 2;
        if (round > (1 << 30)) return hipErrorLaunchTimeOut;
    }
    return hipSuccess;
}

template <int GEOM, int EMODE, int MODE, int SPLIT>
static hipError_t stack_b(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm, unsigned int *flag)
{
    return a.n_probs > 1 ? stack_t<GEOM, EMODE, MODE, SPLIT, true>(a, ws, st, tm, flag)
                         : stack_t<GEOM, EMODE, MODE, SPLIT, false>(a, ws, st, tm, flag);
}

template <int GEOM, int EMODE, int MODE>
static hipError_t stack_s(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm, unsigned int *flag)
{
    return a.split ? stack_b<GEOM, EMODE, MODE, 1>(a, ws, st, tm, flag) : stack_b<GEOM, EMODE, MODE, 0>(a, ws, st, tm, flag);
}

hipError_t launch_stack(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm, unsigned int *flag)
{
    if (a.emode == EMODE_CE) {
        if (a.geom != GEOM_LATTICE || a.mode != MODE_FWD) return hipErrorInvalidValue;
        return stack_s<GEOM_LATTICE, EMODE_CE, MODE_FWD>(a, ws, st, tm, flag);
    }
    if (a.geom == GEOM_BOX) {
        if (a.mode == MODE_FWD) return stack_s<GEOM_BOX, EMODE_MG, MODE_FWD>(a, ws, st, tm, flag);
        if (a.mode == MODE_REPLAY_A) return stack_s<GEOM_BOX, EMODE_MG, MODE_REPLAY_A>(a, ws, st, tm, flag);
        return stack_s<GEOM_BOX, EMODE_MG, MODE_REPLAY_B>(a, ws, st, tm, flag);
    }
    if (a.mode == MODE_FWD) return stack_s<GEOM_LATTICE, EMODE_MG, MODE_FWD>(a, ws, st, tm, flag);
    if (a.mode == MODE_REPLAY_A) return stack_s<GEOM_LATTICE, EMODE_MG, MODE_REPLAY_A>(a, ws, st, tm, flag);
    return stack_s<GEOM_LATTICE, EMODE_MG, MODE_REPLAY_B>(a, ws, st, tm, flag);
}

}  // namespace mcx
