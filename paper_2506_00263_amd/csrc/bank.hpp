// Structure-of-arrays particle storage used between events: the stack
// scheduler's per-event stacks in HBM, the asynchronous scheduler's work
// links in LDS and its spill arena in HBM all share this layout.  A region
// holds `cap` particles as nd arrays of 8-byte fields followed by nu arrays
// of 4-byte fields, so lane i of a wavefront touching particle base+i makes
// one coalesced access per field.
#pragma once
#include "transport.hpp"

namespace mcx {

// Which fields a particle carries for an event program.
template <int EMODE, int MODE, int SPLIT>
struct Layout {
    static constexpr bool CE = EMODE == EMODE_CE;
    static constexpr bool SIG = SPLIT != 0;
    static constexpr bool GG = MODE != MODE_FWD;
    static constexpr bool LL = MODE == MODE_REPLAY_A;
    static constexpr bool DIGEST = MODE == MODE_FWD;   // present only when digests are requested
    static constexpr int D_E = 6;
    static constexpr int D_SIG = D_E + (CE ? 1 : 0);
    static constexpr int D_G = D_SIG + (SIG ? 1 : 0);
    static constexpr int D_L = D_G + (GG ? 1 : 0);
    static constexpr int D_HQ = D_L + (LL ? 1 : 0);
    static constexpr int ND_CORE = D_HQ;                // without the digest field
    static constexpr int NU_CORE = 4;                   // hid, step, gc, prob (+ ncoll)
    __host__ __device__ static int nd(bool dig) { return ND_CORE + ((DIGEST && dig) ? 1 : 0); }
    __host__ __device__ static int nu(bool dig) { return NU_CORE + ((DIGEST && dig) ? 1 : 0); }
    __host__ __device__ static int bytes(bool dig) { return nd(dig) * 8 + nu(dig) * 4; }
};

struct SoA {
    char *base;
    long cap;
    int nd;
};

__device__ __forceinline__ double *dfield(const SoA &s, int f) { return (double *)s.base + (long)f * s.cap; }
__device__ __forceinline__ uint32_t *ufield(const SoA &s, int f)
{
    return (uint32_t *)(s.base + (long)s.nd * s.cap * 8) + (long)f * s.cap;
}

template <class LAY>
__device__ __forceinline__ void put(const SoA &s, long i, const Part &p, bool dig)
{
    dfield(s, 0)[i] = p.x;
    dfield(s, 1)[i] = p.y;
    dfield(s, 2)[i] = p.z;
    dfield(s, 3)[i] = p.u;
    dfield(s, 4)[i] = p.v;
    dfield(s, 5)[i] = p.w;
    if (LAY::CE) dfield(s, LAY::D_E)[i] = p.e;
    if (LAY::SIG) dfield(s, LAY::D_SIG)[i] = p.sigt;
    if (LAY::GG) dfield(s, LAY::D_G)[i] = p.G;
    if (LAY::LL) dfield(s, LAY::D_L)[i] = p.L;
    ufield(s, 0)[i] = p.hid;
    ufield(s, 1)[i] = p.step;
    ufield(s, 2)[i] = p.gc;
    ufield(s, 3)[i] = p.prob;
    if (LAY::DIGEST && dig) {
        ((long long *)dfield(s, LAY::D_HQ))[i] = p.hq;
        ufield(s, 4)[i] = p.ncoll;
    }
}

template <class LAY>
__device__ __forceinline__ void get(const SoA &s, long i, Part &p, bool dig)
{
    p.x = dfield(s, 0)[i];
    p.y = dfield(s, 1)[i];
    p.z = dfield(s, 2)[i];
    p.u = dfield(s, 3)[i];
    p.v = dfield(s, 4)[i];
    p.w = dfield(s, 5)[i];
    p.e = LAY::CE ? dfield(s, LAY::D_E)[i] : 0.0;
    p.sigt = LAY::SIG ? dfield(s, LAY::D_SIG)[i] : 0.0;
    p.G = LAY::GG ? dfield(s, LAY::D_G)[i] : 0.0;
    p.L = LAY::LL ? dfield(s, LAY::D_L)[i] : 0.0;
    p.hid = ufield(s, 0)[i];
    p.step = ufield(s, 1)[i];
    p.gc = ufield(s, 2)[i];
    p.prob = ufield(s, 3)[i];
    p.hq = 0;
    p.ncoll = 0;
    if (LAY::DIGEST && dig) {
        p.hq = ((const long long *)dfield(s, LAY::D_HQ))[i];
        p.ncoll = ufield(s, 4)[i];
    }
}

// copy particle i of one region to particle j of another (same layout)
__device__ __forceinline__ void copy_slot(const SoA &dst, long j, const SoA &src, long i, int nd, int nu)
{
    for (int f = 0; f < nd; ++f) dfield(dst, f)[j] = dfield(src, f)[i];
    for (int f = 0; f < nu; ++f) ufield(dst, f)[j] = ufield(src, f)[i];
}

}  // namespace mcx
