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
template <int EMODE, int MODE, int SPLIT, int EXT>
struct Layout {
    static constexpr bool CE = EMODE == EMODE_CE;
    static constexpr bool GG = MODE != MODE_FWD;
    static constexpr bool TM = EXT != 0;                // particle time and weight
    // pass A: track length; weighted pass B: the running score (the slot is
    // carried by every extended pass B)
    static constexpr bool LL = MODE == MODE_REPLAY_A || (MODE == MODE_REPLAY_B && TM);
    static constexpr bool AA = MODE == MODE_REPLAY_A && TM;   // weighted pass A: absolute score
    static constexpr bool DIGEST = MODE == MODE_FWD;   // present only when digests are requested
    static constexpr int D_E = 6;
    static constexpr int D_G = D_E + (CE ? 1 : 0);
    static constexpr int D_L = D_G + (GG ? 1 : 0);
    static constexpr int D_A = D_L + (LL ? 1 : 0);
    static constexpr int D_T = D_A + (AA ? 1 : 0);
    static constexpr int D_W = D_T + (TM ? 1 : 0);
    static constexpr int D_HQ = D_W + (TM ? 1 : 0);
    static constexpr int ND_CORE = D_HQ;                // without the digest field
    static constexpr int U_NS = 4;                      // extended state: copies split off so far
    static constexpr int NU_CORE = 4 + (TM ? 1 : 0);    // hid, step, gc, prob (+ copies) (+ ncoll)
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
__device__ __forceinline__ double *dptr(const SoA &s, long i, int f) { return dfield(s, f) + i; }
__device__ __forceinline__ uint32_t *uptr(const SoA &s, long i, int f) { return ufield(s, f) + i; }

// 64-particle tiles (the event stacks): particle i lives in tile i/64 at
// lane i%64; in a tile the 8-byte fields take 512 bytes each, then the 4-byte
// fields 256 bytes each.  A wavefront touching 64 consecutive particles makes
// one contiguous access per field, and every field's address is the lane's
// tile address plus a constant, so no per-field base pointers are kept.
struct Tiles {
    char *base;
    long tile_bytes;
    int nd;
};

__device__ __forceinline__ char *tile_of(const Tiles &t, long i) { return t.base + (i >> 6) * t.tile_bytes; }
__device__ __forceinline__ double *dptr(const Tiles &t, long i, int f)
{
    return (double *)(tile_of(t, i) + f * 512) + (i & 63);
}
__device__ __forceinline__ uint32_t *uptr(const Tiles &t, long i, int f)
{
    return (uint32_t *)(tile_of(t, i) + t.nd * 512 + f * 256) + (i & 63);
}

template <class LAY, class R>
__device__ __forceinline__ void put(const R &s, long i, const Part &p, bool dig)
{
    *dptr(s, i, 0) = p.x;
    *dptr(s, i, 1) = p.y;
    *dptr(s, i, 2) = p.z;
    *dptr(s, i, 3) = p.u;
    *dptr(s, i, 4) = p.v;
    *dptr(s, i, 5) = p.w;
    if (LAY::CE) *dptr(s, i, LAY::D_E) = p.e;
    if (LAY::GG) *dptr(s, i, LAY::D_G) = p.G;
    if (LAY::LL) *dptr(s, i, LAY::D_L) = p.L;
    if (LAY::AA) *dptr(s, i, LAY::D_A) = p.A;
    if (LAY::TM) {
        *dptr(s, i, LAY::D_T) = p.t;
        *dptr(s, i, LAY::D_W) = p.wgt;
    }
    *uptr(s, i, 0) = p.hid;
    *uptr(s, i, 1) = p.step;
    *uptr(s, i, 2) = p.gc;
    *uptr(s, i, 3) = p.prob;
    if (LAY::TM) *uptr(s, i, LAY::U_NS) = p.nsplit;
    if (LAY::DIGEST && dig) {
        *(long long *)dptr(s, i, LAY::D_HQ) = p.hq;
        *uptr(s, i, LAY::NU_CORE) = p.ncoll;
    }
}

template <class LAY, class R>
__device__ __forceinline__ void get(const R &s, long i, Part &p, bool dig)
{
    p.x = *dptr(s, i, 0);
    p.y = *dptr(s, i, 1);
    p.z = *dptr(s, i, 2);
    p.u = *dptr(s, i, 3);
    p.v = *dptr(s, i, 4);
    p.w = *dptr(s, i, 5);
    p.e = LAY::CE ? *dptr(s, i, LAY::D_E) : 0.0;
    p.sigt = 0.0;
    p.G = LAY::GG ? *dptr(s, i, LAY::D_G) : 0.0;
    p.L = LAY::LL ? *dptr(s, i, LAY::D_L) : 0.0;
    p.A = LAY::AA ? *dptr(s, i, LAY::D_A) : 0.0;
    p.t = LAY::TM ? *dptr(s, i, LAY::D_T) : 0.0;
    p.wgt = LAY::TM ? *dptr(s, i, LAY::D_W) : 1.0;
    p.hid = *uptr(s, i, 0);
    p.step = *uptr(s, i, 1);
    p.gc = *uptr(s, i, 2);
    p.prob = *uptr(s, i, 3);
    p.nsplit = LAY::TM ? *uptr(s, i, LAY::U_NS) : 0u;
    p.hq = 0;
    p.ncoll = 0;
    if (LAY::DIGEST && dig) {
        p.hq = *(const long long *)dptr(s, i, LAY::D_HQ);
        p.ncoll = *uptr(s, i, LAY::NU_CORE);
    }
}

// copy particle i of one region to particle j of another (same layout)
__device__ __forceinline__ void copy_slot(const SoA &dst, long j, const SoA &src, long i, int nd, int nu)
{
    for (int f = 0; f < nd; ++f) dfield(dst, f)[j] = dfield(src, f)[i];
    for (int f = 0; f < nu; ++f) ufield(dst, f)[j] = ufield(src, f)[i];
}

}  // namespace mcx
