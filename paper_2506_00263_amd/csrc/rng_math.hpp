// Device primitives of the transport kernels: counter-based random numbers
// and deterministic FP64 elementary functions built only from IEEE +, -, *,
// / (no fused multiply-add: the library is compiled with contraction off),
// so every lane, wavefront, scheduler and launch shape computes the same
// bits for the same inputs.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace mcx {

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).  Each round multiplies
// counter words 0 and 2 by the round multipliers; the high halves are xored
// with the other two words and the round key; the key advances by the Weyl
// increments between rounds.
struct Key {
    uint32_t k0, k1;
};

__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, Key k)
{
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t k0 = k.k0, k1 = k.k1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)M0 * c0;     // one 32x32->64 multiply each
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    return make_uint4(c0, c1, c2, c3);
}

// 53 random bits, lowest forced to one: a double in [2^-53, 1 - 2^-53].
__device__ __forceinline__ double to_unit(uint32_t hi, uint32_t lo)
{
    uint64_t v = ((uint64_t)hi << 32) | (uint64_t)lo;
    return (double)((v >> 11) | 1ull) * 0x1p-53;
}

// The two deviates of slots 2*pair and 2*pair+1 of flight `step` of history
// `hist`: one Philox call on counter (hist, step, pair, stream).
__device__ __forceinline__ void uniform_pair(Key k, uint32_t hist, uint32_t step, uint32_t pair, double &a,
                                             double &b, uint32_t stream = 0)
{
    uint4 r = philox4x32_10(hist, step, pair, stream, k);
    a = to_unit(r.x, r.y);
    b = to_unit(r.z, r.w);
}

// ------------------------------------------------ constants (compile time)
// (evaluated by the compiler: every coefficient is a template constant)
constexpr double fact(int n) { return n <= 1 ? 1.0 : fact(n - 1) * (double)n; }   // exact to 22!
template <int K> struct AtanhC { static constexpr double v = 2.0 / (double)(2 * K + 1); };
template <int K> struct CosC { static constexpr double v = ((K & 1) ? -1.0 : 1.0) / fact(2 * K); };
template <int K> struct SinC { static constexpr double v = ((K & 1) ? -1.0 : 1.0) / fact(2 * K + 1); };
#define atanh_coef(k) (AtanhC<k>::v)
#define cos_coef(k) (CosC<k>::v)
#define sin_coef(k) (SinC<k>::v)

// ln 2 split: the head keeps 42 significant bits so e * head is exact for
// every binary64 exponent; tail = ln 2 - head rounded.
constexpr double LN2_HEAD = 0x1.62e42fefa38p-1;
constexpr double LN2_TAIL = 0x1.ef35793c7673p-45;
constexpr double ROOT2 = 0x1.6a09e667f3bcdp+0;
constexpr double HALF_PI = 0x1.921fb54442d18p+0;

// -ln(x), x positive and normal.  x = m 2^e from the bit pattern, m folded
// into [sqrt2/2, sqrt2]; ln m = 2 atanh(s) with s = (m-1)/(m+1), evaluated
// as s * sum_{k=0..10} (2/(2k+1)) s^(2k) by Horner's rule.
__device__ __forceinline__ double neg_log(double x)
{
    uint64_t bits = (uint64_t)__double_as_longlong(x);
    int ex = (int)((bits >> 52) & 0x7ffu) - 1023;
    double m = __longlong_as_double((long long)((bits & 0x000fffffffffffffull) | 0x3ff0000000000000ull));
    if (m > ROOT2) {
        m = m * 0.5;
        ex = ex + 1;
    }
    double s = (m - 1.0) / (m + 1.0);
    double z = s * s;
    double p = atanh_coef(10);
    p = (p * z) + atanh_coef(9);
    p = (p * z) + atanh_coef(8);
    p = (p * z) + atanh_coef(7);
    p = (p * z) + atanh_coef(6);
    p = (p * z) + atanh_coef(5);
    p = (p * z) + atanh_coef(4);
    p = (p * z) + atanh_coef(3);
    p = (p * z) + atanh_coef(2);
    p = (p * z) + atanh_coef(1);
    p = (p * z) + atanh_coef(0);
    double lnm = s * p;
    double de = (double)ex;
    return -((de * LN2_HEAD) + ((de * LN2_TAIL) + lnm));
}

// sqrt(x): reciprocal square root by Newton's method from the binary64
// fast-inverse-square-root guess (0x5FE6EB50C7B537A9 - bits/2), four steps
// y <- y (3/2 - (x/2) y^2), then s = x y and one residual correction
// s <- s + ((x - s^2)/2) y.  Non-positive (and NaN) inputs give 0; inputs
// below 2^-1000 are scaled by 2^1000 (result by 2^-500).
__device__ __forceinline__ double root(double x)
{
    if (!(x > 0.0)) return 0.0;
    double scale = 1.0;
    if (x < 0x1p-1000) {
        x = x * 0x1p+1000;
        scale = 0x1p-500;
    }
    uint64_t bits = (uint64_t)__double_as_longlong(x);
    double y = __longlong_as_double((long long)(0x5FE6EB50C7B537A9ull - (bits >> 1)));
    double hx = 0.5 * x;
    y = y * (1.5 - ((hx * y) * y));
    y = y * (1.5 - ((hx * y) * y));
    y = y * (1.5 - ((hx * y) * y));
    y = y * (1.5 - ((hx * y) * y));
    double s = x * y;
    s = s + ((0.5 * (x - (s * s))) * y);
    return s * scale;
}

// (cos 2 pi t, sin 2 pi t): q = floor(4t), r = 4t - q (exact), recentred to
// |r| <= 1/2; x = r pi/2; Taylor polynomials in x^2 (cos to x^20, sin to
// x^21); the quadrant q mod 4 rotates the pair by exact sign swaps.
__device__ __forceinline__ void turn_cos_sin(double t, double &c, double &s)
{
    double t4 = 4.0 * t;
    double qd = floor(t4);
    double r = t4 - qd;
    int q = (int)qd;
    if (r > 0.5) {
        r = r - 1.0;
        q = q + 1;
    }
    double x = r * HALF_PI;
    double x2 = x * x;
    double cc = cos_coef(10);
    cc = (cc * x2) + cos_coef(9);
    cc = (cc * x2) + cos_coef(8);
    cc = (cc * x2) + cos_coef(7);
    cc = (cc * x2) + cos_coef(6);
    cc = (cc * x2) + cos_coef(5);
    cc = (cc * x2) + cos_coef(4);
    cc = (cc * x2) + cos_coef(3);
    cc = (cc * x2) + cos_coef(2);
    cc = (cc * x2) + cos_coef(1);
    cc = (cc * x2) + cos_coef(0);
    double ss = sin_coef(10);
    ss = (ss * x2) + sin_coef(9);
    ss = (ss * x2) + sin_coef(8);
    ss = (ss * x2) + sin_coef(7);
    ss = (ss * x2) + sin_coef(6);
    ss = (ss * x2) + sin_coef(5);
    ss = (ss * x2) + sin_coef(4);
    ss = (ss * x2) + sin_coef(3);
    ss = (ss * x2) + sin_coef(2);
    ss = (ss * x2) + sin_coef(1);
    ss = (ss * x2) + sin_coef(0);
    ss = x * ss;
    switch (q & 3) {
    case 0: c = cc; s = ss; break;
    case 1: c = -ss; s = cc; break;
    case 2: c = -cc; s = -ss; break;
    default: c = ss; s = -cc; break;
    }
}

// fixed point: rint(x * 2^S), round half to even (v_rndne_f64)
__device__ __forceinline__ int64_t to_fixed(double x, double two_pow_s)
{
    return (int64_t)__builtin_rint(x * two_pow_s);
}

}  // namespace mcx
