// rrs_device.hpp -- device-side random stream and special functions of the
// RRS direction generator (gfx950).
//
// The direction generator of RRS (Alg. S1 sphere, Alg. S4 cap) needs Gaussian
// variates.  They come from a counter-based Philox4x64-10 stream (Salmon et
// al., SC'11) so that any (query, refinement, direction) can be generated
// independently by any lane, and from Box-Muller with log / sin / cos written
// here from their series.  Every operation is a single IEEE binary64 operation
// or an explicit fma, compiled with -ffp-contract=off, so the values are fixed
// by the order written below.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rrs_launch.hpp"

namespace rrs {

// One select that took the exact fallback (profiling only).
__device__ __forceinline__ void stat_fallback(uint32_t *stats) { atomicAdd(&stats[1], 1u); }

// ---------------------------------------------------------------------------
// Philox4x64-10: two 64x64->128 multiplies per round, Weyl key schedule.
// ---------------------------------------------------------------------------
struct Block4 {
    uint64_t w0, w1, w2, w3;
};

__device__ __forceinline__ Block4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2,
                                                uint64_t c3, uint64_t k0, uint64_t k1)
{
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ULL;
    constexpr uint64_t M1 = 0xCA5A826395121157ULL;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ULL;
    constexpr uint64_t W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t lo0 = M0 * c0;
        const uint64_t hi0 = __umul64hi(M0, c0);
        const uint64_t lo1 = M1 * c2;
        const uint64_t hi1 = __umul64hi(M1, c2);
        const uint64_t n0 = hi1 ^ c1 ^ k0;
        const uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return Block4{c0, c1, c2, c3};
}

// Block b of the word stream of direction (q, l, j) under key (seed, 0).
__device__ __forceinline__ Block4 dir_block(uint64_t seed, uint64_t q, uint64_t l,
                                            uint64_t j, uint64_t b)
{
    return philox4x64_10(b, j, l, q, seed, 0);
}

// Open uniform in (0,1) with 52 random bits: ((w >> 12) + 0.5) * 2^-52.
__device__ __forceinline__ double uniform_open(uint64_t w)
{
    return ((double)(w >> 12) + 0.5) * 0x1p-52;
}

// ---------------------------------------------------------------------------
// log x for normal x > 0 from the atanh series: x = m 2^e, m in
// [sqrt(1/2), sqrt(2)), ln m = 2 atanh((m-1)/(m+1)).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double log_series(double x)
{
    constexpr double kLn2 = 0x1.62e42fefa39efp-1;
    constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;
    // split x into mantissa in [0.5, 1) and exponent (x is a normal number)
    const uint64_t bits = (uint64_t)__double_as_longlong(x);
    int e = (int)((bits >> 52) & 0x7FF) - 1022;
    double m = __longlong_as_double((long long)((bits & 0x000FFFFFFFFFFFFFULL) |
                                                0x3FE0000000000000ULL));
    if (m < kSqrtHalf) {
        m = m * 2.0;
        e = e - 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double s2 = s * s;
    double p = 1.0 / 23.0;
    p = fma(p, s2, 1.0 / 21.0);
    p = fma(p, s2, 1.0 / 19.0);
    p = fma(p, s2, 1.0 / 17.0);
    p = fma(p, s2, 1.0 / 15.0);
    p = fma(p, s2, 1.0 / 13.0);
    p = fma(p, s2, 1.0 / 11.0);
    p = fma(p, s2, 1.0 / 9.0);
    p = fma(p, s2, 1.0 / 7.0);
    p = fma(p, s2, 1.0 / 5.0);
    p = fma(p, s2, 1.0 / 3.0);
    const double at = fma(s * s2, p, s);
    return fma((double)e, kLn2, 2.0 * at);
}

// sin and cos of (pi/2) f, f in [0, 1], by Taylor series on [0, pi/4].
__device__ __forceinline__ void sincos_halfpi(double f, double &sn, double &cs)
{
    constexpr double kPio2 = 0x1.921fb54442d18p+0;
    const bool swap = f > 0.5;
    const double g = swap ? 1.0 - f : f;
    const double x = g * kPio2;
    const double z = x * x;
    double ps = 1.0 / 355687428096000.0;
    ps = fma(ps, z, -1.0 / 1307674368000.0);
    ps = fma(ps, z, 1.0 / 6227020800.0);
    ps = fma(ps, z, -1.0 / 39916800.0);
    ps = fma(ps, z, 1.0 / 362880.0);
    ps = fma(ps, z, -1.0 / 5040.0);
    ps = fma(ps, z, 1.0 / 120.0);
    ps = fma(ps, z, -1.0 / 6.0);
    const double s = fma(x * z, ps, x);
    double pc = 1.0 / 20922789888000.0;
    pc = fma(pc, z, -1.0 / 87178291200.0);
    pc = fma(pc, z, 1.0 / 479001600.0);
    pc = fma(pc, z, -1.0 / 3628800.0);
    pc = fma(pc, z, 1.0 / 40320.0);
    pc = fma(pc, z, -1.0 / 720.0);
    pc = fma(pc, z, 1.0 / 24.0);
    pc = fma(pc, z, -1.0 / 2.0);
    const double c = fma(z, pc, 1.0);
    sn = swap ? c : s;
    cs = swap ? s : c;
}

// Area-uniform polar angle in the cap of half-angle (pi/2) phi in d
// dimensions: the angle's density is proportional to sin^(d-2), so with
// x = sin(theta) the distribution function is F = J(x) / J(x_e),
// J(x) = x^(d-1) T(x), T(x) = sum_k c_k x^(2k) / (d - 1 + 2k),
// c_0 = 1, c_(k+1) = c_k (2k + 1) / (2k + 2) (the series of 1 / sqrt(1 - x^2)
// integrated term by term), x_e = sin((pi/2) phi).  For uniform u, Newton's
// method on g(y) = y^(d-1) T(x_e y) - u T(x_e) from y = 1 (g is increasing
// and convex, so the iterates decrease monotonically to the root) gives
// x = x_e y; returns sin(theta) = x and cos(theta) = sqrt((1 - x)(1 + x)).
// The series stops at the first term below 2^-60 of the sum (at most 200000
// terms; the calls accept the law only for cap_shrink <= 0.99 and caps below
// the hemisphere, where this is accurate to about 1e-10).
__device__ __forceinline__ void cap_series(double x, int64_t n1, double &T, double &R)
{
    // T = sum_k t_k, R = sum_k 2k t_k, t_k = c_k x^(2k) / (n1 + 2k)
    const double x2 = x * x;
    double c = 1.0, p = 1.0;
    T = 0.0;
    R = 0.0;
    for (int64_t k = 0; k < 200000; ++k) {
        const double t = (c * p) / (double)(n1 + 2 * k);
        T = T + t;
        R = R + (double)(2 * k) * t;
        if (t <= 0x1p-60 * T) break;
        p = p * x2;
        c = (c * (double)(2 * k + 1)) / (double)(2 * k + 2);
    }
}

__device__ __forceinline__ double pow_int(double y, int64_t e)
{
    double r = 1.0, b = y;
    while (e > 0) {
        if (e & 1) r = r * b;
        e >>= 1;
        if (e > 0) b = b * b;
    }
    return r;
}

__device__ __forceinline__ void area_cap_angle(double u, double phi, int64_t d, double &st,
                                               double &ct)
{
    const int64_t n1 = d - 1;
    double xe, ce;
    sincos_halfpi(phi, xe, ce);
    double Te, Re;
    cap_series(xe, n1, Te, Re);
    const double target = u * Te;
    double y = 1.0;
    for (int it = 0; it < 200; ++it) {
        const double x = xe * y;
        double T, R;
        cap_series(x, n1, T, R);
        const double P = pow_int(y, n1);
        const double g = P * T - target;
        const double gp = (P / y) * ((double)n1 * T + R);
        const double yn = y - g / gp;
        if (!(yn < y)) break;
        y = yn;
    }
    const double x = xe * y;
    st = x;
    ct = sqrt((1.0 - x) * (1.0 + x));
}

// Box-Muller pair from two stream words.
__device__ __forceinline__ void gauss_pair(uint64_t w1, uint64_t w2, double &g1, double &g2)
{
    const double u1 = uniform_open(w1);
    const double u2 = uniform_open(w2);
    const double r = sqrt(-2.0 * log_series(u1));
    const double v = 4.0 * u2;
    const double qd = floor(v);
    const double f = v - qd;
    double s, c;
    sincos_halfpi(f, s, c);
    const int quad = (int)qd;
    double ct, st;
    if (quad == 0) {
        ct = c;
        st = s;
    } else if (quad == 1) {
        ct = -s;
        st = c;
    } else if (quad == 2) {
        ct = -c;
        st = -s;
    } else {
        ct = s;
        st = -c;
    }
    g1 = r * ct;
    g2 = r * st;
}

// Order-preserving map of binary64 to uint64 (total order with -0 < +0).
__device__ __forceinline__ uint64_t order_key(double x)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ULL);
}

__device__ __forceinline__ double key_value(uint64_t k)
{
    const uint64_t b = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFULL) : ~k;
    return __longlong_as_double((long long)b);
}

}  // namespace rrs
