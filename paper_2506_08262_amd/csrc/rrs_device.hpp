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
