// rrs_select_common.hpp -- helpers shared by the order-statistic selects
// (internal): order-preserving 32-bit keys of binary64 values, the bracket
// key with a collapsed neighbourhood of zero, histogram scans and lane
// broadcasts.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace rrs {
namespace sel {

// Value of column entry t in phase PH and whether it takes part (used by the
// global-memory fallback; identical to the in-place register transforms).
template <int PH>
__device__ __forceinline__ bool phase_val(double t, double med, double &x)
{
    if (PH == 0) {
        x = t;
        return true;
    } else if (PH == 1) {
        x = fabs(t - med);
        return true;
    } else {
        x = t - med;
        return x > 0.0;
    }
}

// 32-bit key of a register value in phase PH.  Phase 0 values carry a sign;
// phases 1 and 2 are >= 0 or NaN, whose high words already order correctly.
// Returns 0xFFFFFFFF for NaN (and +inf in phase 0), which never takes part.
template <int PH>
__device__ __forceinline__ uint32_t key32(double x)
{
    const uint32_t hi = (uint32_t)__double2hiint(x);
    if (PH == 0) {
        const uint32_t m = (uint32_t)((int32_t)hi >> 31) | 0x80000000u;
        return hi ^ m;
    }
    return hi;
}

template <int PH>
__device__ __forceinline__ bool key_takes_part(uint32_t k);

// Wave-uniform broadcast of lane `src`'s double.
__device__ __forceinline__ double lane_bcast(double x, int src)
{
    const int lo = __double2loint(x), hi = __double2hiint(x);
    return __hiloint2double(__builtin_amdgcn_readlane(hi, src), __builtin_amdgcn_readlane(lo, src));
}

// Key used for binning.  With mag the high word of |x| (monotone in |x|):
// magnitudes below tau map to the key of zero, larger ones are offset by tau
// so that they start right next to it,
//   |x| < tau: 2^31;   x >= tau: 2^31 + 1 + (mag - tau);
//   x <= -tau: 2^31 - 1 - (mag - tau)           (phase 0 only).
// Monotone in x, and a bracket that straddles zero spends its key range on
// the magnitudes it holds instead of on the empty logarithmic range of tiny
// ones.  NaN keys exceed every finite key.
template <int PH>
__device__ __forceinline__ uint32_t bin_key(double x, uint32_t tau)
{
    const uint32_t hi = (uint32_t)__double2hiint(x);
    const uint32_t mag = hi & 0x7FFFFFFFu;
    const uint32_t dd = mag - tau;
    if (PH == 0) {
        if (mag < tau) return 0x80000000u;
        return (hi >> 31) ? 0x7FFFFFFFu - dd : 0x80000001u + dd;
    }
    return mag < tau ? 0u : 1u + dd;
}

template <int PH>
__device__ __forceinline__ bool key_takes_part(uint32_t k)
{
    // finite values: phase 0 keys < 0xFFF00000, phases 1/2 keys < 0x7FF00000
    return PH == 0 ? k < 0xFFF00000u : k < 0x7FF00000u;
}

// Bucket of a 256-bucket histogram holding rank k when the values below the
// histogram number `base`: lane `lane` of a wave owns buckets 4 lane .. 4 lane
// + 3 and reports found = true when the rank falls in them.
__device__ __forceinline__ void scan_hist(const uint32_t *hist, uint64_t base, uint64_t k,
                                          uint32_t &bin, uint32_t &before_in_bin,
                                          uint32_t &cnt, bool &found)
{
    const int lane = threadIdx.x & 63;
    const uint32_t h0 = hist[4 * lane], h1 = hist[4 * lane + 1];
    const uint32_t h2 = hist[4 * lane + 2], h3 = hist[4 * lane + 3];
    const uint32_t tot = h0 + h1 + h2 + h3;
    uint32_t incl = tot;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = (uint32_t)__shfl_up((int)incl, off);
        if (lane >= off) incl += o;
    }
    const uint64_t ex = base + incl - tot;
    found = ex <= k && k < ex + tot;
    uint64_t c = ex;
    if (k < c + h0) {
        bin = 4 * lane;
        cnt = h0;
    } else if (k < c + h0 + h1) {
        bin = 4 * lane + 1;
        cnt = h1;
        c += h0;
    } else if (k < c + h0 + h1 + h2) {
        bin = 4 * lane + 2;
        cnt = h2;
        c += h0 + h1;
    } else {
        bin = 4 * lane + 3;
        cnt = h3;
        c += h0 + h1 + h2;
    }
    before_in_bin = found ? (uint32_t)(k - c) : 0u;
}

}  // namespace sel
}  // namespace rrs
