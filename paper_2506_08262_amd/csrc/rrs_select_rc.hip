// rrs_select_rc.hip -- step a3 + a4 for projection and asymmetric projection
// depth from reduced-precision projections, with the order statistics made
// exact by recomputing only their neighbours in binary64.
//
// Input per column (query q, direction j): s_i = a_i.u_j in binary32 from the
// matrix cores (a_i = x_i - xbar), the centring term c_j (binary64) and a
// bound E with |(s_i - c_j) - t_i| <= E for every point, where t_i is the
// recipe's binary64 projection (x_i - z).u_j.  Ranks of s are ranks of s - c.
//
// One order statistic of rank k (or the pair k, k + 1):
//   1. 64 sampled approximations bracket the rank; one pass over the column
//      bins the approximations linearly over the bracket (256 bins of a
//      power-of-two width, one fma and a clamp per value), with the values
//      below and above the bracket counted in per-lane slots at either end;
//   2. the bins holding ranks k, k + 1 span approximations [vlo, vhi], so the
//      exact statistics lie in [vlo - E, vhi + E] (shifted by c); every point
//      whose approximation is below vlo - 2E is exactly below them, every one
//      above vhi + 2E exactly above.  A second pass collects the indices
//      inside that window; the points below it (B) are those of the bins
//      below the target ones, less the candidates among them;
//   3. those candidates are recomputed with the binary64 recipe and ranked
//      exactly: the statistics are the candidates of ranks k - B, k + 1 - B.
// MAD (projection depth) is the same select on |s_i - (med + c)| with the
// exact deviations |t_i - med| for the candidates.  MAD_+ (asymmetric
// projection depth) needs no deviation phase: the points above the median are
// the top n - n_le of the order (n_le = #{t <= med}, exact from the median's
// candidates), so MAD_+ = t_(n_le + k') - med for the middle rank k' of the
// positive deviations.
// Anything outside these assumptions (bracket missed, too many candidates)
// falls back to an exact radix select over recomputed values.  In the plain
// form (EXACT = false) E = 0 and the candidates take s - c itself, so the
// result is that of the binary32 projections.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "rrs_device.hpp"
#include "rrs_launch.hpp"
#include "rrs_select_common.hpp"

namespace rrs {

namespace {

using namespace sel;

constexpr int kBins = 256;
constexpr int kCapW = 1024;      // candidates of one window (four waves, streamed columns;
                                 // 18 KB of LDS per workgroup keeps seven per CU)
constexpr int kCapPair = 1024;   // candidates of one window (two waves per column)
constexpr int kCapWave = 512;    // candidates of one window (wave per column)
constexpr int kQuad = 512;       // up to this many, rank candidates by all-pairs counts
constexpr int kRadixCand = 64;
constexpr int kUnroll = 16;     // loads in flight per lane in the streamed passes
constexpr int kDs = 128;         // coordinates kept in LDS for the recomputation

// Histogram layout: 64 per-lane slots for values below the bracket, the 256
// bins, 64 per-lane slots for values above it.
constexpr int kHistLo = 64, kHistN = kHistLo + kBins + 64;

// The threads that share one column: a workgroup of W waves (block
// barriers) or one wave of a 64-thread workgroup.  One wave's LDS accesses
// execute in issue order, so its "barrier" only has to keep the compiler from
// moving memory accesses across it.
template <int W>
struct BlockG {
    static constexpr int kN = 64 * W, kWaves = W;
    __device__ static int tid() { return (int)threadIdx.x; }
    __device__ static void sync() { __syncthreads(); }
};
struct WaveG {
    static constexpr int kN = 64, kWaves = 1;
    __device__ static int tid() { return (int)threadIdx.x & 63; }
    __device__ static void sync()
    {
        __builtin_amdgcn_wave_barrier();
        asm volatile("" ::: "memory");
    }
};

template <int CAP, int STG>
struct alignas(16) RcShared {
    static constexpr int kCap = CAP, kStage = STG;
    static constexpr bool kShared = false;  // no second histogram / candidate list
    static constexpr bool kPP = false;      // one error bound for the whole column
    uint32_t hist[kHistN];
    uint32_t skey[64];
    uint32_t srank[64];
    float sval[64];
    uint32_t cidx[CAP];
    double cval[CAP];
    uint32_t kmin, kmax;         // order keys of the column's range
    uint32_t ncand, nlow;
    uint32_t wcnt[2], wlow[2];   // per-wave candidate counts (one or two waves)
    uint32_t count;
    double resA, resB;
    uint32_t sel_bucket, sel_before, sel_count;
    uint64_t rcand[kRadixCand];
    uint32_t nrcand;
    uint64_t rresult, minkey;
    double zs[kDs], us[kDs];   // the column's query and direction (d <= kDs)
    double xs[STG];            // the candidates' data rows, gathered in one round
};

// Streamed columns: a second histogram and candidate list, so that two order
// statistics of one column share their passes over it.
template <int CAP, int STG>
struct alignas(16) RcSharedS : RcShared<CAP, STG> {
    static constexpr bool kShared = true;
    uint32_t hist2[kHistN];
    uint32_t cidx2[CAP];
    uint32_t ncand2, nlow2;
};

// Per-point bounds (heavy-tailed data; streamed columns only).
template <int CAP, int STG>
struct alignas(16) RcSharedP : RcShared<CAP, STG> {
    static constexpr bool kPP = true;
};

// One column and what its exact recomputation needs.
struct Col {
    const float *s;
    int64_t n;
    double c, E;
    const double *X;   // [n][d]
    int64_t d;
    const double *z;   // [d] query (LDS copy when d <= kDs)
    const double *u;   // [d] direction j, unit stride (LDS copy when d <= kDs)
    int64_t ustride;   // stride of u: 1 for the LDS copy, ldm in global memory
    bool sane;         // binary32 projections finite with room to spare
    // per-point bounds (heavy-tailed data): |(s_i - c) - t_i| <= alpha |a_i| +
    // E with an[i] >= |a_i|; null: E alone bounds every point
    const float *an;
    double alpha;
};

// The recipe's projection of point i (EXACT), or the binary32 one shifted.
// The loads of four coordinates are issued before their fma steps; the fma
// chain itself keeps the recipe's coordinate order.
template <bool EXACT>
__device__ __forceinline__ double exact_t(const Col &C, int64_t i)
{
    if (!EXACT) return (double)C.s[i] - C.c;
    const double *x = C.X + i * C.d;
    const double *z = C.z, *u = C.u;
    const int64_t us = C.ustride, d = C.d;
    double t = 0.0;
    int64_t c = 0;
    for (; c + 4 <= d; c += 4) {
        const double x0 = x[c], x1 = x[c + 1], x2 = x[c + 2], x3 = x[c + 3];
        t = fma(x0 - z[c], u[c * us], t);
        t = fma(x1 - z[c + 1], u[(c + 1) * us], t);
        t = fma(x2 - z[c + 2], u[(c + 2) * us], t);
        t = fma(x3 - z[c + 3], u[(c + 3) * us], t);
    }
    for (; c < d; ++c) t = fma(x[c] - z[c], u[c * us], t);
    return t;
}

// The recipe's projection from a data row held in LDS (same fma order as
// exact_t).
__device__ __forceinline__ double row_t(const double *x, const Col &C)
{
    const double *z = C.z, *u = C.u;
    const int64_t us = C.ustride, d = C.d;
    double t = 0.0;
    for (int64_t c = 0; c < d; ++c) t = fma(x[c] - z[c], u[c * us], t);
    return t;
}

// Approximation of point i's value in phase PH, in binary32 (0: s_i;
// 1: |s_i - sig|, sig rounded to binary32).
template <int PH>
__device__ __forceinline__ float approx_v(float s, float sig)
{
    return PH == 0 ? s : fabsf(s - sig);
}

// Order key of a binary32 value in phase PH (phase 0 values carry a sign,
// phase 1 values are >= 0); finite values only take part.
template <int PH>
__device__ __forceinline__ uint32_t fkey32(float x)
{
    const uint32_t b = __float_as_uint(x);
    if (PH == 0) return b ^ ((uint32_t)((int32_t)b >> 31) | 0x80000000u);
    return b;
}

template <int PH>
__device__ __forceinline__ bool fkey_finite(uint32_t k)
{
    return PH == 0 ? k < 0xFF800000u : k < 0x7F800000u;
}

// Linear bins over a value bracket.  t = fma(x, scale, off) rounds once, so
// it is monotone in x; bin = floor(t) for t in [0, 256).  The clamp limits
// differ per lane (lo = -(lane + 1), hi = 256 + lane), so values outside the
// bracket land in per-lane slots hist[kHistLo + floor(clamped t)] at either
// end of the histogram instead of piling onto one counter.
__device__ __forceinline__ int lin_slot(float x, float scale, float off, float lo, float hi)
{
    return (int)floorf(__builtin_amdgcn_fmed3f(fmaf(x, scale, off), lo, hi));
}

// Bins for the bracket [L, H]: scale = 2^e with (H - L) scale <= 255 and
// max(|L|, |H|) scale < 2^38, off = -L scale.
__device__ void lin_fit(float L, float H, float &scale, float &off)
{
    const double w = (double)H - (double)L;
    const double M = fmax(fabs((double)L), fabs((double)H));
    int e = 0;
    if (w > 0.0) e = ilogb(255.0 / w);
    if (M > 0.0) {
        const int em = 37 - ilogb(M);
        if (w <= 0.0 || em < e) e = em;
    }
    e = e < -126 ? -126 : (e > 126 ? 126 : e);
    scale = ldexpf(1.0f, e);
    off = -L * scale;
}

// Value bounds of bins 0 <= b <= 255: a value in bin b or above satisfies
// x >= lin_lo(b), one in bin b or below x <= lin_hi(b).  t >= b forces
// x scale + off >= b - 2^-17 (half the float spacing below 256), t < b + 1
// forces it below b + 1 + 2^-16; the binary64 evaluation is widened by a
// relative 2^-50 and the division by a power of two is exact.
__device__ __forceinline__ double lin_lo(uint32_t b, float scale, float off)
{
    const double r = ((double)b - 0x1p-14) - (double)off;
    return (r - fabs(r) * 0x1p-50) / (double)scale;
}

__device__ __forceinline__ double lin_hi(uint32_t b, float scale, float off)
{
    const double r = ((double)b + 1.0 + 0x1p-14) - (double)off;
    return (r + fabs(r) * 0x1p-50) / (double)scale;
}

// Inverse of fkey32 for finite keys.
template <int PH>
__device__ __forceinline__ float fkey_value(uint32_t k)
{
    if (PH == 0) return __uint_as_float(k >= 0x80000000u ? k ^ 0x80000000u : ~k);
    return __uint_as_float(k);
}

__device__ __forceinline__ float lane_bcast_f(float x, int src)
{
    return __uint_as_float((uint32_t)__builtin_amdgcn_readlane((int)__float_as_uint(x), src));
}

// Exact value in phase PH from the exact projection t.
template <int PH>
__device__ __forceinline__ double exact_v(double t, double med)
{
    return PH == 0 ? t : fabs(t - med);
}

// Where a select reads the column's binary32 projections from.  Both hand
// every slot to f(i, s_i); slots past n read +inf, which every pass treats as
// above the bracket and outside the window (live values are finite).
// StreamSrc: global memory, kUnroll loads in flight per lane (any n < 2^31):
// each pass rereads the column from HBM, so the passes need enough bytes in
// flight to cover its latency.
template <class G>
struct StreamSrc {
    static constexpr int kMaxLevel = 6;  // rebracket / narrowing passes allowed
    const float *s;
    int64_t n;
    __device__ __forceinline__ float sample(int slot) const
    {
        return s[((2 * (int64_t)slot + 1) * n) / 128];
    }
    template <class F>
    __device__ __forceinline__ void each(F &&f) const
    {
        // the trip count is the same for every thread of the group (the
        // one-wave candidate collection counts with ballots)
        for (int64_t b = 0; b < n; b += (int64_t)kUnroll * G::kN) {
            const int64_t i0 = b + G::tid();
            float t[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int64_t i = i0 + u * G::kN;
                t[u] = i < n ? __builtin_nontemporal_load(s + i) : __builtin_inff();
            }
            // slots past n (+inf) never reach a window, so their index is unused
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) f((int)(i0 + u * G::kN), t[u]);
        }
    }
};

// RegSrc: the column held in registers, VPT values per lane (entry
// tid + G::kN v in slot v, +inf past n).  Every loop over the slots is
// unrolled with compile-time indices, which keeps the array in registers.
template <int VPT, class G>
struct RegSrc {
    static constexpr int kMaxLevel = 0;  // short columns: one pass, misses fall back
    float (&v)[VPT];
    int64_t n;
    __device__ __forceinline__ float sample(int slot) const
    {
        // slots 8 q .. 8 q + 7 (taken by consecutive lanes of one wave) read
        // register (2 q + 1) VPT / 16 of their lane
        const int q = slot >> 3;
        float x = v[VPT / 16];
#pragma unroll
        for (int r = 1; r < 8; ++r) {
            float y = v[((2 * r + 1) * VPT) / 16];
            asm volatile("" : "+v"(y));
            x = q == r ? y : x;
        }
        return x;
    }
    template <class F>
    __device__ __forceinline__ void each(F &&f) const
    {
        // opaque registers: values derived in an earlier pass are recomputed
        // instead of being kept live
#pragma unroll
        for (int u = 0; u < VPT; ++u) asm volatile("" : "+v"(v[u]));
        // likewise the slot indices (only the rare candidates use them)
        int base = G::tid();
        asm volatile("" : "+v"(base));
#pragma unroll
        for (int u = 0; u < VPT; ++u) f(base + G::kN * u, v[u]);
    }
};

// Rank r (and r + 1 when pair) among the n candidate values held in LDS:
// radix select over their order-preserving 64-bit keys, 8 bits per pass.
template <class G, class SH>
__device__ __noinline__ void lds_rank_pair(SH &sh, uint32_t nc, uint64_t r, bool pair)
{
    const int tid = G::tid();
    uint64_t prefix = 0, pmask = 0, k = r;
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int x = tid; x < kBins; x += G::kN) sh.hist[x] = 0;
        G::sync();
        for (uint32_t p = tid; p < nc; p += G::kN) {
            const uint64_t key = order_key(sh.cval[p]);
            if ((key & pmask) == prefix) atomicAdd(&sh.hist[(uint32_t)(key >> shift) & 255u], 1u);
        }
        G::sync();
        if (tid < 64) {
            uint32_t bin, rin, cnt;
            bool found;
            scan_hist(sh.hist, 0, k, bin, rin, cnt, found);
            if (found) {
                sh.sel_bucket = bin;
                sh.sel_before = (uint32_t)(k - rin);
            }
        }
        G::sync();
        k -= sh.sel_before;
        prefix |= (uint64_t)sh.sel_bucket << shift;
        pmask |= 0xFFull << shift;
        G::sync();
    }
    const double a = key_value(prefix);
    if (!pair) {
        if (tid == 0) sh.resA = sh.resB = a;
        G::sync();
        return;
    }
    // the next value: A again if more than r + 1 keys are <= A, else the
    // smallest key above A
    if (tid == 0) {
        sh.count = 0;
        sh.minkey = ~0ull;
    }
    G::sync();
    uint32_t le = 0;
    uint64_t mn = ~0ull;
    for (uint32_t p = tid; p < nc; p += G::kN) {
        const uint64_t key = order_key(sh.cval[p]);
        le += key <= prefix;
        if (key > prefix && key < mn) mn = key;
    }
    if (le) atomicAdd(&sh.count, le);
    if (mn != ~0ull) atomicMin((unsigned long long *)&sh.minkey, (unsigned long long)mn);
    G::sync();
    if (tid == 0) {
        sh.resA = a;
        sh.resB = ((uint64_t)sh.count >= r + 2) ? a : key_value(sh.minkey);
    }
    G::sync();
}

// Exact radix select (rank k) over the recomputed values of phase PH.
template <int PH, bool EXACT, class G, class SH>
__device__ uint64_t rc_radix_kth(const Col &C, double med, uint64_t k, SH &sh)
{
    const int tid = G::tid(), lane = tid & 63;
    uint64_t prefix = 0, pmask = 0;
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int x = tid; x < kBins; x += G::kN) sh.hist[x] = 0;
        G::sync();
        for (int64_t i = tid; i < C.n; i += G::kN) {
            const uint64_t key = order_key(exact_v<PH>(exact_t<EXACT>(C, i), med));
            if ((key & pmask) == prefix) atomicAdd(&sh.hist[(uint32_t)(key >> shift) & 255u], 1u);
        }
        G::sync();
        if (tid < 64) {
            uint32_t bin, rin, cnt;
            bool found;
            scan_hist(sh.hist, 0, k, bin, rin, cnt, found);
            if (found) {
                sh.sel_bucket = bin;
                sh.sel_before = (uint32_t)(k - rin);
                sh.sel_count = cnt;
            }
        }
        G::sync();
        const uint32_t selb = sh.sel_bucket, cntb = sh.sel_count;
        k -= sh.sel_before;
        prefix |= (uint64_t)selb << shift;
        pmask |= 0xFFull << shift;
        if (shift == 0) break;
        if (cntb <= (uint32_t)kRadixCand) {
            if (tid == 0) sh.nrcand = 0;
            G::sync();
            for (int64_t i = tid; i < C.n; i += G::kN) {
                const uint64_t key = order_key(exact_v<PH>(exact_t<EXACT>(C, i), med));
                if ((key & pmask) == prefix) {
                    const uint32_t pos = atomicAdd(&sh.nrcand, 1u);
                    if (pos < (uint32_t)kRadixCand) sh.rcand[pos] = key;
                }
            }
            G::sync();
            if (tid < 64) {
                const uint32_t nc = sh.nrcand < (uint32_t)kRadixCand ? sh.nrcand
                                                                     : (uint32_t)kRadixCand;
                if ((uint32_t)lane < nc) {
                    const uint64_t mine = sh.rcand[lane];
                    uint32_t lt = 0, le = 0;
                    for (uint32_t x = 0; x < nc; ++x) {
                        const uint64_t o = sh.rcand[x];
                        lt += (o < mine);
                        le += (o <= mine);
                    }
                    if (lt <= k && k < le) sh.rresult = mine;
                }
            }
            G::sync();
            const uint64_t r = sh.rresult;
            G::sync();
            return r;
        }
    }
    G::sync();
    return prefix;
}

// Key of the (k+1)-th smallest given the key A of the k-th (exact values).
template <int PH, bool EXACT, class G, class SH>
__device__ uint64_t rc_radix_next(const Col &C, double med, uint64_t k, uint64_t A, SH &sh)
{
    const int tid = G::tid();
    if (tid == 0) {
        sh.count = 0;
        sh.minkey = ~0ull;
    }
    G::sync();
    uint32_t le = 0;
    uint64_t mn = ~0ull;
    for (int64_t i = tid; i < C.n; i += G::kN) {
        const uint64_t key = order_key(exact_v<PH>(exact_t<EXACT>(C, i), med));
        le += (key <= A);
        if (key > A && key < mn) mn = key;
    }
    if (le) atomicAdd(&sh.count, le);
    if (mn != ~0ull) atomicMin((unsigned long long *)&sh.minkey, (unsigned long long)mn);
    G::sync();
    const uint64_t res = ((uint64_t)sh.count >= k + 2) ? A : sh.minkey;
    G::sync();
    return res;
}

// Smallest and largest finite approximation of the column in phase PH (as
// floats); false when there is none.
template <int PH, class G, class SRC, class SH>
__device__ bool rc_range(const SRC &src, float sigf, SH &sh, float &L, float &H)
{
    const int lane = G::tid() & 63;
    if (G::tid() == 0) {
        sh.kmin = 0xFFFFFFFFu;
        sh.kmax = 0u;
    }
    G::sync();
    uint32_t kmin = 0xFFFFFFFFu, kmax = 0u;
    src.each([&](int, float sv) {
        const uint32_t kx = fkey32<PH>(approx_v<PH>(sv, sigf));
        if (fkey_finite<PH>(kx)) {
            kmin = kx < kmin ? kx : kmin;
            kmax = kx > kmax ? kx : kmax;
        }
    });
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t a = (uint32_t)__shfl_xor((int)kmin, o);
        const uint32_t b = (uint32_t)__shfl_xor((int)kmax, o);
        kmin = a < kmin ? a : kmin;
        kmax = b > kmax ? b : kmax;
    }
    if (lane == 0) {
        atomicMin(&sh.kmin, kmin);
        atomicMax(&sh.kmax, kmax);
    }
    G::sync();
    const uint32_t a = sh.kmin, b = sh.kmax;
    G::sync();
    if (a > b) return false;
    L = fkey_value<PH>(a);
    H = fkey_value<PH>(b);
    return true;
}

// Bracket from 64 sampled approximations (slot kPer w + l from lane l < kPer
// of wave w), ranked in LDS: the samples around rank k (and k + 1), 2.5
// binomial standard deviations plus `widen` sample positions either side;
// false when fewer than 16 samples are finite.  sh.srank must be zero.
template <int PH, class G, class SRC, class SH>
__device__ __forceinline__ bool sampled_bracket(const SRC &src, float sigf, int64_t n, uint64_t k,
                                                bool pair, double widen, SH &sh, float &scale,
                                                float &off)
{
    const int tid = G::tid(), lane = tid & 63, wave = tid >> 6;
    constexpr int kPer = 64 / G::kWaves;
    if (lane < kPer) {
        const int slot = wave * kPer + lane;
        const float x = approx_v<PH>(src.sample(slot), sigf);
        const uint32_t kx = fkey32<PH>(x);
        sh.skey[slot] = fkey_finite<PH>(kx) ? kx : 0xFFFFFFFFu;
        sh.sval[slot] = x;
    }
    G::sync();
    {
        const uint32_t mine = sh.skey[lane];
        uint32_t part = 0;
#pragma unroll
        for (int jj = 0; jj < kPer; ++jj) {
            const int o = wave * kPer + jj;
            const uint32_t ko = sh.skey[o];
            part += (ko < mine || (ko == mine && o < lane)) ? 1u : 0u;
        }
        atomicAdd(&sh.srank[lane], part);
    }
    G::sync();
    // every wave derives the bracket itself (same values, no barrier)
    const uint32_t kx = sh.skey[lane];
    const bool ok = kx != 0xFFFFFFFFu;
    const uint32_t rank = sh.srank[lane];
    const uint32_t S = (uint32_t)__popcll(__ballot(ok));
    if (S < 16) return false;
    const double f = ((double)k + 0.5) / (double)n;
    const double pos = f * (double)S;
    const double del = 2.5 * sqrt((double)S * f * (1.0 - f)) + 1.5 + widen;
    double lo = floor(pos - del), hi = ceil(pos + del + (pair ? 1.0 : 0.0));
    if (lo < 0.0) lo = 0.0;
    if (hi > (double)(S - 1)) hi = (double)(S - 1);
    const uint32_t rlo = (uint32_t)lo, rhi = (uint32_t)hi;
    const uint64_t mlo = __ballot(ok && rank == rlo), mhi = __ballot(ok && rank == rhi);
    const float xv = sh.sval[lane];
    const float L = lane_bcast_f(xv, __ffsll((long long)mlo) - 1);
    const float H = lane_bcast_f(xv, __ffsll((long long)mhi) - 1);
    lin_fit(L, H, scale, off);
    return true;
}

// Ranks r and r + 1 (pair) of the nc candidates of a window: their exact
// values (phase PH) in sh.cval, then an all-pairs count (up to kQuadG
// candidates) or a radix select over their keys.  Candidate p's index sits
// at sh.cidx[p] for p < nc0 and at sh.cidx[kCap - 1 - (p - nc0)] above
// (two-wave collection layout; nc0 = nc for a single list).
template <int PH, bool EXACT, class G, class SH>
__device__ __forceinline__ void rank_window(const Col &C, SH &sh, uint32_t nc, uint32_t nc0,
                                            uint64_t r, bool pair, double med, double &a,
                                            double &b)
{
    const int tid = G::tid();
    constexpr uint32_t kCap = (uint32_t)SH::kCap;
    constexpr uint32_t kQuadG = kQuad < SH::kCap / 2 ? kQuad : SH::kCap / 2;
    const bool quad = nc <= kQuadG;
    // index of candidate p in the collection layout
    auto cand = [&](uint32_t p) -> int64_t {
        return (int64_t)sh.cidx[p < nc0 ? p : kCap - 1 - (p - nc0)];
    };
    const uint32_t dd = (uint32_t)C.d, nd = nc * dd;
    if (EXACT && nd <= (uint32_t)SH::kStage) {
        // the candidates' rows in one cooperative round of loads
        // (coordinate c of candidate p at xs[p d + c]), then each
        // thread runs its candidate's fma chain from LDS
        // e / dd = umulhi(e, ceil(2^32 / dd)) for e < 2^16 (d > 1)
        const uint32_t rcp = 0xFFFFFFFFu / dd + 1u;
        for (uint32_t e = tid; e < nd; e += G::kN) {
            const uint32_t p = dd == 1u ? e : __umulhi(e, rcp), c = e - p * dd;
            sh.xs[e] = C.X[cand(p) * C.d + c];
        }
        G::sync();
        for (uint32_t p = tid; p < nc; p += G::kN)
            sh.cval[p] = exact_v<PH>(row_t(sh.xs + p * dd, C), med);
    } else {
        for (uint32_t p = tid; p < nc; p += G::kN)
            sh.cval[p] = exact_v<PH>(exact_t<EXACT>(C, cand(p)), med);
    }
    G::sync();
    if (quad) {
        // the all-pairs ranking counts into cidx[p] (below) and
        // cidx[kCap / 2 + p] (at most)
        for (uint32_t p = tid; p < nc; p += G::kN) {
            sh.cidx[p] = 0u;
            sh.cidx[kCap / 2 + p] = 0u;
        }
        G::sync();
    }
    const uint64_t rA = r, rB = r + 1;
    if (quad) {
        // candidate p against a slice of the others, G slices
        // per candidate spread over the block
        const uint32_t grp = nc >= (uint32_t)G::kN ? 1u : (uint32_t)G::kN / nc;
        const uint32_t span = (nc + grp - 1) / grp;
        for (uint32_t w = tid; w < nc * grp; w += G::kN) {
            const uint32_t g = w / nc, p = w - g * nc;
            const double mine = sh.cval[p];
            const uint32_t x0 = g * span, x1 = x0 + span < nc ? x0 + span : nc;
            uint32_t lt = 0, le = 0;
            for (uint32_t x = x0; x < x1; ++x) {
                const double o = sh.cval[x];
                lt += (o < mine);
                le += (o <= mine);
            }
            if (lt) atomicAdd(&sh.cidx[p], lt);
            if (le) atomicAdd(&sh.cidx[kCap / 2 + p], le);
        }
        G::sync();
        for (uint32_t p = tid; p < nc; p += G::kN) {
            const uint32_t lt = sh.cidx[p], le = sh.cidx[kCap / 2 + p];
            if (lt <= rA && rA < le) sh.resA = sh.cval[p];
            if (pair && lt <= rB && rB < le) sh.resB = sh.cval[p];
        }
        G::sync();
        a = sh.resA;
        b = pair ? sh.resB : a;
    } else {
        lds_rank_pair<G>(sh, nc, rA, pair);
        a = sh.resA;
        b = sh.resB;
    }
}

// Interval [lo, hi] around approximation x (binary32) holding its exact
// counterpart (t_i + c, or |t_i - med| in phase 1), from the point's own
// norm bound an: e = alpha an + E (alpha_f, E_f rounded up), widened by the
// fma's rounding, in phase 1 by the roundings of sig and of s - sig, and by
// the roundings of x -/+ e themselves, all in binary32.
template <int PH>
__device__ __forceinline__ void point_ends(float x, float an, float alpha_f, float E_f,
                                           float sigf, float &lo, float &hi)
{
    float e = fmaf(alpha_f, an, E_f) * (1.0f + 0x1p-22f);
    if (PH == 1) e = fmaf(0x1p-21f, fabsf(sigf) + fabsf(x) + e, e) * (1.0f + 0x1p-22f);
    e = fmaf(0x1p-22f, fabsf(x) + e, e) + 0x1p-149f;
    lo = x - e;
    hi = x + e;
}

// The select with a bound per point (heavy-tailed data, where one bound for
// the whole column would be the largest point's): point i's exact value lies
// in [lo_i, hi_i] = [x_i - e_i, x_i + e_i] (binary32, rounded outwards).  One
// pass bins both ends; with bA the bin of the k-th smallest lower end and bB
// that of the (k + pair)-th smallest upper end, at most k points lie below
// L = lin_lo(bA) and at least k + pair + 1 at or below U = lin_hi(bB), so the
// statistics lie in [L, U].  The window pass counts the points certainly
// below (hi_i < L) and collects those whose interval meets [L, U]; their
// exact values are ranked.  Long columns narrow the bracket while the window
// would hold too many; a miss falls back like the uniform-bound select.
template <int PH, bool EXACT, class G, class SRC, class SH>
__device__ __forceinline__ bool rc_select_pp(const Col &C, const SRC &src, double med, double sig, uint64_t k,
                             bool pair, double &a, double &b, uint64_t *below, SH &sh,
                             uint32_t *stats)
{
    const int tid = G::tid(), lane = tid & 63;
    constexpr uint32_t kCap = (uint32_t)SH::kCap;
    static_assert(SH::kCap >= kHistN, "the upper ends' histogram borrows cidx");
    const float sigf = (float)sig;
    const float *an = C.an;
    const float alpha_f = __double2float_ru(C.alpha), E_f = __double2float_ru(C.E);
    // interval ends of slot i with approximation sv (binary32, outwards)
    auto ends = [&](int i, float sv, float &lo, float &hi) {
        point_ends<PH>(approx_v<PH>(sv, sigf), an[i], alpha_f, E_f, sigf, lo, hi);
    };
    bool fast = C.sane;
    float scale = 1.0f, off = 0.0f;
    bool whole = false;  // bracket over the column's whole range
    if (fast) {
        if (tid < 64) sh.srank[tid] = 0;
        G::sync();
        // the sampled centres' bracket, widened by two sample positions for
        // the interval ends; the column's range when too few are finite
        if (!sampled_bracket<PH, G>(src, sigf, C.n, k, pair, 2.0, sh, scale, off)) {
            float L, H;
            fast = rc_range<PH, G>(src, sigf, sh, L, H);
            if (fast) lin_fit(L, H, scale, off);
            whole = true;
        }
    }
    uint32_t bA = 0, bB = 0;
    const float lo_l = -(float)(lane + 1), hi_l = (float)(kBins + lane);
    for (int level = 0; fast; ++level) {
        for (int x = tid; x < kHistN; x += G::kN) {
            sh.hist[x] = 0;
            sh.cidx[x] = 0;
        }
        G::sync();
        src.each([&](int i, float sv) {
            if (!(sv < __builtin_inff())) return;  // slots past n
            float lo, hi;
            ends(i, sv, lo, hi);
            atomicAdd(&sh.hist[kHistLo + lin_slot(lo, scale, off, lo_l, hi_l)], 1u);
            atomicAdd(&sh.cidx[kHistLo + lin_slot(hi, scale, off, lo_l, hi_l)], 1u);
        });
        G::sync();
        {
            uint32_t blo = sh.hist[lane], bhi = sh.cidx[lane];  // the below slots
            for (int o = 32; o > 0; o >>= 1) {
                blo += (uint32_t)__shfl_xor((int)blo, o);
                bhi += (uint32_t)__shfl_xor((int)bhi, o);
            }
            uint32_t xA, rA, cA, xB, rB, cB;
            bool fA, fB;
            scan_hist(sh.hist + kHistLo, blo, k, xA, rA, cA, fA);
            scan_hist(sh.cidx + kHistLo, bhi, k + (pair ? 1 : 0), xB, rB, cB, fB);
            const uint64_t ma = __ballot(fA), mb = __ballot(fB);
            fast = ma != 0 && mb != 0;
            if (fast) {
                bA = (uint32_t)__builtin_amdgcn_readlane((int)xA, __ffsll((long long)ma) - 1);
                bB = (uint32_t)__builtin_amdgcn_readlane((int)xB, __ffsll((long long)mb) - 1);
            }
        }
        if (level >= SRC::kMaxLevel) break;
        if (!fast) {
            // the sampled bracket missed a rank: bracket the whole column
            // instead (then narrow as usual)
            if (whole) break;
            float L, H;
            fast = rc_range<PH, G>(src, sigf, sh, L, H);
            if (!fast) break;
            lin_fit(L, H, scale, off);
            whole = true;
            G::sync();
            continue;
        }
        // window estimate: the ends falling in bins bA .. bB
        uint32_t held = 0;
        for (uint32_t x = bA; x <= bB; ++x) held += sh.hist[kHistLo + x] + sh.cidx[kHistLo + x];
        if (held <= kCap / 2) break;
        const float nL = __double2float_rd(lin_lo(bA, scale, off));
        const float nH = __double2float_ru(lin_hi(bB, scale, off));
        float ns, no;
        lin_fit(nL, nH, ns, no);
        if (!(ns > scale)) break;  // no finer bins to be had
        scale = ns;
        off = no;
        G::sync();
    }
    if (fast) {
        const float Lf = __double2float_rd(lin_lo(bA, scale, off));
        const float Uf = __double2float_ru(lin_hi(bB, scale, off));
        G::sync();
        if (tid == 0) {
            sh.ncand = 0;
            sh.count = 0;
        }
        G::sync();
        uint32_t nb = 0;  // this lane's points certainly below
        src.each([&](int i, float sv) {
            if (!(sv < __builtin_inff())) return;
            float lo, hi;
            ends(i, sv, lo, hi);
            if (hi < Lf) {
                ++nb;
            } else if (lo <= Uf) {
                const uint32_t p = atomicAdd(&sh.ncand, 1u);
                if (p < kCap) sh.cidx[p] = (uint32_t)i;
            }
        });
        for (int o = 32; o > 0; o >>= 1) nb += (uint32_t)__shfl_xor((int)nb, o);
        if (lane == 0 && nb) atomicAdd(&sh.count, nb);
        G::sync();
        const uint32_t nc = sh.ncand;
        const uint64_t B = sh.count;
        G::sync();
        fast = nc <= kCap && B <= k && k + (pair ? 1 : 0) < B + nc;
        if (fast) {
            rank_window<PH, EXACT, G>(C, sh, nc, nc, k - B, pair, med, a, b);
            *below = B;
            return true;
        }
    }
    G::sync();
    if (SRC::kMaxLevel == 0 && C.sane) {
        // a register-resident column that missed: the streamed select over
        // the same column in global memory
        return rc_select_pp<PH, EXACT, G>(C, StreamSrc<G>{C.s, C.n}, med, sig, k, pair, a, b,
                                          below, sh, stats);
    }
    if (stats && tid == 0) stat_fallback(stats);
    const uint64_t A = rc_radix_kth<PH, EXACT, G>(C, med, k, sh);
    a = key_value(A);
    b = a;
    if (pair) b = key_value(rc_radix_next<PH, EXACT, G>(C, med, k, A, sh));
    return false;
}

// The exact values of ranks k (and k + 1 if pair) in phase PH.  Returns true
// when the window path served them; then sh.cval[0 .. ncand) holds the
// window's exact values and *below the number of points under the window.
template <int PH, bool EXACT, class G, class SRC, class SH>
__device__ __forceinline__ bool rc_select(const Col &C, const SRC &src, double med, double sig,
                                          double E, uint64_t k, bool pair, double &a, double &b,
                                          uint64_t *below, SH &sh, uint32_t *stats)
{
    const int tid = G::tid(), lane = tid & 63, wave = tid >> 6;
    constexpr uint32_t kCap = (uint32_t)SH::kCap;
    const int64_t n = C.n;
    const float sigf = (float)sig;
    if constexpr (SH::kPP)
        return rc_select_pp<PH, EXACT, G>(C, src, med, sig, k, pair, a, b, below, sh, stats);
    bool fast = C.sane;
    float scale = 1.0f, off = 0.0f;
    int fast0 = 0;
    if (fast) {
        for (int x = tid; x < kHistN; x += G::kN) sh.hist[x] = 0;
        if (tid < 64) sh.srank[tid] = 0;
        if (tid == 0) {
            sh.ncand = 0;
            sh.nlow = 0;
        }
        fast0 = sampled_bracket<PH, G>(src, sigf, n, k, pair, 0.0, sh, scale, off) ? 1 : 0;
        // register-resident columns keep a single pass (a miss falls back);
        // streamed columns rebracket and narrow instead
        fast = SRC::kMaxLevel > 0 || fast0 != 0;
    }
    if (fast) {
        bool whole = false;
        uint32_t bA = 0, bB = 0, beforeA = 0;
        if (SRC::kMaxLevel > 0 && fast0 == 0) {
            // too few samples took part: bracket the whole column
            float L, H;
            fast = rc_range<PH, G>(src, sigf, sh, L, H);
            if (fast) lin_fit(L, H, scale, off);
            whole = true;
        }
        // per-lane clamp limits: slots 63 - lane (below) and 320 + lane (above)
        const float lo_l = -(float)(lane + 1), hi_l = (float)(kBins + lane);
        uint32_t *const bins = sh.hist + kHistLo;
        // histogram passes: the first bins the bracket; while the target bins
        // hold more than half the candidate room (long columns), the next pass
        // bins just those bins at least twice finer
        for (int level = 0; fast; ++level) {
            src.each([&](int, float sv) {
                const int t = lin_slot(approx_v<PH>(sv, sigf), scale, off, lo_l, hi_l);
                atomicAdd(&bins[t], 1u);
            });
            G::sync();
            {
                // every wave scans the histogram itself (same results)
                uint32_t lo = sh.hist[lane];  // the below slots
                for (int o = 32; o > 0; o >>= 1) lo += (uint32_t)__shfl_xor((int)lo, o);
                uint32_t xA, rA, cA, xB, rB, cB;
                bool fA, fB;
                scan_hist(bins, lo, k, xA, rA, cA, fA);
                scan_hist(bins, lo, k + 1, xB, rB, cB, fB);
                const uint64_t ma = __ballot(fA), mb = __ballot(fB);
                fast = ma != 0 && (!pair || mb != 0);
                if (fast) {
                    const int la = __ffsll((long long)ma) - 1;
                    bA = (uint32_t)__builtin_amdgcn_readlane((int)xA, la);
                    beforeA = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(k - rA), la);
                    bB = pair ? (uint32_t)__builtin_amdgcn_readlane((int)xB, __ffsll((long long)mb) - 1)
                              : bA;
                }
            }
            if (level >= SRC::kMaxLevel) break;
            float L, H;
            bool rebracket = false;
            if (!fast) {
                // the sampled bracket missed the rank: bracket the whole
                // column instead (then narrow as usual)
                if (whole) break;
                fast = rc_range<PH, G>(src, sigf, sh, L, H);
                if (!fast) break;
                whole = rebracket = true;
            } else {
                uint32_t held = 0;
                for (uint32_t x = bA; x <= bB; ++x) held += bins[x];
                if (held <= kCap / 2) break;
                // narrow to the target bins
                L = __double2float_rd(lin_lo(bA, scale, off));
                H = __double2float_ru(lin_hi(bB, scale, off));
            }
            float ns, no;
            lin_fit(L, H, ns, no);
            if (!rebracket && !(ns > scale)) break;  // no finer bins to be had
            scale = ns;
            off = no;
            G::sync();
            for (int x = tid; x < kHistN; x += G::kN) sh.hist[x] = 0;
            G::sync();
        }
        if (fast) {
            // approximations of the target bins lie in [vlo, vhi]
            const double vlo = lin_lo(bA, scale, off), vhi = lin_hi(bB, scale, off);
            // phase 1 adds the roundings of sig to binary32 and of s - sig
            const double Ew = PH == 0 ? E : E * 1.000001 + 0x1p-22 * (fabs(sig) + fabs(vlo) +
                                                                      fabs(vhi) + E) + 1e-300;
            // the window [wlo, whi] as |x - mid| <= hw, evaluated in binary32
            // with the roundings of mid, hw and x - mid absorbed into hwf
            const double wlo = vlo - 2.0 * Ew, whi = vhi + 2.0 * Ew;
            const double mid = 0.5 * (wlo + whi);
            const float midf = (float)mid;
            const double hw = fmax(mid - wlo, whi - mid) * (1.0 + 0x1p-50);
            const float hwf =
                __double2float_ru((hw + fabs(mid - (double)midf)) * (1.0 + 0x1p-50));
            const float fA = (float)bA;
            // candidates binned below bin A (t < bA is the histogram pass's
            // test, the same fma) are counted apart
            uint32_t nc, nlow, nc0;
            if (G::kWaves <= 2) {
                // one or two waves: slots from ballots, counts in scalar
                // registers; wave 0 fills cidx upwards from 0, wave 1
                // downwards from kCap - 1 (candidate p >= nc0 of the
                // combined list sits at kCap - 1 - (p - nc0))
                uint32_t wc = 0, wl = 0;
                src.each([&](int i, float sv) {
                    const float x = approx_v<PH>(sv, sigf);
                    const bool in = fabsf(x - midf) <= hwf;
                    const uint64_t mask = __ballot(in);
                    if (mask) {
                        const uint64_t ml = __ballot(in && fmaf(x, scale, off) < fA);
                        const uint32_t q =
                            wc + __builtin_amdgcn_mbcnt_hi(
                                     (uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                        if (in && q < kCap) sh.cidx[wave == 0 ? q : kCap - 1 - q] = (uint32_t)i;
                        wc += (uint32_t)__popcll(mask);
                        wl += (uint32_t)__popcll(ml);
                    }
                });
                if (lane == 0) {
                    sh.wcnt[wave] = wc;
                    sh.wlow[wave] = wl;
                }
                G::sync();
                nc0 = sh.wcnt[0];
                nc = G::kWaves == 2 ? nc0 + sh.wcnt[1] : nc0;
                nlow = G::kWaves == 2 ? sh.wlow[0] + sh.wlow[1] : sh.wlow[0];
                if (tid == 0) sh.ncand = nc;  // read by the APD count
            } else {
                src.each([&](int i, float sv) {
                    const float x = approx_v<PH>(sv, sigf);
                    if (fabsf(x - midf) <= hwf) {
                        const bool low = fmaf(x, scale, off) < fA;
                        if (low) atomicAdd(&sh.nlow, 1u);
                        const uint32_t p = atomicAdd(&sh.ncand, 1u);
                        if (p < kCap) sh.cidx[p] = (uint32_t)i;
                    }
                });
                G::sync();
                nc = sh.ncand;
                nlow = sh.nlow;
                nc0 = nc;
            }
            // points below the window: those binned below bin A that are not
            // candidates (a non-candidate under bin A lies below wlo)
            const uint64_t B = (uint64_t)beforeA - nlow;
            fast = nc <= kCap && B <= k && k + (pair ? 1 : 0) < B + nc;
            if (fast) {
                rank_window<PH, EXACT, G>(C, sh, nc, nc0, k - B, pair, med, a, b);
                *below = B;
                return true;
            }
        }
    }
    G::sync();
    if (SRC::kMaxLevel == 0 && C.sane) {
        // a register-resident column that missed: the streamed select over
        // the same column in global memory (rebracketing, narrowing)
        return rc_select<PH, EXACT, G>(C, StreamSrc<G>{C.s, C.n}, med, sig, E, k, pair, a, b,
                                       below, sh, stats);
    }
    if (stats && tid == 0) stat_fallback(stats);
    const uint64_t A = rc_radix_kth<PH, EXACT, G>(C, med, k, sh);
    a = key_value(A);
    b = a;
    if (pair) b = key_value(rc_radix_next<PH, EXACT, G>(C, med, k, A, sh));
    return false;
}


// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Shared passes for streamed APD columns (n > 16384, reread from HBM by every
// pass): one pass bins the brackets of both the median and the MAD_+ rank,
// one pass collects both windows' candidates; the MAD_+ rank is that of the
// tie-free count #{t <= med} (ceil(n / 2)), which the median's window then
// confirms.  Whatever this cannot serve (a bracket that misses, target bins
// that hold too many values for one window, ties at the median) is left to
// the separate selects.  (Projection depth keeps the separate selects: its
// MAD's histogram would have to be binned around an approximation of the
// median, and the resulting window, wider by half a median bin, held so many
// candidates that their binary64 recomputation cost more than the saved
// pass.)
// ---------------------------------------------------------------------------
struct Target {
    float scale, off;    // linear bins of the bracket
    uint32_t bA, bB;     // bins holding ranks k, k + 1
    uint32_t beforeA;    // values below bin A (the below slots included)
    float midf, hwf;     // window |x - mid| <= hw in binary32
};

// The 64 sampled approximations of phase PH (relative to sigf), their keys
// and ranks in LDS.
template <int PH, class G, class SRC, class SH>
__device__ __forceinline__ void take_samples(const SRC &src, float sigf, SH &sh)
{
    const int tid = G::tid(), lane = tid & 63, wave = tid >> 6;
    constexpr int kPer = 64 / G::kWaves;
    if (tid < 64) sh.srank[tid] = 0;
    if (lane < kPer) {
        const int slot = wave * kPer + lane;
        const float x = approx_v<PH>(src.sample(slot), sigf);
        const uint32_t kx = fkey32<PH>(x);
        sh.skey[slot] = fkey_finite<PH>(kx) ? kx : 0xFFFFFFFFu;
        sh.sval[slot] = x;
    }
    G::sync();
    {
        const uint32_t mine = sh.skey[lane];
        uint32_t part = 0;
#pragma unroll
        for (int jj = 0; jj < kPer; ++jj) {
            const int o = wave * kPer + jj;
            const uint32_t ko = sh.skey[o];
            part += (ko < mine || (ko == mine && o < lane)) ? 1u : 0u;
        }
        atomicAdd(&sh.srank[lane], part);
    }
    G::sync();
}

// Linear bins over the sampled bracket of rank k (pair: k and k + 1); false
// when fewer than 16 samples are finite.  Every wave derives it (same values).
template <class SH>
__device__ __forceinline__ bool sample_bracket(const SH &sh, int64_t n, uint64_t k, bool pair,
                                               float &scale, float &off)
{
    const int lane = threadIdx.x & 63;
    const uint32_t kx = sh.skey[lane];
    const bool ok = kx != 0xFFFFFFFFu;
    const uint32_t rank = sh.srank[lane];
    const uint32_t S = (uint32_t)__popcll(__ballot(ok));
    if (S < 16) return false;
    const double f = ((double)k + 0.5) / (double)n;
    const double pos = f * (double)S;
    const double del = 2.5 * sqrt((double)S * f * (1.0 - f)) + 1.5;
    double lo = floor(pos - del), hi = ceil(pos + del + (pair ? 1.0 : 0.0));
    if (lo < 0.0) lo = 0.0;
    if (hi > (double)(S - 1)) hi = (double)(S - 1);
    const uint32_t rlo = (uint32_t)lo, rhi = (uint32_t)hi;
    const uint64_t mlo = __ballot(ok && rank == rlo), mhi = __ballot(ok && rank == rhi);
    const float xv = sh.sval[lane];
    const float L = lane_bcast_f(xv, __ffsll((long long)mlo) - 1);
    const float H = lane_bcast_f(xv, __ffsll((long long)mhi) - 1);
    lin_fit(L, H, scale, off);
    return true;
}

// Bins of ranks k (and k + 1) in a filled histogram; false when the bracket
// missed them or when they hold more than half the candidate room.
template <class SH>
__device__ __forceinline__ bool hist_target(const uint32_t *hist, uint64_t k, bool pair,
                                            Target &t)
{
    const int lane = threadIdx.x & 63;
    const uint32_t *bins = hist + kHistLo;
    uint32_t lo = hist[lane];  // the below slots
    for (int o = 32; o > 0; o >>= 1) lo += (uint32_t)__shfl_xor((int)lo, o);
    uint32_t xA, rA, cA, xB, rB, cB;
    bool fA, fB;
    scan_hist(bins, lo, k, xA, rA, cA, fA);
    scan_hist(bins, lo, k + 1, xB, rB, cB, fB);
    const uint64_t ma = __ballot(fA), mb = __ballot(fB);
    if (ma == 0 || (pair && mb == 0)) return false;
    const int la = __ffsll((long long)ma) - 1;
    t.bA = (uint32_t)__builtin_amdgcn_readlane((int)xA, la);
    t.beforeA = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(k - rA), la);
    t.bB = pair ? (uint32_t)__builtin_amdgcn_readlane((int)xB, __ffsll((long long)mb) - 1) : t.bA;
    uint32_t held = 0;
    for (uint32_t x = t.bA; x <= t.bB; ++x) held += bins[x];
    return held <= (uint32_t)SH::kCap / 2;
}

// Window of the target bins with error bound Ew (already including every
// rounding of the approximations).
__device__ __forceinline__ void target_window(Target &t, double Ew)
{
    const double vlo = lin_lo(t.bA, t.scale, t.off), vhi = lin_hi(t.bB, t.scale, t.off);
    const double wlo = vlo - 2.0 * Ew, whi = vhi + 2.0 * Ew;
    const double mid = 0.5 * (wlo + whi);
    t.midf = (float)mid;
    const double hw = fmax(mid - wlo, whi - mid) * (1.0 + 0x1p-50);
    t.hwf = __double2float_ru((hw + fabs(mid - (double)t.midf)) * (1.0 + 0x1p-50));
}

// Exact values of the nc candidates listed in idx (phase PH), into sh.cval,
// and ranks rA (and rA + 1) among them.
template <int PH, bool EXACT, class G, class SH>
__device__ __forceinline__ void rank_candidates(const Col &C, const uint32_t *idx, uint32_t nc,
                                                double med, uint64_t rA, bool pair, SH &sh,
                                                double &a, double &b)
{
    constexpr uint32_t kCap = (uint32_t)SH::kCap;
    constexpr uint32_t kQuadG = kQuad < SH::kCap / 2 ? kQuad : SH::kCap / 2;
    const int tid = G::tid();
    for (uint32_t p = tid; p < nc; p += G::kN)
        sh.cval[p] = exact_v<PH>(exact_t<EXACT>(C, (int64_t)idx[p]), med);
    G::sync();
    const uint64_t rB = rA + 1;
    if (nc <= kQuadG) {
        // all-pairs ranking; the counts go to cidx[p] (below) and
        // cidx[kCap / 2 + p] (at most) -- the lists are no longer needed
        for (uint32_t p = tid; p < nc; p += G::kN) {
            sh.cidx[p] = 0u;
            sh.cidx[kCap / 2 + p] = 0u;
        }
        G::sync();
        const uint32_t grp = nc >= (uint32_t)G::kN ? 1u : (uint32_t)G::kN / nc;
        const uint32_t span = (nc + grp - 1) / grp;
        for (uint32_t w = tid; w < nc * grp; w += G::kN) {
            const uint32_t g = w / nc, p = w - g * nc;
            const double mine = sh.cval[p];
            const uint32_t x0 = g * span, x1 = x0 + span < nc ? x0 + span : nc;
            uint32_t lt = 0, le = 0;
            for (uint32_t x = x0; x < x1; ++x) {
                const double o = sh.cval[x];
                lt += (o < mine);
                le += (o <= mine);
            }
            if (lt) atomicAdd(&sh.cidx[p], lt);
            if (le) atomicAdd(&sh.cidx[kCap / 2 + p], le);
        }
        G::sync();
        for (uint32_t p = tid; p < nc; p += G::kN) {
            const uint32_t lt = sh.cidx[p], le = sh.cidx[kCap / 2 + p];
            if (lt <= rA && rA < le) sh.resA = sh.cval[p];
            if (pair && lt <= rB && rB < le) sh.resB = sh.cval[p];
        }
        G::sync();
        a = sh.resA;
        b = pair ? sh.resB : a;
        G::sync();
    } else {
        lds_rank_pair<G>(sh, nc, rA, pair);
        a = sh.resA;
        b = sh.resB;
    }
}

// Asymmetric projection depth of a streamed column with shared passes.
// Returns 2 with D when they served the whole column, 1 with the exact
// median and #{t <= med} when only the median's part served (ties at the
// median, or MAD_+'s window missed), 0 when nothing was decided.
template <bool EXACT, class G, class SH>
__device__ __forceinline__ int rc_apd_shared(const Col &C, const StreamSrc<G> &src, SH &sh, double &D,
                             double &med_out, uint64_t &nle_out)
{
    const int tid = G::tid();
    constexpr uint32_t kCap = (uint32_t)SH::kCap;
    const int64_t n = C.n;
    // per-point bounds (heavy tails) take the separate selects
    if (!C.sane || C.an) return 0;
    const bool odd = (n & 1) != 0;
    const uint64_t k = odd ? (uint64_t)n / 2 : (uint64_t)n / 2 - 1;
    // MAD_+'s rank when no other point equals the median
    const uint64_t nle_g = odd ? k + 1 : (uint64_t)n / 2;
    const uint64_t npos_g = (uint64_t)n - nle_g;
    if (npos_g < 2) return 0;
    const bool podd = (npos_g & 1) != 0;
    const uint64_t kp = nle_g + (podd ? npos_g / 2 : npos_g / 2 - 1);
    for (int x = tid; x < kHistN; x += G::kN) {
        sh.hist[x] = 0;
        sh.hist2[x] = 0;
    }
    if (tid == 0) {
        sh.ncand = sh.nlow = sh.ncand2 = sh.nlow2 = 0;
    }
    take_samples<0, G>(src, 0.0f, sh);
    Target t1, t2;
    if (!sample_bracket(sh, n, k, !odd, t1.scale, t1.off)) return 0;
    if (!sample_bracket(sh, n, kp, !podd, t2.scale, t2.off)) return 0;
    // pass 1: both histograms
    {
        const int lane = tid & 63;
        const float lo_l = -(float)(lane + 1), hi_l = (float)(kBins + lane);
        uint32_t *const b1 = sh.hist + kHistLo;
        uint32_t *const b2 = sh.hist2 + kHistLo;
        src.each([&](int, float sv) {
            atomicAdd(&b1[lin_slot(sv, t1.scale, t1.off, lo_l, hi_l)], 1u);
            atomicAdd(&b2[lin_slot(sv, t2.scale, t2.off, lo_l, hi_l)], 1u);
        });
    }
    G::sync();
    const bool ok1 = hist_target<SH>(sh.hist, k, !odd, t1);
    const bool ok2 = hist_target<SH>(sh.hist2, kp, !podd, t2);
    if (!ok1 || !ok2) return 0;
    target_window(t1, C.E);
    target_window(t2, C.E);
    // pass 2: both windows' candidates
    {
        const float fA1 = (float)t1.bA, fA2 = (float)t2.bA;
        src.each([&](int i, float x) {
            if (fabsf(x - t1.midf) <= t1.hwf) {
                if (fmaf(x, t1.scale, t1.off) < fA1) atomicAdd(&sh.nlow, 1u);
                const uint32_t p = atomicAdd(&sh.ncand, 1u);
                if (p < kCap) sh.cidx[p] = (uint32_t)i;
            }
            if (fabsf(x - t2.midf) <= t2.hwf) {
                if (fmaf(x, t2.scale, t2.off) < fA2) atomicAdd(&sh.nlow2, 1u);
                const uint32_t p = atomicAdd(&sh.ncand2, 1u);
                if (p < kCap) sh.cidx2[p] = (uint32_t)i;
            }
        });
    }
    G::sync();
    const uint32_t nc1 = sh.ncand, nc2 = sh.ncand2;
    const uint64_t B1 = (uint64_t)t1.beforeA - sh.nlow, B2 = (uint64_t)t2.beforeA - sh.nlow2;
    G::sync();
    if (!(nc1 <= kCap && B1 <= k && k + (odd ? 0 : 1) < B1 + nc1)) return 0;
    double a, b;
    rank_candidates<0, EXACT, G>(C, sh.cidx, nc1, 0.0, k - B1, !odd, sh, a, b);
    const double med = odd ? a : (a + b) * 0.5;
    // #{t <= med}: the points below the window and the window's candidates
    if (tid == 0) sh.count = 0;
    G::sync();
    {
        uint32_t c = 0;
        for (uint32_t p = tid; p < nc1; p += G::kN) c += sh.cval[p] <= med ? 1u : 0u;
        for (int o = 32; o > 0; o >>= 1) c += (uint32_t)__shfl_xor((int)c, o);
        if ((tid & 63) == 0 && c) atomicAdd(&sh.count, c);
    }
    G::sync();
    const uint64_t nle = B1 + sh.count;
    G::sync();
    med_out = med;
    nle_out = nle;
    if (nle != nle_g || !(nc2 <= kCap && B2 <= kp && kp + (podd ? 0 : 1) < B2 + nc2)) return 1;
    double p1, p2;
    rank_candidates<0, EXACT, G>(C, sh.cidx2, nc2, 0.0, kp - B2, !podd, sh, p1, p2);
    const double madp = podd ? (p1 - med) : ((p1 - med) + (p2 - med)) * 0.5;
    const double num = (med < 0.0) ? -med : 0.0;
    D = 1.0 / (1.0 + num / madp);
    return 2;
}

// Number of points with t <= med: from the median's window when it served,
// else by a counting pass over recomputed values.
template <bool EXACT, class G, class SH>
__device__ __forceinline__ uint64_t rc_count_le(const Col &C, double med, bool window,
                                                uint64_t below, SH &sh)
{
    const int tid = G::tid(), lane = tid & 63;
    if (tid == 0) sh.count = 0;
    G::sync();
    uint32_t c = 0;
    if (window) {
        const uint32_t nc = sh.ncand;
        for (uint32_t p = tid; p < nc; p += G::kN) c += sh.cval[p] <= med ? 1u : 0u;
    } else {
        for (int64_t i = tid; i < C.n; i += G::kN) c += exact_t<EXACT>(C, i) <= med ? 1u : 0u;
    }
    for (int off = 32; off > 0; off >>= 1) c += (uint32_t)__shfl_xor((int)c, off);
    if (lane == 0 && c) atomicAdd(&sh.count, c);
    G::sync();
    const uint64_t r = (window ? below : 0) + sh.count;
    G::sync();
    return r;
}

template <int NOTION, bool EXACT, class G, class SRC, class SH>
__device__ __forceinline__ double rc_depth(const Col &C, const SRC &src, SH &sh,
                                           uint32_t *stats)
{
    // rank k of the s values is rank k of the s - c values: the windows live
    // in s space (|(s - c) - t| <= E moves every statistic by at most E, and
    // c is common to the column), the candidates' exact values in t space
    const int64_t n = C.n;
    const bool odd = (n & 1) != 0;
    const uint64_t k = odd ? (uint64_t)n / 2 : (uint64_t)n / 2 - 1;
    double med = 0.0;
    bool have_med = false;
    uint64_t nle_sh = 0;
    if constexpr (SRC::kMaxLevel > 0 && SH::kShared && NOTION == NOTION_APD) {
        // streamed APD column: the order statistics share passes
        double D;
        const int st = rc_apd_shared<EXACT, G>(C, src, sh, D, med, nle_sh);
        if (stats && G::tid() == 0) atomicAdd(&stats[8 + (2 - st)], 1u);
        if (st == 2) return D;
        have_med = st == 1;
        G::sync();
    }
    bool win = false;
    uint64_t below = 0;
    if (!have_med) {
        double a, b;
        win = rc_select<0, EXACT, G>(C, src, 0.0, 0.0, C.E, k, !odd, a, b, &below, sh, stats);
        med = odd ? a : (a + b) * 0.5;
    }
    if (NOTION == NOTION_PROJECTION) {
        double m1, m2;
        uint64_t b1 = 0;
        rc_select<1, EXACT, G>(C, src, med, med + C.c, C.E, k, !odd, m1, m2, &b1, sh, stats);
        const double mad = odd ? m1 : (m1 + m2) * 0.5;
        if (mad == 0.0) return (med == 0.0) ? 1.0 : 0.0;
        return 1.0 / (1.0 + fabs(med) / mad);
    }
    const uint64_t nle = have_med ? nle_sh : rc_count_le<EXACT, G>(C, med, win, below, sh);
    const uint64_t npos = (uint64_t)n - nle;
    const double num = (med < 0.0) ? -med : 0.0;
    if (npos == 0) return (num == 0.0) ? 1.0 : 0.0;
    const bool podd = (npos & 1) != 0;
    const uint64_t kp = nle + (podd ? npos / 2 : npos / 2 - 1);
    double p1, p2;
    uint64_t b2 = 0;
    rc_select<0, EXACT, G>(C, src, 0.0, 0.0, C.E, kp, !podd, p1, p2, &b2, sh, stats);
    const double madp = podd ? (p1 - med) : ((p1 - med) + (p2 - med)) * 0.5;
    return 1.0 / (1.0 + num / madp);
}

// One column per group G (a workgroup of two or four waves, or a 64-thread
// workgroup of one wave).  VPT > 0: the column in registers (n <= G::kN VPT); VPT == 0:
// streamed.
template <int NOTION, bool EXACT, int VPT, class G, class SH, bool PP>
__device__ __forceinline__ void select_column(const float *__restrict__ S, int64_t n, int64_t m,
                                              int64_t ldm, const double *__restrict__ cq,
                                              const double *__restrict__ eq,
                                              const double *__restrict__ X, int64_t d,
                                              const double *__restrict__ Zb,
                                              const double *__restrict__ UT,
                                              double *__restrict__ Dj, uint32_t *__restrict__ stats,
                                              const float *__restrict__ anorm, double alpha,
                                              SH &sh)
{
    const int tid = G::tid();
    const int64_t j = blockIdx.x;
    const int64_t qi = blockIdx.y;
    Col C;
    C.s = S + (qi * m + j) * n;
    C.n = n;
    C.c = cq[qi * m + j];
    {
        // eq is +inf or NaN when the data's norm bound is out of range
        const double e = eq[qi * m + j];
        C.sane = e < 0x1p100;
        C.E = EXACT ? e : 0.0;
    }
    // heavy-tailed data: a bound per point (E is then the column part)
    C.an = (EXACT && PP) ? anorm : nullptr;
    C.alpha = alpha;
    C.X = X;
    C.d = d;
    if (EXACT && d <= kDs) {
        for (int64_t c = tid; c < d; c += G::kN) {
            sh.zs[c] = Zb[qi * d + c];
            sh.us[c] = UT[qi * d * ldm + c * ldm + j];
        }
        G::sync();
        C.z = sh.zs;
        C.u = sh.us;
        C.ustride = 1;
    } else {
        C.z = Zb + qi * d;
        C.u = UT + qi * d * ldm + j;
        C.ustride = ldm;
    }
    double D;
    if (VPT == 0) {
        D = rc_depth<NOTION, EXACT, G>(C, StreamSrc<G>{C.s, n}, sh, stats);
    } else {
        constexpr int V = VPT > 0 ? VPT : 1;
        float v[V];
#pragma unroll
        for (int u = 0; u < V; ++u) {
            const int64_t i = (int64_t)tid + (int64_t)G::kN * u;
            // the projections are read once: non-temporal, so that they do not
            // push the data rows of the candidates' recomputation out of L2
            v[u] = i < n ? __builtin_nontemporal_load(C.s + i) : __builtin_inff();
        }
        D = rc_depth<NOTION, EXACT, G>(C, RegSrc<V, G>{v, n}, sh, stats);
    }
    if (tid == 0) Dj[qi * ldm + j] = D;
}

template <int NOTION, bool EXACT, int VPT, class G, int CAP, int STG, bool PP>
__global__ __launch_bounds__(G::kN) void k_select_rc(const float *__restrict__ S, int64_t n,
                                                     int64_t m, int64_t ldm,
                                                     const double *__restrict__ cq,
                                                     const double *__restrict__ eq,
                                                     const double *__restrict__ X, int64_t d,
                                                     const double *__restrict__ Zb,
                                                     const double *__restrict__ UT,
                                                     double *__restrict__ Dj,
                                                     uint32_t *__restrict__ stats,
                                                     const float *__restrict__ anorm,
                                                     double alpha)
{
    // streamed APD columns (VPT == 0) carry the second histogram and list;
    // per-point bounds mark their type
    using SH = typename std::conditional<
        PP, RcSharedP<CAP, STG>,
        typename std::conditional<VPT == 0 && NOTION == NOTION_APD, RcSharedS<CAP, STG>,
                                  RcShared<CAP, STG>>::type>::type;
    __shared__ SH sh;
    select_column<NOTION, EXACT, VPT, G, SH, PP>(S, n, m, ldm, cq, eq, X, d, Zb, UT, Dj, stats,
                                                 anorm, alpha, sh);
}

template <int NOTION, bool EXACT, int VPT, class G, int CAP, int STG, bool PP = false>
hipError_t launch_rc(const SelectRcArgs &a, hipStream_t st)
{
    dim3 grid((unsigned)a.m, (unsigned)a.qb);
    hipLaunchKernelGGL((k_select_rc<NOTION, EXACT, VPT, G, CAP, STG, PP>), grid, dim3(G::kN), 0, st,
                       a.S, a.n, a.m, a.ldm, a.cq, a.eq, a.X, a.d, a.Z, a.UT, a.Dj, a.stats,
                       a.anorm, a.alpha);
    return hipGetLastError();
}

// Columns up to 64 x 128 values: one wave (no block barriers; the fixed
// per-column work, sampling, bracket and scans, done once), in registers; up
// to 128 x 128: two waves, in registers; longer: four waves streaming from
// memory.  The register budgets keep two or three waves per SIMD.
template <int NOTION, bool EXACT>
hipError_t launch_rc_vpt(const SelectRcArgs &a, hipStream_t st)
{
    // per-point bounds (heavy-tailed data): the streamed kernel, any n
    if constexpr (EXACT)
        if (a.pp) return launch_rc<NOTION, EXACT, 0, BlockG<4>, kCapW, 64, true>(a, st);
    const int64_t w = (a.n + 63) / 64;
    if (w <= 8) return launch_rc<NOTION, EXACT, 8, WaveG, kCapWave, 512>(a, st);
    if (w <= 16) return launch_rc<NOTION, EXACT, 16, WaveG, kCapWave, 512>(a, st);
    if (w <= 32) return launch_rc<NOTION, EXACT, 32, WaveG, kCapWave, 512>(a, st);
    if (w <= 64) return launch_rc<NOTION, EXACT, 64, WaveG, kCapWave, 512>(a, st);
    if (w <= 96) return launch_rc<NOTION, EXACT, 96, WaveG, kCapWave, 512>(a, st);
    if (w <= 128) return launch_rc<NOTION, EXACT, 128, WaveG, kCapWave, 512>(a, st);
    const int64_t p = (a.n + 127) / 128;
    if (p <= 80) return launch_rc<NOTION, EXACT, 80, BlockG<2>, kCapPair, 1024>(a, st);
    if (p <= 128) return launch_rc<NOTION, EXACT, 128, BlockG<2>, kCapPair, 1024>(a, st);
    return launch_rc<NOTION, EXACT, 0, BlockG<4>, kCapW, 64>(a, st);  // n > 16384
}

}  // namespace

hipError_t launch_select_rc(const SelectRcArgs &a, int notion, bool exact, hipStream_t st)
{
    if (notion == NOTION_PROJECTION)
        return exact ? launch_rc_vpt<NOTION_PROJECTION, true>(a, st)
                     : launch_rc_vpt<NOTION_PROJECTION, false>(a, st);
    return exact ? launch_rc_vpt<NOTION_APD, true>(a, st) : launch_rc_vpt<NOTION_APD, false>(a, st);
}

}  // namespace rrs
