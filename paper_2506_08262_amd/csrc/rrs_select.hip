// rrs_select.hip -- step a3 for projection and asymmetric projection depth:
// exact median, MAD and MAD_+ of one projection column per workgroup, with
// the column held in registers (VPT binary64 values per lane, 256 lanes).
//
// The column goes through three phases, transformed in place:
//   phase 0: t_i                          -> median
//   phase 1: |t_i - med|                  -> MAD (projection depth)
//   phase 2: t_i - med if > 0, else NaN   -> MAD_+ (asymmetric projection depth)
// Unused register slots hold NaN; NaN never takes part in any phase.
//
// Each order statistic (or adjacent pair, for even counts) is found with two
// passes over the registers, both on 32-bit keys: key(x) is the high word of
// the order-preserving 64-bit image of x, so x < y implies key(x) <= key(y)
// and any map that is monotone in the key is monotone in x.
//   1. 64 sampled keys are ranked (all four waves share the comparisons) and
//      two sample order statistics bracket the target rank by [Lk, Hk]; one
//      pass counts the keys below Lk and bins the keys in [Lk, Hk] into at
//      most 256 bins, bin = (key - Lk) >> sh.  Every value of a lower bin is
//      strictly below every value of a higher bin, so the target's bin and
//      its rank inside the bin are exact;
//   2. one pass collects the binary64 values of that bin (a handful), which
//      are ranked exactly by value.
// If the bracket misses the target rank, or the bin holds too many values,
// the pair comes instead from an exact radix select over the 64-bit keys that
// re-reads the column from global memory and applies the phase on the fly
// (rare; it keeps the register array out of the fallback so the register
// footprint stays that of the column).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rrs_device.hpp"
#include "rrs_launch.hpp"
#include "rrs_select_common.hpp"

namespace rrs {

namespace {

using namespace sel;

constexpr int kT = 256;        // lanes per workgroup
constexpr int kBins = 256;     // bins of the bracket
constexpr int kCapA = 256;     // collected values of the target's bin (one per lane)
constexpr int kCapB = 64;      // collected values of the next bin (pairs)
constexpr int kRadixCand = 64;

struct alignas(16) RegShared {
    uint32_t hist[kBins + 64];  // 256 bins, then one dummy slot per lane
    uint32_t skey[64];          // sampled keys
    uint32_t srank[64];         // their ranks
    double candA[kCapA];
    double candB[kCapB];
    double resA, resB;
    double sval[64];            // sampled values
    uint32_t Lk, R, sh, tau;    // bracket: keys Lk..Lk+R, bin shift, collapse
    uint32_t below;
    uint32_t ncandA, ncandB;
    uint32_t binA, binB, rankA, rankB, cntA, cntB;
    int32_t fast;
    uint32_t count;
    uint64_t minkey;
    uint32_t sel_bucket, sel_before, sel_count;
    uint64_t rcand[kRadixCand];
    uint32_t nrcand;
    uint64_t rresult;
};

// Makes every register of the column opaque to the optimiser, so that values
// derived from it before this point are not kept live after it.
template <int VPT>
__device__ __forceinline__ void launder(double (&vals)[VPT])
{
#pragma unroll
    for (int v = 0; v < VPT; ++v) asm volatile("" : "+v"(vals[v]));
}

// ---------------------------------------------------------------------------
// Exact fallback: radix select over the column in global memory.
// ---------------------------------------------------------------------------
template <int PH>
__device__ uint64_t radix_kth_g(const double *__restrict__ col, int64_t n, double med,
                                uint64_t k, RegShared &sh)
{
    const int tid = threadIdx.x, lane = tid & 63;
    uint64_t prefix = 0, pmask = 0;
    for (int shift = 56; shift >= 0; shift -= 8) {
        sh.hist[tid] = 0;
        __syncthreads();
        for (int64_t i = tid; i < n; i += kT) {
            double x;
            if (phase_val<PH>(col[i], med, x)) {
                const uint64_t key = order_key(x);
                if ((key & pmask) == prefix)
                    atomicAdd(&sh.hist[(uint32_t)(key >> shift) & 255u], 1u);
            }
        }
        __syncthreads();
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
        __syncthreads();
        const uint32_t selb = sh.sel_bucket, cntb = sh.sel_count;
        k -= sh.sel_before;
        prefix |= (uint64_t)selb << shift;
        pmask |= 0xFFull << shift;
        if (shift == 0) break;
        if (cntb <= (uint32_t)kRadixCand) {
            if (tid == 0) sh.nrcand = 0;
            __syncthreads();
            for (int64_t i = tid; i < n; i += kT) {
                double x;
                if (phase_val<PH>(col[i], med, x)) {
                    const uint64_t key = order_key(x);
                    if ((key & pmask) == prefix) {
                        const uint32_t pos = atomicAdd(&sh.nrcand, 1u);
                        if (pos < (uint32_t)kRadixCand) sh.rcand[pos] = key;
                    }
                }
            }
            __syncthreads();
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
            __syncthreads();
            const uint64_t r = sh.rresult;
            __syncthreads();
            return r;
        }
    }
    __syncthreads();
    return prefix;
}

// Key of the (k+1)-th smallest given the key A of the k-th.
template <int PH>
__device__ uint64_t radix_next_g(const double *__restrict__ col, int64_t n, double med,
                                 uint64_t k, uint64_t A, RegShared &sh)
{
    const int tid = threadIdx.x;
    if (tid == 0) {
        sh.count = 0;
        sh.minkey = ~0ull;
    }
    __syncthreads();
    uint32_t le = 0;
    uint64_t mn = ~0ull;
    for (int64_t i = tid; i < n; i += kT) {
        double x;
        if (phase_val<PH>(col[i], med, x)) {
            const uint64_t key = order_key(x);
            le += (key <= A);
            if (key > A && key < mn) mn = key;
        }
    }
    if (le) atomicAdd(&sh.count, le);
    if (mn != ~0ull) atomicMin((unsigned long long *)&sh.minkey, (unsigned long long)mn);
    __syncthreads();
    const uint64_t res = ((uint64_t)sh.count >= k + 2) ? A : sh.minkey;
    __syncthreads();
    return res;
}

template <int PH>
__device__ void select_pair_stream(const double *__restrict__ col, int64_t n, double med,
                                   uint64_t cnt, uint64_t k, bool pair, double &a, double &b,
                                   RegShared &sh, uint32_t *stats);

// ---------------------------------------------------------------------------
// The k-th (and, if pair, the (k+1)-th) smallest of the cnt values taking
// part in phase PH; vals holds the column in phase PH.
// ---------------------------------------------------------------------------
template <int PH, int VPT>
__device__ __forceinline__ void select_pair(double (&vals)[VPT],
                                            const double *__restrict__ col, int64_t n,
                                            double med, uint64_t cnt, uint64_t k, bool pair,
                                            double &a, double &b, RegShared &sh,
                                            uint32_t *stats)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    sh.hist[tid] = 0;
    if (tid < 64) sh.srank[tid] = 0;
    if (tid == 0) {
        sh.below = 0;
        sh.ncandA = 0;
        sh.ncandB = 0;
    }
    // sample: lanes 0..15 of wave w publish the key of register (2w+1) VPT / 8
    // (a compile-time index per wave: a lane-dependent index would make the
    // compiler move the whole column to scratch memory)
    if (lane < 16) {
        double x0 = vals[(1 * VPT) / 8], x1 = vals[(3 * VPT) / 8];
        double x2 = vals[(5 * VPT) / 8], x3 = vals[(7 * VPT) / 8];
        asm volatile("" : "+v"(x0), "+v"(x1), "+v"(x2), "+v"(x3));
        const double x = wave == 0 ? x0 : wave == 1 ? x1 : wave == 2 ? x2 : x3;
        const uint32_t kx = key32<PH>(x);
        sh.skey[wave * 16 + lane] = key_takes_part<PH>(kx) ? kx : 0xFFFFFFFFu;
        sh.sval[wave * 16 + lane] = x;
    }
    __syncthreads();
    // ranks of the 64 sampled keys: wave w compares every sample with samples
    // 16w .. 16w+15 (ties broken by sample index)
    {
        const uint32_t mine = sh.skey[lane];
        uint32_t part = 0;
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const int o = wave * 16 + jj;
            const uint32_t ko = sh.skey[o];
            part += (ko < mine || (ko == mine && o < lane)) ? 1u : 0u;
        }
        atomicAdd(&sh.srank[lane], part);
    }
    __syncthreads();
    // wave 0 fixes the bracket [Lk, Lk + R] and the bin shift
    if (tid < 64) {
        const uint32_t kx = sh.skey[lane];
        const bool ok = kx != 0xFFFFFFFFu;
        const uint32_t rank = sh.srank[lane];
        const uint32_t S = (uint32_t)__popcll(__ballot(ok));
        int fast0 = (S >= 16 && cnt > 0) ? 1 : 0;
        uint32_t Lk = 0, Hk = 0, tau = 0;
        if (fast0) {
            const double f = ((double)k + 0.5) / (double)cnt;
            const double pos = f * (double)S;
            const double del = 2.5 * sqrt((double)S * f * (1.0 - f)) + 1.5;
            double lo = floor(pos - del), hi = ceil(pos + del + (pair ? 1.0 : 0.0));
            if (lo < 0.0) lo = 0.0;
            if (hi > (double)(S - 1)) hi = (double)(S - 1);
            const uint32_t rlo = (uint32_t)lo, rhi = (uint32_t)hi;
            const uint64_t mlo = __ballot(ok && rank == rlo), mhi = __ballot(ok && rank == rhi);
            const double xv = sh.sval[lane];
            const double L = lane_bcast(xv, __ffsll((long long)mlo) - 1);
            const double H = lane_bcast(xv, __ffsll((long long)mhi) - 1);
            // magnitudes below max(|L|, |H|) / 64 share one key (see bin_key)
            tau = (uint32_t)__double2hiint(fmax(fabs(L), fabs(H)) * 0x1p-6) & 0x7FFFFFFFu;
            Lk = bin_key<PH>(L, tau);
            Hk = bin_key<PH>(H, tau);
        }
        if (lane == 0) {
            const uint32_t R = Hk - Lk;
            // smallest shift with R >> shift < 256
            const uint32_t nb = 32u - (uint32_t)__clz((int)(R | 1u));   // bits of R
            sh.Lk = Lk;
            sh.R = R;
            sh.sh = nb > 8u ? nb - 8u : 0u;
            sh.tau = tau;
            sh.fast = fast0;
        }
    }
    __syncthreads();
    bool fast = sh.fast != 0;
    if (fast) {
        const uint32_t Lk = sh.Lk, R = sh.R, bsh = sh.sh, tau = sh.tau;
        launder(vals);
        // pass 1: count keys below Lk, bin keys in [Lk, Lk + R]; lanes outside
        // the bracket add to a private dummy slot so the atomic needs no branch
        // (NaN keys exceed every finite key, so they are never counted)
        uint32_t below = 0;
        const uint32_t dummy = (uint32_t)kBins + (uint32_t)lane;
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
            const uint32_t kx = bin_key<PH>(vals[v], tau);
            const uint32_t dk = kx - Lk;
            below += (kx < Lk) ? 1u : 0u;
            atomicAdd(&sh.hist[dk <= R ? (dk >> bsh) : dummy], 1u);
        }
        for (int off = 32; off > 0; off >>= 1) below += (uint32_t)__shfl_xor((int)below, off);
        if (lane == 0 && below) atomicAdd(&sh.below, below);
        __syncthreads();
        // wave 0 finds the bins of ranks k and k+1
        if (tid < 64) {
            const uint64_t base = sh.below;
            uint32_t bA, rA, cA, bB, rB, cB;
            bool fA, fB;
            scan_hist(sh.hist, base, k, bA, rA, cA, fA);
            scan_hist(sh.hist, base, k + 1, bB, rB, cB, fB);
            if (fA) {
                sh.binA = bA;
                sh.rankA = rA;
                sh.cntA = cA;
            }
            if (fB) {
                sh.binB = bB;
                sh.rankB = rB;
                sh.cntB = cB;
            }
            const uint64_t ma = __ballot(fA), mb = __ballot(fB);
            if (lane == 0) sh.fast = (ma != 0 && (!pair || mb != 0)) ? 1 : 0;
        }
        __syncthreads();
        fast = sh.fast != 0;
        uint32_t bA = 0, rA = 0, bB = 0, rB = 0;
        if (fast) {
            bA = sh.binA;
            rA = sh.rankA;
            bB = pair ? sh.binB : bA;
            rB = pair ? sh.rankB : rA;
            const bool same = bB == bA;
            fast = sh.cntA <= (uint32_t)kCapA && (same || sh.cntB <= (uint32_t)kCapB);
        }
        if (fast) {
            launder(vals);
            // pass 2: collect the binary64 values of the target bins
#pragma unroll
            for (int v = 0; v < VPT; ++v) {
                const uint32_t dk = bin_key<PH>(vals[v], tau) - Lk;
                const uint32_t bx = dk >> bsh;
                if (dk <= R && (bx == bA || bx == bB)) {
                    if (bx == bA) {
                        const uint32_t p = atomicAdd(&sh.ncandA, 1u);
                        if (p < (uint32_t)kCapA) sh.candA[p] = vals[v];
                    } else {
                        const uint32_t p = atomicAdd(&sh.ncandB, 1u);
                        if (p < (uint32_t)kCapB) sh.candB[p] = vals[v];
                    }
                }
            }
            __syncthreads();
            // exact ranks inside the bins
            const uint32_t nA = sh.ncandA < (uint32_t)kCapA ? sh.ncandA : (uint32_t)kCapA;
            const uint32_t nB = sh.ncandB < (uint32_t)kCapB ? sh.ncandB : (uint32_t)kCapB;
            if ((uint32_t)tid < nA) {
                const double mine = sh.candA[tid];
                uint32_t lt = 0, le = 0;
                for (uint32_t x = 0; x < nA; ++x) {
                    const double o = sh.candA[x];
                    lt += (o < mine);
                    le += (o <= mine);
                }
                if (lt <= rA && rA < le) sh.resA = mine;
                if (pair && bB == bA && lt <= rB && rB < le) sh.resB = mine;
            }
            if (pair && bB != bA && (uint32_t)tid < nB) {
                const double mine = sh.candB[tid];
                uint32_t lt = 0, le = 0;
                for (uint32_t x = 0; x < nB; ++x) {
                    const double o = sh.candB[x];
                    lt += (o < mine);
                    le += (o <= mine);
                }
                if (lt <= rB && rB < le) sh.resB = mine;
            }
            __syncthreads();
            a = sh.resA;
            b = pair ? sh.resB : a;
            return;
        }
    }
    // a miss: the streamed select over the same column in global memory
    // (rebracketing and narrowing; its own last resort is the exact radix
    // select); the barrier keeps every wave out of the shared histogram until
    // all have finished reading it
    __syncthreads();
    select_pair_stream<PH>(col, n, med, cnt, k, pair, a, b, sh, stats);
}

template <int PH, int VPT>
__device__ __forceinline__ double median_reg(double (&vals)[VPT],
                                             const double *__restrict__ col, int64_t n,
                                             double med, uint64_t cnt, RegShared &sh,
                                             uint32_t *stats)
{
    double a, b;
    if (cnt & 1) {
        select_pair<PH, VPT>(vals, col, n, med, cnt, cnt / 2, false, a, b, sh, stats);
        return a;
    }
    select_pair<PH, VPT>(vals, col, n, med, cnt, cnt / 2 - 1, true, a, b, sh, stats);
    return (a + b) * 0.5;
}

template <int NOTION, int VPT>
__global__ __launch_bounds__(kT) void k_select_reg(const double *__restrict__ T, int64_t n,
                                                   int64_t m, int64_t ldm,
                                                   double *__restrict__ Dj,
                                                   uint32_t *__restrict__ stats)
{
    __shared__ RegShared sh;
    const int64_t j = blockIdx.x;
    const int64_t qi = blockIdx.y;
    const double *col = T + (qi * m + j) * n;
    const int tid = threadIdx.x;
    double vals[VPT];
#pragma unroll
    for (int v = 0; v < VPT; ++v) {
        const int64_t i = tid + (int64_t)kT * v;
        vals[v] = i < n ? col[i] : __builtin_nan("");
    }
    const double med = median_reg<0, VPT>(vals, col, n, 0.0, (uint64_t)n, sh, stats);
    double D;
    if (NOTION == NOTION_PROJECTION) {
#pragma unroll
        for (int v = 0; v < VPT; ++v) vals[v] = fabs(vals[v] - med);
        launder(vals);
        const double mad = median_reg<1, VPT>(vals, col, n, med, (uint64_t)n, sh, stats);
        if (mad == 0.0)
            D = (med == 0.0) ? 1.0 : 0.0;
        else
            D = 1.0 / (1.0 + fabs(med) / mad);
    } else {
        if (tid == 0) sh.count = 0;
        __syncthreads();
        uint32_t np = 0;
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
            const double dv = vals[v] - med;
            np += (dv > 0.0) ? 1u : 0u;
            vals[v] = (dv > 0.0) ? dv : __builtin_nan("");
        }
        launder(vals);
        for (int off = 32; off > 0; off >>= 1) np += (uint32_t)__shfl_xor((int)np, off);
        if ((tid & 63) == 0 && np) atomicAdd(&sh.count, np);
        __syncthreads();
        const uint64_t npos = sh.count;
        __syncthreads();
        const double num = (med < 0.0) ? -med : 0.0;
        if (npos == 0) {
            D = (num == 0.0) ? 1.0 : 0.0;
        } else {
            const double madp = median_reg<2, VPT>(vals, col, n, med, npos, sh, stats);
            D = 1.0 / (1.0 + num / madp);
        }
    }
    if (tid == 0) Dj[qi * ldm + j] = D;
}

// ---------------------------------------------------------------------------
// Streaming form for columns too long for the registers: the same bracket /
// bin / candidate passes, each pass re-reading the column from global memory
// (4 loads in flight per lane) and applying the phase on the fly.
// ---------------------------------------------------------------------------
constexpr int kUnroll = 4;

template <int PH>
__device__ void select_pair_stream(const double *__restrict__ col, int64_t n, double med,
                                   uint64_t cnt, uint64_t k, bool pair, double &a, double &b,
                                   RegShared &sh, uint32_t *stats)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    sh.hist[tid] = 0;
    if (tid < 64) sh.srank[tid] = 0;
    if (tid == 0) {
        sh.below = 0;
        sh.ncandA = 0;
        sh.ncandB = 0;
    }
    // sample: 64 entries spread evenly over the column
    if (tid < 64) {
        const int64_t i = ((2 * (int64_t)tid + 1) * n) / 128;
        double x = 0.0;
        const bool part = phase_val<PH>(col[i], med, x);
        const uint32_t kx = key32<PH>(x);
        sh.skey[tid] = (part && key_takes_part<PH>(kx)) ? kx : 0xFFFFFFFFu;
        sh.sval[tid] = x;
    }
    __syncthreads();
    {
        const uint32_t mine = sh.skey[lane];
        uint32_t part = 0;
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const int o = wave * 16 + jj;
            const uint32_t ko = sh.skey[o];
            part += (ko < mine || (ko == mine && o < lane)) ? 1u : 0u;
        }
        atomicAdd(&sh.srank[lane], part);
    }
    __syncthreads();
    if (tid < 64) {
        const uint32_t kx = sh.skey[lane];
        const bool ok = kx != 0xFFFFFFFFu;
        const uint32_t rank = sh.srank[lane];
        const uint32_t S = (uint32_t)__popcll(__ballot(ok));
        int fast0 = (S >= 16 && cnt > 0) ? 1 : 0;
        uint32_t Lk = 0, Hk = 0, tau = 0;
        if (fast0) {
            const double f = ((double)k + 0.5) / (double)cnt;
            const double pos = f * (double)S;
            const double del = 2.5 * sqrt((double)S * f * (1.0 - f)) + 1.5;
            double lo = floor(pos - del), hi = ceil(pos + del + (pair ? 1.0 : 0.0));
            if (lo < 0.0) lo = 0.0;
            if (hi > (double)(S - 1)) hi = (double)(S - 1);
            const uint32_t rlo = (uint32_t)lo, rhi = (uint32_t)hi;
            const uint64_t mlo = __ballot(ok && rank == rlo), mhi = __ballot(ok && rank == rhi);
            const double xv = sh.sval[lane];
            const double L = lane_bcast(xv, __ffsll((long long)mlo) - 1);
            const double H = lane_bcast(xv, __ffsll((long long)mhi) - 1);
            tau = (uint32_t)__double2hiint(fmax(fabs(L), fabs(H)) * 0x1p-6) & 0x7FFFFFFFu;
            Lk = bin_key<PH>(L, tau);
            Hk = bin_key<PH>(H, tau);
        }
        if (lane == 0) {
            const uint32_t R = Hk - Lk;
            const uint32_t nb = 32u - (uint32_t)__clz((int)(R | 1u));
            sh.Lk = Lk;
            sh.R = R;
            sh.sh = nb > 8u ? nb - 8u : 0u;
            sh.tau = tau;
            sh.fast = fast0;
        }
    }
    __syncthreads();
    bool fast = true;
    {
        // the sampled bracket, or the whole key range when too few samples
        // took part
        uint32_t Lk = sh.Lk, R = sh.R, bsh = sh.sh;
        const uint32_t tau = sh.tau;
        if (sh.fast == 0) {
            Lk = 0u;
            R = 0xFFFFFFFFu;
            bsh = 24u;
        }
        const uint32_t dummy = (uint32_t)kBins + (uint32_t)lane;
        uint32_t bA = 0, rA = 0, bB = 0, rB = 0;
        // histogram passes: the first bins the bracket; while a target bin
        // holds more values than can be collected (long columns), the next
        // pass bins just the target bins 256 times finer
        for (int level = 0;; ++level) {
            uint32_t below = 0;
            for (int64_t i0 = tid; i0 < n; i0 += (int64_t)kUnroll * kT) {
                double t[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const int64_t i = i0 + (int64_t)u * kT;
                    t[u] = i < n ? col[i] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    double x;
                    const bool part = i0 + (int64_t)u * kT < n && phase_val<PH>(t[u], med, x);
                    const uint32_t kx = part ? bin_key<PH>(x, tau) : 0xFFFFFFFFu;
                    const uint32_t dk = kx - Lk;
                    below += (part && kx < Lk) ? 1u : 0u;
                    atomicAdd(&sh.hist[(part && dk <= R) ? (dk >> bsh) : dummy], 1u);
                }
            }
            for (int off = 32; off > 0; off >>= 1)
                below += (uint32_t)__shfl_xor((int)below, off);
            if (lane == 0 && below) atomicAdd(&sh.below, below);
            __syncthreads();
            if (tid < 64) {
                const uint64_t base = sh.below;
                uint32_t fbA, frA, fcA, fbB, frB, fcB;
                bool fA, fB;
                scan_hist(sh.hist, base, k, fbA, frA, fcA, fA);
                scan_hist(sh.hist, base, k + 1, fbB, frB, fcB, fB);
                if (fA) {
                    sh.binA = fbA;
                    sh.rankA = frA;
                    sh.cntA = fcA;
                }
                if (fB) {
                    sh.binB = fbB;
                    sh.rankB = frB;
                    sh.cntB = fcB;
                }
                const uint64_t ma = __ballot(fA), mb = __ballot(fB);
                if (lane == 0) sh.fast = (ma != 0 && (!pair || mb != 0)) ? 1 : 0;
            }
            __syncthreads();
            fast = sh.fast != 0;
            if (!fast) {
                // the sampled bracket missed the rank: bin the whole key range
                // instead (then narrow as usual)
                if (level > 0 || (Lk == 0u && R == 0xFFFFFFFFu)) break;
                Lk = 0u;
                R = 0xFFFFFFFFu;
                bsh = 24u;
            } else {
                bA = sh.binA;
                rA = sh.rankA;
                bB = pair ? sh.binB : bA;
                rB = pair ? sh.rankB : rA;
                const bool same = bB == bA;
                fast = sh.cntA <= (uint32_t)kCapA && (same || sh.cntB <= (uint32_t)kCapB);
                if (fast || bsh == 0 || level == 6) break;
                // narrow to the target bins and start over
                Lk = Lk + (bA << bsh);
                R = ((bB - bA + 1) << bsh) - 1;
                const uint32_t nb = 32u - (uint32_t)__clz((int)(R | 1u));
                bsh = nb > 8u ? nb - 8u : 0u;
            }
            __syncthreads();
            sh.hist[tid] = 0;
            if (tid == 0) sh.below = 0;
            __syncthreads();
        }
        if (fast) {
            for (int64_t i0 = tid; i0 < n; i0 += (int64_t)kUnroll * kT) {
                double t[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const int64_t i = i0 + (int64_t)u * kT;
                    t[u] = i < n ? col[i] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    double x;
                    if (!(i0 + (int64_t)u * kT < n && phase_val<PH>(t[u], med, x))) continue;
                    const uint32_t dk = bin_key<PH>(x, tau) - Lk;
                    const uint32_t bx = dk >> bsh;
                    if (dk <= R && (bx == bA || bx == bB)) {
                        if (bx == bA) {
                            const uint32_t p = atomicAdd(&sh.ncandA, 1u);
                            if (p < (uint32_t)kCapA) sh.candA[p] = x;
                        } else {
                            const uint32_t p = atomicAdd(&sh.ncandB, 1u);
                            if (p < (uint32_t)kCapB) sh.candB[p] = x;
                        }
                    }
                }
            }
            __syncthreads();
            const uint32_t nA = sh.ncandA < (uint32_t)kCapA ? sh.ncandA : (uint32_t)kCapA;
            const uint32_t nB = sh.ncandB < (uint32_t)kCapB ? sh.ncandB : (uint32_t)kCapB;
            if ((uint32_t)tid < nA) {
                const double mine = sh.candA[tid];
                uint32_t lt = 0, le = 0;
                for (uint32_t x = 0; x < nA; ++x) {
                    const double o = sh.candA[x];
                    lt += (o < mine);
                    le += (o <= mine);
                }
                if (lt <= rA && rA < le) sh.resA = mine;
                if (pair && bB == bA && lt <= rB && rB < le) sh.resB = mine;
            }
            if (pair && bB != bA && (uint32_t)tid < nB) {
                const double mine = sh.candB[tid];
                uint32_t lt = 0, le = 0;
                for (uint32_t x = 0; x < nB; ++x) {
                    const double o = sh.candB[x];
                    lt += (o < mine);
                    le += (o <= mine);
                }
                if (lt <= rB && rB < le) sh.resB = mine;
            }
            __syncthreads();
            a = sh.resA;
            b = pair ? sh.resB : a;
            __syncthreads();
            return;
        }
    }
    __syncthreads();
    if (stats && tid == 0) stat_fallback(stats);
    const uint64_t A = radix_kth_g<PH>(col, n, med, k, sh);
    a = key_value(A);
    b = a;
    if (pair) b = key_value(radix_next_g<PH>(col, n, med, k, A, sh));
}

template <int PH>
__device__ double median_stream(const double *__restrict__ col, int64_t n, double med,
                                uint64_t cnt, RegShared &sh, uint32_t *stats)
{
    double a, b;
    if (cnt & 1) {
        select_pair_stream<PH>(col, n, med, cnt, cnt / 2, false, a, b, sh, stats);
        return a;
    }
    select_pair_stream<PH>(col, n, med, cnt, cnt / 2 - 1, true, a, b, sh, stats);
    return (a + b) * 0.5;
}

template <int NOTION>
__global__ __launch_bounds__(kT) void k_select_stream(const double *__restrict__ T, int64_t n,
                                                      int64_t m, int64_t ldm,
                                                      double *__restrict__ Dj,
                                                      uint32_t *__restrict__ stats)
{
    __shared__ RegShared sh;
    const int64_t j = blockIdx.x;
    const int64_t qi = blockIdx.y;
    const double *col = T + (qi * m + j) * n;
    const int tid = threadIdx.x;
    const double med = median_stream<0>(col, n, 0.0, (uint64_t)n, sh, stats);
    double D;
    if (NOTION == NOTION_PROJECTION) {
        const double mad = median_stream<1>(col, n, med, (uint64_t)n, sh, stats);
        if (mad == 0.0)
            D = (med == 0.0) ? 1.0 : 0.0;
        else
            D = 1.0 / (1.0 + fabs(med) / mad);
    } else {
        if (tid == 0) sh.count = 0;
        __syncthreads();
        uint32_t np = 0;
        for (int64_t i = tid; i < n; i += kT) np += (col[i] - med > 0.0) ? 1u : 0u;
        for (int off = 32; off > 0; off >>= 1) np += (uint32_t)__shfl_xor((int)np, off);
        if ((tid & 63) == 0 && np) atomicAdd(&sh.count, np);
        __syncthreads();
        const uint64_t npos = sh.count;
        __syncthreads();
        const double num = (med < 0.0) ? -med : 0.0;
        if (npos == 0) {
            D = (num == 0.0) ? 1.0 : 0.0;
        } else {
            const double madp = median_stream<2>(col, n, med, npos, sh, stats);
            D = 1.0 / (1.0 + num / madp);
        }
    }
    if (tid == 0) Dj[qi * ldm + j] = D;
}

template <int NOTION, int VPT>
hipError_t launch_vpt(const SelectArgs &a, hipStream_t st)
{
    dim3 grid((unsigned)a.m, (unsigned)a.qb);
    hipLaunchKernelGGL((k_select_reg<NOTION, VPT>), grid, dim3(kT), 0, st, a.T, a.n, a.m, a.ldm,
                       a.Dj, a.stats);
    return hipGetLastError();
}

template <int NOTION>
hipError_t launch_reg_t(const SelectArgs &a, hipStream_t st)
{
    const int64_t vpt = (a.n + kT - 1) / kT;
    if (vpt <= 1) return launch_vpt<NOTION, 1>(a, st);
    if (vpt <= 2) return launch_vpt<NOTION, 2>(a, st);
    if (vpt <= 4) return launch_vpt<NOTION, 4>(a, st);
    if (vpt <= 8) return launch_vpt<NOTION, 8>(a, st);
    if (vpt <= 12) return launch_vpt<NOTION, 12>(a, st);
    if (vpt <= 16) return launch_vpt<NOTION, 16>(a, st);
    if (vpt <= 24) return launch_vpt<NOTION, 24>(a, st);
    if (vpt <= 32) return launch_vpt<NOTION, 32>(a, st);
    if (vpt <= 40) return launch_vpt<NOTION, 40>(a, st);
    if (vpt <= 48) return launch_vpt<NOTION, 48>(a, st);
    return launch_vpt<NOTION, 64>(a, st);
}

}  // namespace

int64_t select_reg_max_n() { return (int64_t)kT * 64; }

hipError_t launch_select_stream(const SelectArgs &a, int notion, hipStream_t st)
{
    dim3 grid((unsigned)a.m, (unsigned)a.qb);
    if (notion == NOTION_PROJECTION)
        hipLaunchKernelGGL(k_select_stream<NOTION_PROJECTION>, grid, dim3(kT), 0, st, a.T, a.n,
                           a.m, a.ldm, a.Dj, a.stats);
    else
        hipLaunchKernelGGL(k_select_stream<NOTION_APD>, grid, dim3(kT), 0, st, a.T, a.n, a.m,
                           a.ldm, a.Dj, a.stats);
    return hipGetLastError();
}

hipError_t launch_select_reg(const SelectArgs &a, int notion, hipStream_t st)
{
    if (a.n > select_reg_max_n()) return hipErrorInvalidValue;
    if (notion == NOTION_PROJECTION) return launch_reg_t<NOTION_PROJECTION>(a, st);
    return launch_reg_t<NOTION_APD>(a, st);
}

}  // namespace rrs
