// rrs_mfma.hip -- halfspace depth with the projection on CDNA4 matrix cores
// (BF16 inputs, FP32 accumulation) and an exact FP64 recheck.
//
// Step a2 + a3 (+ a4) for halfspace depth, precision form RRS_BF16_RECHECK:
//   * the data is centred by its mean xbar (binary64), a_i = x_i - xbar, and
//     split into two bfloat16 terms a = a_hi + a_lo (+ remainder);
//   * each direction u_j is split the same way; the query's centring term
//     c_j = (z - xbar).u_j (binary64) is folded into two extra K columns
//     (A: 1, 1; B: -c_hi, -c_lo), so one GEMM row-by-column product is
//     t^_ij ~ a_i.u_j - c_j = (x_i - z).u_j;
//   * t^ = A_hi B_hi + A_hi B_lo + A_lo B_hi on v_mfma_f32_32x32x16_bf16;
//   * the epilogue decides the sign of the recipe's binary64 projection when
//     |t^| exceeds a rigorous margin M_ij = kappa (|a_i| + |c_j|) + e_canon,
//     and queues (query, point, direction) otherwise; the recheck kernel
//     recomputes those projections with the binary64 recipe.
// Counts are integers, so the result is identical to the binary64 form.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rrs_launch.hpp"

namespace rrs {

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr int kNJ = 2;            // 32-direction tiles per wave
constexpr int kRowsPerWave = 32;  // points per wave tile
constexpr int kWaves = 4;

// bfloat16 of a binary64 value, round to nearest even through binary32.
__device__ __forceinline__ __bf16 to_bf16(double v) { return (__bf16)(float)v; }
__device__ __forceinline__ double from_bf16(__bf16 v) { return (double)(float)v; }

// ---------------------------------------------------------------------------
// Data preparation (once per call): column means, centred split operands and
// the norm of every centred point.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_col_mean(const double *__restrict__ X, int64_t n,
                                                  int64_t d, double *__restrict__ xbar)
{
    // one workgroup per coordinate, fixed-order reduction (deterministic)
    __shared__ double red[256];
    const int64_t c = blockIdx.x;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += X[i * d + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) xbar[c] = red[0] / (double)n;
}

__global__ __launch_bounds__(256) void k_split_data(const double *__restrict__ X, int64_t n,
                                                    int64_t d, int64_t kp,
                                                    const double *__restrict__ xbar,
                                                    __bf16 *__restrict__ Ahi,
                                                    __bf16 *__restrict__ Alo,
                                                    float *__restrict__ anorm)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double ss = 0.0;
    for (int64_t c = 0; c < kp; ++c) {
        __bf16 h, l;
        if (c < d) {
            const double a = X[i * d + c] - xbar[c];
            h = to_bf16(a);
            l = to_bf16(a - from_bf16(h));
            ss = fma(a, a, ss);
        } else if (c < d + 2) {
            h = (__bf16)1.0f;  // multiplies the folded centring terms
            l = (__bf16)0.0f;
        } else {
            h = (__bf16)0.0f;
            l = (__bf16)0.0f;
        }
        Ahi[i * kp + c] = h;
        Alo[i * kp + c] = l;
    }
    // upper bound of the norm, rounded up to binary32
    const float nf = (float)sqrt(ss);
    anorm[i] = nf * (1.0f + 1e-6f);
}

// Per refinement: split the directions (binary64, [q][d][ldm] in UT) and fold
// the centring term; cmarg[q][j] = kappa |c_j| + slack (binary32, rounded up).
__global__ __launch_bounds__(64) void k_split_dirs(const double *__restrict__ UT, int64_t d,
                                                   int64_t m, int64_t ldm, int64_t ldb,
                                                   int64_t kp, const double *__restrict__ Zb,
                                                   const double *__restrict__ xbar,
                                                   double kappa, double canon,
                                                   __bf16 *__restrict__ Bhi,
                                                   __bf16 *__restrict__ Blo,
                                                   float *__restrict__ cmarg)
{
    const int64_t j = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int64_t qi = blockIdx.y;
    if (j >= ldb) return;
    __bf16 *bh = Bhi + (qi * ldb + j) * kp;
    __bf16 *bl = Blo + (qi * ldb + j) * kp;
    if (j >= m) {
        for (int64_t c = 0; c < kp; ++c) {
            bh[c] = (__bf16)0.0f;
            bl[c] = (__bf16)0.0f;
        }
        cmarg[qi * ldb + j] = 0.0f;
        return;
    }
    const double *u = UT + qi * d * ldm + j;
    const double *z = Zb + qi * d;
    double cj = 0.0, bn = 0.0;
    for (int64_t c = 0; c < d; ++c) {
        const double uc = u[c * ldm];
        const double b = z[c] - xbar[c];
        cj = fma(b, uc, cj);
        bn = fma(b, b, bn);
        const __bf16 h = to_bf16(uc);
        bh[c] = h;
        bl[c] = to_bf16(uc - from_bf16(h));
    }
    const __bf16 ch = to_bf16(-cj);
    bh[d] = ch;
    bh[d + 1] = to_bf16(-cj - from_bf16(ch));
    bl[d] = (__bf16)0.0f;
    bl[d + 1] = (__bf16)0.0f;
    for (int64_t c = d + 2; c < kp; ++c) {
        bh[c] = (__bf16)0.0f;
        bl[c] = (__bf16)0.0f;
    }
    // margin part that depends on the direction only: kappa |c_j| plus the
    // binary64 recipe's own error through |z - xbar|; the data part
    // kappa' |a_i| is added per element
    const double mc = kappa * fabs(cj) + canon * sqrt(bn) * 1.000001 + 1e-300;
    cmarg[qi * ldb + j] = (float)mc * (1.0f + 1e-6f);
}

// ---------------------------------------------------------------------------
// GEMM + sign epilogue.  Workgroup: 4 waves x 32 points, all sharing
// kNJ x 32 directions of one query.  Lane layout of v_mfma_f32_32x32x16_bf16:
// A row i = lane % 32 holds K elements 8 (lane / 32) .. +7 of the 16-step;
// B column j = lane % 32 likewise; accumulator r holds row
// (r / 4) 8 + (lane / 32) 4 + r % 4 of column lane % 32.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gemm_sign(
    const __bf16 *__restrict__ Ahi, const __bf16 *__restrict__ Alo,
    const float *__restrict__ anorm, int64_t n, int64_t kp,
    const __bf16 *__restrict__ Bhi, const __bf16 *__restrict__ Blo,
    const float *__restrict__ cmarg, int64_t m, int64_t ldm, int64_t ldb, float kappa_a,
    uint32_t *__restrict__ cnt, uint64_t *__restrict__ queue, uint32_t *__restrict__ qcount,
    uint64_t qcap)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t qi = blockIdx.y;
    const int64_t j0 = (int64_t)blockIdx.x * (32 * kNJ);
    const int64_t row0 = (int64_t)blockIdx.z * (kRowsPerWave * kWaves) + wave * kRowsPerWave;
    const int lr = lane & 31, lh = lane >> 5;

    f32x16 acc[kNJ];
#pragma unroll
    for (int t = 0; t < kNJ; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[t][r] = 0.0f;

    int64_t arow = row0 + lr;
    if (arow > n - 1) arow = n - 1;  // clamp; results of rows >= n are ignored
    const __bf16 *ah = Ahi + arow * kp + 8 * lh;
    const __bf16 *al = Alo + arow * kp + 8 * lh;
    const __bf16 *bh[kNJ], *bl[kNJ];
#pragma unroll
    for (int t = 0; t < kNJ; ++t) {
        const int64_t col = qi * ldb + j0 + 32 * t + lr;  // < qb * ldb: ldb covers the grid
        bh[t] = Bhi + col * kp + 8 * lh;
        bl[t] = Blo + col * kp + 8 * lh;
    }
    for (int64_t k = 0; k < kp; k += 16) {
        const bf16x8 a_h = *(const bf16x8 *)(ah + k);
        const bf16x8 a_l = *(const bf16x8 *)(al + k);
#pragma unroll
        for (int t = 0; t < kNJ; ++t) {
            const bf16x8 b_h = *(const bf16x8 *)(bh[t] + k);
            const bf16x8 b_l = *(const bf16x8 *)(bl[t] + k);
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_h, b_h, acc[t], 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_h, b_l, acc[t], 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_l, b_h, acc[t], 0, 0, 0);
        }
    }

    // epilogue: per lane, one column per tile, 16 rows
    float an[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t i = row0 + (r >> 2) * 8 + lh * 4 + (r & 3);
        an[r] = i < n ? anorm[i] : 0.0f;
    }
    __shared__ uint32_t red[kWaves][32 * kNJ][2];
#pragma unroll
    for (int t = 0; t < kNJ; ++t) {
        const int64_t j = j0 + 32 * t + lr;
        const float cm = j < m ? cmarg[qi * ldb + j] : 0.0f;
        uint32_t pos = 0, neg = 0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t i = row0 + (r >> 2) * 8 + lh * 4 + (r & 3);
            const bool live = i < n && j < m;
            const float v = acc[t][r];
            const float marg = fmaf(kappa_a, an[r], cm);
            const bool sp = live && v > marg;
            const bool sn = live && v < -marg;
            pos += sp ? 1u : 0u;
            neg += sn ? 1u : 0u;
            if (live && !sp && !sn) {
                const uint32_t slot = atomicAdd(qcount, 1u);
                if ((uint64_t)slot < qcap)
                    queue[slot] = ((uint64_t)qi << 48) | ((uint64_t)j << 32) | (uint64_t)i;
            }
        }
        // lanes l and l + 32 hold the same column
        pos += (uint32_t)__shfl_xor((int)pos, 32);
        neg += (uint32_t)__shfl_xor((int)neg, 32);
        if (lh == 0) {
            red[wave][32 * t + lr][0] = neg;  // t < 0: counts for "<= 0"
            red[wave][32 * t + lr][1] = pos;  // t > 0: counts for ">= 0"
        }
    }
    __syncthreads();
    if (threadIdx.x < 32 * kNJ * 2) {
        const int jj = threadIdx.x >> 1, w = threadIdx.x & 1;
        const int64_t j = j0 + jj;
        uint32_t s = 0;
#pragma unroll
        for (int wv = 0; wv < kWaves; ++wv) s += red[wv][jj][w];
        if (j < m && s) atomicAdd(&cnt[(qi * ldm + j) * 2 + w], s);
    }
}

// Exact decisions of the queued pairs with the binary64 recipe (grid-stride;
// the queue length is read on the device).
__global__ __launch_bounds__(256) void k_recheck(const uint64_t *__restrict__ queue,
                                                 const uint32_t *__restrict__ qcount,
                                                 uint64_t qcap, const double *__restrict__ X,
                                                 int64_t d, const double *__restrict__ Zb,
                                                 const double *__restrict__ UT, int64_t ldm,
                                                 uint32_t *__restrict__ cnt)
{
    const uint64_t total = *qcount < qcap ? *qcount : qcap;
    for (uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x; e < total;
         e += (uint64_t)gridDim.x * 256) {
        const uint64_t w = queue[e];
        const int64_t qi = (int64_t)(w >> 48);
        const int64_t j = (int64_t)((w >> 32) & 0xFFFF);
        const int64_t i = (int64_t)(w & 0xFFFFFFFFu);
        const double *x = X + i * d;
        const double *z = Zb + qi * d;
        const double *u = UT + qi * d * ldm + j;
        double t = 0.0;
        for (int64_t c = 0; c < d; ++c) t = fma(x[c] - z[c], u[c * ldm], t);
        if (t <= 0.0) atomicAdd(&cnt[(qi * ldm + j) * 2], 1u);
        if (t >= 0.0) atomicAdd(&cnt[(qi * ldm + j) * 2 + 1], 1u);
    }
}

// A queue that overflowed means some pairs were neither counted nor queued:
// the refinement's counts are then recomputed in full with the binary64
// recipe (flag checked on the device; normally a no-op launch).
__global__ __launch_bounds__(256) void k_overflow_reset(const uint32_t *__restrict__ qcount,
                                                        uint64_t qcap, uint32_t *__restrict__ cnt,
                                                        int64_t total, uint32_t *__restrict__ flag)
{
    const bool over = (uint64_t)*qcount > qcap;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i == 0) *flag = over ? 1u : 0u;
    if (over && i < total) cnt[i] = 0u;
}

}  // namespace

// kappa for the three-term bf16 product with binary32 accumulation of K
// terms (see the design doc for the derivation); canon = binary64 recipe slack.
void mfma_margins(int64_t d, int64_t kp, double *kappa, double *canon)
{
    const double split = 3.0 * ldexp(1.0, -17) * 1.5;          // dropped lo*lo + remainders
    const double accum = 2.0 * (double)(3 * kp + 16) * ldexp(1.0, -24);
    *kappa = split + accum;
    *canon = 2.0 * (double)(d + 2) * ldexp(1.0, -53);
}

int64_t mfma_kpad(int64_t d) { return (d + 2 + 15) / 16 * 16; }

hipError_t launch_mfma_prep(const double *X, int64_t n, int64_t d, double *xbar, __bf16 *Ahi,
                            __bf16 *Alo, float *anorm, hipStream_t st)
{
    hipLaunchKernelGGL(k_col_mean, dim3((unsigned)d), dim3(256), 0, st, X, n, d, xbar);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_split_data, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, X, n,
                       d, mfma_kpad(d), xbar, Ahi, Alo, anorm);
    return hipGetLastError();
}

hipError_t launch_mfma_dirs(const double *UT, int64_t d, int64_t m, int64_t ldm, int64_t ldb,
                            int64_t qb, const double *Zb, const double *xbar, __bf16 *Bhi,
                            __bf16 *Blo, float *cmarg, hipStream_t st)
{
    double kappa, canon;
    const int64_t kp = mfma_kpad(d);
    mfma_margins(d, kp, &kappa, &canon);
    dim3 grid((unsigned)((ldb + 63) / 64), (unsigned)qb);
    hipLaunchKernelGGL(k_split_dirs, grid, dim3(64), 0, st, UT, d, m, ldm, ldb, kp, Zb, xbar,
                       kappa, canon, Bhi, Blo, cmarg);
    return hipGetLastError();
}

hipError_t launch_mfma_count(const MfmaArgs &a, hipStream_t st)
{
    double kappa, canon;
    const int64_t kp = mfma_kpad(a.d);
    mfma_margins(a.d, kp, &kappa, &canon);
    const float kappa_a = (float)((kappa + canon) * 1.000001);
    dim3 grid((unsigned)((a.m + 32 * kNJ - 1) / (32 * kNJ)), (unsigned)a.qb,
              (unsigned)((a.n + kRowsPerWave * kWaves - 1) / (kRowsPerWave * kWaves)));
    if (a.ldb < (int64_t)grid.x * 32 * kNJ) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gemm_sign, grid, dim3(256), 0, st, a.Ahi, a.Alo, a.anorm, a.n, kp,
                       a.Bhi, a.Blo, a.cmarg, a.m, a.ldm, a.ldb, kappa_a, a.cnt, a.queue,
                       a.qcount, a.qcap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_recheck, dim3(1024), dim3(256), 0, st, a.queue, a.qcount, a.qcap, a.X,
                       a.d, a.Z, a.UT, a.ldm, a.cnt);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t total = a.qb * a.ldm * 2;
    hipLaunchKernelGGL(k_overflow_reset, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       a.qcount, a.qcap, a.cnt, total, a.flag);
    return hipGetLastError();
}

}  // namespace rrs
