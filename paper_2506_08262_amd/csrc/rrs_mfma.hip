// rrs_mfma.hip -- halfspace depth with the projection on CDNA4 matrix cores
// and, for the exact forms, an FP64 recheck of the uncertain signs.
//
// Step a2 + a3 (+ a4) for halfspace depth.  Every form centres the data by
// its mean xbar (binary64), a_i = x_i - xbar, and folds the query's centring
// term c_j = (z - xbar).u_j (binary64) into extra K columns (A: 1; B: -c), so
// that one GEMM row-by-column product is t^_ij ~ a_i.u_j - c_j = (x_i - z).u_j.
//   RRS_BF16_RECHECK: a and u are split into two bfloat16 terms,
//     t^ = A_hi B_hi + A_hi B_lo + A_lo B_hi on v_mfma_f32_32x32x16_bf16;
//   RRS_F32_RECHECK / RRS_F32_PLAIN: a, u and c rounded to binary32,
//     t^ = A B on v_mfma_f32_32x32x2_f32.
// The recheck forms take the sign of the recipe's binary64 projection from t^
// when |t^| exceeds a rigorous margin M_ij = kappa (|a_i| + |c_j|) + e_canon
// and queue (query, point, direction) otherwise; the recheck kernel
// recomputes those projections with the binary64 recipe, so the counts are
// identical to the binary64 form.  The plain form takes every sign from t^
// (t^ == 0 counts on both sides) and is approximate.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "rrs_launch.hpp"

namespace rrs {

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(16))) float f32x16;


// bfloat16 of a binary64 value, round to nearest even through binary32.
__device__ __forceinline__ __bf16 to_bf16(double v) { return (__bf16)(float)v; }
__device__ __forceinline__ double from_bf16(__bf16 v) { return (double)(float)v; }

// ---------------------------------------------------------------------------
// Data preparation (once per call): column means, centred operands and the
// norm of every centred point.
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

// A0/A1 [n][kp]: bf16 hi/lo terms (BF16) or binary32 values in A0 (F32).
template <int PREC>
__global__ __launch_bounds__(256) void k_prep_data(const double *__restrict__ X, int64_t n,
                                                   int64_t d, int64_t kp,
                                                   const double *__restrict__ xbar,
                                                   void *__restrict__ A0, void *__restrict__ A1,
                                                   float *__restrict__ anorm,
                                                   float *__restrict__ amax)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double ss = 0.0;
    if (i < n) {
        // column d (and d + 1 for BF16) multiplies the folded centring term.
        // The row goes out in 16-byte pieces (8 bf16 or 4 binary32 elements;
        // kp is a multiple of 16 or 8), the loads of a piece's coordinates
        // issued together
        const int64_t nfold = PREC == MFMA_BF16 ? 2 : 1;
        constexpr int kE = PREC == MFMA_BF16 ? 8 : 4;
        typedef __attribute__((ext_vector_type(8))) __bf16 v8bf;
        typedef __attribute__((ext_vector_type(4))) float v4f;
        const double *x = X + i * d;
        for (int64_t g = 0; g < kp / kE; ++g) {
            double xv[kE];
#pragma unroll
            for (int e = 0; e < kE; ++e) {
                const int64_t c = g * kE + e;
                xv[e] = c < d ? x[c] - xbar[c] : 0.0;
            }
            v8bf vh{}, vl{};
            v4f vf{};
#pragma unroll
            for (int e = 0; e < kE; ++e) {
                const int64_t c = g * kE + e;
                double a = 0.0;
                if (c < d) {
                    a = xv[e];
                    ss = fma(a, a, ss);
                } else if (c < d + nfold) {
                    a = 1.0;
                }
                if (PREC == MFMA_BF16) {
                    const __bf16 h = to_bf16(a);
                    vh[e] = h;
                    vl[e] = c < d ? to_bf16(a - from_bf16(h)) : (__bf16)0.0f;
                } else {
                    vf[e] = (float)a;
                }
            }
            if (PREC == MFMA_BF16) {
                ((v8bf *)A0)[i * (kp / kE) + g] = vh;
                ((v8bf *)A1)[i * (kp / kE) + g] = vl;
            } else {
                ((v4f *)A0)[i * (kp / kE) + g] = vf;
            }
        }
        // upper bound of the norm, rounded up to binary32
        const float nf = (float)sqrt(ss);
        anorm[i] = nf * (1.0f + 1e-6f);
        // largest norm bound (non-negative floats order like their bit patterns)
        atomicMax((int *)amax, __float_as_int(anorm[i]));
    }
    // sum of the squared norms: per wave (every lane takes part), then one atomic
    double w = ss;
    for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o);
    if ((threadIdx.x & 63) == 0 && w != 0.0) atomicAdd((double *)(amax + 2), w);
}

// Per refinement: the directions (binary64, [q][d][ldm] in UT) in the GEMM's
// operand format, one operand row per flat column J = q m + j (rows ncols ..
// npad - 1 are zero).  FOLD (sign counts): the centring term is folded in and
// cmarg[J] = kappa |c_j| + slack (binary32, rounded up).  Otherwise (stored
// projections): the centring columns are zero, cq[J] = c_j and eq[J] bounds
// |(s_ij - c_j) - t_ij| for every point i, with t_ij the recipe's binary64
// projection: kappa max|a| + canon (max|a| + 2 |z - xbar|).
//
// Four lanes per column: lane t of the quad converts the 16-byte pieces
// g = t, t + 4, ... of the row (8 bf16 or 4 binary32 elements), so that a
// quad writes 64 contiguous bytes per step and a wave keeps 16 columns' loads
// in flight.  c_j = (z - xbar).u and |z - xbar|^2 are summed per lane and
// then over the quad; the pieces from coordinate d on (centring columns and
// padding) are written after that sum.  The order of the sum only moves c_j
// by rounding, which the canon term of the margin covers for any order.
template <int PREC, bool FOLD>
__global__ __launch_bounds__(256) void k_prep_dirs(const double *__restrict__ UT, int64_t d,
                                                   int64_t m, int64_t ldm, int64_t ncols,
                                                   int64_t npad, int64_t kp,
                                                   const double *__restrict__ Zb,
                                                   const double *__restrict__ xbar, double kappa,
                                                   double canon, void *__restrict__ B0,
                                                   void *__restrict__ B1,
                                                   float *__restrict__ cmarg,
                                                   const float *__restrict__ amax,
                                                   double *__restrict__ cq,
                                                   double *__restrict__ eq, int pp)
{
    const int t = threadIdx.x & 3;
    const int64_t J = (int64_t)blockIdx.x * 64 + (threadIdx.x >> 2);
    if (J >= npad) return;  // uniform within a quad
    constexpr int kE = PREC == MFMA_BF16 ? 8 : 4;
    typedef __attribute__((ext_vector_type(8))) __bf16 v8bf;
    typedef __attribute__((ext_vector_type(4))) float v4f;
    const int64_t pieces = kp / kE;
    v8bf *h8 = (v8bf *)B0 + J * pieces;
    v8bf *l8 = (v8bf *)B1 + J * pieces;
    v4f *f4 = (v4f *)B0 + J * pieces;
    if (J >= ncols) {
        for (int64_t g = t; g < pieces; g += 4) {
            if (PREC == MFMA_BF16) {
                h8[g] = v8bf{};
                l8[g] = v8bf{};
            } else {
                f4[g] = v4f{};
            }
        }
        if (t == 0) {
            if (FOLD) {
                cmarg[J] = 0.0f;
            } else {
                cq[J] = 0.0;
                eq[J] = 0.0;
            }
        }
        return;
    }
    const int64_t qi = J / m, j = J - qi * m;
    const double *u = UT + qi * d * ldm + j;
    const double *z = Zb + qi * d;
    const int64_t gfull = d / kE;  // pieces made of coordinates c < d only
    double cj = 0.0, bn = 0.0;
    for (int64_t g = t; g < pieces; g += 4) {
        v8bf vh{}, vl{};
        v4f vf{};
#pragma unroll
        for (int e = 0; e < kE; ++e) {
            const int64_t c = g * kE + e;
            if (c < d) {
                const double uc = u[c * ldm];
                const double b = z[c] - xbar[c];
                cj = fma(b, uc, cj);
                bn = fma(b, b, bn);
                if (PREC == MFMA_BF16) {
                    const __bf16 h = to_bf16(uc);
                    vh[e] = h;
                    vl[e] = to_bf16(uc - from_bf16(h));
                } else {
                    vf[e] = (float)uc;
                }
            }
        }
        if (g < gfull) {
            if (PREC == MFMA_BF16) {
                h8[g] = vh;
                l8[g] = vl;
            } else {
                f4[g] = vf;
            }
        }
    }
    cj += __shfl_xor(cj, 1);
    bn += __shfl_xor(bn, 1);
    cj += __shfl_xor(cj, 2);
    bn += __shfl_xor(bn, 2);
    // the pieces from coordinate d on, now that c_j is known
    for (int64_t g = gfull + ((t - gfull) & 3); g < pieces; g += 4) {
        v8bf vh{}, vl{};
        v4f vf{};
#pragma unroll
        for (int e = 0; e < kE; ++e) {
            const int64_t c = g * kE + e;
            if (c < d) {
                const double uc = u[c * ldm];
                if (PREC == MFMA_BF16) {
                    const __bf16 h = to_bf16(uc);
                    vh[e] = h;
                    vl[e] = to_bf16(uc - from_bf16(h));
                } else {
                    vf[e] = (float)uc;
                }
            } else if (FOLD && c == d) {
                // the centring term -c_j (bf16: hi in column d, lo in d + 1)
                if (PREC == MFMA_BF16)
                    vh[e] = to_bf16(-cj);
                else
                    vf[e] = (float)(-cj);
            } else if (FOLD && PREC == MFMA_BF16 && c == d + 1) {
                vh[e] = to_bf16(-cj - from_bf16(to_bf16(-cj)));
            }
        }
        if (PREC == MFMA_BF16) {
            h8[g] = vh;
            l8[g] = vl;
        } else {
            f4[g] = vf;
        }
    }
    if (t != 0) return;
    // margin part that depends on the direction only: kappa |c_j| plus the
    // binary64 recipe's own error through |z - xbar|; the data part
    // kappa' |a_i| is added per element
    if (FOLD) {
        const double mc = kappa * fabs(cj) + canon * sqrt(bn) * 1.000001 + 1e-300;
        cmarg[J] = (float)mc * (1.0f + 1e-6f);
    } else {
        cq[J] = cj;
        if (pp) {
            // per-point bounds: the column part only (point i adds
            // mfma_point_alpha * anorm[i])
            eq[J] = canon * 2.0 * sqrt(bn) * 1.000001 * 1.000002;
        } else {
            const double am = (double)*amax;
            eq[J] = (kappa * am + canon * (am + 2.0 * sqrt(bn) * 1.000001)) * 1.000001;
        }
    }
}

// ---------------------------------------------------------------------------
// GEMM with a sign-count or a store epilogue.  C = A B^T with A the centred
// data [n][kp] and B the direction operands [npad][kp] (flat columns
// J = q m + j of the batch).  Workgroup: 4 waves, a tile of kTM = 256 points
// x kTN = 128 columns; wave w owns points 64 w .. 64 w + 63 (two 32-row MFMA
// tiles) against all four 32-column tiles.  B is staged through LDS in K
// chunks of kKC (shared by the four waves); A fragments come straight from
// global memory (each row is read by one wave only).  Lane layouts
// (lr = lane % 32, lh = lane / 32):
//   v_mfma_f32_32x32x16_bf16: A row lr holds K elements 8 lh .. 8 lh + 7 of
//     the 16-step, B column lr likewise;
//   v_mfma_f32_32x32x2_f32: A row lr holds K element lh of the 2-step, B
//     column lr likewise.  Each lane loads 4 consecutive floats of its row
//     (K elements 8 g + 4 lh .. + 3 of group g) and feeds them to 4 MFMAs, so
//     the 4 steps of a group cover its 8 K elements once (A and B use the same
//     assignment, so the sum is the full dot product);
//   both: accumulator r holds row (r / 4) 8 + 4 lh + r % 4 of column lr.
// ---------------------------------------------------------------------------
constexpr int kTM = 256, kTN = 128, kKC = 64;
constexpr int kLdsRow16 = kKC + 8;   // bf16 elements per staged B row (padded)
constexpr int kLdsRow32 = kKC + 4;   // binary32 elements per staged B row (padded)

constexpr int kStg = 64 + 4;          // floats per staged column in the store epilogue

struct alignas(16) GemmLds {
    union {
        __bf16 bh[kTN * kLdsRow16 * 2];  // hi rows, then lo rows
        float bf[kTN * kLdsRow32];
        float stg[4 * 32 * kStg];        // store epilogue: per wave 32 columns x 64 rows
    };
    uint32_t red[4][kTN][2];
    float an[kTM];   // norm bounds of the tile's points (sign epilogue)
};

// Variant 2 (pipelined): both operands staged through LDS in K chunks of
// kKC2, double-buffered; the global loads of chunk c + 1 are in flight while
// the MFMAs of chunk c run.
constexpr int kKC2 = 32;
constexpr int kRow2h = kKC2 + 8;   // bf16 elements per staged row (80 B: 8-lane groups hit
                                   // distinct 16-byte bank groups)
constexpr int kRow2f = kKC2 + 4;   // binary32 elements per staged row (144 B)

struct alignas(16) GemmLds2 {
    union {
        struct {
            __bf16 a[2][2][kTM * kRow2h];  // [buffer][term]
            __bf16 b[2][2][kTN * kRow2h];
        } h;
        struct {
            float a[2][kTM * kRow2f];
            float b[2][kTN * kRow2f];
        } f;
        float stg[4 * 32 * kStg];  // store epilogue (as in GemmLds)
    };
    uint32_t red[4][kTN][2];
    float an[kTM];
};

enum { EPI_SIGN = 0, EPI_STORE = 1 };

// the chunk-prefetch variant stages a B chunk with at most 8 pieces per thread
static_assert(kTN * (kKC / 8) * 2 == 256 * 8 && kKC / 8 == 8,
              "bf16 B chunk: 8 pieces per thread, index math by shifts");
static_assert(kTN * (kKC / 4) == 256 * 8 && kKC / 4 == 16,
              "binary32 B chunk: 8 pieces per thread, index math by shifts");

// Variant 1 (chunk prefetch): per K chunk the B rows go global -> registers
// -> LDS and every A fragment of the chunk is requested before the first
// MFMA, so the global latencies of both overlap and are paid once per chunk
// (more registers, fewer waves per SIMD).
template <int PREC>
__device__ __forceinline__ void gemm_block_chunk(const void *__restrict__ A0,
                                           const void *__restrict__ A1, int64_t n, int64_t kp,
                                           const void *__restrict__ B0,
                                           const void *__restrict__ B1, int64_t J0,
                                           int64_t row0, GemmLds &L, f32x16 (&acc)[2][4])
{
    const int tid = threadIdx.x, lane = tid & 63;
    const int lr = lane & 31, lh = lane >> 5;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[rt][ct][r] = 0.0f;
    int64_t ar[2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
        ar[rt] = row0 + rt * 32 + lr;
        if (ar[rt] > n - 1) ar[rt] = n - 1;  // clamp; rows >= n are ignored
    }
    constexpr int kStep = PREC == MFMA_BF16 ? 16 : 8;   // K per MFMA group
    constexpr int kSteps = kKC / kStep;                  // groups per full chunk
    for (int64_t k0 = 0; k0 < kp; k0 += kKC) {
        const int kc = (int)((kp - k0) < kKC ? (kp - k0) : kKC);
        const int ns = kc / kStep;
        if (PREC == MFMA_BF16) {
            // B chunk: 128 rows x kc, two terms, 16-byte pieces (<= 8 per thread)
            const int vpr = kc / 8;
            bf16x8 bst[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int p = tid + 256 * u;
                const int term = p >> 10, q = p & 1023;
                const int row = q >> 3, piece = q & 7;
                if (piece < vpr)
                    bst[u] = *(const bf16x8 *)((const __bf16 *)(term ? B1 : B0) +
                                               (J0 + row) * kp + k0 + piece * 8);
            }
            bf16x8 ah[kSteps][2], al[kSteps][2];
#pragma unroll
            for (int st = 0; st < kSteps; ++st)
                if (st < ns)
#pragma unroll
                    for (int rt = 0; rt < 2; ++rt) {
                        const int64_t off = ar[rt] * kp + k0 + st * 16 + 8 * lh;
                        ah[st][rt] = *(const bf16x8 *)((const __bf16 *)A0 + off);
                        al[st][rt] = *(const bf16x8 *)((const __bf16 *)A1 + off);
                    }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int p = tid + 256 * u;
                const int term = p >> 10, q = p & 1023;
                const int row = q >> 3, piece = q & 7;
                if (piece < vpr)
                    *(bf16x8 *)(L.bh + (term * kTN + row) * kLdsRow16 + piece * 8) = bst[u];
            }
            __syncthreads();
#pragma unroll
            for (int st = 0; st < kSteps; ++st) {
                if (st >= ns) break;
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) {
                    const int col = ct * 32 + lr;
                    const bf16x8 bh =
                        *(const bf16x8 *)(L.bh + col * kLdsRow16 + st * 16 + 8 * lh);
                    const bf16x8 bl =
                        *(const bf16x8 *)(L.bh + (kTN + col) * kLdsRow16 + st * 16 + 8 * lh);
#pragma unroll
                    for (int rt = 0; rt < 2; ++rt) {
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            ah[st][rt], bh, acc[rt][ct], 0, 0, 0);
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            ah[st][rt], bl, acc[rt][ct], 0, 0, 0);
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            al[st][rt], bh, acc[rt][ct], 0, 0, 0);
                    }
                }
            }
        } else {
            const int vpr = kc / 4;
            f32x4 bst[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int p = tid + 256 * u;
                const int row = p >> 4, piece = p & 15;
                if (piece < vpr)
                    bst[u] = *(const f32x4 *)((const float *)B0 + (J0 + row) * kp + k0 +
                                              piece * 4);
            }
            f32x4 a[kSteps][2];
#pragma unroll
            for (int st = 0; st < kSteps; ++st)
                if (st < ns)
#pragma unroll
                    for (int rt = 0; rt < 2; ++rt)
                        a[st][rt] = *(const f32x4 *)((const float *)A0 + ar[rt] * kp + k0 +
                                                     st * 8 + 4 * lh);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int p = tid + 256 * u;
                const int row = p >> 4, piece = p & 15;
                if (piece < vpr) *(f32x4 *)(L.bf + row * kLdsRow32 + piece * 4) = bst[u];
            }
            __syncthreads();
#pragma unroll
            for (int st = 0; st < kSteps; ++st) {
                if (st >= ns) break;
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) {
                    const int col = ct * 32 + lr;
                    const f32x4 b = *(const f32x4 *)(L.bf + col * kLdsRow32 + st * 8 + 4 * lh);
#pragma unroll
                    for (int rt = 0; rt < 2; ++rt) {
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[st][rt][0], b[0],
                                                                           acc[rt][ct], 0, 0, 0);
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[st][rt][1], b[1],
                                                                           acc[rt][ct], 0, 0, 0);
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[st][rt][2], b[2],
                                                                           acc[rt][ct], 0, 0, 0);
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[st][rt][3], b[3],
                                                                           acc[rt][ct], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();  // the next chunk overwrites the staged B
    }
}

// Variant 0 (per-step loads): B chunks staged through LDS, A fragments
// loaded right before the MFMAs of each K step (fewer registers).
template <int PREC>
__device__ __forceinline__ void gemm_block_steps(const void *__restrict__ A0,
                                           const void *__restrict__ A1, int64_t n, int64_t kp,
                                           const void *__restrict__ B0,
                                           const void *__restrict__ B1, int64_t J0,
                                           int64_t row0, GemmLds &L, f32x16 (&acc)[2][4])
{
    const int tid = threadIdx.x, lane = tid & 63;
    const int lr = lane & 31, lh = lane >> 5;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[rt][ct][r] = 0.0f;
    int64_t ar[2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
        ar[rt] = row0 + rt * 32 + lr;
        if (ar[rt] > n - 1) ar[rt] = n - 1;  // clamp; rows >= n are ignored
    }
    for (int64_t k0 = 0; k0 < kp; k0 += kKC) {
        const int kc = (int)((kp - k0) < kKC ? (kp - k0) : kKC);
        // stage B[J0 .. J0 + 127][k0 .. k0 + kc) in LDS, 16 bytes per copy
        if (PREC == MFMA_BF16) {
            // 8 pieces of 16 bytes per row and term in a full chunk
            const int vpr = kc / 8;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int p = tid + 256 * u;
                const int term = p >> 10, q = p & 1023;
                const int row = q >> 3, piece = q & 7;
                if (piece < vpr) {
                    const __bf16 *src = (const __bf16 *)(term ? B1 : B0) + (J0 + row) * kp +
                                        k0 + piece * 8;
                    *(bf16x8 *)(L.bh + (term * kTN + row) * kLdsRow16 + piece * 8) =
                        *(const bf16x8 *)src;
                }
            }
        } else {
            // 16 pieces of 16 bytes per row in a full chunk
            const int vpr = kc / 4;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int p = tid + 256 * u;
                const int row = p >> 4, piece = p & 15;
                if (piece < vpr) {
                    const float *src = (const float *)B0 + (J0 + row) * kp + k0 + piece * 4;
                    *(f32x4 *)(L.bf + row * kLdsRow32 + piece * 4) = *(const f32x4 *)src;
                }
            }
        }
        __syncthreads();
        if (PREC == MFMA_BF16) {
            for (int kk = 0; kk < kc; kk += 16) {
                bf16x8 ah[2], al[2];
#pragma unroll
                for (int rt = 0; rt < 2; ++rt) {
                    ah[rt] = *(const bf16x8 *)((const __bf16 *)A0 + ar[rt] * kp + k0 + kk + 8 * lh);
                    al[rt] = *(const bf16x8 *)((const __bf16 *)A1 + ar[rt] * kp + k0 + kk + 8 * lh);
                }
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) {
                    const int col = ct * 32 + lr;
                    const bf16x8 bh = *(const bf16x8 *)(L.bh + col * kLdsRow16 + kk + 8 * lh);
                    const bf16x8 bl =
                        *(const bf16x8 *)(L.bh + (kTN + col) * kLdsRow16 + kk + 8 * lh);
#pragma unroll
                    for (int rt = 0; rt < 2; ++rt) {
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[rt], bh,
                                                                              acc[rt][ct], 0, 0, 0);
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[rt], bl,
                                                                              acc[rt][ct], 0, 0, 0);
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[rt], bh,
                                                                              acc[rt][ct], 0, 0, 0);
                    }
                }
            }
        } else {
            for (int kk = 0; kk < kc; kk += 8) {
                f32x4 a[2];
#pragma unroll
                for (int rt = 0; rt < 2; ++rt)
                    a[rt] = *(const f32x4 *)((const float *)A0 + ar[rt] * kp + k0 + kk + 4 * lh);
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) {
                    const int col = ct * 32 + lr;
                    const f32x4 b = *(const f32x4 *)(L.bf + col * kLdsRow32 + kk + 4 * lh);
#pragma unroll
                    for (int rt = 0; rt < 2; ++rt) {
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[rt][0], b[0],
                                                                           acc[rt][ct], 0, 0, 0);
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[rt][1], b[1],
                                                                           acc[rt][ct], 0, 0, 0);
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[rt][2], b[2],
                                                                           acc[rt][ct], 0, 0, 0);
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[rt][3], b[3],
                                                                           acc[rt][ct], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();  // the next chunk overwrites the staged B
    }
}

// Variant 2: see GemmLds2.  Each thread moves 8 A pieces and 4 B pieces of
// 16 bytes per chunk (256 rows x 64 B x 2 terms, 128 rows x 64 B x 2 terms for
// bf16; 256 x 128 B and 128 x 128 B for binary32).
template <int PREC>
__device__ __forceinline__ void gemm_block_pipe(const void *__restrict__ A0,
                                                const void *__restrict__ A1, int64_t n,
                                                int64_t kp, const void *__restrict__ B0,
                                                const void *__restrict__ B1, int64_t J0,
                                                int64_t rowblk, GemmLds2 &L,
                                                f32x16 (&acc)[2][4])
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 31, lh = lane >> 5;
    constexpr bool kH = PREC == MFMA_BF16;
    constexpr int kEl = kH ? 2 : 4;                 // bytes per element
    constexpr int kPieceEl = 16 / kEl;              // elements per 16-byte piece
    constexpr int kPR = kKC2 * kEl / 16;            // pieces per row and term
    constexpr int kRow = kH ? kRow2h : kRow2f;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[rt][ct][r] = 0.0f;
    const int nchunks = (int)((kp + kKC2 - 1) / kKC2);
    f32x4 ra[8], rb[4];  // staging registers (16 bytes each, reinterpreted)

    // piece u of this thread: A pieces p = tid + 256 u (u < 8), B pieces likewise
    auto load = [&](int c) {
        const int64_t k0 = (int64_t)c * kKC2;
        const int kc = (int)((kp - k0) < kKC2 ? (kp - k0) : kKC2);
        const int vpr = kc * kEl / 16;  // valid pieces per row
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int p = tid + 256 * u;
            const int term = kH ? p / (kTM * kPR) : 0;
            const int q = p - term * kTM * kPR;
            const int row = q / kPR, part = q - row * kPR;
            if ((kH || p < kTM * kPR) && part < vpr) {
                int64_t g = rowblk + row;
                if (g > n - 1) g = n - 1;
                const char *src = (const char *)(term ? A1 : A0) +
                                  ((g * kp + k0) * kEl + part * 16);
                ra[u] = *(const f32x4 *)src;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int p = tid + 256 * u;
            const int term = kH ? p / (kTN * kPR) : 0;
            const int q = p - term * kTN * kPR;
            const int row = q / kPR, part = q - row * kPR;
            if ((kH || p < kTN * kPR) && part < vpr) {
                const char *src = (const char *)(term ? B1 : B0) +
                                  (((J0 + row) * kp + k0) * kEl + part * 16);
                rb[u] = *(const f32x4 *)src;
            }
        }
    };
    auto store = [&](int c, int buf) {
        const int64_t k0 = (int64_t)c * kKC2;
        const int kc = (int)((kp - k0) < kKC2 ? (kp - k0) : kKC2);
        const int vpr = kc * kEl / 16;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int p = tid + 256 * u;
            const int term = kH ? p / (kTM * kPR) : 0;
            const int q = p - term * kTM * kPR;
            const int row = q / kPR, part = q - row * kPR;
            if ((kH || p < kTM * kPR) && part < vpr) {
                char *dst = kH ? (char *)(L.h.a[buf][term] + row * kRow + part * kPieceEl)
                               : (char *)(L.f.a[buf] + row * kRow + part * kPieceEl);
                *(f32x4 *)dst = ra[u];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int p = tid + 256 * u;
            const int term = kH ? p / (kTN * kPR) : 0;
            const int q = p - term * kTN * kPR;
            const int row = q / kPR, part = q - row * kPR;
            if ((kH || p < kTN * kPR) && part < vpr) {
                char *dst = kH ? (char *)(L.h.b[buf][term] + row * kRow + part * kPieceEl)
                               : (char *)(L.f.b[buf] + row * kRow + part * kPieceEl);
                *(f32x4 *)dst = rb[u];
            }
        }
    };

    load(0);
    store(0, 0);
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
        const int buf = c & 1;
        if (c + 1 < nchunks) load(c + 1);  // in flight during this chunk's MFMAs
        const int64_t k0 = (int64_t)c * kKC2;
        const int kc = (int)((kp - k0) < kKC2 ? (kp - k0) : kKC2);
        if (kH) {
            for (int kk = 0; kk < kc; kk += 16) {
                bf16x8 ah[2], al[2];
#pragma unroll
                for (int rt = 0; rt < 2; ++rt) {
                    const int row = wave * 64 + rt * 32 + lr;
                    ah[rt] = *(const bf16x8 *)(L.h.a[buf][0] + row * kRow + kk + 8 * lh);
                    al[rt] = *(const bf16x8 *)(L.h.a[buf][1] + row * kRow + kk + 8 * lh);
                }
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) {
                    const int col = ct * 32 + lr;
                    const bf16x8 bh = *(const bf16x8 *)(L.h.b[buf][0] + col * kRow + kk + 8 * lh);
                    const bf16x8 bl = *(const bf16x8 *)(L.h.b[buf][1] + col * kRow + kk + 8 * lh);
#pragma unroll
                    for (int rt = 0; rt < 2; ++rt) {
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[rt], bh,
                                                                              acc[rt][ct], 0, 0, 0);
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[rt], bl,
                                                                              acc[rt][ct], 0, 0, 0);
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[rt], bh,
                                                                              acc[rt][ct], 0, 0, 0);
                    }
                }
            }
        } else {
            for (int kk = 0; kk < kc; kk += 8) {
                f32x4 a[2];
#pragma unroll
                for (int rt = 0; rt < 2; ++rt) {
                    const int row = wave * 64 + rt * 32 + lr;
                    a[rt] = *(const f32x4 *)(L.f.a[buf] + row * kRow + kk + 4 * lh);
                }
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) {
                    const int col = ct * 32 + lr;
                    const f32x4 b = *(const f32x4 *)(L.f.b[buf] + col * kRow + kk + 4 * lh);
#pragma unroll
                    for (int rt = 0; rt < 2; ++rt) {
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[rt][0], b[0],
                                                                           acc[rt][ct], 0, 0, 0);
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[rt][1], b[1],
                                                                           acc[rt][ct], 0, 0, 0);
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[rt][2], b[2],
                                                                           acc[rt][ct], 0, 0, 0);
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[rt][3], b[3],
                                                                           acc[rt][ct], 0, 0, 0);
                    }
                }
            }
        }
        if (c + 1 < nchunks) store(c + 1, buf ^ 1);  // the other buffer: free since the
                                                     // barrier that ended chunk c - 1
        __syncthreads();
    }
}

template <int PREC, int EPI, int PF>
__global__ __launch_bounds__(256) void k_gemm(
    const void *__restrict__ A0, const void *__restrict__ A1,
    const float *__restrict__ anorm, int64_t n, int64_t kp,
    const void *__restrict__ B0, const void *__restrict__ B1,
    const float *__restrict__ cmarg, int64_t m, int64_t ncols, int64_t ldm, float kappa_a,
    uint32_t *__restrict__ cnt, uint64_t *__restrict__ queue, uint32_t *__restrict__ qcount,
    uint64_t qcap, float *__restrict__ S)
{
    using Lds = typename std::conditional<PF == 2, GemmLds2, GemmLds>::type;
    __shared__ Lds L;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 31, lh = lane >> 5;
    const int64_t J0 = (int64_t)blockIdx.x * kTN;
    const int64_t row0 = (int64_t)blockIdx.y * kTM + wave * 64;
    if (EPI == EPI_SIGN && PREC != MFMA_F32_PLAIN) {
        const int64_t i = (int64_t)blockIdx.y * kTM + tid;  // 256 threads = kTM rows
        L.an[tid] = i < n ? anorm[i] : 0.0f;
    }
    f32x16 acc[2][4];
    // the block's barriers publish L.an
    if constexpr (PF == 2)
        gemm_block_pipe<PREC>(A0, A1, n, kp, B0, B1, J0, (int64_t)blockIdx.y * kTM, L, acc);
    else if constexpr (PF == 1)
        gemm_block_chunk<PREC>(A0, A1, n, kp, B0, B1, J0, row0, L, acc);
    else
        gemm_block_steps<PREC>(A0, A1, n, kp, B0, B1, J0, row0, L, acc);

    if (EPI == EPI_STORE) {
        const bool full = (int64_t)(blockIdx.y + 1) * kTM <= n && (n & 3) == 0;
        if (full) {
            // through LDS, per column tile: the wave's 64 x 32 block is
            // written column-major (stride kStg floats), then read back as 16
            // lanes x 16 bytes per column, so each store instruction covers
            // four whole 256-byte column segments
            float *stg = L.stg + wave * 32 * kStg;
            const int rc = lane >> 4, rr = (lane & 15) * 4;
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                __syncthreads();  // the previous tile's reads (or the K loop) are done
#pragma unroll
                for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        const f32x4 v = {acc[rt][ct][4 * g], acc[rt][ct][4 * g + 1],
                                         acc[rt][ct][4 * g + 2], acc[rt][ct][4 * g + 3]};
                        *(f32x4 *)(stg + lr * kStg + rt * 32 + g * 8 + lh * 4) = v;
                    }
                __syncthreads();
#pragma unroll
                for (int it = 0; it < 8; ++it) {
                    const int c = it * 4 + rc;
                    const int64_t J = J0 + ct * 32 + c;
                    const f32x4 v = *(const f32x4 *)(stg + c * kStg + rr);
                    // written once, read by the select: non-temporal
                    if (J < ncols) __builtin_nontemporal_store(v, (f32x4 *)(S + J * n + row0 + rr));
                }
            }
            return;
        }
        // S[J][i]: lane lr writes rows (r / 4) 8 + 4 lh .. + 3 of column J
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int64_t J = J0 + ct * 32 + lr;
            if (J >= ncols) continue;
            float *col = S + J * n;
#pragma unroll
            for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int64_t i = row0 + rt * 32 + g * 8 + lh * 4;
                    if (i + 3 < n && (n & 3) == 0) {
                        f32x4 v = {acc[rt][ct][4 * g], acc[rt][ct][4 * g + 1],
                                   acc[rt][ct][4 * g + 2], acc[rt][ct][4 * g + 3]};
                        *(f32x4 *)(col + i) = v;
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (i + e < n) col[i + e] = acc[rt][ct][4 * g + e];
                    }
                }
        }
        return;
    }

    constexpr bool kPlain = PREC == MFMA_F32_PLAIN;
    const int rows_left = (int)(n - (int64_t)blockIdx.y * kTM);  // > 0
    float cm[4];
    bool jl[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const int64_t J = J0 + ct * 32 + lr;
        jl[ct] = J < ncols;
        cm[ct] = (!kPlain && jl[ct]) ? cmarg[J] : 0.0f;
    }
    // counts: per element one margin, two compares and two adds; rows past n
    // occur in the last row block only (a uniform test per workgroup)
    uint32_t pos[4] = {0u, 0u, 0u, 0u}, neg[4] = {0u, 0u, 0u, 0u};
    auto count = [&](auto full) {
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int il = wave * 64 + rt * 32 + (r >> 2) * 8 + lh * 4 + (r & 3);
                const bool rl = decltype(full)::value || il < rows_left;
                const float an_r = kPlain ? 0.0f : L.an[il];
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) {
                    const float v = acc[rt][ct][r];
                    if (kPlain) {
                        // sign of t^ itself; zero counts on both sides
                        pos[ct] += (rl && v >= 0.0f) ? 1u : 0u;
                        neg[ct] += (rl && v <= 0.0f) ? 1u : 0u;
                    } else {
                        const float marg = fmaf(kappa_a, an_r, cm[ct]);
                        pos[ct] += (rl && v > marg) ? 1u : 0u;
                        neg[ct] += (rl && v < -marg) ? 1u : 0u;
                    }
                }
            }
    };
    const bool rows_full = rows_left >= kTM;
    if (rows_full)
        count(std::true_type{});
    else
        count(std::false_type{});
    int lrows = 32;  // this lane's live rows per column tile
    if (!rows_full) {
        lrows = 0;
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                lrows += (wave * 64 + rt * 32 + (r >> 2) * 8 + lh * 4 + (r & 3)) < rows_left;
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        if (!kPlain && jl[ct] && pos[ct] + neg[ct] < (uint32_t)lrows) {
            // some sign of this column is uncertain (rare): queue (query,
            // direction, point) for the binary64 recheck
            const int64_t J = J0 + ct * 32 + lr;
            const int64_t qi = J / m, j = J - qi * m;
            for (int rt = 0; rt < 2; ++rt)
                for (int r = 0; r < 16; ++r) {
                    const int il = wave * 64 + rt * 32 + (r >> 2) * 8 + lh * 4 + (r & 3);
                    if (il >= rows_left) continue;
                    const float v = acc[rt][ct][r];
                    const float marg = fmaf(kappa_a, L.an[il], cm[ct]);
                    if (v > marg || v < -marg) continue;
                    const int64_t i = (int64_t)blockIdx.y * kTM + il;
                    const uint32_t slot = atomicAdd(qcount, 1u);
                    if ((uint64_t)slot < qcap)
                        queue[slot] = ((uint64_t)qi << 48) | ((uint64_t)j << 32) | (uint64_t)i;
                }
        }
        uint32_t pc = jl[ct] ? pos[ct] : 0u, nc = jl[ct] ? neg[ct] : 0u;
        // lanes l and l + 32 hold the same column
        pc += (uint32_t)__shfl_xor((int)pc, 32);
        nc += (uint32_t)__shfl_xor((int)nc, 32);
        if (lh == 0) {
            L.red[wave][ct * 32 + lr][0] = nc;  // t < 0: counts for "<= 0"
            L.red[wave][ct * 32 + lr][1] = pc;  // t > 0: counts for ">= 0"
        }
    }
    __syncthreads();
    {
        const int jj = tid >> 1, w = tid & 1;  // 256 threads = 128 columns x 2 sides
        const int64_t J = J0 + jj;
        uint32_t s = 0;
#pragma unroll
        for (int wv = 0; wv < 4; ++wv) s += L.red[wv][jj][w];
        if (J < ncols && s) {
            const int64_t qi = J / m, j = J - qi * m;
            atomicAdd(&cnt[(qi * ldm + j) * 2 + w], s);
        }
    }
}

// Exact decisions of the queued pairs with the binary64 recipe (grid-stride;
// the queue length is read on the device).
__global__ __launch_bounds__(256) void k_recheck(const uint64_t *__restrict__ queue,
                                                 const uint32_t *__restrict__ qcount,
                                                 uint64_t qcap, const double *__restrict__ X,
                                                 int64_t d, const double *__restrict__ Zb,
                                                 const double *__restrict__ UT, int64_t ldm,
                                                 uint32_t *__restrict__ cnt,
                                                 unsigned long long *__restrict__ tally)
{
    const uint64_t total = *qcount < qcap ? *qcount : qcap;
    if (tally && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(tally, (unsigned long long)total);
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

// Error bounds of the matrix-core forms (kappa multiplies |a_i| + |c_j|).
//
// BF16: split |a - a_hi| <= 2^-8 |a| and the remainder |a - a_hi - a_lo| <=
// 2^-17 |a| (a_lo lies one binade below 2^-8 |a|), so the dropped a_lo b_lo
// and the two remainder products miss at most (2^-16 + 2 * 2^-17)(1 + 2^-8)
// |a||b| <= 4.5 * 2^-17 |a||b|; summed over the coordinates this is bounded
// by |a|_2 |u|_2 (Cauchy-Schwarz).  The bf16 products are exact in binary32
// and each of the 3 kp + 16 additions adds at most 2^-24 of the running sum
// of magnitudes (doubled for slack).
//
// F32: a, u and c are each rounded once to binary32 (relative 2^-24), each
// product is rounded at most once and each of the kp additions adds at most
// 2^-24 of the sum of magnitudes: (kp + 4) 2^-24, doubled for slack.
//
// canon bounds the binary64 recipe's own distance from the exact product.
void mfma_margins(int prec, int64_t d, int64_t kp, double *kappa, double *canon)
{
    if (prec == MFMA_BF16) {
        const double split = 3.0 * ldexp(1.0, -17) * 1.5;
        const double accum = 2.0 * (double)(3 * kp + 16) * ldexp(1.0, -24);
        *kappa = split + accum;
    } else if (prec == MFMA_F32) {
        *kappa = 2.0 * (double)(kp + 4) * ldexp(1.0, -24);
    } else {
        *kappa = 0.0;
    }
    *canon = prec == MFMA_F32_PLAIN ? 0.0 : 2.0 * (double)(d + 2) * ldexp(1.0, -53);
}

int64_t mfma_kpad(int prec, int64_t d)
{
    return prec == MFMA_BF16 ? (d + 2 + 15) / 16 * 16 : (d + 1 + 7) / 8 * 8;
}

size_t mfma_elem_bytes(int prec) { return prec == MFMA_BF16 ? 2 : 4; }
int mfma_terms(int prec) { return prec == MFMA_BF16 ? 2 : 1; }

hipError_t launch_mfma_prep(int prec, const double *X, int64_t n, int64_t d, double *xbar,
                            void *A0, void *A1, float *anorm, float *amax, hipStream_t st)
{
    hipError_t e = launch_fill_u32((uint32_t *)amax, 4, 0u, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_col_mean, dim3((unsigned)d), dim3(256), 0, st, X, n, d, xbar);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)((n + 255) / 256));
    const int64_t kp = mfma_kpad(prec, d);
    if (prec == MFMA_BF16)
        hipLaunchKernelGGL(k_prep_data<MFMA_BF16>, grid, dim3(256), 0, st, X, n, d, kp, xbar,
                           A0, A1, anorm, amax);
    else
        hipLaunchKernelGGL(k_prep_data<MFMA_F32>, grid, dim3(256), 0, st, X, n, d, kp, xbar, A0,
                           A1, anorm, amax);
    return hipGetLastError();
}

double mfma_point_alpha(int prec, int64_t d)
{
    double kappa, canon;
    mfma_margins(prec, d, mfma_kpad(prec, d), &kappa, &canon);
    return (kappa + canon) * 1.000001 * 1.000002;
}

hipError_t launch_mfma_dirs(int prec, bool fold, const double *UT, int64_t d, int64_t m,
                            int64_t ldm, int64_t ncols, int64_t npad, const double *Zb,
                            const double *xbar, void *B0, void *B1, float *cmarg,
                            const float *amax, double *cq, double *eq, hipStream_t st,
                            bool pp)
{
    double kappa, canon;
    const int64_t kp = mfma_kpad(prec, d);
    mfma_margins(prec, d, kp, &kappa, &canon);
    dim3 grid((unsigned)((npad + 63) / 64));
#define RRS_DIRS(P, F)                                                                         \
    hipLaunchKernelGGL((k_prep_dirs<P, F>), grid, dim3(256), 0, st, UT, d, m, ldm, ncols, npad, \
                       kp, Zb, xbar, kappa, canon, B0, B1, cmarg, amax, cq, eq, pp ? 1 : 0)
    if (prec == MFMA_BF16) {
        if (fold)
            RRS_DIRS(MFMA_BF16, true);
        else
            RRS_DIRS(MFMA_BF16, false);
    } else {
        if (fold)
            RRS_DIRS(MFMA_F32, true);
        else
            RRS_DIRS(MFMA_F32, false);
    }
#undef RRS_DIRS
    return hipGetLastError();
}

int64_t mfma_col_pad(int64_t ncols) { return (ncols + kTN - 1) / kTN * kTN; }

namespace {

constexpr int kVariants = 3;

// Launch of one GEMM variant (PF = variant) for either epilogue.
struct GemmLaunch {
    int prec, epi;
    dim3 grid;
    const void *A0, *A1;
    const float *anorm;
    int64_t n, kp;
    const void *B0, *B1;
    const float *cmarg;
    int64_t m, ncols, ldm;
    float kappa_a;
    uint32_t *cnt;
    uint64_t *queue;
    uint32_t *qcount;
    uint64_t qcap;
    float *S;

    template <int P, int E, int V>
    void go(hipStream_t st) const
    {
        hipLaunchKernelGGL((k_gemm<P, E, V>), grid, dim3(256), 0, st, A0, A1, anorm, n, kp, B0,
                           B1, cmarg, m, ncols, ldm, kappa_a, cnt, queue, qcount, qcap, S);
    }
    template <int V>
    void go_v(hipStream_t st) const
    {
        if (epi == EPI_STORE) {
            if (prec == MFMA_BF16)
                go<MFMA_BF16, EPI_STORE, V>(st);
            else
                go<MFMA_F32, EPI_STORE, V>(st);
        } else if (prec == MFMA_BF16) {
            go<MFMA_BF16, EPI_SIGN, V>(st);
        } else if (prec == MFMA_F32) {
            go<MFMA_F32, EPI_SIGN, V>(st);
        } else {
            go<MFMA_F32_PLAIN, EPI_SIGN, V>(st);
        }
    }
    hipError_t run(int v, hipStream_t st) const
    {
        if (v == 2)
            go_v<2>(st);
        else if (v == 1)
            go_v<1>(st);
        else
            go_v<0>(st);
        return hipGetLastError();
    }
};

// ---------------------------------------------------------------------------
// Autotuner.  The variant of a GEMM launch is chosen per key (epilogue,
// format, padded K, log2 buckets of n and of the column count) by timing
// every variant on the first launch with that key, on that launch's own
// operands (the sign epilogue's counters and queue are cleared after each
// trial, so the launch that follows starts from zero as usual).  Choices are
// kept for the process; with RRS_TUNE_CACHE=<file> they are also read from
// and appended to that file (lines: epi prec kp nbucket cbucket variant).
// RRS_TUNE=0 turns timing off (variant 0), RRS_TUNE=v+1 forces variant v.
// A stream under graph capture is never timed.
// ---------------------------------------------------------------------------
struct TuneKey {
    int epi, prec;
    int64_t kp;
    int nb, cb;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(epi, prec, kp, nb, cb) < std::tie(o.epi, o.prec, o.kp, o.nb, o.cb);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;
bool g_tune_loaded = false;

int log2_bucket(int64_t x)
{
    int b = 0;
    while (x > 1) {
        x >>= 1;
        ++b;
    }
    return b;
}

int tune_mode()
{
    const char *e = getenv("RRS_TUNE");
    if (!e || !*e) return -1;  // tune
    return atoi(e);            // 0: off, v + 1: force v
}

void tune_load_locked()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = getenv("RRS_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    TuneKey k;
    long long kp;
    int v;
    while (fscanf(f, "%d %d %lld %d %d %d", &k.epi, &k.prec, &kp, &k.nb, &k.cb, &v) == 6) {
        k.kp = kp;
        if (v >= 0 && v < kVariants) g_tune[k] = v;
    }
    fclose(f);
}

void tune_store_locked(const TuneKey &k, int v)
{
    g_tune[k] = v;
    const char *path = getenv("RRS_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%d %d %lld %d %d %d\n", k.epi, k.prec, (long long)k.kp, k.nb, k.cb, v);
    fclose(f);
}

thread_local bool t_tune_suspended = false;

hipError_t tuned_launch(const GemmLaunch &g, int64_t cnt_words, hipStream_t st)
{
    const int mode = tune_mode();
    if (mode >= 0) return g.run(mode == 0 ? 0 : (mode - 1) % kVariants, st);
    const TuneKey key{g.epi, g.prec, g.kp, log2_bucket(g.n), log2_bucket(g.ncols)};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) return g.run(it->second, st);
    }
    if (t_tune_suspended) return g.run(0, st);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
        return g.run(0, st);
    hipEvent_t ev[2];
    if (hipEventCreate(&ev[0]) != hipSuccess) return g.run(0, st);
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        return g.run(0, st);
    }
    float best_ms = 0.f;
    int best = 0;
    hipError_t e = hipSuccess;
    for (int v = 0; v < kVariants && e == hipSuccess; ++v) {
        float ms = 0.f;
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the first loads the code
            e = hipEventRecord(ev[0], st);
            if (e == hipSuccess) e = g.run(v, st);
            if (e == hipSuccess) e = hipEventRecord(ev[1], st);
            if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
        }
        if (e == hipSuccess && (v == 0 || ms < best_ms)) {
            best_ms = ms;
            best = v;
        }
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (e != hipSuccess) return e;
    if (g.epi == EPI_SIGN) {
        // trials accumulated into the counters and the queue: start over
        e = launch_fill_u32(g.cnt, cnt_words, 0u, st);
        if (e == hipSuccess) e = launch_fill_u32(g.qcount, 2, 0u, st);
        if (e != hipSuccess) return e;
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_store_locked(key, best);
    }
    return g.run(best, st);
}

}  // namespace

void mfma_tune_suspend(bool on) { t_tune_suspended = on; }

hipError_t launch_mfma_store(int prec, const void *A0, const void *A1, int64_t n, int64_t d,
                             const void *B0, const void *B1, int64_t m, int64_t ncols,
                             int64_t npad, float *S, hipStream_t st)
{
    GemmLaunch g{};
    g.prec = prec == MFMA_BF16 ? MFMA_BF16 : MFMA_F32;
    g.epi = EPI_STORE;
    g.kp = mfma_kpad(prec, d);
    g.grid = dim3((unsigned)((ncols + kTN - 1) / kTN), (unsigned)((n + kTM - 1) / kTM));
    if (npad < (int64_t)g.grid.x * kTN) return hipErrorInvalidValue;
    g.A0 = A0;
    g.A1 = A1;
    g.n = n;
    g.B0 = B0;
    g.B1 = B1;
    g.m = m;
    g.ncols = ncols;
    g.S = S;
    return tuned_launch(g, 0, st);
}

hipError_t launch_mfma_gemm(const MfmaArgs &a, hipStream_t st)
{
    double kappa, canon;
    GemmLaunch g{};
    g.prec = a.prec;
    g.epi = EPI_SIGN;
    g.kp = mfma_kpad(a.prec, a.d);
    mfma_margins(a.prec, a.d, g.kp, &kappa, &canon);
    g.kappa_a = (float)((kappa + canon) * 1.000001);
    g.ncols = a.qb * a.m;
    g.grid = dim3((unsigned)((g.ncols + kTN - 1) / kTN), (unsigned)((a.n + kTM - 1) / kTM));
    if (a.npad < (int64_t)g.grid.x * kTN) return hipErrorInvalidValue;
    g.A0 = a.A0;
    g.A1 = a.A1;
    g.anorm = a.anorm;
    g.n = a.n;
    g.B0 = a.B0;
    g.B1 = a.B1;
    g.cmarg = a.cmarg;
    g.m = a.m;
    g.ldm = a.ldm;
    g.cnt = a.cnt;
    g.queue = a.queue;
    g.qcount = a.qcount;
    g.qcap = a.qcap;
    return tuned_launch(g, a.qb * a.ldm * 2, st);
}

hipError_t launch_mfma_recheck(const MfmaArgs &a, hipStream_t st)
{
    if (a.prec == MFMA_F32_PLAIN) return hipSuccess;
    hipLaunchKernelGGL(k_recheck, dim3(1024), dim3(256), 0, st, a.queue, a.qcount, a.qcap, a.X,
                       a.d, a.Z, a.UT, a.ldm, a.cnt, (unsigned long long *)a.tally);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_queue_overflow(a.qcount, a.qcap, a.cnt, a.qb * a.ldm * 2, a.flag, st);
}

hipError_t launch_queue_overflow(const uint32_t *qcount, uint64_t qcap, uint32_t *cnt,
                                 int64_t cnt_words, uint32_t *flag, hipStream_t st)
{
    hipLaunchKernelGGL(k_overflow_reset, dim3((unsigned)((cnt_words + 255) / 256)), dim3(256), 0,
                       st, qcount, qcap, cnt, cnt_words, flag);
    return hipGetLastError();
}

}  // namespace rrs
