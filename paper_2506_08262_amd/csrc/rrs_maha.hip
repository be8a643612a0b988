// rrs_maha.hip -- Mahalanobis depth D_M(L), the closed-form comparator of the
// paper's center-outward ranking study (Sec. "Center-outward ordering
// precision and depth benchmark"):
//
//     D_M(z | X) = (1 + (z - mu)' Sigma^-1 (z - mu))^-1,
//
// with mu the sample mean and Sigma the maximum-likelihood covariance (divisor
// n) of X.  Every step runs on the device in binary64:
//   1. mu: column means (fixed-order tree reduction per coordinate);
//   2. A = X - mu [n][d];
//   3. Sigma = A' A / n on the FP64 matrix cores (v_mfma_f64_16x16x4_f64),
//      split over the points into fixed chunks whose partial sums are added
//      in chunk order (deterministic);
//   4. Sigma = L L' (Cholesky, one workgroup) and W = L^-1 (forward
//      substitution, one column per thread, stored transposed);
//   5. Y = W B with B = (Z - mu)' [d][m] on the matrix cores, and
//      D_q = 1 / (1 + sum_j Y[j][q]^2).
// A covariance that is not positive definite (n <= d, collinear data) is
// reported through a device flag and the call fails with RRS_E_INVAL.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rrs_launch.hpp"

namespace rrs {

namespace {

typedef __attribute__((ext_vector_type(4))) double f64x4;

// Column means of X [n][d] (one workgroup per coordinate).
__global__ __launch_bounds__(256) void k_maha_mean(const double *__restrict__ X, int64_t n,
                                                   int64_t d, double *__restrict__ mu)
{
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
    if (threadIdx.x == 0) mu[c] = red[0] / (double)n;
}

// V [rows][d] minus mu: row-major (T[i][c], trans = 0) or coordinate-major
// (T[c][i], trans = 1).
__global__ __launch_bounds__(256) void k_maha_center(const double *__restrict__ V, int64_t rows,
                                                     int64_t d, const double *__restrict__ mu,
                                                     int trans, double *__restrict__ T)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= rows * d) return;
    const int64_t i = e / d, c = e - i * d;
    T[trans ? c * rows + i : e] = V[e] - mu[c];
}

// Partial products C_s[M][N] = sum over k in chunk s of P[k][m] Q[k][n]
// (P: [K][ldp], Q: [K][ldq], both K-major).  One wave per 16 x 16 tile and
// chunk; v_mfma_f64_16x16x4_f64 takes A[i][k] from lane 16 k + i and B[k][j]
// from lane 16 k + j, and returns D[4 v + lane / 16][lane % 16] in element v
// of each lane (binary64 accumulators hold one row per register, unlike the
// four consecutive rows of the binary32 layouts).
__global__ __launch_bounds__(64) void k_maha_gemm(const double *__restrict__ P, int64_t ldp,
                                                  const double *__restrict__ Q, int64_t ldq,
                                                  int64_t M, int64_t N, int64_t K,
                                                  int64_t chunk, double *__restrict__ part)
{
    const int lane = threadIdx.x;
    const int64_t m0 = (int64_t)blockIdx.x * 16, n0 = (int64_t)blockIdx.y * 16;
    const int64_t k0 = (int64_t)blockIdx.z * chunk;
    const int64_t k1 = k0 + chunk < K ? k0 + chunk : K;
    const int64_t mi = m0 + (lane & 15), nj = n0 + (lane & 15);
    const int kk = lane >> 4;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int64_t k = k0; k < k1; k += 4) {
        const int64_t kr = k + kk;
        const double a = (kr < k1 && mi < M) ? P[kr * ldp + mi] : 0.0;
        const double b = (kr < k1 && nj < N) ? Q[kr * ldq + nj] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    double *out = part + (int64_t)blockIdx.z * M * N;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t i = m0 + 4 * v + (lane >> 4), j = n0 + (lane & 15);
        if (i < M && j < N) out[i * N + j] = acc[v];
    }
}

// C[M][N] = scale * sum over the chunks (in chunk order) of the partials.
__global__ __launch_bounds__(256) void k_maha_reduce(const double *__restrict__ part,
                                                     int64_t MN, int64_t chunks, double scale,
                                                     double *__restrict__ C)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= MN) return;
    double s = 0.0;
    for (int64_t c = 0; c < chunks; ++c) s += part[c * MN + e];
    C[e] = s * scale;
}

// Cholesky factor L (lower, in place of S [d][d]) and WT = (L^-1)' (upper,
// [d][d], WT[c][i] = (L^-1)[i][c]).  One workgroup; flag = 1 when a pivot is
// not positive.
__global__ __launch_bounds__(256) void k_maha_chol(double *__restrict__ S, int64_t d,
                                                   double *__restrict__ WT,
                                                   uint32_t *__restrict__ flag)
{
    __shared__ double piv;
    __shared__ int bad;
    const int tid = threadIdx.x;
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int64_t j = 0; j < d; ++j) {
        if (tid == 0) {
            double s = S[j * d + j];
            for (int64_t k = 0; k < j; ++k) s = fma(-S[j * d + k], S[j * d + k], s);
            if (!(s > 0.0)) bad = 1;
            piv = s > 0.0 ? sqrt(s) : 1.0;
            S[j * d + j] = piv;
        }
        __syncthreads();
        for (int64_t i = j + 1 + tid; i < d; i += 256) {
            double s = S[i * d + j];
            for (int64_t k = 0; k < j; ++k) s = fma(-S[i * d + k], S[j * d + k], s);
            S[i * d + j] = s / piv;
        }
        __syncthreads();
    }
    // L^-1: column c solves L w = e_c by forward substitution (row c of WT)
    for (int64_t c = tid; c < d; c += 256) {
        double *w = WT + c * d;
        for (int64_t i = 0; i < c; ++i) w[i] = 0.0;
        for (int64_t i = c; i < d; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int64_t k = c; k < i; ++k) s = fma(-S[i * d + k], w[k], s);
            w[i] = s / S[i * d + i];
        }
    }
    if (tid == 0 && flag) *flag = bad ? 1u : 0u;
}

// D_q = 1 / (1 + sum_j Y[j][q]^2), Y [d][m].
__global__ __launch_bounds__(256) void k_maha_depth(const double *__restrict__ Y, int64_t d,
                                                    int64_t m, double *__restrict__ depth)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= m) return;
    double s = 0.0;
    for (int64_t j = 0; j < d; ++j) s = fma(Y[j * m + q], Y[j * m + q], s);
    depth[q] = 1.0 / (1.0 + s);
}

int64_t ceil_div64(int64_t a, int64_t b) { return (a + b - 1) / b; }

constexpr int64_t kChunk = 4096;  // points per partial sum of the covariance

}  // namespace

size_t maha_ws_bytes(int64_t n, int64_t d, int64_t m)
{
    const int64_t chunks = ceil_div64(n, kChunk);
    size_t b = 0;
    auto add = [&](size_t x) { b += (x + 255) / 256 * 256; };
    add((size_t)d * 8);               // mu
    add((size_t)n * d * 8);           // A = X - mu
    add((size_t)d * m * 8);           // B = (Z - mu)'
    add((size_t)d * d * 8);           // Sigma, then L
    add((size_t)d * d * 8);           // WT
    add((size_t)d * m * 8);           // Y
    add((size_t)chunks * d * d * 8);  // partial sums of Sigma
    add(64);                          // flag
    return b + 256;
}

hipError_t maha_enqueue(const double *X, int64_t n, int64_t d, const double *Z, int64_t m,
                        double *depth, void *ws, uint32_t **flag_out, hipStream_t st)
{
    char *p = (char *)ws;
    size_t off = 0;
    auto take = [&](size_t x) {
        off = (off + 255) / 256 * 256;
        void *r = p + off;
        off += x;
        return r;
    };
    const int64_t chunks = ceil_div64(n, kChunk);
    double *mu = (double *)take((size_t)d * 8);
    double *A = (double *)take((size_t)n * d * 8);
    double *B = (double *)take((size_t)d * m * 8);
    double *S = (double *)take((size_t)d * d * 8);
    double *WT = (double *)take((size_t)d * d * 8);
    double *Y = (double *)take((size_t)d * m * 8);
    double *part = (double *)take((size_t)chunks * d * d * 8);
    uint32_t *flag = (uint32_t *)take(64);
    *flag_out = flag;
    const unsigned td = (unsigned)ceil_div64(d, 16);
    hipLaunchKernelGGL(k_maha_mean, dim3((unsigned)d), dim3(256), 0, st, X, n, d, mu);
    hipLaunchKernelGGL(k_maha_center, dim3((unsigned)ceil_div64(n * d, 256)), dim3(256), 0, st,
                       X, n, d, mu, 0, A);
    hipLaunchKernelGGL(k_maha_center, dim3((unsigned)ceil_div64(m * d, 256)), dim3(256), 0, st,
                       Z, m, d, mu, 1, B);
    // Sigma[i][j] = sum_r A[r][i] A[r][j] / n (K = n points, chunked)
    hipLaunchKernelGGL(k_maha_gemm, dim3(td, td, (unsigned)chunks), dim3(64), 0, st, A, d, A, d,
                       d, d, n, kChunk, part);
    hipLaunchKernelGGL(k_maha_reduce, dim3((unsigned)ceil_div64(d * d, 256)), dim3(256), 0, st,
                       part, d * d, chunks, 1.0 / (double)n, S);
    hipLaunchKernelGGL(k_maha_chol, dim3(1), dim3(256), 0, st, S, d, WT, flag);
    // Y[j][q] = sum_c W[j][c] B[c][q] = sum_c WT[c][j] B[c][q] (K = d, one chunk)
    hipLaunchKernelGGL(k_maha_gemm, dim3(td, (unsigned)ceil_div64(m, 16), 1), dim3(64), 0, st,
                       WT, d, B, m, d, m, d, d, Y);
    hipLaunchKernelGGL(k_maha_depth, dim3((unsigned)ceil_div64(m, 256)), dim3(256), 0, st, Y, d,
                       m, depth);
    return hipGetLastError();
}

}  // namespace rrs
