// rrs_kernels.hip -- HIP kernels of the RRS depth hot path on gfx950.
//
// One refinement of RRS for a batch of queries (Alg. 4 / Alg. S5) is:
//   k_gen_dirs      step a1: directions (Alg. S1 sphere / Alg. S4 cap)
//   k_proj_f64      step a2: centred projections t = (x - z).u, binary64
//                   fma chain in coordinate order; for halfspace depth the
//                   sign counts are fused into the epilogue (no projection
//                   matrix is stored), otherwise columns go to scratch
//   (step a3, the median / MAD / MAD_+ selects, is in rrs_select.hip for
//                   binary64 columns and rrs_select_rc.hip for the matrix-core
//                   forms)
//   k_argmin_pole   step a5: first index of the minimum, strict pole update
//
// Layouts (all device memory):
//   XT  [d][ldx]        data transposed, ldx = n rounded up to 512 (pad = 0)
//   Z   [Qb][d]         queries of the batch
//   UT  [Qb][d][ldm]    directions, direction index fastest, ldm = m
//                       rounded up to 16 (pad = 0)
//   cnt [Qb][ldm][2]    halfspace counts #{t <= 0}, #{t >= 0} (uint32)
//   T   [Qb][m][n]      projection columns (projection / APD only)
//   Dj  [Qb][ldm]       univariate depth per direction
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rrs_device.hpp"
#include "rrs_launch.hpp"

namespace rrs {

// ---------------------------------------------------------------------------
// a1: directions.  Four lanes per (query, direction): in iteration i lane t
// of the quad draws Philox block 4 i + t of the direction and writes its
// coordinates into UT (coalesced over directions); the quad exchanges the
// values with shuffles so that every lane adds the squared norm, and later
// the reflection's dot product, in coordinate order exactly as a single
// sequential pass does; normalisation and reflection then touch each lane's
// own coordinates.  Lanes past m compute a dummy direction and write nothing.
// ---------------------------------------------------------------------------
__device__ __forceinline__ Block4 shfl_block(const Block4 &b, int src)
{
    return Block4{(uint64_t)__shfl((long long)b.w0, src), (uint64_t)__shfl((long long)b.w1, src),
                  (uint64_t)__shfl((long long)b.w2, src), (uint64_t)__shfl((long long)b.w3, src)};
}

__global__ __launch_bounds__(64) void k_gen_dirs(int64_t d, int64_t m, int64_t ldm, int32_t l,
                                                 double phi, uint64_t seed, uint64_t qbase,
                                                 const double *__restrict__ pole,
                                                 double *__restrict__ UT, int32_t first_cap,
                                                 int32_t area_cap, double *__restrict__ UR)
{
    const int lane = threadIdx.x, t = lane & 3, q4 = lane & ~3;
    const int64_t j = (int64_t)blockIdx.x * 16 + (lane >> 2);
    const int64_t qi = blockIdx.y;
    const bool live = j < m;  // uniform within a quad
    const int64_t jj = live ? j : 0;
    const uint64_t q = qbase + (uint64_t)qi;
    const uint64_t ul = (uint64_t)l;
    double *u = UT + qi * d * ldm + jj;
    double *ur = (UR && live) ? UR + (qi * m + jj) * d : nullptr;

    if (l == 1 && !first_cap) {
        // Alg. S1: block b gives the Gaussians of coordinates 4 b .. 4 b + 3
        // from word pairs (0,1), (2,3); then divide by the Euclidean norm.
        // (first_cap: refinement 1 also draws from Alg. S4, in the half-angle
        // pi/2 cap around the initial pole e1.)
        const int64_t nb = (d + 3) / 4;
        double s = 0.0;
        for (int64_t i = 0; 4 * i < nb; ++i) {
            const int64_t b = 4 * i + t;
            double g[4] = {0.0, 0.0, 0.0, 0.0};
            if (b < nb) {
                const Block4 w = dir_block(seed, q, ul, (uint64_t)jj, (uint64_t)b);
                gauss_pair(w.w0, w.w1, g[0], g[1]);
                if (4 * b + 2 < d) gauss_pair(w.w2, w.w3, g[2], g[3]);
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (live && 4 * b + e < d) u[(4 * b + e) * ldm] = g[e];
            }
#pragma unroll
            for (int tt = 0; tt < 4; ++tt)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const double v = __shfl(g[e], q4 + tt);
                    if (4 * (4 * i + tt) + e < d) s = fma(v, v, s);
                }
        }
        const double nrm = sqrt(s);
        for (int64_t b = t; b < nb; b += 4)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t c = 4 * b + e;
                if (live && c < d) {
                    const double v = u[c * ldm] / nrm;
                    u[c * ldm] = v;
                    if (ur) ur[c] = v;
                }
            }
        return;
    }

    // Alg. S4: polar angle (pi/2) * U * phi from word 0 of block 0, tangent
    // Gaussians h_1..h_{d-1} from word pairs (1,2), (3,4), ...: block b gives
    // coordinates 4 b + 1, 4 b + 2 from its words 1, 2 and 4 b + 3, 4 b + 4
    // from its word 3 and word 0 of block b + 1.  Lane t draws block
    // 4 i + t + 1 in iteration i: its own next block, lane t + 1's block, and
    // (lane 3) lane 0's block of the next iteration.
    const Block4 b0 = dir_block(seed, q, ul, (uint64_t)jj, 0);
    double st, ct;
    if (area_cap)
        area_cap_angle(uniform_open(b0.w0), phi, d, st, ct);  // area-uniform in the cap
    else
        sincos_halfpi(uniform_open(b0.w0) * phi, st, ct);
    const int64_t nbk = (d - 1 + 3) / 4;  // blocks holding tangent coordinates
    double s = 0.0;
    Block4 carry = b0;
    for (int64_t i = 0; 4 * i < nbk; ++i) {
        const int64_t b = 4 * i + t;
        const Block4 nxt = dir_block(seed, q, ul, (uint64_t)jj, (uint64_t)(b + 1));
        const Block4 fromprev = shfl_block(nxt, q4 + ((t + 3) & 3));
        const Block4 cur = t == 0 ? carry : fromprev;
        carry = shfl_block(nxt, q4 + 3);
        double h[4] = {0.0, 0.0, 0.0, 0.0};
        if (b < nbk) {
            const int64_t c = 1 + 4 * b;
            gauss_pair(cur.w1, cur.w2, h[0], h[1]);
            if (c + 2 <= d - 1) gauss_pair(cur.w3, nxt.w0, h[2], h[3]);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (live && c + e <= d - 1) u[(c + e) * ldm] = h[e];
        }
#pragma unroll
        for (int tt = 0; tt < 4; ++tt)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double v = __shfl(h[e], q4 + tt);
                if (1 + 4 * (4 * i + tt) + e <= d - 1) s = fma(v, v, s);
            }
    }
    const double nrm = sqrt(s);
    for (int64_t b = t; b < nbk; b += 4)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t c = 1 + 4 * b + e;
            if (live && c <= d - 1) u[c * ldm] = st * (u[c * ldm] / nrm);
        }
    const double v0 = ct;

    // Householder reflection taking e1 to the pole p: w = e1 - p,
    // u = v - (2 w.v / w.w) w.
    const double *p = pole + qi * d;
    const double am = 1.0 - p[0];
    double ww = am * am;
    for (int64_t c = 1; c < d; ++c) ww = fma(p[c], p[c], ww);
    if (ww == 0.0) {
        if (live && t == 0) u[0] = v0;
        if (ur) {
            if (t == 0) ur[0] = v0;
            for (int64_t b = t; b < nbk; b += 4)
                for (int e = 0; e < 4; ++e) {
                    const int64_t c = 1 + 4 * b + e;
                    if (c <= d - 1) ur[c] = u[c * ldm];
                }
        }
        return;
    }
    double wv = am * v0;
    for (int64_t i = 0; 4 * i < nbk; ++i) {
        const int64_t b = 4 * i + t;
        double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t c = 1 + 4 * b + e;
            if (live && b < nbk && c <= d - 1) v[e] = u[c * ldm];
        }
#pragma unroll
        for (int tt = 0; tt < 4; ++tt)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double x = __shfl(v[e], q4 + tt);
                const int64_t c = 1 + 4 * (4 * i + tt) + e;
                if (c <= d - 1) wv = fma(-p[c], x, wv);
            }
    }
    const double beta = (2.0 * wv) / ww;
    if (live && t == 0) {
        const double u0 = fma(-beta, am, v0);
        u[0] = u0;
        if (ur) ur[0] = u0;
    }
    for (int64_t b = t; b < nbk; b += 4)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t c = 1 + 4 * b + e;
            if (live && c <= d - 1) {
                const double x = fma(beta, p[c], u[c * ldm]);
                u[c * ldm] = x;
                if (ur) ur[c] = x;
            }
        }
}

// ---------------------------------------------------------------------------
// Data transpose X[n][d] -> XT[d][ldx] with zero padding.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_transpose(const double *__restrict__ X, int64_t n,
                                                   int64_t d, int64_t ldx,
                                                   double *__restrict__ XT)
{
    __shared__ double tile[32][33];
    const int64_t i0 = (int64_t)blockIdx.x * 32;
    const int64_t c0 = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = i0 + r, c = c0 + tx;
        tile[r][tx] = (i < n && c < d) ? X[i * d + c] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t c = c0 + r, i = i0 + tx;
        if (c < d && i < ldx) XT[c * ldx + i] = tile[tx][r];
    }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *__restrict__ p, int64_t count,
                                                  uint32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) p[i] = v;
}

// ---------------------------------------------------------------------------
// a2 (+ a3 for halfspace): binary64 projection tile.  A workgroup of 4 waves
// owns JT directions of one query; each lane owns 2 points per 512-point
// slab.  The direction values and the query coordinate are wave-uniform, so
// they are read through the scalar cache; each lane keeps 2 x JT
// accumulators, every one the recipe's fma chain over c = 0..d-1.
// ---------------------------------------------------------------------------
template <int JT, bool COUNT>
__global__ __launch_bounds__(256) void k_proj_f64(
    const double *__restrict__ XT, int64_t ldx, int64_t n, int64_t d,
    const double *__restrict__ Zb, const double *__restrict__ UT, int64_t ldm, int64_t m,
    uint32_t *__restrict__ cnt, double *__restrict__ T, int64_t pts_per_block,
    const uint32_t *__restrict__ only_if)
{
    if (only_if && *only_if == 0u) return;  // conditional launch (whole grid exits)
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t qi = blockIdx.y;
    const int64_t j0 = (int64_t)blockIdx.x * JT;
    const double *zq = Zb + qi * d;
    const double *ut = UT + qi * d * ldm + j0;
    const int64_t pbeg = (int64_t)blockIdx.z * pts_per_block;
    const int64_t pend = min(n, pbeg + pts_per_block);

    uint32_t le[JT], ge[JT];
#pragma unroll
    for (int jj = 0; jj < JT; ++jj) le[jj] = ge[jj] = 0;

    for (int64_t base = pbeg + wave * 128; base < pend; base += 512) {
        const int64_t i0 = base + lane, i1 = base + 64 + lane;
        double acc0[JT], acc1[JT];
#pragma unroll
        for (int jj = 0; jj < JT; ++jj) acc0[jj] = acc1[jj] = 0.0;
        const double *x0 = XT + i0;
        const double *x1 = XT + i1;
        for (int64_t c = 0; c < d; ++c) {
            const double zc = zq[c];
            const double a0 = x0[c * ldx] - zc;
            const double a1 = x1[c * ldx] - zc;
            const double *ur = ut + c * ldm;
#pragma unroll
            for (int jj = 0; jj < JT; ++jj) {
                const double uu = ur[jj];
                acc0[jj] = fma(a0, uu, acc0[jj]);
                acc1[jj] = fma(a1, uu, acc1[jj]);
            }
        }
        const bool v0 = i0 < pend, v1 = i1 < pend;
        if (COUNT) {
#pragma unroll
            for (int jj = 0; jj < JT; ++jj) {
                le[jj] += (uint32_t)__popcll(__ballot(v0 && acc0[jj] <= 0.0)) +
                          (uint32_t)__popcll(__ballot(v1 && acc1[jj] <= 0.0));
                ge[jj] += (uint32_t)__popcll(__ballot(v0 && acc0[jj] >= 0.0)) +
                          (uint32_t)__popcll(__ballot(v1 && acc1[jj] >= 0.0));
            }
        } else {
#pragma unroll
            for (int jj = 0; jj < JT; ++jj) {
                if (j0 + jj < m) {
                    double *col = T + (qi * m + j0 + jj) * n;
                    if (v0) col[i0] = acc0[jj];
                    if (v1) col[i1] = acc1[jj];
                }
            }
        }
    }
    if (COUNT) {
        __shared__ uint32_t red[4][JT][2];
        if (lane == 0) {
#pragma unroll
            for (int jj = 0; jj < JT; ++jj) {
                red[wave][jj][0] = le[jj];
                red[wave][jj][1] = ge[jj];
            }
        }
        __syncthreads();
        if (threadIdx.x < 2 * JT) {
            const int jj = threadIdx.x >> 1, w = threadIdx.x & 1;
            const uint32_t sum = red[0][jj][w] + red[1][jj][w] + red[2][jj][w] + red[3][jj][w];
            if (j0 + jj < m && sum) atomicAdd(&cnt[(qi * ldm + j0 + jj) * 2 + w], sum);
        }
    }
}

// ---------------------------------------------------------------------------
// a5: per query, the first direction index attaining the minimum; strict
// improvement moves the pole and the running minimum.
// ---------------------------------------------------------------------------
template <bool HALF>
__global__ __launch_bounds__(256) void k_argmin_pole(
    int64_t m, int64_t ldm, int64_t d, const uint32_t *__restrict__ cnt,
    const double *__restrict__ Dj, const double *__restrict__ UT, double *__restrict__ pole,
    double *__restrict__ best_d, int64_t *__restrict__ best_c, int64_t *__restrict__ trace,
    int32_t l, int32_t r)
{
    const int64_t qi = blockIdx.x;
    const int tid = threadIdx.x;
    __shared__ double sv[256];
    __shared__ int64_t sc[256];
    __shared__ int64_t sj[256];
    __shared__ int improved_s;
    __shared__ int64_t jbest_s;
    double bv = 0.0;
    int64_t bc = 0;
    int64_t bj = -1;
    for (int64_t j = tid; j < m; j += 256) {
        if (HALF) {
            const uint32_t a = cnt[(qi * ldm + j) * 2], b = cnt[(qi * ldm + j) * 2 + 1];
            const int64_t c = (int64_t)(a < b ? a : b);
            if (bj < 0 || c < bc) {
                bc = c;
                bj = j;
            }
        } else {
            const double v = Dj[qi * ldm + j];
            if (bj < 0 || v < bv) {
                bv = v;
                bj = j;
            }
        }
    }
    sv[tid] = bv;
    sc[tid] = bc;
    sj[tid] = bj;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) {
            const int64_t oj = sj[tid + off];
            if (oj >= 0) {
                bool take;
                if (sj[tid] < 0)
                    take = true;
                else if (HALF)
                    take = sc[tid + off] < sc[tid] || (sc[tid + off] == sc[tid] && oj < sj[tid]);
                else
                    take = sv[tid + off] < sv[tid] || (sv[tid + off] == sv[tid] && oj < sj[tid]);
                if (take) {
                    sv[tid] = sv[tid + off];
                    sc[tid] = sc[tid + off];
                    sj[tid] = oj;
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        const int64_t js = sj[0];
        int imp;
        int64_t tv;
        if (HALF) {
            imp = sc[0] < best_c[qi];
            if (imp) best_c[qi] = sc[0];
            tv = sc[0];
        } else {
            imp = sv[0] < best_d[qi];
            if (imp) best_d[qi] = sv[0];
            tv = __double_as_longlong(sv[0]);
        }
        improved_s = imp;
        jbest_s = js;
        if (trace) {
            int64_t *tr = trace + (qi * r + (l - 1)) * 3;
            tr[0] = js;
            tr[1] = imp;
            tr[2] = tv;
        }
    }
    __syncthreads();
    if (improved_s) {
        const int64_t js = jbest_s;
        for (int64_t c = tid; c < d; c += 256) pole[qi * d + c] = UT[(qi * d + c) * ldm + js];
    }
}

__global__ __launch_bounds__(256) void k_init_state(int64_t qb, int64_t d, int64_t n,
                                                    double *__restrict__ pole,
                                                    double *__restrict__ best_d,
                                                    int64_t *__restrict__ best_c)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < qb * d) pole[i] = ((i % d) == 0) ? 1.0 : 0.0;
    if (i < qb) {
        best_d[i] = 1.0;
        best_c[i] = n;
    }
}

__global__ __launch_bounds__(256) void k_finalize(int64_t qb, int64_t d, int64_t n, int half,
                                                  const double *__restrict__ pole,
                                                  const double *__restrict__ best_d,
                                                  const int64_t *__restrict__ best_c,
                                                  double *__restrict__ depth,
                                                  int64_t *__restrict__ count,
                                                  double *__restrict__ poles_out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < qb) {
        if (half) {
            depth[i] = (double)best_c[i] / (double)n;
            if (count) count[i] = best_c[i];
        } else {
            depth[i] = best_d[i];
        }
    }
    if (poles_out && i < qb * d) poles_out[i] = pole[i];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline unsigned ceil_div(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

hipError_t launch_gen_dirs(const GenArgs &a, hipStream_t st)
{
    dim3 grid(ceil_div(a.m, 16), (unsigned)a.qb);
    hipLaunchKernelGGL(k_gen_dirs, grid, dim3(64), 0, st, a.d, a.m, a.ldm, a.l, a.phi, a.seed,
                       a.qbase, a.pole, a.UT, a.first_cap, a.area_cap, a.UR);
    return hipGetLastError();
}

hipError_t launch_transpose(const double *X, int64_t n, int64_t d, int64_t ldx, double *XT,
                            hipStream_t st)
{
    dim3 grid(ceil_div(ldx, 32), ceil_div(d, 32));
    hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, st, X, n, d, ldx, XT);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t count, uint32_t v, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(ceil_div(count, 256)), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}

hipError_t launch_proj_f64(const ProjArgs &a, bool count_mode, hipStream_t st)
{
    constexpr int JT = kProjJT;
    const unsigned gx = ceil_div(a.m, JT);
    const int64_t slabs = (a.n + 511) / 512;
    int64_t chunks;
    if (count_mode) {
        // enough workgroups to fill the chip; each covers whole 512-point slabs
        const int64_t want = 4096;
        const int64_t have = (int64_t)gx * a.qb;
        chunks = (want + have - 1) / have;
        if (chunks > slabs) chunks = slabs;
        if (chunks < 1) chunks = 1;
    } else {
        chunks = slabs;
    }
    const int64_t per = ((slabs + chunks - 1) / chunks) * 512;
    chunks = (a.n + per - 1) / per;
    dim3 grid(gx, (unsigned)a.qb, (unsigned)chunks);
    if (count_mode)
        hipLaunchKernelGGL((k_proj_f64<JT, true>), grid, dim3(256), 0, st, a.XT, a.ldx, a.n, a.d,
                           a.Z, a.UT, a.ldm, a.m, a.cnt, a.T, per, a.only_if);
    else
        hipLaunchKernelGGL((k_proj_f64<JT, false>), grid, dim3(256), 0, st, a.XT, a.ldx, a.n,
                           a.d, a.Z, a.UT, a.ldm, a.m, a.cnt, a.T, per, a.only_if);
    return hipGetLastError();
}

hipError_t launch_argmin(const ArgminArgs &a, bool half, hipStream_t st)
{
    if (half)
        hipLaunchKernelGGL(k_argmin_pole<true>, dim3((unsigned)a.qb), dim3(256), 0, st, a.m,
                           a.ldm, a.d, a.cnt, a.Dj, a.UT, a.pole, a.best_d, a.best_c, a.trace,
                           a.l, a.r);
    else
        hipLaunchKernelGGL(k_argmin_pole<false>, dim3((unsigned)a.qb), dim3(256), 0, st, a.m,
                           a.ldm, a.d, a.cnt, a.Dj, a.UT, a.pole, a.best_d, a.best_c, a.trace,
                           a.l, a.r);
    return hipGetLastError();
}

hipError_t launch_init_state(int64_t qb, int64_t d, int64_t n, double *pole, double *best_d,
                             int64_t *best_c, hipStream_t st)
{
    hipLaunchKernelGGL(k_init_state, dim3(ceil_div(qb * d, 256)), dim3(256), 0, st, qb, d, n,
                       pole, best_d, best_c);
    return hipGetLastError();
}

hipError_t launch_finalize(int64_t qb, int64_t d, int64_t n, bool half, const double *pole,
                           const double *best_d, const int64_t *best_c, double *depth,
                           int64_t *count, double *poles_out, hipStream_t st)
{
    hipLaunchKernelGGL(k_finalize, dim3(ceil_div(qb * d, 256)), dim3(256), 0, st, qb, d, n,
                       half ? 1 : 0, pole, best_d, best_c, depth, count, poles_out);
    return hipGetLastError();
}

}  // namespace rrs
