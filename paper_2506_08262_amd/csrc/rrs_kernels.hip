// rrs_kernels.hip -- HIP kernels of the RRS depth hot path on gfx950.
//
// One refinement of RRS for a batch of queries (Alg. 4 / Alg. S5) is:
//   k_gen_dirs      step a1: directions (Alg. S1 sphere / Alg. S4 cap)
//   k_proj_f64      step a2: centred projections t = (x - z).u, binary64
//                   fma chain in coordinate order; for halfspace depth the
//                   sign counts are fused into the epilogue (no projection
//                   matrix is stored), otherwise columns go to scratch
//   k_select        step a3: median / MAD / MAD_+ per column by LDS radix
//                   select on order-preserving 64-bit keys (exact)
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
// a1: directions.  One lane per (query, direction); the lane writes its
// direction straight into UT (coalesced over directions) and re-reads it for
// the normalisation and the reflection.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_gen_dirs(int64_t d, int64_t m, int64_t ldm, int32_t l,
                                                 double phi, uint64_t seed, uint64_t qbase,
                                                 const double *__restrict__ pole,
                                                 double *__restrict__ UT, int32_t first_cap,
                                                 int32_t area_cap)
{
    const int64_t j = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int64_t qi = blockIdx.y;
    if (j >= m) return;
    const uint64_t q = qbase + (uint64_t)qi;
    const uint64_t ul = (uint64_t)l;
    double *u = UT + qi * d * ldm + j;

    if (l == 1 && !first_cap) {
        // Alg. S1: d Gaussians from word pairs (0,1), (2,3), ... then divide
        // by the Euclidean norm.  (first_cap: refinement 1 also draws from
        // Alg. S4, in the half-angle pi/2 cap around the initial pole e1.)
        double s = 0.0;
        for (int64_t c = 0, b = 0; c < d; c += 4, ++b) {
            const Block4 w = dir_block(seed, q, ul, (uint64_t)j, (uint64_t)b);
            double g0, g1;
            gauss_pair(w.w0, w.w1, g0, g1);
            u[c * ldm] = g0;
            s = fma(g0, g0, s);
            if (c + 1 < d) {
                u[(c + 1) * ldm] = g1;
                s = fma(g1, g1, s);
            }
            if (c + 2 < d) {
                double g2, g3;
                gauss_pair(w.w2, w.w3, g2, g3);
                u[(c + 2) * ldm] = g2;
                s = fma(g2, g2, s);
                if (c + 3 < d) {
                    u[(c + 3) * ldm] = g3;
                    s = fma(g3, g3, s);
                }
            }
        }
        const double nrm = sqrt(s);
        for (int64_t c = 0; c < d; ++c) u[c * ldm] = u[c * ldm] / nrm;
        return;
    }

    // Alg. S4: polar angle (pi/2) * U * phi from word 0, tangent Gaussians
    // h_1..h_{d-1} from word pairs (1,2), (3,4), ...; pair 2k uses words
    // 4k+1, 4k+2 of block k and pair 2k+1 uses word 4k+3 of block k and word
    // 4k+4 (= word 0 of block k+1).
    Block4 a = dir_block(seed, q, ul, (uint64_t)j, 0);
    double st, ct;
    if (area_cap)
        area_cap_angle(uniform_open(a.w0), phi, d, st, ct);  // area-uniform in the cap
    else
        sincos_halfpi(uniform_open(a.w0) * phi, st, ct);
    double s = 0.0;
    for (int64_t c = 1, b = 0;; c += 4, ++b) {
        if (c > d - 1) break;
        double h0, h1;
        gauss_pair(a.w1, a.w2, h0, h1);
        u[c * ldm] = h0;
        s = fma(h0, h0, s);
        if (c + 1 <= d - 1) {
            u[(c + 1) * ldm] = h1;
            s = fma(h1, h1, s);
        }
        if (c + 2 > d - 1) break;
        const Block4 nb = dir_block(seed, q, ul, (uint64_t)j, (uint64_t)(b + 1));
        double h2, h3;
        gauss_pair(a.w3, nb.w0, h2, h3);
        u[(c + 2) * ldm] = h2;
        s = fma(h2, h2, s);
        if (c + 3 <= d - 1) {
            u[(c + 3) * ldm] = h3;
            s = fma(h3, h3, s);
        }
        a = nb;
    }
    const double nrm = sqrt(s);
    for (int64_t c = 1; c < d; ++c) u[c * ldm] = st * (u[c * ldm] / nrm);
    const double v0 = ct;

    // Householder reflection taking e1 to the pole p: w = e1 - p,
    // u = v - (2 w.v / w.w) w.
    const double *p = pole + qi * d;
    const double am = 1.0 - p[0];
    double ww = am * am;
    for (int64_t c = 1; c < d; ++c) ww = fma(p[c], p[c], ww);
    if (ww == 0.0) {
        u[0] = v0;
        return;
    }
    double wv = am * v0;
    for (int64_t c = 1; c < d; ++c) wv = fma(-p[c], u[c * ldm], wv);
    const double beta = (2.0 * wv) / ww;
    u[0] = fma(-beta, am, v0);
    for (int64_t c = 1; c < d; ++c) u[c * ldm] = fma(beta, p[c], u[c * ldm]);
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
// a3 for projection / APD: exact order statistics of one column by radix
// select over order-preserving 64-bit keys, 8 bits per pass, stopping as soon
// as the selected bucket holds at most kCand elements (they are then ranked
// directly).  The column sits in LDS when it fits, otherwise it is read from
// the scratch buffer on every pass.
// ---------------------------------------------------------------------------
constexpr int kSelThreads = 512;
constexpr int kCand = 64;

struct SelShared {
    uint32_t hist[256];
    uint64_t cand[kCand];
    uint32_t ncand;
    uint32_t sel_bucket, sel_before, sel_count;
    uint64_t result;
    uint64_t minkey;
    uint32_t count;
};

enum { KEY_T = 0, KEY_ABSDEV = 1, KEY_POSDEV = 2 };

template <bool LDS>
__device__ __forceinline__ double col_load(const double *g, const double *s, int64_t i)
{
    return LDS ? s[i] : g[i];
}

template <int MODE>
__device__ __forceinline__ bool make_key(double t, double med, uint64_t &key)
{
    if (MODE == KEY_T) {
        key = order_key(t);
        return true;
    } else if (MODE == KEY_ABSDEV) {
        key = order_key(fabs(t - med));
        return true;
    } else {
        const double dv = t - med;
        key = order_key(dv);
        return dv > 0.0;
    }
}

__device__ __forceinline__ void block_sync() { __syncthreads(); }

// Key of the k-th smallest (0-based) included element.
template <int MODE, bool LDS>
__device__ uint64_t select_kth(const double *g, const double *s, int64_t n, double med,
                               uint64_t k, SelShared &sh)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    uint64_t prefix = 0, pmask = 0;
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int b = tid; b < 256; b += kSelThreads) sh.hist[b] = 0;
        block_sync();
        for (int64_t i0 = 0; i0 < n; i0 += kSelThreads) {
            const int64_t i = i0 + tid;
            uint64_t key = 0;
            bool act = false;
            if (i < n) {
                act = make_key<MODE>(col_load<LDS>(g, s, i), med, key);
                act = act && ((key & pmask) == prefix);
            }
            const uint32_t bucket = (uint32_t)(key >> shift) & 255u;
            if (shift == 56) {
                // first pass: few distinct buckets, aggregate per wave
                uint64_t am = __ballot(act);
                while (am) {
                    const int leader = __ffsll((long long)am) - 1;
                    const uint32_t lb = (uint32_t)__shfl((int)bucket, leader);
                    const uint64_t same = __ballot(act && bucket == lb);
                    if (lane == leader) atomicAdd(&sh.hist[lb], (uint32_t)__popcll(same));
                    if (bucket == lb) act = false;
                    am &= ~same;
                }
            } else if (act) {
                atomicAdd(&sh.hist[bucket], 1u);
            }
        }
        block_sync();
        if (tid < 64) {
            const uint32_t h0 = sh.hist[4 * lane], h1 = sh.hist[4 * lane + 1];
            const uint32_t h2 = sh.hist[4 * lane + 2], h3 = sh.hist[4 * lane + 3];
            const uint32_t tot = h0 + h1 + h2 + h3;
            uint32_t incl = tot;
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t v = (uint32_t)__shfl_up((int)incl, off);
                if (lane >= off) incl += v;
            }
            const uint64_t excl = incl - tot;
            if (excl <= k && k < (uint64_t)incl) {
                uint64_t c = excl;
                uint32_t sel = 0, cntb = 0;
                const uint32_t hs[4] = {h0, h1, h2, h3};
                for (int b = 0; b < 4; ++b) {
                    if (k < c + hs[b]) {
                        sel = 4 * lane + b;
                        cntb = hs[b];
                        break;
                    }
                    c += hs[b];
                }
                sh.sel_bucket = sel;
                sh.sel_before = (uint32_t)c;
                sh.sel_count = cntb;
            }
        }
        block_sync();
        const uint32_t selb = sh.sel_bucket;
        const uint32_t cntb = sh.sel_count;
        k -= sh.sel_before;
        prefix |= (uint64_t)selb << shift;
        pmask |= 0xFFull << shift;
        if (shift == 0) break;
        if (cntb <= (uint32_t)kCand) {
            if (tid == 0) sh.ncand = 0;
            block_sync();
            for (int64_t i0 = 0; i0 < n; i0 += kSelThreads) {
                const int64_t i = i0 + tid;
                if (i < n) {
                    uint64_t key;
                    bool act = make_key<MODE>(col_load<LDS>(g, s, i), med, key);
                    if (act && (key & pmask) == prefix) {
                        const uint32_t pos = atomicAdd(&sh.ncand, 1u);
                        if (pos < (uint32_t)kCand) sh.cand[pos] = key;
                    }
                }
            }
            block_sync();
            if (tid < 64) {
                const uint32_t nc = sh.ncand < (uint32_t)kCand ? sh.ncand : (uint32_t)kCand;
                if ((uint32_t)lane < nc) {
                    const uint64_t mine = sh.cand[lane];
                    uint32_t lt = 0, le = 0;
                    for (uint32_t x = 0; x < nc; ++x) {
                        const uint64_t o = sh.cand[x];
                        lt += (o < mine);
                        le += (o <= mine);
                    }
                    if (lt <= k && k < le) sh.result = mine;
                }
            }
            block_sync();
            const uint64_t r = sh.result;
            block_sync();
            return r;
        }
    }
    block_sync();
    return prefix;
}

// Given the key A of the k-th smallest included element, the key of the
// (k+1)-th: A again if more than k+1 included keys are <= A, else the
// smallest included key above A.
template <int MODE, bool LDS>
__device__ uint64_t select_next(const double *g, const double *s, int64_t n, double med,
                                uint64_t k, uint64_t A, SelShared &sh)
{
    const int tid = threadIdx.x;
    if (tid == 0) {
        sh.count = 0;
        sh.minkey = ~0ull;
    }
    block_sync();
    uint32_t le = 0;
    uint64_t mn = ~0ull;
    for (int64_t i = tid; i < n; i += kSelThreads) {
        uint64_t key;
        if (make_key<MODE>(col_load<LDS>(g, s, i), med, key)) {
            le += (key <= A);
            if (key > A && key < mn) mn = key;
        }
    }
    if (le) atomicAdd(&sh.count, le);
    if (mn != ~0ull) atomicMin((unsigned long long *)&sh.minkey, (unsigned long long)mn);
    block_sync();
    const uint64_t res = ((uint64_t)sh.count >= k + 2) ? A : sh.minkey;
    block_sync();
    return res;
}

template <int MODE, bool LDS>
__device__ double median_of(const double *g, const double *s, int64_t cnt, int64_t n,
                            double med, SelShared &sh)
{
    if (cnt & 1) {
        return key_value(select_kth<MODE, LDS>(g, s, n, med, (uint64_t)(cnt / 2), sh));
    }
    const uint64_t k = (uint64_t)(cnt / 2 - 1);
    const uint64_t A = select_kth<MODE, LDS>(g, s, n, med, k, sh);
    const uint64_t B = select_next<MODE, LDS>(g, s, n, med, k, A, sh);
    return (key_value(A) + key_value(B)) * 0.5;
}

template <int NOTION, bool LDS>
__global__ __launch_bounds__(kSelThreads) void k_select(const double *__restrict__ T, int64_t n,
                                                        int64_t m, int64_t ldm,
                                                        double *__restrict__ Dj)
{
    extern __shared__ double scol[];
    __shared__ SelShared sh;
    const int64_t j = blockIdx.x;
    const int64_t qi = blockIdx.y;
    const double *g = T + (qi * m + j) * n;
    if (LDS) {
        for (int64_t i = threadIdx.x; i < n; i += kSelThreads) scol[i] = g[i];
        block_sync();
    }
    const double med = median_of<KEY_T, LDS>(g, scol, n, n, 0.0, sh);
    double D;
    if (NOTION == NOTION_PROJECTION) {
        const double mad = median_of<KEY_ABSDEV, LDS>(g, scol, n, n, med, sh);
        if (mad == 0.0)
            D = (med == 0.0) ? 1.0 : 0.0;
        else
            D = 1.0 / (1.0 + fabs(med) / mad);
    } else {
        // APD: count the strictly positive deviations, then their median
        if (threadIdx.x == 0) sh.count = 0;
        block_sync();
        uint32_t np = 0;
        for (int64_t i = threadIdx.x; i < n; i += kSelThreads)
            np += (col_load<LDS>(g, scol, i) - med > 0.0);
        if (np) atomicAdd(&sh.count, np);
        block_sync();
        const int64_t npos = sh.count;
        block_sync();
        const double num = (med < 0.0) ? -med : 0.0;
        if (npos == 0) {
            D = (num == 0.0) ? 1.0 : 0.0;
        } else {
            const double madp = median_of<KEY_POSDEV, LDS>(g, scol, npos, n, med, sh);
            D = 1.0 / (1.0 + num / madp);
        }
    }
    if (threadIdx.x == 0) Dj[qi * ldm + j] = D;
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
    dim3 grid(ceil_div(a.m, 64), (unsigned)a.qb);
    hipLaunchKernelGGL(k_gen_dirs, grid, dim3(64), 0, st, a.d, a.m, a.ldm, a.l, a.phi, a.seed,
                       a.qbase, a.pole, a.UT, a.first_cap, a.area_cap);
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

int64_t select_lds_max_n(int device)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return 0;
    const int64_t avail = (int64_t)prop.sharedMemPerBlock - (int64_t)sizeof(SelShared) - 1024;
    return avail > 0 ? avail / 8 : 0;
}

template <int NOTION>
static hipError_t launch_select_t(const SelectArgs &a, bool lds, hipStream_t st)
{
    dim3 grid((unsigned)a.m, (unsigned)a.qb);
    if (lds) {
        const size_t bytes = (size_t)a.n * sizeof(double);
        hipError_t e = hipFuncSetAttribute((const void *)k_select<NOTION, true>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_select<NOTION, true>), grid, dim3(kSelThreads), bytes, st, a.T, a.n,
                           a.m, a.ldm, a.Dj);
    } else {
        hipLaunchKernelGGL((k_select<NOTION, false>), grid, dim3(kSelThreads), 0, st, a.T, a.n,
                           a.m, a.ldm, a.Dj);
    }
    return hipGetLastError();
}

hipError_t launch_select(const SelectArgs &a, int notion, bool lds, hipStream_t st)
{
    if (notion == NOTION_PROJECTION) return launch_select_t<NOTION_PROJECTION>(a, lds, st);
    return launch_select_t<NOTION_APD>(a, lds, st);
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
