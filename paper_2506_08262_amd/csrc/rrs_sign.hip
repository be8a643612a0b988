// rrs_sign.hip -- halfspace counts of the bfloat16 form (steps a2 + a3 + a4)
// on the CDNA4 matrix cores: a persistent sign-count GEMM and cap culling.
//
// Sign GEMM.  As in rrs_mfma.hip, every element is t^_ij = A_i . B_j with the
// data centred by its mean (a_i = x_i - xbar, split into bfloat16 hi + lo) and
// the direction operands carrying the query's centring term in two extra K
// columns, three bf16 products per K step (A_hi B_hi + A_hi B_lo + A_lo B_hi)
// accumulated in binary32; a sign is taken from t^ only outside a rigorous
// margin, and the rows inside it are queued, as a row mask per half column of
// a wave tile, for the binary64 recheck.  Here the
// kernel is persistent: a fixed grid (two workgroups per CU) walks a list of
// items, each item one tile of 128 directions kept in LDS for up to `rpi`
// tiles of 256 points, with the per-column counts held in registers across
// the point tiles and added to the global counts once per item.  Items are
// handed out in contiguous ranges per XCD (workgroup b runs on XCD b mod 8),
// so the workgroups of one XCD share their points and directions in its L2.
//
// Cap culling (refinements l >= 2).  Every direction of refinement l lies in
// the cap around the query's pole p: u_j = p + delta_j with
// |delta_j| <= Delta_q = max_j |u_j - p|.  For a point with
// |(x_i - z).p| > |x_i - z| Delta_q (plus the error bounds), every
// (x_i - z).u_j has the sign of (x_i - z).p, so the point adds one to the
// same side of every direction's count without entering the GEMM.  A small
// GEMM of the points against the poles decides this per (query, point),
// counts the decided points per query and appends the others to the query's
// list; the sign GEMM then runs over (query, list tile, direction tile) items
// only.  The counts, and therefore every result, are identical to the full
// GEMM's (and to the binary64 recipe's).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rrs_launch.hpp"

namespace rrs {

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr int kTM = 256;  // points per point tile (4 waves x 64)
constexpr int kTN = 128;  // directions per item

// LDS of one workgroup: the item's direction operands (hi, lo) with rows
// padded by 16 bytes (row pitch 2 KS + 1 pieces of 16 bytes: the 8 lanes of
// one ds_read_b128 phase hit distinct bank groups), count reduction, and, for
// the cull epilogue, the norms of each wave tile's rows and the list positions.
template <int KS>
struct alignas(16) SignLds {
    bf16x8 b[2][kTN][2 * KS + 1];
    uint32_t red[4][kTN][2];
    float an[4][64];
    // cull epilogue: undecided points per (wave, lane half, column) and the
    // list positions they are written at
    uint32_t ucnt[4][2][kTN];
};

struct SignParams {
    const __bf16 *A0, *A1;     // [n][kp] centred data, bf16 hi / lo
    const float *anorm;        // [n] norm bounds of the centred points
    int32_t n, kp;
    const __bf16 *B0, *B1;     // [npad][kp] column operands (flat columns), hi / lo
    const float *cmarg;        // [npad] column part of the margin
    int32_t npad, ncols;       // operand rows; live flat columns
    int32_t m, ldm, qb;        // directions per query, count stride, queries
    float kappa_a;             // data part of the margin (times |a_i|)
    int32_t rpi;               // point tiles per item (list mode)
    int32_t rpi_dense;         // point tiles per item (dense mode)
    const uint32_t *mode;      // list mode only when *mode != 0 (null: lists decide)
    // sign epilogue: counts, and per wave of the grid a queue segment of
    // `seg` entries (two words each) with its fill in segcnt; a segment that
    // overflows sets bit 31 of *qflag
    uint32_t *cnt;             // [qb][ldm][2]
    uint64_t *queue;
    uint32_t *segcnt;
    uint32_t *qflag;
    uint32_t seg;
    // list mode (sign GEMM after culling); lists == nullptr: all points
    const uint32_t *lists;     // [qb][n] undecided points per query
    const uint32_t *lcount;    // [qb]
    const uint32_t *offs;      // [qb + 1] first item of each query; offs[qb] = total
    const uint32_t *items;     // [total][4] q | tile << 16, first and end list position
    // cull epilogue (columns are the queries' poles)
    const float *lam, *mu;     // [qb] threshold = |a_i| lam_q + mu_q
    uint32_t *lists_out;       // [qb][n]
    uint32_t *lcount_out;      // [qb]
    uint32_t *base;            // [qb][2]: decided points with t < 0, with t > 0
};

// Buffer resources (base, size in bytes): loads take 32-bit offsets, and a
// load past the size returns zero.
typedef __amdgpu_buffer_rsrc_t Rsrc;
__device__ __forceinline__ Rsrc rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                             0x00020000);
}
__device__ __forceinline__ bf16x8 ld_b128(Rsrc r, uint32_t off)
{
    return __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
__device__ __forceinline__ uint32_t ld_u32(Rsrc r, uint32_t off)
{
    return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}
typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;
__device__ __forceinline__ u32x4 ld_u32x4(Rsrc r, uint32_t off)
{
    return __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
__device__ __forceinline__ float ld_f32(Rsrc r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// Item range of this workgroup: contiguous per XCD (workgroups b and b + 8
// share an XCD), strided by the workgroups of the XCD inside it.
struct Sched {
    int32_t lo, hi, step;
};
__device__ __forceinline__ Sched schedule(int32_t total)
{
    const int G = gridDim.x, b = blockIdx.x;
    Sched s;
    if ((G & 7) == 0) {
        const int x = b & 7, k = b >> 3, G8 = G >> 3;
        const int32_t per = (total + 7) >> 3;
        s.lo = x * per + k;
        s.hi = (x + 1) * per < total ? (x + 1) * per : total;
        s.step = G8;
    } else {
        s.lo = b;
        s.hi = total;
        s.step = G;
    }
    return s;
}

// Query of list-mode item `it` (offs ascending, offs[qb] = total).
__device__ __forceinline__ int32_t item_query(const uint32_t *__restrict__ offs, int32_t qb,
                                              int32_t it)
{
    int32_t lo = 0, hi = qb - 1;  // largest q with offs[q] <= it
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if ((int32_t)offs[mid] <= it)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Stages operand rows J0 .. J0 + 127 (both terms) in LDS; rows past npad
// read as zero.
template <int KS>
__device__ __forceinline__ void stage_b(Rsrc B0, Rsrc B1, uint32_t J0, SignLds<KS> &L)
{
    constexpr int kPieces = 2 * KS;  // 16-byte pieces per row and term
    const int tid = threadIdx.x;
    const uint32_t base = J0 * (uint32_t)(KS * 32);
#pragma unroll
    for (int u = 0; u < KS; ++u) {  // kTN * kPieces / 256 = KS pieces per thread and term
        const int p = tid + 256 * u;
        const int row = p / kPieces, part = p - row * kPieces;
        const uint32_t off = base + (uint32_t)p * 16u;
        L.b[0][row][part] = ld_b128(B0, off);
        L.b[1][row][part] = ld_b128(B1, off);
    }
}

// The 64 x 128 block of one wave: its 64 rows of the point tile (idx: this
// lane's two point indices, rows lr and 32 + lr), all KS K steps, three
// products each.
template <int KS>
__device__ __forceinline__ void wave_mma(Rsrc A0, Rsrc A1, const uint32_t (&idx)[2],
                                         const SignLds<KS> &L, f32x16 (&acc)[2][4])
{
    const int lane = threadIdx.x & 63, lr = lane & 31, lh = lane >> 5;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[rt][ct][r] = 0.0f;
    // A fragments one K step ahead: step ks + 1 is in flight during step ks
    bf16x8 ah[2][2], al[2][2];
    uint32_t aoff[2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) aoff[rt] = idx[rt] * (uint32_t)(KS * 32) + (uint32_t)lh * 16u;
    auto load = [&](int ks, int stg) {
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            ah[stg][rt] = ld_b128(A0, aoff[rt] + ks * 32);
            al[stg][rt] = ld_b128(A1, aoff[rt] + ks * 32);
        }
    };
    // B fragments one (K step, column tile) ahead: the LDS reads of step
    // s + 1 are in flight during the MFMAs of step s
    bf16x8 bh[2], bl[2];
    auto ldb = [&](int ks, int ct, int buf) {
        const int col = ct * 32 + lr;
        bh[buf] = L.b[0][col][2 * ks + lh];
        bl[buf] = L.b[1][col][2 * ks + lh];
    };
    load(0, 0);
    ldb(0, 0, 0);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int stg = ks & 1;
        if (ks + 1 < KS) load(ks + 1, stg ^ 1);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int cur = (ks * 4 + ct) & 1;
            const bool more = ct < 3 || ks + 1 < KS;
            if (ct < 3)
                ldb(ks, ct + 1, cur ^ 1);
            else if (ks + 1 < KS)
                ldb(ks + 1, 0, cur ^ 1);
            // issue order: the next step's B reads (and, at ct = 0, the next
            // K step's A loads), then this step's six MFMAs
            if (ct == 0 && ks + 1 < KS) __builtin_amdgcn_sched_group_barrier(0x020, 4, 0);
            if (more) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, 6, 0);
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[stg][rt], bh[cur],
                                                                      acc[rt][ct], 0, 0, 0);
                acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[stg][rt], bl[cur],
                                                                      acc[rt][ct], 0, 0, 0);
                acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[stg][rt], bh[cur],
                                                                      acc[rt][ct], 0, 0, 0);
            }
            // keep the scheduler from hoisting every column tile's operands
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// Wave-local row of accumulator element r of row tile rt for lane half lh.
__device__ __forceinline__ int acc_row(int rt, int r, int lh)
{
    return rt * 32 + (r >> 2) * 8 + lh * 4 + (r & 3);
}

// Bits of `b` set below this lane.
__device__ __forceinline__ uint32_t lane_rank(uint64_t b)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    return v;
}

// Signs of column tile ct of a wave tile against the margin M of this lane's
// column, as bit masks over the lane half's 32 rows (bit 16 rt + r): rows
// with t^ above the margin (above) and rows with |t^| above it (sure).  The
// tests take sign bits of differences (M - v < 0 exactly when v > M: a
// difference of two binary32 values is zero only when they are equal), so
// they stay in vector registers; a NaN, were there one, would not read as
// sure.
__device__ __forceinline__ void column_masks(const f32x16 (&acc)[2][4], int ct, float M,
                                             uint32_t &above, uint32_t &sure)
{
    above = 0u;
    sure = 0u;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int k = rt * 16 + r;
            const float v = acc[rt][ct][r];
            above |= (__float_as_uint(M - v) >> 31) << k;
            sure |= (__float_as_uint(M - fabsf(v)) >> 31) << k;
            if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // bounded live ranges
        }
}

// Cheap statistics of column tile ct against the margin M: whether all of
// the lane half's 32 rows have |t^| above M (bit 31 of the AND of the bit
// patterns of M - |t^|), and how many have the sign bit of t^ set.
__device__ __forceinline__ void column_stats(const f32x16 (&acc)[2][4], int ct, float M,
                                             bool &certain, uint32_t &nneg)
{
    uint32_t all = 0xFFFFFFFFu, c0 = 0u, c1 = 0u;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int r = 0; r < 16; r += 4) {
            const float v0 = acc[rt][ct][r], v1 = acc[rt][ct][r + 1];
            const float v2 = acc[rt][ct][r + 2], v3 = acc[rt][ct][r + 3];
            all &= __float_as_uint(M - fabsf(v0)) & __float_as_uint(M - fabsf(v1));
            all &= __float_as_uint(M - fabsf(v2)) & __float_as_uint(M - fabsf(v3));
            c0 += (__float_as_uint(v0) >> 31) + (__float_as_uint(v1) >> 31);
            c1 += (__float_as_uint(v2) >> 31) + (__float_as_uint(v3) >> 31);
        }
    certain = (all >> 31) != 0u;
    nneg = c0 + c1;
}

// Rows of the wave tile that lane half lh holds (bit 16 rt + r) below wl.
__device__ __forceinline__ uint32_t live_rows(int wl, int lh)
{
    if (wl >= 64) return 0xFFFFFFFFu;
    uint32_t m = 0u;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int r = 0; r < 16; ++r)
            if (acc_row(rt, r, lh) < wl) m |= 1u << (rt * 16 + r);
    return m;
}

// ---------------------------------------------------------------------------
// Sign GEMM: counts of certain signs per (query, direction); uncertain pairs
// go to the recheck queue.
// ---------------------------------------------------------------------------
template <int KS>
__global__ __launch_bounds__(256, 2) void k_sign(SignParams P)
{
    __shared__ SignLds<KS> L;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 31, lh = lane >> 5;
    const bool list = P.lists != nullptr && (P.mode == nullptr || *P.mode != 0u);
    const uint32_t rowb = (uint32_t)(KS * 32);  // bytes per operand row
    const Rsrc A0 = rsrc(P.A0, (uint32_t)P.n * rowb), A1 = rsrc(P.A1, (uint32_t)P.n * rowb);
    const Rsrc B0 = rsrc(P.B0, (uint32_t)P.npad * rowb), B1 = rsrc(P.B1, (uint32_t)P.npad * rowb);
    const Rsrc AN = rsrc(P.anorm, (uint32_t)P.n * 4u), CM = rsrc(P.cmarg, (uint32_t)P.npad * 4u);
    const int32_t rows_per_item = kTM * (list ? P.rpi : P.rpi_dense);
    // items: list mode (query, point chunk, direction tile of the query);
    // otherwise (point chunk, direction tile over the flat columns)
    const int32_t nct_all = (P.ncols + kTN - 1) / kTN;
    const int32_t total = list ? (int32_t)P.offs[P.qb]
                               : ((P.n + rows_per_item - 1) / rows_per_item) * nct_all;
    const Sched sc = schedule(total);
    const uint32_t gw = blockIdx.x * 4u + (uint32_t)wave;  // this wave's queue segment
    uint64_t *const myq = P.queue + 2ull * (uint64_t)gw * (uint64_t)P.seg;
    uint32_t nq = 0;
    // list mode: the item records, each loaded one item ahead
    const Rsrc IT = rsrc(P.items, list ? (uint32_t)total * 16u : 0u);
    u32x4 rec = ld_u32x4(IT, (uint32_t)sc.lo * 16u);
    for (int32_t it = sc.lo; it < sc.hi; it += sc.step) {
        int32_t J0, jend, rbeg, rend;
        Rsrc LS = rsrc(nullptr, 0u);
        const u32x4 cur = rec;
        if (list && it + sc.step < sc.hi) rec = ld_u32x4(IT, (uint32_t)(it + sc.step) * 16u);
        if (list) {
            const int32_t q = (int32_t)(cur[0] & 0xFFFFu), ct = (int32_t)(cur[0] >> 16);
            J0 = q * P.m + ct * kTN;
            const int32_t je = (ct + 1) * kTN < P.m ? (ct + 1) * kTN : P.m;
            jend = q * P.m + je;
            rbeg = (int32_t)cur[1];
            rend = (int32_t)cur[2];
            LS = rsrc(P.lists + (size_t)q * (size_t)P.n, (uint32_t)rend * 4u);
        } else {
            const int32_t rc = it / nct_all, ct = it - rc * nct_all;
            J0 = ct * kTN;
            jend = J0 + kTN < P.ncols ? J0 + kTN : P.ncols;
            rbeg = rc * rows_per_item;
            rend = rbeg + rows_per_item < P.n ? rbeg + rows_per_item : P.n;
        }
        __syncthreads();  // the previous item's reads of L are done
        stage_b<KS>(B0, B1, (uint32_t)J0, L);
        // column part of the margin; -inf for columns past jend, which then
        // never look uncertain (their counts are dropped at the end)
        float cm[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int32_t J = J0 + ct * 32 + lr;
            cm[ct] = J < jend ? ld_f32(CM, (uint32_t)J * 4u) : -INFINITY;
        }
        __syncthreads();
        uint32_t pos[4] = {0u, 0u, 0u, 0u}, neg[4] = {0u, 0u, 0u, 0u};
        // point indices of this wave's rows of a tile (list mode: read from
        // the query's list), fetched one tile ahead so that the A loads do
        // not wait on the list; the norms follow once the indices are in
        auto rows_of = [&](int32_t t0, uint32_t (&ix)[2]) {
            const int32_t r0 = t0 + wave * 64;
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                const int32_t pr = r0 + rt * 32 + lr;
                const uint32_t prc = (uint32_t)(pr < rend ? pr : rbeg);
                ix[rt] = list ? ld_u32(LS, prc * 4u) : prc;
            }
        };
        uint32_t idx[2];
        rows_of(rbeg, idx);
        for (int32_t t0 = rbeg; t0 < rend; t0 += kTM) {
            const int32_t r0 = t0 + wave * 64;
            const int wl = rend - r0 >= 64 ? 64 : (rend - r0 > 0 ? rend - r0 : 0);
            uint32_t nidx[2] = {0u, 0u};
            if (t0 + kTM < rend) rows_of(t0 + kTM, nidx);
            if (wl == 0) {  // wave-uniform: this wave has no rows in the tile
                idx[0] = nidx[0];
                idx[1] = nidx[1];
                continue;
            }
            float an = 0.0f;
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                const float a = ld_f32(AN, idx[rt] * 4u);
                if (rt * 32 + lr < wl) an = fmaxf(an, a);
            }
            f32x16 acc[2][4];
            wave_mma<KS>(A0, A1, idx, L, acc);
            idx[0] = nidx[0];
            idx[1] = nidx[1];
            // margin: largest norm of the tile's points, column part per lane
            const float amax = wave_max(an);
            float M[4];
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) M[ct] = fmaf(P.kappa_a, amax, cm[ct]);
            // per column tile: when no row of the wave's 64 is within the
            // margin (and all are live), the counts follow from the sign
            // bits; otherwise the masks of certain and uncertain rows
            uint32_t um[4];
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                bool certain;
                uint32_t nneg;
                column_stats(acc, ct, M[ct], certain, nneg);
                if (wl == 64 && __builtin_amdgcn_ballot_w64(!certain) == 0ull) {
                    pos[ct] += 32u - nneg;
                    neg[ct] += nneg;
                    um[ct] = 0u;
                } else {
                    uint32_t above, sure;
                    column_masks(acc, ct, M[ct], above, sure);
                    const uint32_t live = live_rows(wl, lh);
                    sure &= live;
                    above &= live;
                    pos[ct] += (uint32_t)__builtin_popcount(above);
                    neg[ct] += (uint32_t)__builtin_popcount(sure & ~above);
                    um[ct] = live & ~sure;  // uncertain rows
                }
            }
            // half columns with uncertain rows (rare): one entry each,
            // appended to this wave's queue segment
            uint32_t off = nq;
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                const uint64_t bal = __builtin_amdgcn_ballot_w64(um[ct] != 0u);
                const uint32_t slot = off + lane_rank(bal);
                if (um[ct] != 0u && slot < P.seg) {
                    const int32_t J = J0 + ct * 32 + lr;
                    const int32_t qi = J / P.m, j = J - qi * P.m;
                    uint64_t *e = myq + 2 * (uint64_t)slot;
                    e[0] = ((uint64_t)qi << 48) | ((uint64_t)j << 32) |
                           (uint64_t)((uint32_t)r0 | (uint32_t)lh);
                    e[1] = (uint64_t)um[ct];
                }
                off += (uint32_t)__builtin_popcountll(bal);
            }
            nq = off;
        }
        // counts of the item: lanes l and l + 32 hold the same column
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const bool jl = J0 + ct * 32 + lr < jend;
            uint32_t pc = jl ? pos[ct] : 0u, nc = jl ? neg[ct] : 0u;
            pc += (uint32_t)__shfl_xor((int)pc, 32);
            nc += (uint32_t)__shfl_xor((int)nc, 32);
            if (lh == 0) {
                L.red[wave][ct * 32 + lr][0] = nc;  // t < 0: counts for "<= 0"
                L.red[wave][ct * 32 + lr][1] = pc;  // t > 0: counts for ">= 0"
            }
        }
        __syncthreads();
        {
            const int jj = tid >> 1, w = tid & 1;
            const int32_t J = J0 + jj;
            const uint32_t s = L.red[0][jj][w] + L.red[1][jj][w] + L.red[2][jj][w] +
                               L.red[3][jj][w];
            if (J < jend && s) {
                const int32_t qi = J / P.m, j = J - qi * P.m;
                atomicAdd(&P.cnt[((size_t)qi * P.ldm + j) * 2 + w], s);
            }
        }
    }
    if (lane == 0) {
        P.segcnt[gw] = nq < P.seg ? nq : P.seg;
        if (nq > P.seg) atomicOr(P.qflag, kSignQueueOverflow);  // overflow: recount in binary64
    }
}

// ---------------------------------------------------------------------------
// Cull GEMM: points x poles.  Decided points are counted per query (base),
// undecided ones appended to the query's list.
// ---------------------------------------------------------------------------
template <int KS>
__global__ __launch_bounds__(256, 2) void k_cull(SignParams P)
{
    __shared__ SignLds<KS> L;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 31, lh = lane >> 5;
    const uint32_t rowb = (uint32_t)(KS * 32);
    const Rsrc A0 = rsrc(P.A0, (uint32_t)P.n * rowb), A1 = rsrc(P.A1, (uint32_t)P.n * rowb);
    const Rsrc B0 = rsrc(P.B0, (uint32_t)P.npad * rowb), B1 = rsrc(P.B1, (uint32_t)P.npad * rowb);
    const Rsrc AN = rsrc(P.anorm, (uint32_t)P.n * 4u);
    const int32_t nct_all = (P.ncols + kTN - 1) / kTN;
    const int32_t total = ((P.n + kTM - 1) / kTM) * nct_all;
    const Sched sc = schedule(total);
    for (int32_t it = sc.lo; it < sc.hi; it += sc.step) {
        const int32_t rc = it / nct_all, ct0 = it - rc * nct_all;
        const int32_t J0 = ct0 * kTN;
        const int32_t jend = J0 + kTN < P.ncols ? J0 + kTN : P.ncols;
        const int32_t r0 = rc * kTM + wave * 64;
        const int wl = P.n - r0 >= 64 ? 64 : (P.n - r0 > 0 ? P.n - r0 : 0);
        __syncthreads();
        stage_b<KS>(B0, B1, (uint32_t)J0, L);
        uint32_t idx[2];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            const int wr = rt * 32 + lr;
            idx[rt] = (uint32_t)(wr < wl ? r0 + wr : 0);
            if (lh == 0) L.an[wave][wr] = wr < wl ? ld_f32(AN, idx[rt] * 4u) : 0.0f;
        }
        float lam[4], mu[4];
        bool jl[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int32_t J = J0 + ct * 32 + lr;
            jl[ct] = J < jend;
            lam[ct] = jl[ct] ? P.lam[J] : 0.0f;
            mu[ct] = jl[ct] ? P.mu[J] : 0.0f;
        }
        __syncthreads();
        // per column: undecided rows as a bit mask (bit 16 rt + r), decided counts
        uint32_t um[4] = {0u, 0u, 0u, 0u}, dp[4] = {0u, 0u, 0u, 0u}, dn[4] = {0u, 0u, 0u, 0u};
        if (wl > 0) {
            f32x16 acc[2][4];
            wave_mma<KS>(A0, A1, idx, L, acc);
#pragma unroll
            for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int wr = acc_row(rt, r, lh);
                    const bool rl = wr < wl;
                    const float a = L.an[wave][wr];
#pragma unroll
                    for (int ct = 0; ct < 4; ++ct) {
                        const float v = acc[rt][ct][r];
                        const float thr = fmaf(a, lam[ct], mu[ct]);
                        const bool p = v > thr, ng = v < -thr;
                        dp[ct] += (rl && p) ? 1u : 0u;
                        dn[ct] += (rl && ng) ? 1u : 0u;
                        um[ct] |= (rl && !p && !ng) ? (1u << (rt * 16 + r)) : 0u;
                    }
                }
        }
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int col = ct * 32 + lr;
            L.ucnt[wave][lh][col] = jl[ct] ? (uint32_t)__builtin_popcount(um[ct]) : 0u;
            uint32_t pc = jl[ct] ? dp[ct] : 0u, nc = jl[ct] ? dn[ct] : 0u;
            pc += (uint32_t)__shfl_xor((int)pc, 32);
            nc += (uint32_t)__shfl_xor((int)nc, 32);
            if (lh == 0) {
                L.red[wave][col][0] = nc;
                L.red[wave][col][1] = pc;
            }
        }
        __syncthreads();
        if (tid < kTN) {
            // list positions: contributors in (wave, lane half) order
            const int col = tid;
            const int32_t J = J0 + col;
            uint32_t tot = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w)
#pragma unroll
                for (int h = 0; h < 2; ++h) tot += L.ucnt[w][h][col];
            if (J < jend) {
                uint32_t basepos = tot ? atomicAdd(&P.lcount_out[J], tot) : 0u;
#pragma unroll
                for (int w = 0; w < 4; ++w)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const uint32_t c = L.ucnt[w][h][col];
                        L.ucnt[w][h][col] = basepos;
                        basepos += c;
                    }
                const uint32_t nneg = L.red[0][col][0] + L.red[1][col][0] + L.red[2][col][0] +
                                      L.red[3][col][0];
                const uint32_t npos = L.red[0][col][1] + L.red[1][col][1] + L.red[2][col][1] +
                                      L.red[3][col][1];
                if (nneg) atomicAdd(&P.base[J * 2], nneg);
                if (npos) atomicAdd(&P.base[J * 2 + 1], npos);
            }
        }
        __syncthreads();
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            uint32_t bits = jl[ct] ? um[ct] : 0u;
            if (!bits) continue;
            const int col = ct * 32 + lr;
            const int32_t J = J0 + col;
            uint32_t w = L.ucnt[wave][lh][col];
            uint32_t *dst = P.lists_out + (size_t)J * (size_t)P.n;
            while (bits) {
                const int k = __builtin_ctz(bits);
                bits &= bits - 1u;
                dst[w++] = (uint32_t)(r0 + acc_row(k >> 4, k & 15, lh));
            }
        }
    }
}

// Recheck of the uncertain rows: a queue entry is two words, (query,
// direction, wave tile row r0, lane half h) and the mask of the half column's
// uncertain rows (bit 16 rt + r: row 32 rt + 8 (r / 4) + 4 h + r % 4 of the
// wave tile), nearly always a single row.  One lane per entry: each masked
// row gets the binary64 recipe value (the recipe's fma chain over the point's
// row and the direction's row, both contiguous) and both counts from it; the other rows of the half column were
// counted by the sign GEMM.  Workgroup b takes the entries of queue segment
// b (those of one wave of the sign GEMM, in the order it met them), so a
// wave's lanes mostly share the query and read nearby directions.  Rows index
// the query's list in list mode, the points otherwise.
__global__ __launch_bounds__(256) void k_block_recheck(
    const uint64_t *__restrict__ queue, const uint32_t *__restrict__ segcnt, uint32_t seg,
    const double *__restrict__ X, int64_t n, int64_t d, const double *__restrict__ Zb,
    const double *__restrict__ UR, int64_t m, const uint32_t *__restrict__ lists_in,
    const uint32_t *__restrict__ mode, int64_t ldm, uint32_t *__restrict__ cnt,
    unsigned long long *__restrict__ tally)
{
    const uint32_t *const lists = (mode == nullptr || *mode != 0u) ? lists_in : nullptr;
    // workgroup b: the entries of queue segment b
    const uint64_t *q = queue + 2ull * (uint64_t)blockIdx.x * (uint64_t)seg;
    const uint32_t total = segcnt[blockIdx.x];
    uint32_t pairs = 0;
    for (uint32_t e = threadIdx.x; e < total; e += 256) {
        const uint64_t w = q[2 * (uint64_t)e];
        const uint32_t mask = (uint32_t)q[2 * (uint64_t)e + 1];
        const int64_t qi = (int64_t)(w >> 48);
        const int64_t j = (int64_t)((w >> 32) & 0xFFFF);
        const uint32_t lo = (uint32_t)(w & 0xFFFFFFFFu);
        const int64_t r0 = (int64_t)(lo & ~63u) + 4 * (int64_t)(lo & 1u);
        const double *z = Zb + qi * d;
        const double *u = UR + (qi * m + j) * d;
        uint32_t le = 0, ge = 0;
        for (uint32_t bits = mask; bits; bits &= bits - 1u) {
            const int k = __builtin_ctz(bits);
            const int64_t row = r0 + (k >> 4) * 32 + ((k >> 2) & 3) * 8 + (k & 3);
            const int64_t i = lists ? (int64_t)lists[qi * n + row] : row;
            const double *x = X + i * d;
            // the recipe's fma chain in coordinate order, with the loads of
            // eight coordinates issued ahead of their steps
            double t = 0.0;
            int64_t c = 0;
            for (; c + 8 <= d; c += 8) {
                double xv[8], uv[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    xv[k] = x[c + k];
                    uv[k] = u[c + k];
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) t = fma(xv[k] - z[c + k], uv[k], t);
            }
            for (; c < d; ++c) t = fma(x[c] - z[c], u[c], t);
            le += t <= 0.0 ? 1u : 0u;
            ge += t >= 0.0 ? 1u : 0u;
        }
        if (le) atomicAdd(&cnt[(qi * ldm + j) * 2], le);
        if (ge) atomicAdd(&cnt[(qi * ldm + j) * 2 + 1], ge);
        pairs += (uint32_t)__builtin_popcount(mask);
    }
    if (tally) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) pairs += (uint32_t)__shfl_xor((int)pairs, off);
        if ((threadIdx.x & 63) == 0 && pairs) atomicAdd(tally, (unsigned long long)pairs);
    }
}

// Per query: Delta_q = max_j |u_j - p_q| and |z_q - xbar| (binary32, rounded
// up), and the cull thresholds lam_q, mu_q; also zeroes the query's list
// count and decided counts, which the cull GEMM then accumulates.  One
// workgroup per query; the loads of eight coordinates go out before their fma
// steps, and wave 0 sums |z_q - xbar|^2 over its lanes while the others
// finish their directions.
__global__ __launch_bounds__(256) void k_cull_bounds(const double *__restrict__ UT, int64_t d,
                                                     int64_t m, int64_t ldm,
                                                     const double *__restrict__ pole,
                                                     const double *__restrict__ Zb,
                                                     const double *__restrict__ xbar,
                                                     const float *__restrict__ pmarg,
                                                     float kappa_a, double gamma,
                                                     float *__restrict__ lam,
                                                     float *__restrict__ mu,
                                                     uint32_t *__restrict__ lcount,
                                                     uint32_t *__restrict__ base)
{
    const int64_t q = blockIdx.x;
    const int tid = threadIdx.x;
    if (tid == 0) {
        lcount[q] = 0u;
        base[2 * q] = 0u;
        base[2 * q + 1] = 0u;
    }
    __shared__ double red[256];
    __shared__ double bn_sh;
    const double *u = UT + q * d * ldm;
    const double *p = pole + q * d;
    double mx = 0.0;
    for (int64_t j = tid; j < m; j += 256) {
        double s = 0.0;
        int64_t c = 0;
        for (; c + 8 <= d; c += 8) {
            double e[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) e[k] = u[(c + k) * ldm + j] - p[c + k];
#pragma unroll
            for (int k = 0; k < 8; ++k) s = fma(e[k], e[k], s);
        }
        for (; c < d; ++c) {
            const double e = u[c * ldm + j] - p[c];
            s = fma(e, e, s);
        }
        mx = fmax(mx, s);
    }
    if (tid < 64) {
        // |z_q - xbar|^2 in lane-strided partial sums (the order only moves
        // the sum by rounding, far inside the slack applied below)
        double bn = 0.0;
        for (int64_t c = tid; c < d; c += 64) {
            const double b = Zb[q * d + c] - xbar[c];
            bn = fma(b, b, bn);
        }
        for (int o = 32; o > 0; o >>= 1) bn += __shfl_xor(bn, o);
        if (tid == 0) bn_sh = bn;
    }
    red[tid] = mx;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) red[tid] = fmax(red[tid], red[tid + off]);
        __syncthreads();
    }
    if (tid == 0) {
        // the binary64 sums above are within a relative 1e-13 of the exact
        // squared norms; the factors below absorb that and the roundings to
        // binary32
        const double delta = sqrt(red[0]) * (1.0 + 1e-9);
        const double bnorm = sqrt(bn_sh) * (1.0 + 1e-9);
        // |t^ - (x - z).p| <= kappa_a |a_i| + pmarg_q (the sign GEMM's
        // margin for the pole column), |x_i - z| <= |a_i| + |z - xbar|, and
        // the binary64 recipe of a projection is within gamma |x_i - z| of
        // the exact value
        const double dg = delta + gamma;
        lam[q] = (float)(((double)kappa_a + dg) * (1.0 + 1e-6));
        mu[q] = (float)(((double)pmarg[q] + bnorm * dg) * (1.0 + 1e-6));
    }
}

// Exclusive prefix of the items per query (one workgroup): items_q =
// ceil(lcount_q / (256 rpi)) * ceil(m / 128); offs[qb] = total.  Also picks
// the mode of the refinement's sign GEMM: lists (*mode = 1) when their
// matrix-core work (rows padded to 64, each query's directions to tiles of
// 128) is below list_pct percent of the dense GEMM's over every point and
// the flat columns, dense (*mode = 0) otherwise.
__global__ __launch_bounds__(1024) void k_worklist(const uint32_t *__restrict__ lcount,
                                                   int64_t qb, int64_t m, int rpi, int64_t n,
                                                   int64_t dense_cols, int list_pct,
                                                   uint32_t *__restrict__ offs,
                                                   uint32_t *__restrict__ mode,
                                                   unsigned long long *__restrict__ pairs)
{
    __shared__ uint32_t part[1024];
    __shared__ unsigned long long work, lpairs;
    const int tid = threadIdx.x;
    if (tid == 0) work = lpairs = 0ull;
    const int64_t per = (qb + 1023) / 1024;
    const int64_t q0 = tid * per, q1 = q0 + per < qb ? q0 + per : qb;
    const uint32_t nctq = (uint32_t)((m + kTN - 1) / kTN);
    const uint32_t rows = (uint32_t)(kTM * rpi);
    uint32_t s = 0;
    unsigned long long w = 0, lp = 0;
    for (int64_t q = q0; q < q1; ++q) {
        s += (lcount[q] + rows - 1) / rows * nctq;
        w += (unsigned long long)((lcount[q] + 63u) / 64u) * 64ull * nctq * (unsigned long long)kTN;
        lp += lcount[q];
    }
    part[tid] = s;
    __syncthreads();
    if (w) atomicAdd(&work, w);
    if (lp) atomicAdd(&lpairs, lp);
    // inclusive scan over the 1024 partial sums
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = tid >= off ? part[tid - off] : 0u;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    uint32_t run = tid ? part[tid - 1] : 0u;
    for (int64_t q = q0; q < q1; ++q) {
        offs[q] = run;
        run += (lcount[q] + rows - 1) / rows * nctq;
    }
    if (tid == 1023) offs[qb] = part[1023];
    if (tid == 0) {
        const double dense = (double)((n + 63) / 64 * 64) * (double)dense_cols;
        const bool lists = (double)work * 100.0 < dense * (double)list_pct;
        *mode = lists ? 1u : 0u;
        if (pairs) atomicAdd(pairs, lists ? lpairs * (unsigned long long)m
                                          : (unsigned long long)qb * (unsigned long long)m *
                                                (unsigned long long)n);
    }
}

// The list-mode items as records: q | tile << 16, first list position,
// end list position (the GEMM reads one record per item instead of searching
// the offsets).
__global__ __launch_bounds__(256) void k_item_table(const uint32_t *__restrict__ offs,
                                                    const uint32_t *__restrict__ lcount,
                                                    int64_t qb, int64_t m, int rpi,
                                                    const uint32_t *__restrict__ mode,
                                                    uint32_t *__restrict__ items)
{
    if (*mode == 0u) return;
    const uint32_t total = offs[qb];
    const uint32_t nctq = (uint32_t)((m + kTN - 1) / kTN);
    const uint32_t rows = (uint32_t)(kTM * rpi);
    for (uint32_t it = blockIdx.x * 256u + threadIdx.x; it < total; it += gridDim.x * 256u) {
        const int32_t q = item_query(offs, (int32_t)qb, (int32_t)it);
        const uint32_t loc = it - offs[q];
        const uint32_t rc = loc / nctq, ct = loc - rc * nctq;
        const uint32_t rb = rc * rows, lc = lcount[q];
        uint32_t *r = items + 4ull * it;
        r[0] = (uint32_t)q | (ct << 16);
        r[1] = rb;
        r[2] = rb + rows < lc ? rb + rows : lc;
        r[3] = 0u;
    }
}

// Counts start from the decided points: cnt[q][j] = base[q] (j < m), 0 for
// the padding directions; from zero when the refinement runs the dense GEMM.
__global__ __launch_bounds__(256) void k_spread_base(const uint32_t *__restrict__ base,
                                                     int64_t qb, int64_t m, int64_t ldm,
                                                     const uint32_t *__restrict__ mode,
                                                     uint32_t *__restrict__ cnt)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;  // (q, j, side)
    if (e >= qb * ldm * 2) return;
    const int64_t q = e / (ldm * 2), j = (e / 2) % ldm, side = e & 1;
    cnt[e] = (j < m && *mode != 0u) ? base[q * 2 + side] : 0u;
}

int g_cus = 0;

int grid_size()
{
    if (g_cus == 0) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) ==
                hipSuccess &&
            cus > 0)
            g_cus = cus;
        else
            g_cus = 256;
    }
    return ((2 * g_cus + 7) / 8) * 8;
}

// Recheck queue of the sign GEMM (qcap words): one segment of `seg` entries
// (two words each) per wave of the grid, then the segment fills (one word per
// two segments) at the end.
struct SignQueue {
    uint32_t *segcnt;
    uint32_t seg, nseg;
};
SignQueue sign_queue(const SignArgs &a, int grid)
{
    const uint64_t nseg = (uint64_t)grid * 4;
    const uint64_t cw = (nseg + 1) / 2;
    const uint64_t seg = a.qcap > cw ? (a.qcap - cw) / 2 / nseg : 0;
    return {(uint32_t *)(a.queue + (a.qcap - cw)), (uint32_t)seg, (uint32_t)nseg};
}

#define RRS_SIGN_KS_SWITCH(KS_VAR, F, ...)                                                  \
    switch (KS_VAR) {                                                                       \
    case 1: F<1>(__VA_ARGS__); break;                                                       \
    case 2: F<2>(__VA_ARGS__); break;                                                       \
    case 3: F<3>(__VA_ARGS__); break;                                                       \
    case 4: F<4>(__VA_ARGS__); break;                                                       \
    case 5: F<5>(__VA_ARGS__); break;                                                       \
    case 6: F<6>(__VA_ARGS__); break;                                                       \
    case 7: F<7>(__VA_ARGS__); break;                                                       \
    default: F<8>(__VA_ARGS__); break;                                                      \
    }

template <int KS>
void go_sign(const SignParams &p, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_sign<KS>, dim3((unsigned)grid), dim3(256), 0, st, p);
}
template <int KS>
void go_cull(const SignParams &p, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_cull<KS>, dim3((unsigned)grid), dim3(256), 0, st, p);
}

}  // namespace

bool sign_supported(int prec, int64_t d)
{
    return prec == MFMA_BF16 && mfma_kpad(prec, d) <= 16 * kSignMaxKS;
}

hipError_t launch_sign(const SignArgs &a, hipStream_t st)
{
    double kappa, canon;
    const int64_t kp = mfma_kpad(MFMA_BF16, a.d);
    if (kp > 16 * kSignMaxKS || kp % 16) return hipErrorInvalidValue;
    mfma_margins(MFMA_BF16, a.d, kp, &kappa, &canon);
    SignParams p{};
    p.A0 = (const __bf16 *)a.A0;
    p.A1 = (const __bf16 *)a.A1;
    p.anorm = a.anorm;
    p.n = (int32_t)a.n;
    p.kp = (int32_t)kp;
    p.B0 = (const __bf16 *)a.B0;
    p.B1 = (const __bf16 *)a.B1;
    p.cmarg = a.cmarg;
    p.npad = (int32_t)a.npad;
    p.ncols = (int32_t)(a.qb * a.m);
    p.m = (int32_t)a.m;
    p.ldm = (int32_t)a.ldm;
    p.qb = (int32_t)a.qb;
    p.kappa_a = (float)((kappa + canon) * 1.000001);
    p.cnt = a.cnt;
    const int grid = grid_size();
    const SignQueue sq = sign_queue(a, grid);
    p.queue = a.queue;
    p.segcnt = sq.segcnt;
    p.qflag = a.qcount;
    p.seg = sq.seg;
    p.lists = a.lists;
    p.lcount = a.lcount;
    p.offs = a.offs;
    p.items = a.items;
    // point tiles per item of the dense GEMM: keep about four items per
    // workgroup at least
    int rpi = 4;
    {
        const int64_t nct = (p.ncols + kTN - 1) / kTN;
        while (rpi > 1 && ((a.n + (int64_t)kTM * rpi - 1) / ((int64_t)kTM * rpi)) * nct <
                              4 * (int64_t)grid)
            rpi >>= 1;
    }
    p.rpi = a.lists ? a.rpi : rpi;
    p.rpi_dense = rpi;
    p.mode = a.lists ? a.mode : nullptr;
    const int ks = (int)(kp / 16);
    RRS_SIGN_KS_SWITCH(ks, go_sign, p, grid, st)
    return hipGetLastError();
}

hipError_t launch_block_recheck(const SignArgs &a, const double *X, uint64_t *tally,
                                hipStream_t st)
{
    const SignQueue sq = sign_queue(a, grid_size());
    hipLaunchKernelGGL(k_block_recheck, dim3(sq.nseg), dim3(256), 0, st, a.queue, sq.segcnt, sq.seg,
                       X, a.n, a.d, a.Z, a.UR, a.m, a.lists, a.mode, a.ldm, a.cnt,
                       (unsigned long long *)tally);
    return hipGetLastError();
}

hipError_t launch_cull(const SignArgs &a, const CullArgs &c, hipStream_t st)
{
    double kappa, canon;
    const int64_t kp = mfma_kpad(MFMA_BF16, a.d);
    if (kp > 16 * kSignMaxKS || kp % 16) return hipErrorInvalidValue;
    mfma_margins(MFMA_BF16, a.d, kp, &kappa, &canon);
    const float kappa_a = (float)((kappa + canon) * 1.000001);
    // thresholds per query
    const double gamma = 4.0 * (double)(a.d + 2) * ldexp(1.0, -53);
    hipLaunchKernelGGL(k_cull_bounds, dim3((unsigned)a.qb), dim3(256), 0, st, a.UT, a.d, a.m,
                       a.ldm, c.pole, a.Z, c.xbar, c.pmarg, kappa_a, gamma, c.lam, c.mu,
                       c.lcount, c.base);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    SignParams p{};
    p.A0 = (const __bf16 *)a.A0;
    p.A1 = (const __bf16 *)a.A1;
    p.anorm = a.anorm;
    p.n = (int32_t)a.n;
    p.kp = (int32_t)kp;
    p.B0 = (const __bf16 *)c.P0;
    p.B1 = (const __bf16 *)c.P1;
    p.npad = (int32_t)c.npad_pole;
    p.ncols = (int32_t)a.qb;
    p.m = 1;
    p.ldm = 1;
    p.qb = (int32_t)a.qb;
    p.kappa_a = kappa_a;
    p.rpi = 1;
    p.lam = c.lam;
    p.mu = c.mu;
    p.lists_out = c.lists;
    p.lcount_out = c.lcount;
    p.base = c.base;
    const int ks = (int)(kp / 16);
    RRS_SIGN_KS_SWITCH(ks, go_cull, p, grid_size(), st)
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_worklist, dim3(1), dim3(1024), 0, st, c.lcount, a.qb, a.m, a.rpi, a.n,
                       mfma_col_pad(a.qb * a.m), c.list_pct, c.offs, c.mode, c.pairs);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_item_table, dim3(512), dim3(256), 0, st, c.offs, c.lcount, a.qb, a.m,
                       a.rpi, c.mode, c.items);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t tot = a.qb * a.ldm * 2;
    hipLaunchKernelGGL(k_spread_base, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                       c.base, a.qb, a.m, a.ldm, c.mode, a.cnt);
    return hipGetLastError();
}

}  // namespace rrs
