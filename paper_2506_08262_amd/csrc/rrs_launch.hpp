// rrs_launch.hpp -- host-side launchers of the RRS kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rrs {

// Profiling counters of one job (device, uint32 words): [1] selects that took
// the exact fallback (rare, so one address suffices), [4..5] the recheck
// tally (uint64), [6..7] the pairs the culled sign GEMM evaluated (uint64).  Selects that took the window path are counted on the host:
// one device count per column would serialize a launch on one address.
constexpr int kStatWords = 16;


enum { NOTION_HALFSPACE = 0, NOTION_PROJECTION = 1, NOTION_APD = 2 };

constexpr int kProjJT = 16;  // directions per projection workgroup

struct GenArgs {
    int64_t d, m, ldm, qb;
    int32_t l;
    double phi;
    uint64_t seed, qbase;
    const double *pole;
    double *UT;
    int32_t first_cap = 0;  // 1: refinement 1 draws from Alg. S4's cap (phi = 1) too
    int32_t area_cap = 0;   // 1: cap directions uniform in area instead of in angle
    double *UR = nullptr;   // optional [qb][m][d] copy, one contiguous row per direction
};

struct ProjArgs {
    const double *XT;
    int64_t ldx, n, d;
    const double *Z;
    const double *UT;
    int64_t ldm, m, qb;
    uint32_t *cnt;
    double *T;
    const uint32_t *only_if;  // count mode: run only when *only_if != 0 (may be null)
};

// Halfspace counts on matrix cores (rrs_mfma.hip).
enum { MFMA_BF16 = 0, MFMA_F32 = 1, MFMA_F32_PLAIN = 2 };

struct MfmaArgs {
    int prec;                  // MFMA_*
    const void *A0, *A1;       // [n][kp] centred data: bf16 hi/lo, or binary32 in A0
    const float *anorm;        // [n] norm bound of the centred points
    int64_t n, d;
    const void *B0, *B1;       // [npad][kp] directions + centring (flat columns q m + j)
    const float *cmarg;        // [npad] direction part of the margin
    int64_t m, ldm, npad, qb;
    uint32_t *cnt;             // [qb][ldm][2]
    uint64_t *queue;           // uncertain (query, direction, point)
    uint32_t *qcount;
    uint64_t qcap;
    uint32_t *flag;            // set when the queue overflowed
    const double *X;           // [n][d] binary64 data (recheck)
    const double *Z;           // [qb][d] queries of the batch
    const double *UT;          // [qb][d][ldm] binary64 directions
    uint64_t *tally;           // optional: running total of rechecked pairs
};

struct SelectArgs {
    const double *T;
    int64_t n, m, ldm, qb;
    double *Dj;
    uint32_t *stats;  // optional [2]: pairs resolved by the bracket / the fallback
};

// Projection / APD depth from binary32 projections (rrs_select_rc.hip).
struct SelectRcArgs {
    const float *S;            // [qb][m][n] s_ij = a_i.u_j
    int64_t n, m, ldm, qb;
    const double *cq, *eq;     // [qb m] centring terms and error bounds (flat columns)
    const double *X;           // [n][d] binary64 data (recompute)
    int64_t d;
    const double *Z;           // [qb][d]
    const double *UT;          // [qb][d][ldm]
    double *Dj;
    uint32_t *stats;
    // per-point bounds (heavy-tailed data; eq then holds the column part and
    // point i adds alpha anorm[i])
    const float *anorm;
    bool pp;
    double alpha;
};

struct ArgminArgs {
    int64_t m, ldm, d, qb;
    const uint32_t *cnt;
    const double *Dj;
    const double *UT;
    double *pole;
    double *best_d;
    int64_t *best_c;
    int64_t *trace;
    int32_t l, r;
};

hipError_t launch_gen_dirs(const GenArgs &a, hipStream_t st);
hipError_t launch_transpose(const double *X, int64_t n, int64_t d, int64_t ldx, double *XT,
                            hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, int64_t count, uint32_t v, hipStream_t st);
hipError_t launch_proj_f64(const ProjArgs &a, bool count_mode, hipStream_t st);
int64_t select_reg_max_n();
hipError_t launch_select_reg(const SelectArgs &a, int notion, hipStream_t st);
hipError_t launch_select_stream(const SelectArgs &a, int notion, hipStream_t st);
hipError_t launch_select_rc(const SelectRcArgs &a, int notion, bool exact, hipStream_t st);
hipError_t launch_argmin(const ArgminArgs &a, bool half, hipStream_t st);
int64_t mfma_kpad(int prec, int64_t d);
size_t mfma_elem_bytes(int prec);
int mfma_terms(int prec);
void mfma_margins(int prec, int64_t d, int64_t kp, double *kappa, double *canon);
// amax: 16 words; [0] the largest norm bound, [2..3] the sum of squared
// norms (binary64).
hipError_t launch_mfma_prep(int prec, const double *X, int64_t n, int64_t d, double *xbar,
                            void *A0, void *A1, float *anorm, float *amax, hipStream_t st);
// Per-point factor of the stored-projection bound: point i's bound is
// alpha anorm[i] plus the column part.
double mfma_point_alpha(int prec, int64_t d);
// pp (stored projections): eq holds only the column part of per-point
// bounds (alpha anorm[i] + eq[J], alpha = mfma_point_alpha).
hipError_t launch_mfma_dirs(int prec, bool fold, const double *UT, int64_t d, int64_t m,
                            int64_t ldm, int64_t ncols, int64_t npad, const double *Zb,
                            const double *xbar, void *B0, void *B1, float *cmarg,
                            const float *amax, double *cq, double *eq, hipStream_t st,
                            bool pp = false);
hipError_t launch_mfma_store(int prec, const void *A0, const void *A1, int64_t n, int64_t d,
                             const void *B0, const void *B1, int64_t m, int64_t ncols,
                             int64_t npad, float *S, hipStream_t st);
int64_t mfma_col_pad(int64_t ncols);
hipError_t launch_mfma_gemm(const MfmaArgs &a, hipStream_t st);
// While suspended (per thread), GEMM launches use the variant already chosen
// for their key, else variant 0, and never time variants (no events).
void mfma_tune_suspend(bool on);
hipError_t launch_mfma_recheck(const MfmaArgs &a, hipStream_t st);
// Sets *flag when the recheck queue overflowed, and then zeroes the counts
// (cnt_words words) for the binary64 recount that follows.
hipError_t launch_queue_overflow(const uint32_t *qcount, uint64_t qcap, uint32_t *cnt,
                                 int64_t cnt_words, uint32_t *flag, hipStream_t st);

// Persistent sign GEMM and cap culling of the bfloat16 form (rrs_sign.hip).
constexpr int kSignMaxKS = 8;  // padded K up to 128 (d <= 126)
struct SignArgs {
    int64_t n, d;
    const void *A0, *A1;       // [n][kp] centred data, bf16 hi / lo
    const float *anorm;        // [n]
    const void *B0, *B1;       // [npad][kp] direction operands (flat columns q m + j)
    const float *cmarg;        // [npad]
    int64_t npad, m, ldm, qb;
    uint32_t *cnt;             // [qb][ldm][2]
    uint64_t *queue;           // qcap words: recheck entries
    uint32_t *qcount;          // zeroed by the caller; kSignQueueOverflow on overflow
    uint64_t qcap;
    const double *UT;          // [qb][d][ldm] binary64 directions (cull bounds)
    const double *UR;          // [qb][m][d] the same, a row per direction (recheck)
    const double *Z;           // [qb][d]
    // list mode: the undecided points of each query (null: every point), and
    // the items of the list-mode GEMM (four words each: q | tile << 16, first
    // and end list position)
    const uint32_t *lists, *lcount, *offs, *items;
    const uint32_t *mode;      // list mode only when *mode != 0 (written by launch_cull)
    int rpi;                   // point tiles of 256 per list-mode item
};
struct CullArgs {
    const double *pole;        // [qb][d] current poles
    const double *xbar;        // [d]
    const void *P0, *P1;       // [npad_pole][kp] pole operands (centring folded)
    const float *pmarg;        // [npad_pole] column part of their margin
    int64_t npad_pole;
    float *lam, *mu;           // [qb] cull thresholds
    uint32_t *lists;           // [qb][n] out: undecided points
    uint32_t *lcount;          // [qb] out (launch_cull zeroes it first)
    uint32_t *base;            // [qb][2] out: decided points below / above (zeroed first)
    uint32_t *offs;            // [qb + 1] out: item offsets of the list-mode GEMM
    uint32_t *items;           // [sign_max_items][4] out: the items themselves
    uint32_t *mode;            // out: 1 = the sign GEMM runs over the lists, 0 = dense
    int list_pct;              // lists when their work is below this percent of dense
    unsigned long long *pairs; // optional: adds sum_q lcount_q * m (pairs the GEMM evaluates)
};
bool sign_supported(int prec, int64_t d);
// Most items the list-mode sign GEMM can have (every point undecided).
inline int64_t sign_max_items(int64_t qb, int64_t n, int64_t m, int rpi)
{
    return qb * ((n + 256 * (int64_t)rpi - 1) / (256 * (int64_t)rpi)) * ((m + 127) / 128);
}
// A queue segment of the sign GEMM that overflowed sets this bit of *qcount
// (the queue's words are split into one segment per wave of its grid).
constexpr uint32_t kSignQueueOverflow = 0x80000000u;
// Sign counts (cnt must hold the starting counts) and the recheck queue.
hipError_t launch_sign(const SignArgs &a, hipStream_t st);
// Binary64 recount of the (query, direction, half tile of 32 rows) blocks
// the sign GEMM queued; adds both counts of every live row.  X: [n][d].
hipError_t launch_block_recheck(const SignArgs &a, const double *X, uint64_t *tally,
                                hipStream_t st);
// Culls the points of every query against its cap: lists, item offsets, and
// cnt set to the decided points' counts.
hipError_t launch_cull(const SignArgs &a, const CullArgs &c, hipStream_t st);
// Mahalanobis depth D_M(L) (rrs_maha.hip): workspace bytes and the enqueue
// of the whole computation; *flag_out (device word) is 1 afterwards when the
// covariance was not positive definite.
size_t maha_ws_bytes(int64_t n, int64_t d, int64_t m);
hipError_t maha_enqueue(const double *X, int64_t n, int64_t d, const double *Z, int64_t m,
                        double *depth, void *ws, uint32_t **flag_out, hipStream_t st);
hipError_t launch_init_state(int64_t qb, int64_t d, int64_t n, double *pole, double *best_d,
                             int64_t *best_c, hipStream_t st);
hipError_t launch_finalize(int64_t qb, int64_t d, int64_t n, bool half, const double *pole,
                           const double *best_d, const int64_t *best_c, double *depth,
                           int64_t *count, double *poles_out, hipStream_t st);

}  // namespace rrs
