// rrs_engine.hip -- planning and enqueueing of one RRS depth job.
//
// For each batch of queries the job runs the refinement loop of Alg. 4 /
// Alg. S5 -- directions, projection, univariate depth, argmin and pole
// update -- on one HIP stream.  The refinement chain stays on the device; the
// host only enqueues kernels.
#include "rrs_engine.hpp"

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <math.h>

namespace rrs {

namespace {
thread_local std::string t_last_error;
}

std::string &last_error() { return t_last_error; }

rrs_status fail(rrs_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    t_last_error = buf;
    return s;
}

size_t carve_size(const size_t *sizes, int k)
{
    size_t off = 0;
    for (int i = 0; i < k; ++i) {
        off = (off + 255) & ~(size_t)255;
        off += sizes[i];
    }
    return off + 256;
}

const char *const kKernelNames[K_COUNT] = {"k_gen_dirs",    "k_proj_f64", "k_select",
                                           "k_argmin_pole", "k_gemm",     "k_recheck",
                                           "k_misc",        "k_cull"};

hipEvent_t Profiler::get()
{
    if (used == pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        pool.push_back(e);
    }
    return pool[used++];
}

void Profiler::reserve2()
{
    if (used + 2 <= kPoolCap) return;
    collect();
}

void Profiler::collect()
{
    for (const Rec &r : recs) {
        float t = 0.f;
        // the events may belong to several streams: wait for each end event
        if (hipEventSynchronize(r.b) == hipSuccess &&
            hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
            launches[r.kind] += 1;
            ms[r.kind] += t;
            work[r.kind] += r.work;
        }
    }
    recs.clear();
    used = 0;
}

void Profiler::clear()
{
    recs.clear();
    used = 0;
    for (int k = 0; k < K_COUNT; ++k) {
        launches[k] = 0;
        ms[k] = 0.0;
        work[k] = 0.0;
    }
    sel_total = sel_fallback = recheck_pairs = gemm_pairs = 0.0;
    shared[0] = shared[1] = shared[2] = 0.0;
}

namespace {

bool env_flag(const char *name, bool dflt)
{
    const char *e = std::getenv(name);
    if (!e || !*e) return dflt;
    return std::atoi(e) != 0;
}

double env_double(const char *name, double dflt)
{
    const char *e = std::getenv(name);
    if (!e || !*e) return dflt;
    return std::atof(e);
}

// HIP events around one launch on its stream (when profiling).
struct ProfScope {
    Profiler *p;
    Profiler::Rec rec{};
    hipStream_t st;
    bool live = false;
    ProfScope(Profiler *prof, int kind, double work, hipStream_t s) : p(prof), st(s)
    {
        if (!p || !p->on) return;
        rec.kind = kind;
        rec.work = work;
        p->reserve2();
        rec.a = p->get();
        rec.b = p->get();
        if (rec.a && rec.b && hipEventRecord(rec.a, st) == hipSuccess) live = true;
    }
    ~ProfScope()
    {
        if (live && hipEventRecord(rec.b, st) == hipSuccess) p->recs.push_back(rec);
    }
};

}  // namespace

size_t data_bytes(int64_t n, int64_t d, int prec)
{
    const int64_t ldx = (n + 511) / 512 * 512;
    size_t sizes[6] = {(size_t)d * ldx * 8, 0, 0, 0, 0, 0};
    if (prec >= 0) {
        const int64_t kp = mfma_kpad(prec, d);
        const size_t eb = mfma_elem_bytes(prec);
        sizes[1] = (size_t)d * 8;
        sizes[2] = (size_t)n * kp * eb;
        sizes[3] = mfma_terms(prec) == 2 ? (size_t)n * kp * eb : 0;
        sizes[4] = (size_t)n * 4;
        sizes[5] = 64;
    }
    return carve_size(sizes, 6);
}

hipError_t data_prepare(DataDev &D, void *mem, int prec, hipStream_t st)
{
    const int64_t n = D.n, d = D.d;
    D.ldx = (n + 511) / 512 * 512;
    Carver cv(mem);
    D.XT = cv.take<double>((size_t)d * D.ldx);
    D.prec = prec;
    if (prec >= 0) {
        const int64_t kp = mfma_kpad(prec, d);
        const size_t eb = mfma_elem_bytes(prec);
        D.xbar = cv.take<double>((size_t)d);
        D.A0 = cv.take<char>((size_t)n * kp * eb);
        D.A1 = mfma_terms(prec) == 2 ? (void *)cv.take<char>((size_t)n * kp * eb) : nullptr;
        D.anorm = cv.take<float>((size_t)n);
        D.amax = cv.take<float>(16);
    } else {
        D.xbar = nullptr;
        D.A0 = D.A1 = nullptr;
        D.anorm = nullptr;
        D.amax = nullptr;
    }
    hipError_t e = launch_transpose(D.X, n, d, D.ldx, D.XT, st);
    if (e != hipSuccess || prec < 0) return e;
    return launch_mfma_prep(prec, D.X, n, d, D.xbar, D.A0, D.A1, D.anorm, D.amax, st);
}

hipError_t data_point_bounds(DataDev &D, hipStream_t st)
{
    D.pp = false;
    if (D.prec < 0 || D.prec == MFMA_F32_PLAIN || !D.amax) return hipSuccess;
    const double force = env_double("RRS_POINT_BOUNDS", -1.0);
    if (force >= 0.0) {
        D.pp = force > 0.0;
        return hipSuccess;
    }
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    hipError_t e = hipMemcpyAsync(w, D.amax, sizeof(w), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    // candidates a column-wide bound E = alpha max|a| would put in a window
    // around the median: about 4 E times the points per unit near it,
    // n / (2.5 rms / sqrt(d)) for a projection of spread rms / sqrt(d);
    // per-point bounds once that passes a quarter of the candidate room
    float amax;
    double sum;
    std::memcpy(&amax, &w[0], sizeof(amax));
    std::memcpy(&sum, &w[2], sizeof(sum));
    const double rms = sqrt(sum / (double)(D.n > 0 ? D.n : 1));
    if (rms > 0.0) {
        const double est = 4.0 * mfma_point_alpha(D.prec, D.d) * (double)amax * (double)D.n *
                           sqrt((double)D.d) / (2.5 * rms);
        D.pp = est > 256.0;
    }
    return hipSuccess;
}

int job_mfma_prec(int precision)
{
    switch (precision) {
    case RRS_BF16_RECHECK: return MFMA_BF16;
    case RRS_F32_RECHECK: return MFMA_F32;
    case RRS_F32_PLAIN: return MFMA_F32_PLAIN;
    default: return -1;
    }
}

rrs_status job_validate(const JobSpec &s, int64_t n, int64_t d)
{
    if (s.nq < 0) return fail(RRS_E_INVAL, "number of queries must be >= 0 (got %lld)", (long long)s.nq);
    if (n < 1) return fail(RRS_E_INVAL, "n must be >= 1 (got %lld)", (long long)n);
    if (d < 2) return fail(RRS_E_INVAL, "d must be >= 2 (got %lld)", (long long)d);
    if (s.K < 1) return fail(RRS_E_INVAL, "K must be >= 1 (got %lld)", (long long)s.K);
    if (s.r < 1) return fail(RRS_E_INVAL, "n_refine must be >= 1 (got %d)", s.r);
    if (!(s.alpha > 0.0 && s.alpha <= 1.0))
        return fail(RRS_E_INVAL, "cap_shrink must be in (0, 1] (got %g)", s.alpha);
    if (s.notion != NOTION_HALFSPACE && s.notion != NOTION_PROJECTION && s.notion != NOTION_APD)
        return fail(RRS_E_INVAL, "unknown depth notion %d", s.notion);
    if (s.precision != RRS_F64 && s.precision != RRS_F32_RECHECK &&
        s.precision != RRS_BF16_RECHECK && s.precision != RRS_F32_PLAIN)
        return fail(RRS_E_INVAL, "unknown precision %d", s.precision);
    const bool mfma = s.precision != RRS_F64;
    if (mfma && ((s.K + s.r - 1) / s.r >= 65536 || s.nq > 65535))
        return fail(RRS_E_INVAL,
                    "matrix-core precisions need ceil(K/n_refine) < 65536 directions and at "
                    "most 65535 queries");
    if (n > 0x7FFFFFFFLL || d > 0x7FFFFFFFLL)
        return fail(RRS_E_INVAL, "n and d must fit in 31 bits");
    if ((s.K + s.r - 1) / s.r > 0x7FFFFFFFLL)
        return fail(RRS_E_INVAL, "ceil(K / n_refine) too large");
    if (s.qoff < 0) return fail(RRS_E_INVAL, "query_offset must be >= 0");
    return RRS_OK;
}

namespace {

// Workspace pieces of a job with query batch qb (order = carve order).
int job_sizes(const JobSpec &s, int64_t n, int64_t d, const Plan &p, int64_t qb, size_t *sz)
{
    const bool half = s.notion == NOTION_HALFSPACE;
    const bool mfma = p.prec >= 0;
    int k = 0;
    sz[k++] = (size_t)qb * d * p.ldm * 8;                       // UT
    sz[k++] = (size_t)qb * d * 8;                               // pole
    sz[k++] = (size_t)qb * 8;                                   // best_d
    sz[k++] = (size_t)qb * 8;                                   // best_c
    sz[k++] = half ? (size_t)qb * p.ldm * 2 * 4 : 0;            // cnt
    sz[k++] = (half || mfma) ? 0 : (size_t)qb * p.m * n * 8;    // T (binary64)
    sz[k++] = half ? 0 : (size_t)qb * p.ldm * 8;                // Dj
    sz[k++] = (size_t)kStatWords * 4;                           // stats
    const size_t npad = mfma ? (size_t)mfma_col_pad(qb * p.m) : 0;
    sz[k++] = mfma ? npad * p.kp * p.eb : 0;                    // B0
    sz[k++] = (mfma && p.terms == 2) ? npad * p.kp * p.eb : 0;  // B1
    sz[k++] = (mfma && half) ? npad * 4 : 0;                    // cmarg
    sz[k++] = (mfma && half) ? (size_t)p.qcap * 8 : 0;          // queue
    sz[k++] = 64;                                               // qctl
    sz[k++] = (mfma && !half) ? (size_t)qb * p.m * n * 4 : 0;   // S (binary32)
    sz[k++] = (mfma && !half) ? npad * 8 : 0;                   // cq
    sz[k++] = (mfma && !half) ? npad * 8 : 0;                   // eq
    // cap culling (halfspace bfloat16 form)
    const size_t npp = p.cull ? (size_t)mfma_col_pad(qb) : 0;
    sz[k++] = npp * p.kp * p.eb;                                // P0 (pole operands)
    sz[k++] = npp * p.kp * p.eb;                                // P1
    sz[k++] = npp * 4;                                          // pmarg
    sz[k++] = p.cull ? (size_t)qb * 4 : 0;                      // lam
    sz[k++] = p.cull ? (size_t)qb * 4 : 0;                      // mu
    sz[k++] = p.cull ? (size_t)qb * n * 4 : 0;                  // lists
    sz[k++] = p.cull ? (size_t)qb * 4 : 0;                      // lcount
    sz[k++] = p.cull ? (size_t)qb * 8 : 0;                      // base
    sz[k++] = p.cull ? (size_t)(qb + 1) * 4 : 0;                // offs
    sz[k++] = p.cull ? (size_t)sign_max_items(qb, n, p.m, p.rpi) * 16 : 0;  // items
    sz[k++] = p.sign ? (size_t)qb * p.m * d * 8 : 0;            // UR (direction rows)
    return k;
}

uint64_t job_qcap(const Plan &p, int64_t n, int64_t qb)
{
    // recheck queue: 1% of the pairs of a launch, at least 1M words;
    // RRS_QUEUE_WORDS overrides the size (at least 4096 words), e.g. to
    // exercise the overflow recount
    uint64_t qcap = (uint64_t)qb * (uint64_t)p.m * (uint64_t)n / 100;
    if (qcap < (1u << 20)) qcap = 1u << 20;
    if (qcap > 0xFFFFFFF0ull) qcap = 0xFFFFFFF0ull;
    const double force = env_double("RRS_QUEUE_WORDS", 0.0);
    if (force > 0.0) qcap = force < 4096.0 ? 4096u : (force > 4.0e9 ? 4000000000ull : (uint64_t)force);
    return qcap;
}

}  // namespace

rrs_status job_plan(const JobSpec &s, int64_t n, int64_t d, size_t limit, Plan *out)
{
    Plan p;
    p.prec = job_mfma_prec(s.precision);
    p.m = (s.K + s.r - 1) / s.r;
    p.ldm = (p.m + kProjJT - 1) / kProjJT * kProjJT;

    if (p.prec >= 0) {
        p.kp = mfma_kpad(p.prec, d);
        p.eb = mfma_elem_bytes(p.prec);
        p.terms = mfma_terms(p.prec);
    }
    // the persistent sign GEMM: bfloat16 halfspace form with K up to 128 and
    // operands addressable with 32-bit offsets (RRS_SIGN=0 selects the
    // tile-per-workgroup GEMM of rrs_mfma.hip instead)
    int64_t hi = s.nq < 65535 ? (s.nq > 0 ? s.nq : 1) : 65535;
    if (s.notion == NOTION_HALFSPACE && sign_supported(p.prec, d) && env_flag("RRS_SIGN", true)) {
        const double rowb = (double)p.kp * 2.0;
        const double cols = (double)mfma_col_pad(hi * p.m) + 128.0;
        if ((double)n * rowb < 2147483648.0 && cols * rowb < 2147483648.0 &&
            (double)hi * (double)p.m < 2147483648.0) {
            p.sign = true;
            // culling's item table (16 bytes per item) must stay below 2 GiB
            const double items = (double)hi * ((double)n / 256.0 + 1.0) *
                                 (double)((p.m + 127) / 128);
            p.cull = env_flag("RRS_CULL", true) && items < 134217728.0;
        }
    }
    // largest batch whose workspace fits the limit (the size grows with qb)
    int64_t lo = 1;
    size_t sz[32];
    auto bytes = [&](int64_t qb) {
        Plan t = p;
        t.qcap = (p.prec >= 0 && s.notion == NOTION_HALFSPACE) ? job_qcap(p, n, qb) : 0;
        const int k = job_sizes(s, n, d, t, qb, sz);
        return carve_size(sz, k);
    };
    if (bytes(hi) > limit) {
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo + 1) / 2;
            if (bytes(mid) <= limit)
                lo = mid;
            else
                hi = mid - 1;
        }
    } else {
        lo = hi;
    }
    p.qb = lo;
    p.qcap = (p.prec >= 0 && s.notion == NOTION_HALFSPACE) ? job_qcap(p, n, p.qb) : 0;
    p.ws_bytes = bytes(p.qb);
    *out = p;
    return RRS_OK;
}

rrs_status enqueue_job(const JobSpec &s, const DataDev &D, const Plan &p, const JobIO &io,
                       void *ws, hipStream_t st, Profiler *prof, uint32_t **stats_out)
{
    const int64_t n = D.n, d = D.d, nq = s.nq, m = p.m, ldm = p.ldm, qb = p.qb;
    const int64_t npad = p.prec >= 0 ? mfma_col_pad(qb * m) : 0;
    const int32_t r = s.r;
    const bool half = s.notion == NOTION_HALFSPACE;
    const bool mfma = p.prec >= 0;
    const bool profiling = prof && prof->on;
    if (mfma && D.prec != p.prec)
        return fail(RRS_E_INTERNAL, "data set not prepared for matrix-core format %d", p.prec);
    size_t sz[32];
    job_sizes(s, n, d, p, qb, sz);
    Carver cv(ws);
    double *UT = cv.take<double>(sz[0] / 8);
    double *pole = cv.take<double>(sz[1] / 8);
    double *best_d = cv.take<double>(sz[2] / 8);
    int64_t *best_c = cv.take<int64_t>(sz[3] / 8);
    uint32_t *cnt = cv.take<uint32_t>(sz[4] / 4);
    double *T = cv.take<double>(sz[5] / 8);
    double *Dj = cv.take<double>(sz[6] / 8);
    uint32_t *stats = cv.take<uint32_t>(kStatWords);
    void *B0 = cv.take<char>(sz[8]);
    void *B1 = cv.take<char>(sz[9]);
    float *cmarg = cv.take<float>(sz[10] / 4);
    uint64_t *queue = cv.take<uint64_t>(sz[11] / 8);
    uint32_t *qctl = cv.take<uint32_t>(16);  // [0] queue length, [1] overflow flag
    float *S32 = cv.take<float>(sz[13] / 4);
    double *cq = cv.take<double>(sz[14] / 8);
    double *eq = cv.take<double>(sz[15] / 8);
    void *P0 = cv.take<char>(sz[16]);
    void *P1 = cv.take<char>(sz[17]);
    float *pmarg = cv.take<float>(sz[18] / 4);
    float *lam = cv.take<float>(sz[19] / 4);
    float *mu = cv.take<float>(sz[20] / 4);
    uint32_t *lists = cv.take<uint32_t>(sz[21] / 4);
    uint32_t *lcount = cv.take<uint32_t>(sz[22] / 4);
    uint32_t *base = cv.take<uint32_t>(sz[23] / 4);
    uint32_t *offs = cv.take<uint32_t>(sz[24] / 4);
    uint32_t *items = cv.take<uint32_t>(sz[25] / 4);
    double *UR = p.sign ? cv.take<double>(sz[26] / 8) : nullptr;
    const int64_t npad_pole = p.cull ? mfma_col_pad(qb) : 0;
    // Culling at refinement l decides the points whose angle to the pole's
    // hyperplane exceeds the cap's half-angle eps_l; for data spread over d
    // dimensions that angle's sine is about |N(0,1)| / sqrt(d), so caps with
    // sin(eps_l) > 3 / sqrt(d) decide almost nothing and the cull pass is
    // skipped there (the dense GEMM follows either way).  RRS_CULL_ANGLE
    // overrides the largest half-angle.
    const double cull_angle = env_double(
        "RRS_CULL_ANGLE", asin(fmin(1.0, 3.0 / sqrt((double)(d > 0 ? d : 1)))));
    // lists when their matrix-core work is below this percent of the dense
    // GEMM's (RRS_LIST_PCT: 0 always dense, 1000 always lists)
    const int list_pct = (int)env_double("RRS_LIST_PCT", 80.0);
    if (stats_out) *stats_out = stats;
    if (profiling) RRS_HIP_TRY(launch_fill_u32(stats, kStatWords, 0u, st));

    // zero the direction padding once (the generator writes j < m only)
    RRS_HIP_TRY(launch_fill_u32((uint32_t *)UT, qb * d * ldm * 2, 0u, st));
    for (int64_t q0 = 0; q0 < nq; q0 += qb) {
        const int64_t nb = (nq - q0 < qb) ? nq - q0 : qb;
        const double *Zb = io.Z + q0 * d;
        RRS_HIP_TRY(launch_init_state(nb, d, n, pole, best_d, best_c, st));
        double phi = 1.0;
        for (int32_t l = 1; l <= r; ++l) {
            const double proj_units = (double)nb * (double)m * (double)n;
            GenArgs ga{d, m, ldm, nb, l, phi, s.seed, (uint64_t)(s.qoff + q0), pole, UT,
                       s.first_cap ? 1 : 0, s.area_cap ? 1 : 0, (half && mfma && p.sign) ? UR : nullptr};
            {
                ProfScope ps(prof, K_GEN, (double)nb * m * d, st);
                RRS_HIP_TRY(launch_gen_dirs(ga, st));
            }
            ProjArgs pa{D.XT, D.ldx, n, d, Zb, UT, ldm, m, nb, cnt, T, nullptr};
            if (half && mfma && p.sign) {
                // bfloat16 form: persistent sign GEMM, with the points of
                // refinements l >= 2 culled against each query's cap first
                RRS_HIP_TRY(launch_fill_u32(qctl, 16, 0u, st));
                RRS_HIP_TRY(launch_mfma_dirs(p.prec, true, UT, d, m, ldm, nb * m, npad, Zb, D.xbar,
                                             B0, B1, cmarg, D.amax, nullptr, nullptr, st));
                SignArgs sa{n,     d,     D.A0,  D.A1,   D.anorm, B0,     B1,     cmarg,
                            npad,  m,     ldm,   nb,     cnt,     queue,  qctl,   p.qcap,
                            UT,    UR,    Zb,    nullptr, nullptr, nullptr, nullptr, nullptr,
                            p.rpi};
                const bool cull_l = p.cull && l >= 2 && 1.5707963267948966 * phi <= cull_angle;
                if (cull_l) {
                    RRS_HIP_TRY(launch_mfma_dirs(p.prec, true, pole, d, 1, 1, nb, npad_pole, Zb,
                                                 D.xbar, P0, P1, pmarg, D.amax, nullptr, nullptr,
                                                 st));
                    CullArgs ca{pole,  D.xbar, P0,     P1,   pmarg,
                                npad_pole, lam, mu,   lists, lcount,
                                base,  offs,  items, qctl + 4, list_pct,
                                profiling ? (unsigned long long *)(stats + 6) : nullptr};
                    {
                        ProfScope ps(prof, K_CULL, (double)nb * (double)n, st);
                        RRS_HIP_TRY(launch_cull(sa, ca, st));
                    }
                    sa.lists = lists;
                    sa.lcount = lcount;
                    sa.offs = offs;
                    sa.items = items;
                    sa.mode = qctl + 4;
                } else {
                    RRS_HIP_TRY(launch_fill_u32(cnt, nb * ldm * 2, 0u, st));
                    if (profiling) prof->gemm_pairs += proj_units;
                }
                {
                    ProfScope ps(prof, K_MFMA, proj_units, st);
                    RRS_HIP_TRY(launch_sign(sa, st));
                }
                {
                    ProfScope ps(prof, K_RECHECK, 0.0, st);
                    RRS_HIP_TRY(launch_block_recheck(
                        sa, D.X, profiling ? (uint64_t *)(stats + 4) : nullptr, st));
                }
                // queue overflow (never expected): recount in binary64
                RRS_HIP_TRY(launch_queue_overflow(qctl, kSignQueueOverflow - 1u, cnt,
                                                  nb * ldm * 2, qctl + 1, st));
                pa.only_if = qctl + 1;
                RRS_HIP_TRY(launch_proj_f64(pa, true, st));
            } else if (half && mfma) {
                RRS_HIP_TRY(launch_fill_u32(cnt, nb * ldm * 2, 0u, st));
                RRS_HIP_TRY(launch_fill_u32(qctl, 16, 0u, st));
                RRS_HIP_TRY(launch_mfma_dirs(p.prec, true, UT, d, m, ldm, nb * m, npad, Zb, D.xbar,
                                             B0, B1, cmarg, D.amax, nullptr, nullptr, st));
                MfmaArgs ma{p.prec, D.A0,   D.A1,   D.anorm, n,    d,    B0,
                            B1,     cmarg,  m,      ldm,     npad, nb,   cnt,
                            queue,  qctl,   p.qcap, qctl + 1, D.X, Zb,   UT,
                            profiling ? (uint64_t *)(stats + 4) : nullptr};
                {
                    ProfScope ps(prof, K_MFMA, proj_units, st);
                    RRS_HIP_TRY(launch_mfma_gemm(ma, st));
                }
                if (p.prec != MFMA_F32_PLAIN) {
                    {
                        ProfScope ps(prof, K_RECHECK, 0.0, st);
                        RRS_HIP_TRY(launch_mfma_recheck(ma, st));
                    }
                    // queue overflow (never expected): recount in binary64
                    pa.only_if = qctl + 1;
                    RRS_HIP_TRY(launch_proj_f64(pa, true, st));
                }
            } else if (mfma) {
                // projection / APD from binary32 projections on the matrix cores
                RRS_HIP_TRY(launch_mfma_dirs(p.prec, false, UT, d, m, ldm, nb * m, npad, Zb,
                                             D.xbar, B0, B1, nullptr, D.amax, cq, eq, st, D.pp));
                {
                    ProfScope ps(prof, K_MFMA, proj_units, st);
                    RRS_HIP_TRY(launch_mfma_store(p.prec, D.A0, D.A1, n, d, B0, B1, m, nb * m,
                                                  npad, S32, st));
                }
                SelectRcArgs ra{S32, n, m, ldm, nb, cq, eq, D.X, d, Zb, UT, Dj,
                                profiling ? stats : nullptr, D.anorm, D.pp,
                                mfma_point_alpha(p.prec, d)};
                ProfScope ps(prof, K_SELECT, proj_units, st);
                if (profiling) prof->sel_total += 2.0 * (double)(nb * m);
                RRS_HIP_TRY(launch_select_rc(ra, s.notion, p.prec != MFMA_F32_PLAIN, st));
            } else if (half) {
                RRS_HIP_TRY(launch_fill_u32(cnt, nb * ldm * 2, 0u, st));
                ProfScope ps(prof, K_PROJ, proj_units, st);
                RRS_HIP_TRY(launch_proj_f64(pa, true, st));
            } else {
                {
                    ProfScope ps(prof, K_PROJ, proj_units, st);
                    RRS_HIP_TRY(launch_proj_f64(pa, false, st));
                }
                SelectArgs sa{T, n, m, ldm, nb, Dj, profiling ? stats : nullptr};
                ProfScope ps(prof, K_SELECT, proj_units, st);
                if (profiling) prof->sel_total += 2.0 * (double)(nb * m);
                if (n <= select_reg_max_n())
                    RRS_HIP_TRY(launch_select_reg(sa, s.notion, st));
                else
                    RRS_HIP_TRY(launch_select_stream(sa, s.notion, st));
            }
            ArgminArgs aa{m, ldm, d, nb, cnt, Dj, UT, pole, best_d, best_c,
                          io.trace ? io.trace + q0 * r * 3 : nullptr, l, r};
            {
                ProfScope ps(prof, K_ARGMIN, (double)nb * m, st);
                RRS_HIP_TRY(launch_argmin(aa, half, st));
            }
            phi = phi * s.alpha;
        }
        RRS_HIP_TRY(launch_finalize(nb, d, n, half, pole, best_d, best_c, io.depth + q0,
                                    io.count ? io.count + q0 : nullptr,
                                    io.poles ? io.poles + q0 * d : nullptr, st));
    }
    return RRS_OK;
}

}  // namespace rrs
