// rrs_api.hip -- the C ABI of librrs (declared in include/rrs.h).
//
// Host side of one call: validate, stage inputs on the device, then for each
// batch of queries run the RRS refinement loop of Alg. 4 / Alg. S5 --
// directions, projection, univariate depth, argmin and pole update -- on one
// HIP stream, and write the per-query results.  The refinement chain stays on
// the device; the host only enqueues kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rrs.h"
#include "rrs_launch.hpp"

namespace {

thread_local std::string g_last_error;
std::mutex g_mutex;

rrs_status fail(rrs_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

// Per-device workspace: one arena, grown on demand, carved per call.
struct Arena {
    void *base = nullptr;
    size_t cap = 0;
};
std::map<int, Arena> g_arenas;

struct Carver {
    char *p;
    size_t off = 0;
    explicit Carver(void *b) : p((char *)b) {}
    template <class T>
    T *take(size_t count)
    {
        off = (off + 255) & ~(size_t)255;
        T *r = (T *)(p + off);
        off += count * sizeof(T);
        return r;
    }
};

size_t carve_size(const size_t *sizes, int k)
{
    size_t off = 0;
    for (int i = 0; i < k; ++i) {
        off = (off + 255) & ~(size_t)255;
        off += sizes[i];
    }
    return off + 256;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t _e = (expr);                                                          \
        if (_e != hipSuccess)                                                            \
            return fail(_e == hipErrorOutOfMemory ? RRS_E_NOMEM : RRS_E_DEVICE,          \
                        "%s failed: %s", #expr, hipGetErrorString(_e));                  \
    } while (0)

rrs_status ensure_arena(int dev, size_t need, void **out)
{
    Arena &a = g_arenas[dev];
    if (a.cap < need) {
        if (a.base) {
            HIP_TRY(hipDeviceSynchronize());
            HIP_TRY(hipFree(a.base));
            a.base = nullptr;
            a.cap = 0;
        }
        size_t cap = need + need / 8;
        hipError_t e = hipMalloc(&a.base, cap);
        if (e != hipSuccess) {
            a.base = nullptr;
            e = hipMalloc(&a.base, need);
            if (e != hipSuccess) {
                a.base = nullptr;
                return fail(RRS_E_NOMEM, "hipMalloc of %zu bytes failed: %s", need,
                            hipGetErrorString(e));
            }
            cap = need;
        }
        a.cap = cap;
    }
    *out = a.base;
    return RRS_OK;
}

// Optional per-kernel timing: HIP events recorded around every launch on the
// launch stream, read back once the call has synchronised the stream.
enum { K_GEN = 0, K_PROJ, K_SELECT, K_ARGMIN, K_MFMA, K_OTHER, K_COUNT };
const char *const kKernelNames[K_COUNT] = {"k_gen_dirs", "k_proj_f64", "k_select",
                                           "k_argmin_pole", "k_gemm_sign", "k_misc"};
struct ProfRec {
    int kind;
    hipEvent_t a, b;
    double work;
};
struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<ProfRec> recs;
    int64_t launches[K_COUNT] = {};
    double ms[K_COUNT] = {};
    double work[K_COUNT] = {};
    double sel_fast = 0.0, sel_fallback = 0.0;
    hipEvent_t get()
    {
        if (used == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
};
Profiler g_prof;

struct ProfScope {
    ProfRec rec{};
    hipStream_t st;
    bool live = false;
    ProfScope(int kind, double work, hipStream_t s) : st(s)
    {
        if (!g_prof.on) return;
        rec.kind = kind;
        rec.work = work;
        rec.a = g_prof.get();
        rec.b = g_prof.get();
        if (rec.a && rec.b && hipEventRecord(rec.a, st) == hipSuccess) live = true;
    }
    ~ProfScope()
    {
        if (live && hipEventRecord(rec.b, st) == hipSuccess) g_prof.recs.push_back(rec);
    }
};

void prof_collect()
{
    for (const ProfRec &r : g_prof.recs) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            g_prof.launches[r.kind] += 1;
            g_prof.ms[r.kind] += ms;
            g_prof.work[r.kind] += r.work;
        }
    }
    g_prof.recs.clear();
    g_prof.used = 0;
}

bool all_finite(const double *p, int64_t count)
{
    for (int64_t i = 0; i < count; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

rrs_status run(int notion, const double *X, int64_t n, int64_t d, const double *Z, int64_t nq,
               int64_t K, int32_t r, double alpha, uint64_t seed, double *depth,
               int64_t *count, const rrs_opts *opts)
{
    rrs_opts o{};
    if (opts) o = *opts;
    if (nq < 0) return fail(RRS_E_INVAL, "number of queries must be >= 0 (got %lld)", (long long)nq);
    if (nq == 0) return RRS_OK;
    if (!X || !Z || !depth) return fail(RRS_E_INVAL, "X, Z and depth must be non-NULL");
    if (n < 1) return fail(RRS_E_INVAL, "n must be >= 1 (got %lld)", (long long)n);
    if (d < 2) return fail(RRS_E_INVAL, "d must be >= 2 (got %lld)", (long long)d);
    if (K < 1) return fail(RRS_E_INVAL, "K must be >= 1 (got %lld)", (long long)K);
    if (r < 1) return fail(RRS_E_INVAL, "n_refine must be >= 1 (got %d)", r);
    if (!(alpha > 0.0 && alpha <= 1.0))
        return fail(RRS_E_INVAL, "cap_shrink must be in (0, 1] (got %g)", alpha);
    if (o.precision != RRS_F64 && o.precision != RRS_BF16_RECHECK)
        return fail(RRS_E_INVAL, "unknown precision %d", o.precision);
    const bool mfma = o.precision == RRS_BF16_RECHECK;
    if (mfma && notion != rrs::NOTION_HALFSPACE)
        return fail(RRS_E_INVAL, "precision RRS_BF16_RECHECK is available for halfspace depth only");
    if (mfma && ((K + r - 1) / r >= 65536 || nq > 65535))
        return fail(RRS_E_INVAL,
                    "precision RRS_BF16_RECHECK needs ceil(K/n_refine) < 65536 directions");
    if (n > 0x7FFFFFFFLL || d > 0x7FFFFFFFLL)
        return fail(RRS_E_INVAL, "n and d must fit in 31 bits");
    if (o.query_offset < 0) return fail(RRS_E_INVAL, "query_offset must be >= 0");
    const bool dev_ptrs = o.device_ptrs != 0;
    if (!dev_ptrs) {
        if (!all_finite(X, n * d)) return fail(RRS_E_INVAL, "X holds a non-finite value");
        if (!all_finite(Z, nq * d)) return fail(RRS_E_INVAL, "Z holds a non-finite value");
    }

    std::lock_guard<std::mutex> lock(g_mutex);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipStream_t st = (hipStream_t)o.stream;

    const bool half = notion == rrs::NOTION_HALFSPACE;
    const int64_t m = (K + r - 1) / r;
    if (m > 0x7FFFFFFFLL) return fail(RRS_E_INVAL, "ceil(K / n_refine) too large");
    const int64_t ldm = (m + rrs::kProjJT - 1) / rrs::kProjJT * rrs::kProjJT;
    const int64_t ldx = (n + 511) / 512 * 512;

    // batch size: per-query scratch must fit the workspace limit
    size_t limit = o.workspace_limit ? o.workspace_limit : ((size_t)16 << 30);
    size_t freeb = 0, totb = 0;
    if (hipMemGetInfo(&freeb, &totb) == hipSuccess && freeb > ((size_t)2 << 30)) {
        const size_t cap = (freeb - ((size_t)1 << 30)) / 10 * 8;
        if (limit > cap) limit = cap;
    }
    // matrix-core form: split operands, K padded to 16, directions to 64
    const int64_t kp = mfma ? rrs::mfma_kpad(d) : 0;
    const int64_t ldb = (m + rrs::kMfmaCols - 1) / rrs::kMfmaCols * rrs::kMfmaCols;
    size_t per_q = (size_t)d * ldm * 8 + (size_t)d * 8 + 16;
    if (half)
        per_q += (size_t)ldm * 8;
    else
        per_q += (size_t)m * n * 8 + (size_t)ldm * 8;
    if (mfma) per_q += (size_t)ldb * kp * 4 + (size_t)ldb * 4 + (size_t)m * n * 8 / 100;
    int64_t qb = (int64_t)(limit / per_q);
    if (qb < 1) qb = 1;
    if (qb > nq) qb = nq;
    if (qb > 65535) qb = 65535;
    // recheck queue: 1% of the pairs of a launch, at least 1M entries
    uint64_t qcap = (uint64_t)qb * (uint64_t)m * (uint64_t)n / 100;
    if (qcap < (1u << 20)) qcap = 1u << 20;
    if (qcap > 0xFFFFFFF0ull) qcap = 0xFFFFFFF0ull;

    // workspace layout
    const bool stage_in = !dev_ptrs;
    size_t sizes[22];
    int k = 0;
    sizes[k++] = (size_t)d * ldx * 8;                          // XT
    sizes[k++] = stage_in ? (size_t)n * d * 8 : 0;             // X staging
    sizes[k++] = stage_in ? (size_t)nq * d * 8 : 0;            // Z staging
    sizes[k++] = (size_t)qb * d * ldm * 8;                     // UT
    sizes[k++] = (size_t)qb * d * 8;                           // pole
    sizes[k++] = (size_t)qb * 8;                               // best_d
    sizes[k++] = (size_t)qb * 8;                               // best_c
    sizes[k++] = half ? (size_t)qb * ldm * 2 * 4 : 0;          // cnt
    sizes[k++] = half ? 0 : (size_t)qb * m * n * 8;            // T
    sizes[k++] = half ? 0 : (size_t)qb * ldm * 8;              // Dj
    const bool want_trace = o.trace != nullptr, want_poles = o.poles != nullptr;
    sizes[k++] = stage_in ? (size_t)nq * (8 + 8 + (want_poles ? d * 8 : 0)) : 0;  // outputs
    sizes[k++] = (stage_in && want_trace) ? (size_t)nq * r * 3 * 8 : 0;         // trace
    sizes[k++] = 64;                                                             // stats
    sizes[k++] = mfma ? (size_t)d * 8 : 0;                                       // xbar
    sizes[k++] = mfma ? (size_t)n * kp * 2 : 0;                                  // Ahi
    sizes[k++] = mfma ? (size_t)n * kp * 2 : 0;                                  // Alo
    sizes[k++] = mfma ? (size_t)n * 4 : 0;                                       // anorm
    sizes[k++] = mfma ? (size_t)qb * ldb * kp * 2 : 0;                           // Bhi
    sizes[k++] = mfma ? (size_t)qb * ldb * kp * 2 : 0;                           // Blo
    sizes[k++] = mfma ? (size_t)qb * ldb * 4 : 0;                                // cmarg
    sizes[k++] = mfma ? (size_t)qcap * 8 : 0;                                    // queue
    sizes[k++] = 64;                                                             // qcount, flag
    void *base = nullptr;
    rrs_status s = ensure_arena(dev, carve_size(sizes, k), &base);
    if (s != RRS_OK) return s;
    Carver cv(base);
    double *XT = cv.take<double>((size_t)d * ldx);
    double *Xs = cv.take<double>(stage_in ? (size_t)n * d : 0);
    double *Zs = cv.take<double>(stage_in ? (size_t)nq * d : 0);
    double *UT = cv.take<double>((size_t)qb * d * ldm);
    double *pole = cv.take<double>((size_t)qb * d);
    double *best_d = cv.take<double>((size_t)qb);
    int64_t *best_c = cv.take<int64_t>((size_t)qb);
    uint32_t *cnt = cv.take<uint32_t>(half ? (size_t)qb * ldm * 2 : 0);
    double *T = cv.take<double>(half ? 0 : (size_t)qb * m * n);
    double *Dj = cv.take<double>(half ? 0 : (size_t)qb * ldm);
    double *out_depth = cv.take<double>(stage_in ? (size_t)nq : 0);
    int64_t *out_count = cv.take<int64_t>(stage_in ? (size_t)nq : 0);
    double *out_poles = cv.take<double>((stage_in && want_poles) ? (size_t)nq * d : 0);
    int64_t *out_trace = cv.take<int64_t>((stage_in && want_trace) ? (size_t)nq * r * 3 : 0);
    uint32_t *stats = cv.take<uint32_t>(16);
    double *xbar = cv.take<double>(mfma ? (size_t)d : 0);
    __bf16 *Ahi = cv.take<__bf16>(mfma ? (size_t)n * kp : 0);
    __bf16 *Alo = cv.take<__bf16>(mfma ? (size_t)n * kp : 0);
    float *anorm = cv.take<float>(mfma ? (size_t)n : 0);
    __bf16 *Bhi = cv.take<__bf16>(mfma ? (size_t)qb * ldb * kp : 0);
    __bf16 *Blo = cv.take<__bf16>(mfma ? (size_t)qb * ldb * kp : 0);
    float *cmarg = cv.take<float>(mfma ? (size_t)qb * ldb : 0);
    uint64_t *queue = cv.take<uint64_t>(mfma ? (size_t)qcap : 0);
    uint32_t *qctl = cv.take<uint32_t>(16);  // [0] queue length, [1] overflow flag
    if (g_prof.on) HIP_TRY(rrs::launch_fill_u32(stats, 16, 0u, st));

    const double *Xd = X, *Zd = Z;
    double *depth_d = depth;
    int64_t *count_d = count;
    double *poles_d = o.poles;
    int64_t *trace_d = o.trace;
    if (stage_in) {
        HIP_TRY(hipMemcpyAsync(Xs, X, (size_t)n * d * 8, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(Zs, Z, (size_t)nq * d * 8, hipMemcpyHostToDevice, st));
        Xd = Xs;
        Zd = Zs;
        depth_d = out_depth;
        count_d = count ? out_count : nullptr;
        poles_d = want_poles ? out_poles : nullptr;
        trace_d = want_trace ? out_trace : nullptr;
    }
    HIP_TRY(rrs::launch_transpose(Xd, n, d, ldx, XT, st));
    if (mfma) HIP_TRY(rrs::launch_mfma_prep(Xd, n, d, xbar, Ahi, Alo, anorm, st));
    // zero the direction padding once (the generator writes j < m only)
    HIP_TRY(rrs::launch_fill_u32((uint32_t *)UT, qb * d * ldm * 2, 0u, st));

    const bool lds = !half && n <= rrs::select_lds_max_n(dev);
    for (int64_t q0 = 0; q0 < nq; q0 += qb) {
        const int64_t nb = (nq - q0 < qb) ? nq - q0 : qb;
        HIP_TRY(rrs::launch_init_state(nb, d, n, pole, best_d, best_c, st));
        double phi = 1.0;
        for (int32_t l = 1; l <= r; ++l) {
            const double proj_units = (double)nb * (double)m * (double)n;
            rrs::GenArgs ga{d, m, ldm, nb, l, phi, seed, (uint64_t)(o.query_offset + q0), pole, UT};
            {
                ProfScope ps(K_GEN, (double)nb * m * d, st);
                HIP_TRY(rrs::launch_gen_dirs(ga, st));
            }
            rrs::ProjArgs pa{XT, ldx, n, d, Zd + q0 * d, UT, ldm, m, nb, cnt, T, nullptr};
            if (half && mfma) {
                HIP_TRY(rrs::launch_fill_u32(cnt, nb * ldm * 2, 0u, st));
                HIP_TRY(rrs::launch_fill_u32(qctl, 16, 0u, st));
                HIP_TRY(rrs::launch_mfma_dirs(UT, d, m, ldm, ldb, nb, Zd + q0 * d, xbar, Bhi, Blo,
                                              cmarg, st));
                rrs::MfmaArgs ma{Ahi,  Alo,    anorm, n,    d,      Bhi,     Blo,
                                 cmarg, m,     ldm,   ldb,  nb,     cnt,     queue,
                                 qctl, qcap,   qctl + 1, Xd, Zd + q0 * d, UT};
                {
                    ProfScope ps(K_MFMA, proj_units, st);
                    HIP_TRY(rrs::launch_mfma_count(ma, st));
                }
                // queue overflow (never expected): recount in binary64
                pa.only_if = qctl + 1;
                HIP_TRY(rrs::launch_proj_f64(pa, true, st));
            } else if (half) {
                HIP_TRY(rrs::launch_fill_u32(cnt, nb * ldm * 2, 0u, st));
                ProfScope ps(K_PROJ, proj_units, st);
                HIP_TRY(rrs::launch_proj_f64(pa, true, st));
            } else {
                {
                    ProfScope ps(K_PROJ, proj_units, st);
                    HIP_TRY(rrs::launch_proj_f64(pa, false, st));
                }
                rrs::SelectArgs sa{T, n, m, ldm, nb, Dj, g_prof.on ? stats : nullptr};
                ProfScope ps(K_SELECT, proj_units, st);
                if (n <= rrs::select_reg_max_n())
                    HIP_TRY(rrs::launch_select_reg(sa, notion, st));
                else
                    HIP_TRY(rrs::launch_select(sa, notion, lds, st));
            }
            rrs::ArgminArgs aa{m, ldm, d, nb, cnt, Dj, UT, pole, best_d, best_c,
                               trace_d ? trace_d + q0 * r * 3 : nullptr, l, r};
            {
                ProfScope ps(K_ARGMIN, (double)nb * m, st);
                HIP_TRY(rrs::launch_argmin(aa, half, st));
            }
            phi = phi * alpha;
        }
        HIP_TRY(rrs::launch_finalize(nb, d, n, half, pole, best_d, best_c, depth_d + q0,
                                     count_d ? count_d + q0 : nullptr,
                                     poles_d ? poles_d + q0 * d : nullptr, st));
    }
    if (stage_in) {
        HIP_TRY(hipMemcpyAsync(depth, out_depth, (size_t)nq * 8, hipMemcpyDeviceToHost, st));
        if (count)
            HIP_TRY(hipMemcpyAsync(count, out_count, (size_t)nq * 8, hipMemcpyDeviceToHost, st));
        if (want_poles)
            HIP_TRY(hipMemcpyAsync(o.poles, out_poles, (size_t)nq * d * 8, hipMemcpyDeviceToHost,
                                   st));
        if (want_trace)
            HIP_TRY(hipMemcpyAsync(o.trace, out_trace, (size_t)nq * r * 3 * 8,
                                   hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    if (g_prof.on) {
        prof_collect();
        uint32_t hs[2] = {0, 0};
        HIP_TRY(hipMemcpy(hs, stats, sizeof(hs), hipMemcpyDeviceToHost));
        g_prof.sel_fast += hs[0];
        g_prof.sel_fallback += hs[1];
    }
    return RRS_OK;
}

}  // namespace

extern "C" {

rrs_status rrs_depth_halfspace(const double *X, int64_t n, int64_t d, const double *Z, int64_t m,
                               int64_t K, int32_t n_refine, double cap_shrink, uint64_t seed,
                               double *depth, int64_t *count, const rrs_opts *opts)
{
    return run(rrs::NOTION_HALFSPACE, X, n, d, Z, m, K, n_refine, cap_shrink, seed, depth, count,
               opts);
}

rrs_status rrs_depth_projection(const double *X, int64_t n, int64_t d, const double *Z,
                                int64_t m, int64_t K, int32_t n_refine, double cap_shrink,
                                uint64_t seed, double *depth, const rrs_opts *opts)
{
    return run(rrs::NOTION_PROJECTION, X, n, d, Z, m, K, n_refine, cap_shrink, seed, depth,
               nullptr, opts);
}

rrs_status rrs_depth_apd(const double *X, int64_t n, int64_t d, const double *Z, int64_t m,
                         int64_t K, int32_t n_refine, double cap_shrink, uint64_t seed,
                         double *depth, const rrs_opts *opts)
{
    return run(rrs::NOTION_APD, X, n, d, Z, m, K, n_refine, cap_shrink, seed, depth, nullptr,
               opts);
}

const char *rrs_last_error(void) { return g_last_error.c_str(); }

rrs_status rrs_release_workspace(void)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) cur = 0;
    for (auto &kv : g_arenas) {
        if (kv.second.base) {
            if (hipSetDevice(kv.first) == hipSuccess) {
                (void)hipDeviceSynchronize();
                (void)hipFree(kv.second.base);
            }
        }
    }
    g_arenas.clear();
    (void)hipSetDevice(cur);
    return RRS_OK;
}

int32_t rrs_version(void) { return 100; }

rrs_status rrs_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    g_prof.on = on != 0;
    g_prof.recs.clear();
    g_prof.used = 0;
    for (int k = 0; k < K_COUNT; ++k) {
        g_prof.launches[k] = 0;
        g_prof.ms[k] = 0.0;
        g_prof.work[k] = 0.0;
    }
    g_prof.sel_fast = 0.0;
    g_prof.sel_fallback = 0.0;
    return RRS_OK;
}

int32_t rrs_profile_counter(const char *name, double *value)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!name || !value) return -1;
    if (std::strcmp(name, "select_fast") == 0) {
        *value = g_prof.sel_fast;
        return 0;
    }
    if (std::strcmp(name, "select_fallback") == 0) {
        *value = g_prof.sel_fallback;
        return 0;
    }
    return -1;
}

int32_t rrs_profile_read(rrs_kernel_stat *out, int32_t max_entries)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    int32_t k = 0;
    for (int i = 0; i < K_COUNT && k < max_entries; ++i) {
        if (!g_prof.launches[i]) continue;
        if (out) {
            std::memset(&out[k], 0, sizeof(rrs_kernel_stat));
            std::strncpy(out[k].name, kKernelNames[i], sizeof(out[k].name) - 1);
            out[k].launches = g_prof.launches[i];
            out[k].total_ms = g_prof.ms[i];
            out[k].work_units = g_prof.work[i];
        }
        ++k;
    }
    return k;
}

rrs_status rrs_debug_directions(int64_t d, int64_t m_dir, int32_t l, double phi, uint64_t seed,
                                uint64_t q, const double *pole, double *out)
{
    if (d < 2 || m_dir < 1 || l < 1 || !pole || !out)
        return fail(RRS_E_INVAL, "rrs_debug_directions: invalid arguments");
    std::lock_guard<std::mutex> lock(g_mutex);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    const int64_t ldm = (m_dir + rrs::kProjJT - 1) / rrs::kProjJT * rrs::kProjJT;
    size_t sizes[2] = {(size_t)d * ldm * 8, (size_t)d * 8};
    void *base = nullptr;
    rrs_status s = ensure_arena(dev, carve_size(sizes, 2), &base);
    if (s != RRS_OK) return s;
    Carver cv(base);
    double *UT = cv.take<double>((size_t)d * ldm);
    double *pd = cv.take<double>((size_t)d);
    HIP_TRY(hipMemcpy(pd, pole, (size_t)d * 8, hipMemcpyHostToDevice));
    rrs::GenArgs ga{d, m_dir, ldm, 1, l, phi, seed, q, pd, UT};
    HIP_TRY(rrs::launch_gen_dirs(ga, 0));
    double *host = new double[(size_t)d * ldm];
    hipError_t e = hipMemcpy(host, UT, (size_t)d * ldm * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) {
        for (int64_t j = 0; j < m_dir; ++j)
            for (int64_t c = 0; c < d; ++c) out[j * d + c] = host[c * ldm + j];
    }
    delete[] host;
    HIP_TRY(e);
    return RRS_OK;
}

}  // extern "C"
