// rrs_api.hip -- the synchronous C entry points of librrs (include/rrs.h).
//
// Host side of one call: validate, stage inputs on the device, prepare the
// data set, enqueue the job (rrs_engine.hip) on the caller's stream and wait
// for it.  Device memory comes from one per-device arena that grows on demand.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>

#include "../../include/rrs.h"
#include "rrs_engine.hpp"

using rrs::fail;

namespace {

std::mutex g_mutex;
rrs::Profiler g_prof;

struct Arena {
    void *base = nullptr;
    size_t cap = 0;
};
std::map<int, Arena> g_arenas;

// Captured calls (RRS_FLAG_GRAPH), keyed by every argument that shapes the
// captured work, including the pointers the kernels were given.
struct GraphKey {
    int64_t v[20];
    bool operator<(const GraphKey &o) const
    {
        return std::lexicographical_compare(v, v + 20, o.v, o.v + 20);
    }
};
std::map<GraphKey, hipGraphExec_t> g_graphs;

// The library's extra streams per device (default priority) and their fork /
// join events: a large call runs its queries in kMaxParts parts concurrently.
constexpr int kMaxParts = 4;
struct Side {
    hipStream_t st[kMaxParts - 1] = {};
    hipEvent_t fork = nullptr, join[kMaxParts - 1] = {};
};
std::map<int, Side> g_side;

rrs_status side_streams(int dev, Side **out)
{
    Side &sd = g_side[dev];
    if (!sd.fork) {
        RRS_HIP_TRY(hipEventCreateWithFlags(&sd.fork, hipEventDisableTiming));
        for (int i = 0; i < kMaxParts - 1; ++i) {
            RRS_HIP_TRY(hipStreamCreateWithFlags(&sd.st[i], hipStreamNonBlocking));
            RRS_HIP_TRY(hipEventCreateWithFlags(&sd.join[i], hipEventDisableTiming));
        }
    }
    *out = &sd;
    return RRS_OK;
}

// Calls with at least this many projections per refinement (queries x
// directions x points) split their queries into parts on separate streams;
// RRS_SPLIT_WORK overrides the threshold (tests force the split with 1) and
// RRS_SPLIT_PARTS the number of parts (1 .. 4).  Default: four for halfspace
// depth (concurrent sign GEMMs keep the matrix cores busier: -15% on a
// 1e5 x 100 data set); none for projection / APD depth, where a projection
// GEMM beside a select gained under 2%.
constexpr double kSplitWork = 268435456.0;

double split_work()
{
    const char *e = std::getenv("RRS_SPLIT_WORK");
    return (e && *e) ? std::atof(e) : kSplitWork;
}

int split_parts(int notion, int precision)
{
    // the bfloat16 halfspace form runs a persistent GEMM that fills the chip
    // by itself; the other halfspace forms gain from concurrent GEMMs
    const char *e = std::getenv("RRS_SPLIT_PARTS");
    const int dflt =
        (notion == rrs::NOTION_HALFSPACE && precision != RRS_BF16_RECHECK) ? 4 : 1;
    const int p = (e && *e) ? std::atoi(e) : dflt;
    return p < 1 ? 1 : (p > kMaxParts ? kMaxParts : p);
}

void drop_graphs()
{
    for (auto &kv : g_graphs) (void)hipGraphExecDestroy(kv.second);
    g_graphs.clear();
}

rrs_status ensure_arena(int dev, size_t need, void **out)
{
    Arena &a = g_arenas[dev];
    if (a.cap < need) {
        drop_graphs();  // they point into the arena
        if (a.base) {
            RRS_HIP_TRY(hipDeviceSynchronize());
            RRS_HIP_TRY(hipFree(a.base));
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
    rrs::JobSpec s;
    s.notion = notion;
    s.precision = o.precision;
    s.nq = nq;
    s.K = K;
    s.r = r;
    s.alpha = alpha;
    s.seed = seed;
    s.qoff = o.query_offset;
    s.want_trace = o.trace != nullptr;
    if (nq < 0) return fail(RRS_E_INVAL, "number of queries must be >= 0 (got %lld)", (long long)nq);
    if (nq == 0) return RRS_OK;
    if (!X || !Z || !depth) return fail(RRS_E_INVAL, "X, Z and depth must be non-NULL");
    rrs_status vs = rrs::job_validate(s, n, d);
    if (vs != RRS_OK) return vs;
    const bool dev_ptrs = o.device_ptrs != 0;
    if (o.reserved != 0 ||
        (o.flags & ~(RRS_FLAG_GRAPH | RRS_FLAG_FIRST_CAP | RRS_FLAG_AREA_CAP)) != 0)
        return fail(RRS_E_INVAL, "unknown flags or non-zero reserved field in opts");
    s.first_cap = (o.flags & RRS_FLAG_FIRST_CAP) != 0;
    s.area_cap = (o.flags & RRS_FLAG_AREA_CAP) != 0;
    if (s.area_cap && (s.first_cap || !(alpha <= 0.99)))
        return fail(RRS_E_INVAL,
                    "RRS_FLAG_AREA_CAP needs cap_shrink <= 0.99 and no RRS_FLAG_FIRST_CAP (caps "
                    "below the hemisphere)");
    if ((o.flags & RRS_FLAG_GRAPH) && (!dev_ptrs || o.stream == nullptr))
        return fail(RRS_E_INVAL, "RRS_FLAG_GRAPH needs device pointers and a non-default stream");
    if (!dev_ptrs) {
        if (!all_finite(X, n * d)) return fail(RRS_E_INVAL, "X holds a non-finite value");
        if (!all_finite(Z, nq * d)) return fail(RRS_E_INVAL, "Z holds a non-finite value");
    }

    std::lock_guard<std::mutex> lock(g_mutex);
    int dev = 0;
    RRS_HIP_TRY(hipGetDevice(&dev));
    hipStream_t st = (hipStream_t)o.stream;

    // workspace limit: the caller's, else 16 GiB, and at most 80% of free HBM
    size_t limit = o.workspace_limit ? o.workspace_limit : ((size_t)16 << 30);
    size_t freeb = 0, totb = 0;
    if (hipMemGetInfo(&freeb, &totb) == hipSuccess && freeb > ((size_t)2 << 30)) {
        const size_t cap = (freeb - ((size_t)1 << 30)) / 10 * 8;
        if (limit > cap) limit = cap;
    }
    rrs::Plan plan;
    rrs_status ps = rrs::job_plan(s, n, d, limit, &plan);
    if (ps != RRS_OK) return ps;
    // large calls: two query halves, each with its own workspace and stream;
    // the queries' refinement chains are independent, so the projection
    // GEMM of one half overlaps the select of the other (query offsets keep
    // every direction and result unchanged)
    int parts = 1;
    int64_t qa = nq;  // queries per part (the last part takes the rest)
    if (!(o.flags & RRS_FLAG_GRAPH) && nq >= 2 &&
        (double)nq * (double)plan.m * (double)n >= split_work()) {
        int p = split_parts(notion, o.precision);
        if (p > nq) p = (int)nq;
        rrs::JobSpec sh = s;
        sh.nq = (nq + p - 1) / p;
        rrs::Plan ph;
        if (p >= 2 && rrs::job_plan(sh, n, d, limit / (size_t)p, &ph) == RRS_OK) {
            plan = ph;
            qa = sh.nq;
            parts = (int)((nq + qa - 1) / qa);
        }
    }
    const bool split = parts > 1;

    const bool stage_in = !dev_ptrs;
    const bool want_trace = o.trace != nullptr, want_poles = o.poles != nullptr;
    size_t sizes[8];
    int k = 0;
    sizes[k++] = rrs::data_bytes(n, d, plan.prec);                           // prepared data
    sizes[k++] = stage_in ? (size_t)n * d * 8 : 0;                           // X staging
    sizes[k++] = stage_in ? (size_t)nq * d * 8 : 0;                          // Z staging
    sizes[k++] = stage_in ? (size_t)nq * (8 + 8 + (want_poles ? d * 8 : 0)) : 0;  // outputs
    sizes[k++] = (stage_in && want_trace) ? (size_t)nq * r * 3 * 8 : 0;      // trace
    sizes[k++] = plan.ws_bytes;                                              // job workspace
    sizes[k++] = split ? plan.ws_bytes * (size_t)(parts - 1) : 0;           // other parts'
    void *base = nullptr;
    rrs_status as = ensure_arena(dev, rrs::carve_size(sizes, k), &base);
    if (as != RRS_OK) return as;
    rrs::Carver cv(base);
    void *data_mem = cv.take<char>(sizes[0]);
    double *Xs = cv.take<double>(stage_in ? (size_t)n * d : 0);
    double *Zs = cv.take<double>(stage_in ? (size_t)nq * d : 0);
    double *out_depth = cv.take<double>(stage_in ? (size_t)nq : 0);
    int64_t *out_count = cv.take<int64_t>(stage_in ? (size_t)nq : 0);
    double *out_poles = cv.take<double>((stage_in && want_poles) ? (size_t)nq * d : 0);
    int64_t *out_trace = cv.take<int64_t>((stage_in && want_trace) ? (size_t)nq * r * 3 : 0);
    void *ws = cv.take<char>(plan.ws_bytes);
    char *ws_rest = cv.take<char>(split ? plan.ws_bytes * (size_t)(parts - 1) : 0);

    rrs::JobIO io;
    io.Z = Z;
    io.depth = depth;
    io.count = count;
    io.poles = o.poles;
    io.trace = o.trace;
    const double *Xd = X;
    if (stage_in) {
        RRS_HIP_TRY(hipMemcpyAsync(Xs, X, (size_t)n * d * 8, hipMemcpyHostToDevice, st));
        RRS_HIP_TRY(hipMemcpyAsync(Zs, Z, (size_t)nq * d * 8, hipMemcpyHostToDevice, st));
        Xd = Xs;
        io.Z = Zs;
        io.depth = out_depth;
        io.count = count ? out_count : nullptr;
        io.poles = want_poles ? out_poles : nullptr;
        io.trace = want_trace ? out_trace : nullptr;
    }
    rrs::DataDev D;
    D.X = Xd;
    D.n = n;
    D.d = d;
    if ((o.flags & RRS_FLAG_GRAPH) && !g_prof.on) {
        // the whole device side as one graph: captured on first use, then replayed
        GraphKey key{};
        int64_t *v = key.v;
        double abits = alpha;
        int64_t ab;
        std::memcpy(&ab, &abits, sizeof(ab));
        const int64_t vals[20] = {notion,
                                  o.precision + 256 * (int64_t)s.first_cap +
                                      512 * (int64_t)s.area_cap,
                                  n, d, nq, K, r,
                                  ab, (int64_t)seed,
                                  o.query_offset, (int64_t)X, (int64_t)Z, (int64_t)depth,
                                  (int64_t)count, (int64_t)o.poles, (int64_t)o.trace,
                                  (int64_t)st, (int64_t)base, (int64_t)plan.qb, dev};
        std::memcpy(v, vals, sizeof(vals));
        auto it = g_graphs.find(key);
        if (it == g_graphs.end()) {
            RRS_HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            hipError_t pe = rrs::data_prepare(D, data_mem, plan.prec, st);
            rrs_status es = pe == hipSuccess
                                ? rrs::enqueue_job(s, D, plan, io, ws, st, nullptr, nullptr)
                                : fail(RRS_E_DEVICE, "data preparation failed: %s",
                                       hipGetErrorString(pe));
            hipGraph_t graph = nullptr;
            const hipError_t ce = hipStreamEndCapture(st, &graph);
            if (es != RRS_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return es;
            }
            RRS_HIP_TRY(ce);
            hipGraphExec_t exec = nullptr;
            const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            RRS_HIP_TRY(ie);
            it = g_graphs.emplace(key, exec).first;
        }
        RRS_HIP_TRY(hipGraphLaunch(it->second, st));
        RRS_HIP_TRY(hipStreamSynchronize(st));
        return RRS_OK;
    }
    RRS_HIP_TRY(rrs::data_prepare(D, data_mem, plan.prec, st));
    // per-point bounds for heavy-tailed data (the graph path above keeps the
    // column bound: its preparation runs inside the captured graph)
    if (notion != rrs::NOTION_HALFSPACE) RRS_HIP_TRY(rrs::data_point_bounds(D, st));
    uint32_t *pstats[kMaxParts] = {};
    rrs_status es = RRS_OK;
    if (!split) {
        es = rrs::enqueue_job(s, D, plan, io, ws, st, &g_prof, &pstats[0]);
    } else {
        Side *sd = nullptr;
        const rrs_status ss = side_streams(dev, &sd);
        if (ss != RRS_OK) return ss;
        RRS_HIP_TRY(hipEventRecord(sd->fork, st));
        for (int pi = 1; pi < parts; ++pi)
            RRS_HIP_TRY(hipStreamWaitEvent(sd->st[pi - 1], sd->fork, 0));
        for (int pi = 0; pi < parts && es == RRS_OK; ++pi) {
            const int64_t q0 = qa * pi;
            rrs::JobSpec sp = s;
            sp.nq = (pi == parts - 1) ? nq - q0 : qa;
            sp.qoff = s.qoff + q0;
            rrs::JobIO ip = io;
            ip.Z = io.Z + q0 * d;
            ip.depth = io.depth + q0;
            if (io.count) ip.count = io.count + q0;
            if (io.poles) ip.poles = io.poles + q0 * d;
            if (io.trace) ip.trace = io.trace + q0 * (int64_t)r * 3;
            void *wsp = pi == 0 ? ws : (void *)(ws_rest + plan.ws_bytes * (size_t)(pi - 1));
            es = rrs::enqueue_job(sp, D, plan, ip, wsp, pi == 0 ? st : sd->st[pi - 1], &g_prof,
                                  &pstats[pi]);
        }
        // join even after a failure: the caller's stream never runs ahead of
        // work still using the workspace
        for (int pi = 1; pi < parts; ++pi) {
            RRS_HIP_TRY(hipEventRecord(sd->join[pi - 1], sd->st[pi - 1]));
            RRS_HIP_TRY(hipStreamWaitEvent(st, sd->join[pi - 1], 0));
        }
    }
    if (es != RRS_OK) return es;
    if (stage_in) {
        RRS_HIP_TRY(hipMemcpyAsync(depth, out_depth, (size_t)nq * 8, hipMemcpyDeviceToHost, st));
        if (count)
            RRS_HIP_TRY(
                hipMemcpyAsync(count, out_count, (size_t)nq * 8, hipMemcpyDeviceToHost, st));
        if (want_poles)
            RRS_HIP_TRY(hipMemcpyAsync(o.poles, out_poles, (size_t)nq * d * 8,
                                       hipMemcpyDeviceToHost, st));
        if (want_trace)
            RRS_HIP_TRY(hipMemcpyAsync(o.trace, out_trace, (size_t)nq * r * 3 * 8,
                                       hipMemcpyDeviceToHost, st));
    }
    RRS_HIP_TRY(hipStreamSynchronize(st));
    if (g_prof.on) {
        g_prof.collect();
        for (uint32_t *sp : pstats) {
            if (!sp) continue;
            uint32_t hs[rrs::kStatWords] = {};
            RRS_HIP_TRY(hipMemcpy(hs, sp, sizeof(hs), hipMemcpyDeviceToHost));
            g_prof.sel_fallback += hs[1];
            for (int w = 0; w < 3; ++w) g_prof.shared[w] += hs[8 + w];
            uint64_t rp = 0, gp = 0;
            std::memcpy(&rp, hs + 4, sizeof(rp));
            std::memcpy(&gp, hs + 6, sizeof(gp));
            g_prof.recheck_pairs += (double)rp;
            g_prof.gemm_pairs += (double)gp;
        }
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

rrs_status rrs_depth_mahalanobis(const double *X, int64_t n, int64_t d, const double *Z,
                                 int64_t m, double *depth, const rrs_opts *opts)
{
    rrs_opts o{};
    if (opts) o = *opts;
    if (m < 0) return fail(RRS_E_INVAL, "number of queries must be >= 0 (got %lld)", (long long)m);
    if (m == 0) return RRS_OK;
    if (!X || !Z || !depth) return fail(RRS_E_INVAL, "X, Z and depth must be non-NULL");
    if (n < 1 || d < 1) return fail(RRS_E_INVAL, "need n >= 1 and d >= 1");
    if (o.reserved != 0 || o.flags != 0)
        return fail(RRS_E_INVAL, "rrs_depth_mahalanobis takes no flags");
    const bool dev_ptrs = o.device_ptrs != 0;
    if (!dev_ptrs) {
        if (!all_finite(X, n * d)) return fail(RRS_E_INVAL, "X holds a non-finite value");
        if (!all_finite(Z, m * d)) return fail(RRS_E_INVAL, "Z holds a non-finite value");
    }
    std::lock_guard<std::mutex> lock(g_mutex);
    int dev = 0;
    RRS_HIP_TRY(hipGetDevice(&dev));
    hipStream_t st = (hipStream_t)o.stream;
    size_t sizes[5];
    int k = 0;
    sizes[k++] = rrs::maha_ws_bytes(n, d, m);
    sizes[k++] = dev_ptrs ? 0 : (size_t)n * d * 8;
    sizes[k++] = dev_ptrs ? 0 : (size_t)m * d * 8;
    sizes[k++] = dev_ptrs ? 0 : (size_t)m * 8;
    void *base = nullptr;
    rrs_status as = ensure_arena(dev, rrs::carve_size(sizes, k), &base);
    if (as != RRS_OK) return as;
    rrs::Carver cv(base);
    void *ws = cv.take<char>(sizes[0]);
    double *Xs = cv.take<double>(dev_ptrs ? 0 : (size_t)n * d);
    double *Zs = cv.take<double>(dev_ptrs ? 0 : (size_t)m * d);
    double *Ds = cv.take<double>(dev_ptrs ? 0 : (size_t)m);
    const double *Xd = X, *Zd = Z;
    double *Dd = depth;
    if (!dev_ptrs) {
        RRS_HIP_TRY(hipMemcpyAsync(Xs, X, (size_t)n * d * 8, hipMemcpyHostToDevice, st));
        RRS_HIP_TRY(hipMemcpyAsync(Zs, Z, (size_t)m * d * 8, hipMemcpyHostToDevice, st));
        Xd = Xs;
        Zd = Zs;
        Dd = Ds;
    }
    uint32_t *flag = nullptr;
    RRS_HIP_TRY(rrs::maha_enqueue(Xd, n, d, Zd, m, Dd, ws, &flag, st));
    uint32_t hflag = 0;
    RRS_HIP_TRY(hipMemcpyAsync(&hflag, flag, sizeof(hflag), hipMemcpyDeviceToHost, st));
    if (!dev_ptrs)
        RRS_HIP_TRY(hipMemcpyAsync(depth, Ds, (size_t)m * 8, hipMemcpyDeviceToHost, st));
    RRS_HIP_TRY(hipStreamSynchronize(st));
    if (hflag)
        return fail(RRS_E_INVAL, "the covariance of X is not positive definite (n = %lld, d = %lld)",
                    (long long)n, (long long)d);
    return RRS_OK;
}

const char *rrs_last_error(void) { return rrs::last_error().c_str(); }

rrs_status rrs_release_workspace(void)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    drop_graphs();
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

int32_t rrs_version(void) { return 200; }

rrs_status rrs_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    g_prof.clear();
    g_prof.on = on != 0;
    return RRS_OK;
}

int32_t rrs_profile_counter(const char *name, double *value)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!name || !value) return -1;
    if (std::strcmp(name, "select_fast") == 0) {
        *value = g_prof.sel_total - g_prof.sel_fallback;
        return 0;
    }
    if (std::strcmp(name, "select_fallback") == 0) {
        *value = g_prof.sel_fallback;
        return 0;
    }
    if (std::strcmp(name, "recheck_pairs") == 0) {
        *value = g_prof.recheck_pairs;
        return 0;
    }
    if (std::strcmp(name, "gemm_pairs") == 0) {
        *value = g_prof.gemm_pairs;
        return 0;
    }
    static const char *const kShared[3] = {"shared_full", "shared_median", "shared_none"};
    for (int w = 0; w < 3; ++w)
        if (std::strcmp(name, kShared[w]) == 0) {
            *value = g_prof.shared[w];
            return 0;
        }
    return -1;
}

int32_t rrs_profile_read(rrs_kernel_stat *out, int32_t max_entries)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    int32_t k = 0;
    for (int i = 0; i < rrs::K_COUNT && k < max_entries; ++i) {
        if (!g_prof.launches[i]) continue;
        if (out) {
            std::memset(&out[k], 0, sizeof(rrs_kernel_stat));
            std::strncpy(out[k].name, rrs::kKernelNames[i], sizeof(out[k].name) - 1);
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
    RRS_HIP_TRY(hipGetDevice(&dev));
    const int64_t ldm = (m_dir + rrs::kProjJT - 1) / rrs::kProjJT * rrs::kProjJT;
    size_t sizes[2] = {(size_t)d * ldm * 8, (size_t)d * 8};
    void *base = nullptr;
    rrs_status s = ensure_arena(dev, rrs::carve_size(sizes, 2), &base);
    if (s != RRS_OK) return s;
    rrs::Carver cv(base);
    double *UT = cv.take<double>((size_t)d * ldm);
    double *pd = cv.take<double>((size_t)d);
    RRS_HIP_TRY(hipMemcpy(pd, pole, (size_t)d * 8, hipMemcpyHostToDevice));
    rrs::GenArgs ga{d, m_dir, ldm, 1, l, phi, seed, q, pd, UT};
    RRS_HIP_TRY(rrs::launch_gen_dirs(ga, 0));
    double *host = new double[(size_t)d * ldm];
    hipError_t e = hipMemcpy(host, UT, (size_t)d * ldm * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) {
        for (int64_t j = 0; j < m_dir; ++j)
            for (int64_t c = 0; c < d; ++c) out[j * d + c] = host[c * ldm + j];
    }
    delete[] host;
    RRS_HIP_TRY(e);
    return RRS_OK;
}

}  // extern "C"
