// rrs_serve.hip -- serving context: resident data sets, a device-memory
// budget with a first-fit sub-allocator, and a scheduler thread that admits
// requests into stream slots as slots and memory free up (continuous
// batching across requests: a request that arrives while others run starts as
// soon as it fits, and its kernels overlap theirs on the device).
//
// Threads: callers submit and wait from any thread; one scheduler thread per
// context makes every admission decision and enqueues every request; HIP's
// callback thread only reports completions.  The scheduler never holds the
// context lock across a HIP call, and the completion callback takes only that
// lock, so neither can block the other.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "../../include/rrs.h"
#include "rrs_engine.hpp"

using rrs::fail;

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// First-fit allocator over one device block; neighbouring free ranges are
// merged on release.  Not thread-safe (the context lock guards it).
class DevicePool {
public:
    void init(char *base, size_t cap)
    {
        base_ = base;
        cap_ = cap;
        free_.clear();
        live_.clear();
        if (cap) free_[0] = cap;
        used_ = peak_ = 0;
    }
    char *alloc(size_t bytes)
    {
        bytes = align256(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, rem = it->second - bytes;
            free_.erase(it);
            if (rem) free_[off + bytes] = rem;
            live_[off] = bytes;
            used_ += bytes;
            if (used_ > peak_) peak_ = used_;
            return base_ + off;
        }
        return nullptr;
    }
    void release(char *p)
    {
        if (!p) return;
        const size_t off = (size_t)(p - base_);
        auto lv = live_.find(off);
        if (lv == live_.end()) return;
        size_t bytes = lv->second;
        live_.erase(lv);
        used_ -= bytes;
        size_t start = off;
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && off + bytes == nx->first) {
            bytes += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                start = pv->first;
                bytes += pv->second;
                free_.erase(pv);
            }
        }
        free_[start] = bytes;
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t cap() const { return cap_; }

private:
    char *base_ = nullptr;
    size_t cap_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;  // offset -> bytes
    std::map<size_t, size_t> live_;
};

constexpr int kMaxSkips = 8;  // times a pending head may be passed over

}  // namespace

struct rrs_dataset {
    rrs_ctx *ctx = nullptr;
    int64_t n = 0, d = 0;
    char *mem = nullptr;        // X copy + transposed data
    rrs::DataDev base;          // binary64 data and its transpose
    struct Ops {                // matrix-core operands of one format
        char *mem = nullptr;
        double *xbar = nullptr;
        void *A0 = nullptr, *A1 = nullptr;
        float *anorm = nullptr;
        float *amax = nullptr;
        bool pp = false;
        hipEvent_t ready = nullptr;
    } ops[3];
    int refs = 0;               // requests submitted and not finished
    bool released = false;
};

struct rrs_request {
    rrs::JobSpec spec;
    rrs_dataset *ds = nullptr;
    rrs::Plan plan;
    size_t bytes = 0;           // device block: Z, outputs, workspace
    double *Zh = nullptr;       // pinned host copies
    double *depth_h = nullptr;
    int64_t *count_h = nullptr;
    char *mem = nullptr;
    int skipped = 0;
    rrs_request_info info{};
    std::mutex mu;
    std::condition_variable cv;
    bool done = false;
    rrs_status status = RRS_OK;
    std::string err;
};

struct CbArg {
    rrs_ctx *ctx;
    int slot;
};

struct rrs_ctx {
    int device = 0;
    char *base = nullptr;
    DevicePool pool;
    size_t ws_limit = 0;
    hipStream_t aux = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<rrs_request *> running;  // per slot
    std::vector<CbArg> cbargs;
    std::vector<double> done_time;       // per slot, set by the callback
    std::mutex mu;
    std::condition_variable cv;
    std::deque<rrs_request *> pending;
    std::vector<int> done_slots;
    std::set<rrs_dataset *> datasets;
    bool dirty = false, stop = false;
    int64_t completed = 0, failed = 0;
    std::thread th;
};

namespace {

void finish(rrs_request *r, rrs_status st, const std::string &err)
{
    std::lock_guard<std::mutex> lk(r->mu);
    r->status = st;
    r->err = err;
    r->done = true;
    r->cv.notify_all();
}

void free_request(rrs_request *r)
{
    if (r->Zh) (void)hipHostFree(r->Zh);
    if (r->depth_h) (void)hipHostFree(r->depth_h);
    if (r->count_h) (void)hipHostFree(r->count_h);
    delete r;
}

// Frees a released data set once nothing uses it (context lock held).
void maybe_free_dataset(rrs_ctx *c, rrs_dataset *ds)
{
    if (!ds->released || ds->refs > 0) return;
    c->pool.release(ds->mem);
    for (auto &o : ds->ops) {
        c->pool.release(o.mem);
        if (o.ready) (void)hipEventDestroy(o.ready);
    }
    c->datasets.erase(ds);
    delete ds;
}

size_t ops_bytes(int64_t n, int64_t d, int prec)
{
    return rrs::data_bytes(n, d, prec) - rrs::data_bytes(n, d, -1) + 1024;
}

void on_done(void *p)
{
    CbArg *a = (CbArg *)p;
    rrs_ctx *c = a->ctx;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        c->done_time[a->slot] = now_s();
        c->done_slots.push_back(a->slot);
        c->dirty = true;
    }
    c->cv.notify_all();
}

// Enqueues an admitted request on its slot's stream (no context lock held;
// only the scheduler thread calls this).
rrs_status launch_request(rrs_ctx *c, rrs_request *r, int slot, bool prep_ops)
{
    hipStream_t st = c->streams[slot];
    rrs_dataset *ds = r->ds;
    const int64_t nq = r->spec.nq, d = ds->d;
    rrs::Carver cv(r->mem);
    double *Zd = cv.take<double>((size_t)nq * d);
    double *depth_d = cv.take<double>((size_t)nq);
    int64_t *count_d = cv.take<int64_t>((size_t)nq);
    void *ws = cv.take<char>(r->plan.ws_bytes);
    RRS_HIP_TRY(hipMemcpyAsync(Zd, r->Zh, (size_t)nq * d * 8, hipMemcpyHostToDevice, st));
    rrs::DataDev D = ds->base;
    const int prec = r->plan.prec;
    if (prec >= 0) {
        rrs_dataset::Ops &o = ds->ops[prec];
        if (prep_ops) {
            rrs::Carver oc(o.mem);
            const int64_t kp = rrs::mfma_kpad(prec, d);
            const size_t eb = rrs::mfma_elem_bytes(prec);
            o.xbar = oc.take<double>((size_t)d);
            o.A0 = oc.take<char>((size_t)ds->n * kp * eb);
            o.A1 = rrs::mfma_terms(prec) == 2 ? (void *)oc.take<char>((size_t)ds->n * kp * eb)
                                               : nullptr;
            o.anorm = oc.take<float>((size_t)ds->n);
            o.amax = oc.take<float>(16);
            RRS_HIP_TRY(rrs::launch_mfma_prep(prec, ds->base.X, ds->n, d, o.xbar, o.A0, o.A1,
                                              o.anorm, o.amax, st));
            // per-point bounds for heavy-tailed data (a one-time wait for
            // this data set's preparation)
            rrs::DataDev t;
            t.prec = prec;
            t.amax = o.amax;
            RRS_HIP_TRY(rrs::data_point_bounds(t, st));
            o.pp = t.pp;
            RRS_HIP_TRY(hipEventCreateWithFlags(&o.ready, hipEventDisableTiming));
            RRS_HIP_TRY(hipEventRecord(o.ready, st));
        } else {
            RRS_HIP_TRY(hipStreamWaitEvent(st, o.ready, 0));
        }
        D.prec = prec;
        D.xbar = o.xbar;
        D.A0 = o.A0;
        D.A1 = o.A1;
        D.anorm = o.anorm;
        D.amax = o.amax;
        D.pp = o.pp;
    }
    rrs::JobIO io;
    io.Z = Zd;
    io.depth = depth_d;
    io.count = r->spec.notion == rrs::NOTION_HALFSPACE ? count_d : nullptr;
    rrs_status s = rrs::enqueue_job(r->spec, D, r->plan, io, ws, st, nullptr, nullptr);
    if (s != RRS_OK) return s;
    RRS_HIP_TRY(hipMemcpyAsync(r->depth_h, depth_d, (size_t)nq * 8, hipMemcpyDeviceToHost, st));
    if (io.count)
        RRS_HIP_TRY(
            hipMemcpyAsync(r->count_h, count_d, (size_t)nq * 8, hipMemcpyDeviceToHost, st));
    RRS_HIP_TRY(hipLaunchHostFunc(st, on_done, &c->cbargs[slot]));
    return RRS_OK;
}

void scheduler(rrs_ctx *c)
{
    (void)hipSetDevice(c->device);
    std::unique_lock<std::mutex> lk(c->mu);
    for (;;) {
        // completions: release memory, publish results
        while (!c->done_slots.empty()) {
            const int s = c->done_slots.back();
            c->done_slots.pop_back();
            rrs_request *r = c->running[s];
            c->running[s] = nullptr;
            c->pool.release(r->mem);
            r->mem = nullptr;
            r->info.done_s = c->done_time[s];
            r->ds->refs--;
            maybe_free_dataset(c, r->ds);
            c->completed++;
            finish(r, RRS_OK, "");
        }
        int busy = 0;
        for (rrs_request *r : c->running) busy += r != nullptr;
        if (c->stop) {
            while (!c->pending.empty()) {
                rrs_request *r = c->pending.front();
                c->pending.pop_front();
                r->ds->refs--;
                maybe_free_dataset(c, r->ds);
                finish(r, RRS_E_CANCELLED, "context destroyed before the request ran");
            }
            if (busy == 0) break;
        }
        // admission in arrival order; a later request may pass a head that
        // does not fit yet, at most kMaxSkips times in all
        c->dirty = false;
        for (bool progress = true; progress && !c->stop;) {
            progress = false;
            int slot = -1;
            for (size_t s = 0; s < c->running.size(); ++s)
                if (!c->running[s]) {
                    slot = (int)s;
                    break;
                }
            if (slot < 0) break;
            bool head_blocked = false;
            for (auto it = c->pending.begin(); it != c->pending.end(); ++it) {
                rrs_request *r = *it;
                rrs_dataset *ds = r->ds;
                const int prec = r->plan.prec;
                const bool prep = prec >= 0 && ds->ops[prec].mem == nullptr;
                char *opsmem = prep ? c->pool.alloc(ops_bytes(ds->n, ds->d, prec)) : nullptr;
                char *mem = (prep && !opsmem) ? nullptr : c->pool.alloc(r->bytes);
                if (!mem) {
                    c->pool.release(opsmem);
                    if (it == c->pending.begin()) {
                        if (r->skipped >= kMaxSkips) break;  // wait for the head
                        head_blocked = true;
                    }
                    continue;
                }
                if (head_blocked) c->pending.front()->skipped++;
                if (prep) ds->ops[prec].mem = opsmem;
                c->pending.erase(it);
                c->running[slot] = r;
                r->mem = mem;
                r->info.admit_s = now_s();
                r->info.bytes = r->bytes;
                lk.unlock();
                rrs_status s = launch_request(c, r, slot, prep);
                std::string err = s == RRS_OK ? "" : rrs::last_error();
                if (s != RRS_OK) (void)hipStreamSynchronize(c->streams[slot]);
                lk.lock();
                if (s != RRS_OK) {
                    if (prep && ds->ops[prec].ready == nullptr) {
                        c->pool.release(ds->ops[prec].mem);
                        ds->ops[prec].mem = nullptr;
                    }
                    c->running[slot] = nullptr;
                    c->pool.release(r->mem);
                    r->mem = nullptr;
                    r->ds->refs--;
                    maybe_free_dataset(c, r->ds);
                    c->failed++;
                    finish(r, s, err);
                }
                progress = true;
                break;  // the list may have changed while unlocked: rescan
            }
        }
        // woken by a submission, a completion or the stop request (each sets
        // dirty); never spins while work is still on the device
        c->cv.wait(lk, [c] { return c->dirty || !c->done_slots.empty(); });
    }
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

extern "C" {

rrs_status rrs_ctx_create(const rrs_ctx_config *cfg, rrs_ctx **out)
{
    if (!out) return fail(RRS_E_INVAL, "out must be non-NULL");
    *out = nullptr;
    rrs_ctx_config k{};
    if (cfg) k = *cfg;
    int ndev = 0;
    RRS_HIP_TRY(hipGetDeviceCount(&ndev));
    if (k.device < 0 || k.device >= ndev)
        return fail(RRS_E_INVAL, "device %d out of range (%d devices)", k.device, ndev);
    if (k.slots < 0 || k.slots > 64) return fail(RRS_E_INVAL, "slots must be in 0..64");
    const int slots = k.slots ? k.slots : 4;
    DeviceGuard g(k.device);
    size_t budget = k.hbm_budget;
    if (!budget) {
        size_t freeb = 0, totb = 0;
        RRS_HIP_TRY(hipMemGetInfo(&freeb, &totb));
        budget = freeb / 2;
    }
    budget = align256(budget);
    rrs_ctx *c = new rrs_ctx();
    c->device = k.device;
    hipError_t e = hipMalloc(&c->base, budget);
    if (e != hipSuccess) {
        delete c;
        return fail(RRS_E_NOMEM, "budget of %zu bytes could not be allocated: %s", budget,
                    hipGetErrorString(e));
    }
    c->pool.init(c->base, budget);
    c->ws_limit = k.request_ws_limit ? k.request_ws_limit : budget / (2 * (size_t)slots);
    c->streams.resize(slots, nullptr);
    c->running.assign(slots, nullptr);
    c->done_time.assign(slots, 0.0);
    c->cbargs.resize(slots);
    for (int s = 0; s < slots; ++s) {
        c->cbargs[s] = CbArg{c, s};
        e = hipStreamCreateWithFlags(&c->streams[s], hipStreamNonBlocking);
        if (e == hipSuccess) continue;
        for (int t = 0; t < s; ++t) (void)hipStreamDestroy(c->streams[t]);
        (void)hipFree(c->base);
        delete c;
        return fail(RRS_E_DEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e));
    }
    e = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking);
    if (e != hipSuccess) {
        for (int t = 0; t < slots; ++t) (void)hipStreamDestroy(c->streams[t]);
        (void)hipFree(c->base);
        delete c;
        return fail(RRS_E_DEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e));
    }
    c->th = std::thread(scheduler, c);
    *out = c;
    return RRS_OK;
}

rrs_status rrs_ctx_destroy(rrs_ctx *c)
{
    if (!c) return fail(RRS_E_INVAL, "ctx must be non-NULL");
    {
        std::lock_guard<std::mutex> lk(c->mu);
        c->stop = true;
        c->dirty = true;
    }
    c->cv.notify_all();
    c->th.join();
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->aux);
    for (hipStream_t s : c->streams) (void)hipStreamDestroy(s);
    (void)hipStreamDestroy(c->aux);
    for (rrs_dataset *ds : c->datasets) {
        for (auto &o : ds->ops)
            if (o.ready) (void)hipEventDestroy(o.ready);
        delete ds;
    }
    c->datasets.clear();
    (void)hipFree(c->base);
    delete c;
    return RRS_OK;
}

rrs_status rrs_dataset_put(rrs_ctx *c, const double *X, int64_t n, int64_t d, rrs_dataset **out)
{
    if (!c || !X || !out) return fail(RRS_E_INVAL, "ctx, X and out must be non-NULL");
    *out = nullptr;
    if (n < 1 || d < 2 || n > 0x7FFFFFFFLL || d > 0x7FFFFFFFLL)
        return fail(RRS_E_INVAL, "need n >= 1 and d >= 2 (got n=%lld d=%lld)", (long long)n,
                    (long long)d);
    for (int64_t i = 0; i < n * d; ++i)
        if (!std::isfinite(X[i])) return fail(RRS_E_INVAL, "X holds a non-finite value");
    const size_t xbytes = align256((size_t)n * d * 8);
    const size_t bytes = xbytes + rrs::data_bytes(n, d, -1);
    rrs_dataset *ds = new rrs_dataset();
    ds->ctx = c;
    ds->n = n;
    ds->d = d;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        ds->mem = c->pool.alloc(bytes);
        if (!ds->mem) {
            delete ds;
            return fail(RRS_E_NOMEM, "data set of %zu bytes does not fit the budget (%zu of %zu "
                                     "bytes in use)", bytes, c->pool.used(), c->pool.cap());
        }
        ds->refs = 1;  // held until the data is in place
        c->datasets.insert(ds);
    }
    DeviceGuard g(c->device);
    ds->base.X = (const double *)ds->mem;
    ds->base.n = n;
    ds->base.d = d;
    hipError_t e = hipMemcpyAsync(ds->mem, X, (size_t)n * d * 8, hipMemcpyHostToDevice, c->aux);
    if (e == hipSuccess) e = rrs::data_prepare(ds->base, ds->mem + xbytes, -1, c->aux);
    if (e == hipSuccess) e = hipStreamSynchronize(c->aux);
    std::lock_guard<std::mutex> lk(c->mu);
    ds->refs = 0;
    if (e != hipSuccess) {
        ds->released = true;
        maybe_free_dataset(c, ds);
        return fail(RRS_E_DEVICE, "copying the data set failed: %s", hipGetErrorString(e));
    }
    *out = ds;
    return RRS_OK;
}

rrs_status rrs_dataset_release(rrs_ctx *c, rrs_dataset *ds)
{
    if (!c || !ds) return fail(RRS_E_INVAL, "ctx and ds must be non-NULL");
    std::lock_guard<std::mutex> lk(c->mu);
    if (!c->datasets.count(ds) || ds->released)
        return fail(RRS_E_INVAL, "unknown or released data set");
    ds->released = true;
    maybe_free_dataset(c, ds);
    return RRS_OK;
}

rrs_status rrs_submit(rrs_ctx *c, rrs_dataset *ds, int32_t notion, const double *Z, int64_t m,
                      int64_t K, int32_t n_refine, double cap_shrink, uint64_t seed,
                      const rrs_opts *opts, rrs_request **out)
{
    if (!c || !ds || !out) return fail(RRS_E_INVAL, "ctx, ds and out must be non-NULL");
    *out = nullptr;
    rrs_opts o{};
    if (opts) o = *opts;
    if (o.device_ptrs || o.stream || o.poles || o.trace)
        return fail(RRS_E_INVAL, "rrs_submit takes host queries and no stream, poles or trace");
    rrs::JobSpec s;
    s.notion = notion;
    s.precision = o.precision;
    s.nq = m;
    s.K = K;
    s.r = n_refine;
    s.alpha = cap_shrink;
    s.seed = seed;
    s.qoff = o.query_offset;
    rrs_status vs = rrs::job_validate(s, ds->n, ds->d);
    if (vs != RRS_OK) return vs;
    if (m < 1 || !Z) return fail(RRS_E_INVAL, "need m >= 1 queries and Z non-NULL");
    for (int64_t i = 0; i < m * ds->d; ++i)
        if (!std::isfinite(Z[i])) return fail(RRS_E_INVAL, "Z holds a non-finite value");
    rrs_request *r = new rrs_request();
    r->spec = s;
    r->ds = ds;
    const size_t limit = o.workspace_limit ? o.workspace_limit : c->ws_limit;
    rrs_status ps = rrs::job_plan(s, ds->n, ds->d, limit, &r->plan);
    if (ps != RRS_OK) {
        delete r;
        return ps;
    }
    size_t sizes[4] = {(size_t)m * ds->d * 8, (size_t)m * 8, (size_t)m * 8, r->plan.ws_bytes};
    r->bytes = rrs::carve_size(sizes, 4);
    const size_t extra = r->plan.prec >= 0 ? ops_bytes(ds->n, ds->d, r->plan.prec) : 0;
    if (r->bytes + extra > c->pool.cap()) {
        const size_t need = r->bytes + extra;
        delete r;
        return fail(RRS_E_NOMEM, "request needs %zu bytes, more than the budget of %zu", need,
                    c->pool.cap());
    }
    hipError_t e = hipHostMalloc((void **)&r->Zh, (size_t)m * ds->d * 8, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&r->depth_h, (size_t)m * 8, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&r->count_h, (size_t)m * 8, hipHostMallocDefault);
    if (e != hipSuccess) {
        free_request(r);
        return fail(RRS_E_NOMEM, "pinned host memory: %s", hipGetErrorString(e));
    }
    std::memcpy(r->Zh, Z, (size_t)m * ds->d * 8);
    r->info.projections = m * (int64_t)n_refine * ((K + n_refine - 1) / n_refine) * ds->n;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        if (c->stop || !c->datasets.count(ds) || ds->released) {
            free_request(r);
            return fail(RRS_E_INVAL, "data set released or context stopping");
        }
        ds->refs++;
        r->info.submit_s = now_s();
        c->pending.push_back(r);
        c->dirty = true;
    }
    c->cv.notify_all();
    *out = r;
    return RRS_OK;
}

rrs_status rrs_wait(rrs_request *r, double timeout_s, double *depth, int64_t *count,
                    rrs_request_info *info)
{
    if (!r) return fail(RRS_E_INVAL, "request must be non-NULL");
    {
        std::unique_lock<std::mutex> lk(r->mu);
        if (timeout_s < 0) {
            r->cv.wait(lk, [r] { return r->done; });
        } else if (!r->cv.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                   [r] { return r->done; })) {
            return fail(RRS_E_BUSY, "request not finished after %g s", timeout_s);
        }
    }
    const rrs_status st = r->status;
    const std::string err = r->err;
    if (st == RRS_OK) {
        const int64_t m = r->spec.nq;
        if (depth) std::memcpy(depth, r->depth_h, (size_t)m * 8);
        if (count && r->spec.notion == rrs::NOTION_HALFSPACE)
            std::memcpy(count, r->count_h, (size_t)m * 8);
    }
    if (info) *info = r->info;
    free_request(r);
    if (st != RRS_OK) return fail(st, "%s", err.c_str());
    return RRS_OK;
}

rrs_status rrs_ctx_get_stats(rrs_ctx *c, rrs_ctx_stats *out)
{
    if (!c || !out) return fail(RRS_E_INVAL, "ctx and out must be non-NULL");
    std::lock_guard<std::mutex> lk(c->mu);
    std::memset(out, 0, sizeof(*out));
    out->pending = (int64_t)c->pending.size();
    for (rrs_request *r : c->running) out->running += r != nullptr;
    out->completed = c->completed;
    out->failed = c->failed;
    out->datasets = 0;
    for (rrs_dataset *ds : c->datasets) out->datasets += !ds->released;
    out->bytes_in_use = c->pool.used();
    out->bytes_peak = c->pool.peak();
    out->budget = c->pool.cap();
    return RRS_OK;
}

}  // extern "C"
