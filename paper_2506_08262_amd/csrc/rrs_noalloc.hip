// rrs_noalloc.hip -- rrs_depth_halfspace_noalloc: the halfspace depth call for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, hosts that forbid allocation during a call).
//
// Every byte of device memory the call needs beyond the caller's inputs and
// outputs -- the prepared data (transpose, centred matrix-core operands) and
// the job workspace (directions, operands, counts, recheck queue, pole state)
// -- is carved from one file-scope device array, `scratch`, of kScratchBytes.
// Each device the library runs on holds its own copy of the array until the
// process ends.  Host code never passes the array's name to a kernel: the
// name is a host-side stand-in, so the array's device address is looked up
// once per device with hipGetSymbolAddress (with that device current) and
// that address is what the kernels receive.
//
// The call enqueues its work on the caller's stream and returns without
// waiting; nothing in it allocates (no hipMalloc / hipFree, no events, no
// GEMM variant timing).  All calls on one device share that device's array,
// which keeps the last call's contents: everything that must start at zero
// is cleared by fill kernels inside the call, and calls whose work overlaps
// on one device (different streams, or another thread) race.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "../../include/rrs.h"
#include "rrs_engine.hpp"

using rrs::fail;

namespace {

constexpr size_t kScratchBytes = (size_t)RRS_NOALLOC_SCRATCH_MIB << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
std::map<int, void *> g_scratch;  // device ordinal -> device address of `scratch`

// Device address of this device's copy of `scratch` (looked up once per
// device, with that device current).
rrs_status scratch_address(int dev, void **out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) {
        *out = it->second;
        return RRS_OK;
    }
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
        return fail(RRS_E_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                    hipGetErrorString(e));
    g_scratch.emplace(dev, ptr);
    *out = ptr;
    return RRS_OK;
}

}  // namespace

extern "C" rrs_status rrs_depth_halfspace_noalloc(const double *X, int64_t n, int64_t d,
                                                  const double *Z, int64_t m, int64_t K,
                                                  int32_t n_refine, double cap_shrink,
                                                  uint64_t seed, double *depth, int64_t *count,
                                                  const rrs_opts *opts)
{
    if (!opts || opts->device_ptrs == 0)
        return fail(RRS_E_INVAL,
                    "rrs_depth_halfspace_noalloc needs opts with device_ptrs = 1 (device "
                    "inputs and outputs)");
    const rrs_opts &o = *opts;
    if (o.reserved != 0 || o.flags != 0)
        return fail(RRS_E_INVAL, "rrs_depth_halfspace_noalloc takes no flags");
    rrs::JobSpec s;
    s.notion = rrs::NOTION_HALFSPACE;
    s.precision = o.precision;
    s.nq = m;
    s.K = K;
    s.r = n_refine;
    s.alpha = cap_shrink;
    s.seed = seed;
    s.qoff = o.query_offset;
    s.want_trace = o.trace != nullptr;
    if (m < 0) return fail(RRS_E_INVAL, "number of queries must be >= 0 (got %lld)", (long long)m);
    if (m == 0) return RRS_OK;
    if (!X || !Z || !depth) return fail(RRS_E_INVAL, "X, Z and depth must be non-NULL");
    rrs_status vs = rrs::job_validate(s, n, d);
    if (vs != RRS_OK) return vs;

    int dev = 0;
    RRS_HIP_TRY(hipGetDevice(&dev));
    void *base = nullptr;
    vs = scratch_address(dev, &base);
    if (vs != RRS_OK) return vs;

    // the prepared data first, then the job workspace in what is left
    const size_t data_sz = rrs::data_bytes(n, d, rrs::job_mfma_prec(s.precision));
    if (data_sz + 256 > kScratchBytes)
        return fail(RRS_E_NOMEM,
                    "data set of %lld x %lld needs %zu bytes of prepared data, more than the "
                    "%zu-byte static scratch of rrs_depth_halfspace_noalloc",
                    (long long)n, (long long)d, data_sz, kScratchBytes);
    size_t limit = kScratchBytes - data_sz - 256;
    if (o.workspace_limit && o.workspace_limit < limit) limit = o.workspace_limit;
    rrs::Plan plan;
    vs = rrs::job_plan(s, n, d, limit, &plan);
    if (vs != RRS_OK) return vs;
    if (plan.ws_bytes > limit)
        return fail(RRS_E_NOMEM,
                    "one query's workspace (%zu bytes) does not fit the %zu bytes left in the "
                    "static scratch of rrs_depth_halfspace_noalloc",
                    plan.ws_bytes, limit);
    rrs::Carver cv(base);
    void *data_mem = cv.take<char>(data_sz);
    void *ws = cv.take<char>(plan.ws_bytes);
    if (cv.off > kScratchBytes)
        return fail(RRS_E_INTERNAL, "scratch carve overran (%zu > %zu)", cv.off, kScratchBytes);

    hipStream_t st = (hipStream_t)o.stream;
    rrs::JobIO io;
    io.Z = Z;
    io.depth = depth;
    io.count = count;
    io.poles = o.poles;
    io.trace = o.trace;
    rrs::DataDev D;
    D.X = X;
    D.n = n;
    D.d = d;
    RRS_HIP_TRY(rrs::data_prepare(D, data_mem, plan.prec, st));
    // GEMM variants are never timed here (timing creates events)
    rrs::mfma_tune_suspend(true);
    const rrs_status es = rrs::enqueue_job(s, D, plan, io, ws, st, nullptr, nullptr);
    rrs::mfma_tune_suspend(false);
    return es;
}
