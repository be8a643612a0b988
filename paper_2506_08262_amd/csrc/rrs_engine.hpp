// rrs_engine.hpp -- one RRS depth job, planned and enqueued on a HIP stream
// (internal).  The synchronous C entry points and the serving context both
// drive this: they differ only in where device memory comes from and in when
// the host waits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/rrs.h"
#include "rrs_launch.hpp"

namespace rrs {

// Records the failure text for the calling thread and returns s.
rrs_status fail(rrs_status s, const char *fmt, ...);
std::string &last_error();

#define RRS_HIP_TRY(expr)                                                                \
    do {                                                                                 \
        hipError_t _e = (expr);                                                          \
        if (_e != hipSuccess)                                                            \
            return ::rrs::fail(_e == hipErrorOutOfMemory ? RRS_E_NOMEM : RRS_E_DEVICE,   \
                               "%s failed: %s", #expr, hipGetErrorString(_e));           \
    } while (0)

// Bump allocator over one block; every piece is 256-byte aligned.
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
size_t carve_size(const size_t *sizes, int k);

// Per-kernel HIP-event timing (kinds as reported by rrs_profile_read).
enum { K_GEN = 0, K_PROJ, K_SELECT, K_ARGMIN, K_MFMA, K_RECHECK, K_OTHER, K_CULL, K_COUNT };
extern const char *const kKernelNames[K_COUNT];

struct Profiler {
    struct Rec {
        int kind;
        hipEvent_t a, b;
        double work;
    };
    // events in flight at most: a long call (thousands of launches) waits
    // for its recorded launches and reuses their events once the pool is full
    static constexpr size_t kPoolCap = 256;
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<Rec> recs;
    int64_t launches[K_COUNT] = {};
    double ms[K_COUNT] = {};
    double work[K_COUNT] = {};
    // selects issued (two per projection / APD column, counted on the host)
    // and those that took the exact fallback (counted on the device)
    double sel_total = 0.0, sel_fallback = 0.0, recheck_pairs = 0.0;
    // (query, direction, point) pairs the sign GEMM evaluated: all of them
    // without culling (counted on the host), the listed points' pairs after
    // culling (counted on the device, stats words 6..7)
    double gemm_pairs = 0.0;
    // streamed APD columns whose shared passes served the whole column,
    // only the median, or nothing (stats words 8..10)
    double shared[3] = {0.0, 0.0, 0.0};
    hipEvent_t get();
    // makes room for two more events (waits for the recorded launches)
    void reserve2();
    void collect();
    void clear();
};

// ---------------------------------------------------------------------------
// The data set on the device, prepared once and shared by every job on it.
// ---------------------------------------------------------------------------
struct DataDev {
    const double *X = nullptr;   // [n][d] row-major binary64
    double *XT = nullptr;        // [d][ldx] transposed, ldx = n rounded up to 512 (pad 0)
    int64_t n = 0, d = 0, ldx = 0;
    // matrix-core operands of one MFMA_* format (prec < 0: none)
    int prec = -1;
    double *xbar = nullptr;      // [d] column means
    void *A0 = nullptr, *A1 = nullptr;  // [n][kp] centred operands
    float *anorm = nullptr;      // [n] norm bounds of the centred points
    float *amax = nullptr;       // largest of them, flag, sum of squares (16 words)
    bool pp = false;             // stored-projection selects with per-point bounds
};

// Bytes of the prepared data beyond X itself: XT, plus the operands of one
// matrix-core format when prec >= 0.
size_t data_bytes(int64_t n, int64_t d, int prec);
// Carves the prepared arrays from mem (data_bytes(n, d, prec) bytes) and
// enqueues their preparation from D.X on st.
hipError_t data_prepare(DataDev &D, void *mem, int prec, hipStream_t st);
// Whether the stored-projection selects take per-point bounds on this data:
// when the column-wide bound, set by the largest norm, would fill a window
// with too many candidates (waits for the preparation; RRS_POINT_BOUNDS =
// 0 / 1 forces it off / on).
hipError_t data_point_bounds(DataDev &D, hipStream_t st);

// ---------------------------------------------------------------------------
// One job: nq queries of one notion on a data set.
// ---------------------------------------------------------------------------
struct JobSpec {
    int notion = NOTION_HALFSPACE;
    int precision = RRS_F64;     // rrs_precision
    int64_t nq = 0, K = 0;
    int32_t r = 1;
    double alpha = 1.0;
    uint64_t seed = 0;
    int64_t qoff = 0;            // stream index of the first query
    bool want_trace = false;
    bool first_cap = false;      // RRS_FLAG_FIRST_CAP: refinement 1 in the pi/2 cap of Alg. S4
    bool area_cap = false;       // RRS_FLAG_AREA_CAP: caps uniform in area
};

// Validates the arguments of a job on an n x d data set (everything that
// does not need the data values).
rrs_status job_validate(const JobSpec &s, int64_t n, int64_t d);
// MFMA_* format of a precision, or -1 for the binary64 form.
int job_mfma_prec(int precision);

struct Plan {
    int64_t m = 0, ldm = 0, kp = 0, qb = 0;
    size_t eb = 0;
    int terms = 0, prec = -1;
    uint64_t qcap = 0;
    size_t ws_bytes = 0;         // workspace of enqueue_job
    // halfspace bfloat16 form: persistent sign GEMM (rrs_sign.hip) and cap
    // culling of the refinements l >= 2
    bool sign = false, cull = false;
    int rpi = 4;                 // point tiles per list-mode item
};
// Chooses the query batch so that the workspace fits `limit` bytes.
rrs_status job_plan(const JobSpec &s, int64_t n, int64_t d, size_t limit, Plan *p);

struct JobIO {
    const double *Z = nullptr;   // device [nq][d]
    double *depth = nullptr;     // device [nq]
    int64_t *count = nullptr;    // device [nq] or null (halfspace)
    double *poles = nullptr;     // device [nq][d] or null
    int64_t *trace = nullptr;    // device [nq][r][3] or null
};

// Enqueues the whole refinement chain of the job on st (no host wait).  ws
// holds plan.ws_bytes bytes of device memory that stays untouched by others
// until the stream has passed the job.  With prof->on, kernels are timed and
// the event counters accumulate into *stats_out (device, 16 words) -- the
// caller reads them after synchronising.
rrs_status enqueue_job(const JobSpec &s, const DataDev &D, const Plan &p, const JobIO &io,
                       void *ws, hipStream_t st, Profiler *prof, uint32_t **stats_out);

}  // namespace rrs
