"""Python binding of librrs (the C ABI in include/rrs.h).

Argument marshalling only: numpy arrays are passed as host pointers, torch
tensors on a ROCm device as device pointers together with torch's current HIP
stream.  Every step of the depth computation runs in the library's HIP
kernels; there is no fallback path -- if the library is missing or fails to
load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librrs.so")

RRS_OK, RRS_E_INVAL, RRS_E_NOMEM, RRS_E_DEVICE = 0, 1, 2, 3
RRS_FLAG_GRAPH = 1
RRS_FLAG_FIRST_CAP = 2
RRS_FLAG_AREA_CAP = 4
RRS_E_BUSY, RRS_E_CANCELLED, RRS_E_INTERNAL = 4, 5, 6
RRS_F64, RRS_F32_RECHECK, RRS_BF16_RECHECK, RRS_F32_PLAIN = 0, 1, 2, 3
PRECISIONS = {"f64": RRS_F64, "f32": RRS_F32_RECHECK, "bf16": RRS_BF16_RECHECK,
              "f32_plain": RRS_F32_PLAIN}
STATUS_NAMES = {0: "RRS_OK", 1: "RRS_E_INVAL", 2: "RRS_E_NOMEM", 3: "RRS_E_DEVICE",
                4: "RRS_E_BUSY", 5: "RRS_E_CANCELLED", 6: "RRS_E_INTERNAL"}
NOTIONS = {"halfspace": 0, "projection": 1, "apd": 2}

EXPORTED = ["rrs_depth_halfspace", "rrs_depth_projection", "rrs_depth_apd",
            "rrs_last_error", "rrs_release_workspace", "rrs_version", "rrs_debug_directions",
            "rrs_profile_enable", "rrs_profile_read", "rrs_profile_counter",
            "rrs_ctx_create", "rrs_ctx_destroy", "rrs_dataset_put", "rrs_dataset_release",
            "rrs_submit", "rrs_wait", "rrs_ctx_get_stats", "rrs_depth_halfspace_noalloc",
            "rrs_depth_mahalanobis"]


class RRSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class rrs_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32),
                ("device_ptrs", ctypes.c_int32),
                ("stream", ctypes.c_void_p),
                ("query_offset", ctypes.c_int64),
                ("poles", ctypes.c_void_p),
                ("trace", ctypes.c_void_p),
                ("workspace_limit", ctypes.c_size_t),
                ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class rrs_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32),
                ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double),
                ("work_units", ctypes.c_double)]


class rrs_ctx_config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32),
                ("slots", ctypes.c_int32),
                ("hbm_budget", ctypes.c_size_t),
                ("request_ws_limit", ctypes.c_size_t)]


class rrs_request_info(ctypes.Structure):
    _fields_ = [("submit_s", ctypes.c_double),
                ("admit_s", ctypes.c_double),
                ("done_s", ctypes.c_double),
                ("projections", ctypes.c_int64),
                ("bytes", ctypes.c_size_t)]


class rrs_ctx_stats(ctypes.Structure):
    _fields_ = [("pending", ctypes.c_int64),
                ("running", ctypes.c_int64),
                ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64),
                ("datasets", ctypes.c_int64),
                ("bytes_in_use", ctypes.c_size_t),
                ("bytes_peak", ctypes.c_size_t),
                ("budget", ctypes.c_size_t)]


_lib = None


def load(path: str = LIB_PATH):
    """Load librrs.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"librrs.so not built at {path}; run __graft_entry__.build()")
    # One HIP runtime per process: torch ships its own libamdhip64 (same
    # soname as the system one librrs links against).  Loading torch first
    # makes librrs bind to torch's copy, so device pointers and streams from
    # torch are valid in the library; loading librrs first would make torch
    # load a second runtime that cannot see the GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(path)
    p, i64, i32, u64, dbl = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                             ctypes.c_double)
    common = [p, i64, i64, p, i64, i64, i32, dbl, u64, p]
    L.rrs_depth_halfspace.argtypes = common + [p, ctypes.POINTER(rrs_opts)]
    L.rrs_depth_halfspace.restype = ctypes.c_int
    L.rrs_depth_halfspace_noalloc.argtypes = common + [p, ctypes.POINTER(rrs_opts)]
    L.rrs_depth_halfspace_noalloc.restype = ctypes.c_int
    L.rrs_depth_projection.argtypes = common + [ctypes.POINTER(rrs_opts)]
    L.rrs_depth_projection.restype = ctypes.c_int
    L.rrs_depth_apd.argtypes = common + [ctypes.POINTER(rrs_opts)]
    L.rrs_depth_apd.restype = ctypes.c_int
    L.rrs_depth_mahalanobis.argtypes = [p, i64, i64, p, i64, p, ctypes.POINTER(rrs_opts)]
    L.rrs_depth_mahalanobis.restype = ctypes.c_int
    L.rrs_last_error.restype = ctypes.c_char_p
    L.rrs_release_workspace.restype = ctypes.c_int
    L.rrs_version.restype = ctypes.c_int32
    L.rrs_debug_directions.argtypes = [i64, i64, i32, dbl, u64, u64, p, p]
    L.rrs_debug_directions.restype = ctypes.c_int
    L.rrs_profile_enable.argtypes = [i32]
    L.rrs_profile_enable.restype = ctypes.c_int
    L.rrs_profile_read.argtypes = [ctypes.POINTER(rrs_kernel_stat), i32]
    L.rrs_profile_read.restype = i32
    L.rrs_profile_counter.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double)]
    L.rrs_profile_counter.restype = i32
    L.rrs_ctx_create.argtypes = [ctypes.POINTER(rrs_ctx_config), ctypes.POINTER(p)]
    L.rrs_ctx_create.restype = ctypes.c_int
    L.rrs_ctx_destroy.argtypes = [p]
    L.rrs_ctx_destroy.restype = ctypes.c_int
    L.rrs_dataset_put.argtypes = [p, p, i64, i64, ctypes.POINTER(p)]
    L.rrs_dataset_put.restype = ctypes.c_int
    L.rrs_dataset_release.argtypes = [p, p]
    L.rrs_dataset_release.restype = ctypes.c_int
    L.rrs_submit.argtypes = [p, p, i32, p, i64, i64, i32, dbl, u64, ctypes.POINTER(rrs_opts),
                             ctypes.POINTER(p)]
    L.rrs_submit.restype = ctypes.c_int
    L.rrs_wait.argtypes = [p, dbl, p, p, ctypes.POINTER(rrs_request_info)]
    L.rrs_wait.restype = ctypes.c_int
    L.rrs_ctx_get_stats.argtypes = [p, ctypes.POINTER(rrs_ctx_stats)]
    L.rrs_ctx_get_stats.restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int):
    if status != RRS_OK:
        raise RRSError(status, load().rrs_last_error().decode())


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _prep(a, name, dtype):
    """Returns (pointer, keepalive, on_device)."""
    if _is_torch(a):
        import torch
        if a.dtype != dtype[1]:
            raise TypeError(f"{name} must be {dtype[1]}")
        if not a.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return ctypes.c_void_p(a.data_ptr()), a, a.is_cuda
    arr = np.ascontiguousarray(a, dtype=dtype[0])
    return arr.ctypes.data_as(ctypes.c_void_p), arr, False


def _alloc_like(X, shape, np_dtype, torch_dtype):
    if _is_torch(X):
        import torch
        return torch.empty(shape, dtype=torch_dtype, device=X.device)
    return np.empty(shape, dtype=np_dtype)


def _run(fn_name, X, Z, K, n_refine, cap_shrink, seed, precision, query_offset,
         want_count, want_poles, want_trace, stream, workspace_limit, graph=False,
         first_cap=False, area_cap=False):
    import_torch = _is_torch(X) or _is_torch(Z)
    f64 = (np.float64, None)
    i64 = (np.int64, None)
    if import_torch:
        import torch
        f64 = (np.float64, torch.float64)
        i64 = (np.int64, torch.int64)
    Xp, Xk, Xdev = _prep(X, "X", f64)
    Zp, Zk, Zdev = _prep(Z, "Z", f64)
    if Xdev != Zdev:
        raise ValueError("X and Z must both be host or both be device arrays")
    n, d = int(Xk.shape[0]), int(Xk.shape[1])
    nq = int(Zk.shape[0])
    if Zk.shape[1] != d:
        raise ValueError("Z must have d columns")
    tdt = None
    if import_torch:
        import torch
        tdt = (torch.float64, torch.int64)
    depth = _alloc_like(Xk, (nq,), np.float64, tdt[0] if tdt else None)
    count = _alloc_like(Xk, (nq,), np.int64, tdt[1] if tdt else None) if want_count else None
    poles = _alloc_like(Xk, (nq, d), np.float64, tdt[0] if tdt else None) if want_poles else None
    trace = (_alloc_like(Xk, (nq, n_refine, 3), np.int64, tdt[1] if tdt else None)
             if want_trace else None)

    def ptr(a):
        if a is None:
            return None
        return ctypes.c_void_p(a.data_ptr()) if _is_torch(a) else a.ctypes.data_as(ctypes.c_void_p)

    o = rrs_opts()
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.device_ptrs = 1 if Xdev else 0
    if Xdev:
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(Xk.device)
        o.stream = ctypes.c_void_p(s.cuda_stream if hasattr(s, "cuda_stream") else int(s))
    o.query_offset = int(query_offset)
    o.poles = ptr(poles)
    o.trace = ptr(trace)
    o.workspace_limit = int(workspace_limit or 0)
    o.flags = ((RRS_FLAG_GRAPH if graph else 0) | (RRS_FLAG_FIRST_CAP if first_cap else 0)
               | (RRS_FLAG_AREA_CAP if area_cap else 0))
    L = load()
    args = [Xp, n, d, Zp, nq, int(K), int(n_refine), float(cap_shrink), int(seed), ptr(depth)]
    if fn_name == "rrs_depth_halfspace":
        args.append(ptr(count))
    args.append(ctypes.byref(o))
    _check(getattr(L, fn_name)(*args))
    out = {"depth": depth}
    if want_count:
        out["count"] = count
    if want_poles:
        out["poles"] = poles
    if want_trace:
        out["trace"] = trace
    return out


def rrs_depth_halfspace(X, Z, K, n_refine, cap_shrink, seed=0, precision="f64", query_offset=0,
                        want_poles=False, want_trace=False, stream=None, workspace_limit=0,
                        graph=False, first_cap=False, area_cap=False):
    """Halfspace depth of each row of Z; returns dict(depth, count[, poles, trace])."""
    return _run("rrs_depth_halfspace", X, Z, K, n_refine, cap_shrink, seed, precision,
                query_offset, True, want_poles, want_trace, stream, workspace_limit, graph,
                first_cap, area_cap)


def rrs_depth_projection(X, Z, K, n_refine, cap_shrink, seed=0, precision="f64", query_offset=0,
                         want_poles=False, want_trace=False, stream=None, workspace_limit=0,
                         graph=False, first_cap=False, area_cap=False):
    """Projection depth of each row of Z; returns dict(depth[, poles, trace])."""
    return _run("rrs_depth_projection", X, Z, K, n_refine, cap_shrink, seed, precision,
                query_offset, False, want_poles, want_trace, stream, workspace_limit, graph,
                first_cap, area_cap)


def rrs_depth_apd(X, Z, K, n_refine, cap_shrink, seed=0, precision="f64", query_offset=0,
                  want_poles=False, want_trace=False, stream=None, workspace_limit=0,
                  graph=False, first_cap=False, area_cap=False):
    """Asymmetric projection depth of each row of Z; returns dict(depth[, poles, trace])."""
    return _run("rrs_depth_apd", X, Z, K, n_refine, cap_shrink, seed, precision, query_offset,
                False, want_poles, want_trace, stream, workspace_limit, graph, first_cap,
                area_cap)


def rrs_depth_halfspace_noalloc(X, Z, K, n_refine, cap_shrink, seed=0, precision="f64",
                                query_offset=0, out=None, want_poles=False, want_trace=False,
                                stream=None, workspace_limit=0):
    """rrs_depth_halfspace_noalloc: X and Z are torch tensors on the device;
    the outputs are written into `out` (dict of device tensors depth [m],
    count [m], optional poles [m, d], trace [m, n_refine, 3]) or into new
    tensors allocated here by torch (the library allocates nothing).  The
    call only enqueues the work on `stream` (default: torch's current
    stream) and returns the output dict at once."""
    import torch
    for a, name in ((X, "X"), (Z, "Z")):
        if not (_is_torch(a) and a.is_cuda and a.dtype == torch.float64 and a.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous float64 tensor on the device")
    nq, d = int(Z.shape[0]), int(X.shape[1])
    if int(Z.shape[1]) != d:
        raise ValueError("Z must have d columns")
    if out is None:
        out = {"depth": torch.empty(nq, dtype=torch.float64, device=X.device),
               "count": torch.empty(nq, dtype=torch.int64, device=X.device)}
        if want_poles:
            out["poles"] = torch.empty((nq, d), dtype=torch.float64, device=X.device)
        if want_trace:
            out["trace"] = torch.empty((nq, int(n_refine), 3), dtype=torch.int64,
                                       device=X.device)
    o = rrs_opts()
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.device_ptrs = 1
    s = stream if stream is not None else torch.cuda.current_stream(X.device)
    o.stream = ctypes.c_void_p(s.cuda_stream if hasattr(s, "cuda_stream") else int(s))
    o.query_offset = int(query_offset)
    o.poles = ctypes.c_void_p(out["poles"].data_ptr()) if "poles" in out else None
    o.trace = ctypes.c_void_p(out["trace"].data_ptr()) if "trace" in out else None
    o.workspace_limit = int(workspace_limit or 0)
    cnt = out.get("count")
    _check(load().rrs_depth_halfspace_noalloc(
        ctypes.c_void_p(X.data_ptr()), int(X.shape[0]), d, ctypes.c_void_p(Z.data_ptr()), nq,
        int(K), int(n_refine), float(cap_shrink), int(seed),
        ctypes.c_void_p(out["depth"].data_ptr()),
        ctypes.c_void_p(cnt.data_ptr()) if cnt is not None else None, ctypes.byref(o)))
    return out


def rrs_depth_mahalanobis(X, Z, stream=None):
    """Mahalanobis depth D_M(L) of each row of Z (sample mean, maximum-likelihood
    covariance of X); numpy arrays (host) or torch device tensors."""
    f64 = (np.float64, None)
    if _is_torch(X) or _is_torch(Z):
        import torch
        f64 = (np.float64, torch.float64)
    Xp, Xk, Xdev = _prep(X, "X", f64)
    Zp, Zk, Zdev = _prep(Z, "Z", f64)
    if Xdev != Zdev:
        raise ValueError("X and Z must both be host or both be device arrays")
    n, d = int(Xk.shape[0]), int(Xk.shape[1])
    nq = int(Zk.shape[0])
    if int(Zk.shape[1]) != d:
        raise ValueError("Z must have d columns")
    o = rrs_opts()
    if Xdev:
        import torch
        depth = torch.empty(nq, dtype=torch.float64, device=Xk.device)
        o.device_ptrs = 1
        s = stream if stream is not None else torch.cuda.current_stream(Xk.device)
        o.stream = ctypes.c_void_p(s.cuda_stream if hasattr(s, "cuda_stream") else int(s))
        dptr = ctypes.c_void_p(depth.data_ptr())
    else:
        depth = np.empty(nq, dtype=np.float64)
        dptr = depth.ctypes.data_as(ctypes.c_void_p)
    _check(load().rrs_depth_mahalanobis(Xp, n, d, Zp, nq, dptr, ctypes.byref(o)))
    return depth


DEPTH_FUNCS = {"halfspace": rrs_depth_halfspace, "projection": rrs_depth_projection,
               "apd": rrs_depth_apd}


def depth(notion, X, Z, K, n_refine, cap_shrink, seed=0, **kw):
    return DEPTH_FUNCS[notion](X, Z, K, n_refine, cap_shrink, seed, **kw)


def rrs_debug_directions(d, m_dir, l, phi, seed, q, pole) -> np.ndarray:
    """Directions of refinement l for stream query index q, from the device."""
    pole = np.ascontiguousarray(pole, dtype=np.float64)
    out = np.zeros((m_dir, d), dtype=np.float64)
    _check(load().rrs_debug_directions(int(d), int(m_dir), int(l), float(phi), int(seed), int(q),
                                       pole.ctypes.data_as(ctypes.c_void_p),
                                       out.ctypes.data_as(ctypes.c_void_p)))
    return out


def rrs_release_workspace():
    _check(load().rrs_release_workspace())


def rrs_version() -> int:
    return int(load().rrs_version())


def rrs_profile_enable(on: bool = True):
    _check(load().rrs_profile_enable(1 if on else 0))


def rrs_profile_read() -> dict:
    """{kernel name: {launches, total_ms, avg_ms, work_units}} of the timed launches."""
    L = load()
    arr = (rrs_kernel_stat * 16)()
    k = L.rrs_profile_read(arr, 16)
    out = {}
    for i in range(k):
        e = arr[i]
        out[e.name.decode()] = {"launches": int(e.launches), "total_ms": float(e.total_ms),
                                "avg_ms": float(e.total_ms) / max(int(e.launches), 1),
                                "work_units": float(e.work_units)}
    return out


def rrs_profile_counter(name: str):
    """Value of a diagnostic event counter (None if unknown)."""
    v = ctypes.c_double()
    rc = load().rrs_profile_counter(name.encode(), ctypes.byref(v))
    return float(v.value) if rc == 0 else None


# --------------------------------------------------------------------------
# Serving: resident data sets and continuously batched requests
# --------------------------------------------------------------------------
class Dataset:
    """A data set resident in a Context (rrs_dataset_put)."""

    def __init__(self, ctx, handle, n, d):
        self.ctx, self.handle, self.n, self.d = ctx, handle, n, d

    def release(self):
        if self.handle is not None:
            _check(load().rrs_dataset_release(self.ctx.handle, self.handle))
            self.handle = None


class Request:
    """A submitted depth request (rrs_submit); wait() returns its result."""

    def __init__(self, handle, nq, notion):
        self.handle, self.nq, self.notion = handle, nq, notion
        self.result = None

    def wait(self, timeout=None):
        """dict(depth, count (halfspace), info) once done; raises RRSError with
        status RRS_E_BUSY if still running after `timeout` seconds."""
        if self.result is not None:
            return self.result
        depth = np.empty(self.nq, dtype=np.float64)
        count = np.empty(self.nq, dtype=np.int64)
        info = rrs_request_info()
        st = load().rrs_wait(self.handle, -1.0 if timeout is None else float(timeout),
                             depth.ctypes.data_as(ctypes.c_void_p),
                             count.ctypes.data_as(ctypes.c_void_p), ctypes.byref(info))
        if st == RRS_E_BUSY:
            raise RRSError(st, load().rrs_last_error().decode())
        self.handle = None
        _check(st)
        self.result = {"depth": depth, "info": {k: getattr(info, k) for k, _ in info._fields_}}
        if self.notion == "halfspace":
            self.result["count"] = count
        return self.result


class Context:
    """Serving context on one device: a memory budget, `slots` concurrent
    request streams and a scheduler thread (rrs_ctx_create)."""

    def __init__(self, device=0, slots=0, hbm_budget=0, request_ws_limit=0):
        cfg = rrs_ctx_config(int(device), int(slots), int(hbm_budget), int(request_ws_limit))
        h = ctypes.c_void_p()
        _check(load().rrs_ctx_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h

    def put(self, X) -> Dataset:
        X = np.ascontiguousarray(X, dtype=np.float64)
        h = ctypes.c_void_p()
        _check(load().rrs_dataset_put(self.handle, X.ctypes.data_as(ctypes.c_void_p),
                                      X.shape[0], X.shape[1], ctypes.byref(h)))
        return Dataset(self, h, X.shape[0], X.shape[1])

    def submit(self, ds: Dataset, notion, Z, K, n_refine, cap_shrink, seed=0, precision="f64",
               query_offset=0, workspace_limit=0) -> Request:
        Z = np.ascontiguousarray(Z, dtype=np.float64)
        o = rrs_opts()
        o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        o.query_offset = int(query_offset)
        o.workspace_limit = int(workspace_limit)
        h = ctypes.c_void_p()
        _check(load().rrs_submit(self.handle, ds.handle, NOTIONS[notion],
                                 Z.ctypes.data_as(ctypes.c_void_p), Z.shape[0], int(K),
                                 int(n_refine), float(cap_shrink), int(seed), ctypes.byref(o),
                                 ctypes.byref(h)))
        return Request(h, Z.shape[0], notion)

    def stats(self) -> dict:
        st = rrs_ctx_stats()
        _check(load().rrs_ctx_get_stats(self.handle, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in st._fields_}

    def close(self):
        if self.handle is not None:
            _check(load().rrs_ctx_destroy(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
