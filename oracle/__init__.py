"""FP64 CPU oracle for Refined Random Search depths -- test infrastructure.

This package is the independent, slow reference that the GPU library is
checked against.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import it; the product package never does, and this
package never imports the product package.

The arithmetic lives in ``rrs_oracle.c`` (plain C, FP64, explicit ``fma``,
built with ``-ffp-contract=off``); this module only builds it and marshals
arguments with ctypes.  See the C file's header for the paper passage each
function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rrs_oracle.c")
LIB = os.path.join(HERE, "librrs_oracle.so")

HALFSPACE, PROJECTION, APD = 0, 1, 2
NOTIONS = {"halfspace": HALFSPACE, "projection": PROJECTION, "apd": APD}


# -O3 with the x86-64-v3 level (AVX2 and hardware FMA, so fma() is one
# correctly rounded instruction instead of a library call); no -ffast-math and
# no contraction, so results are bit-identical to any IEEE build of the file.
# Not -march=native: the library is built once and may run on other x86 hosts.
CFLAGS = ["-O3", "-march=x86-64-v3", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp"]
CFLAGS_TEXT = "gcc " + " ".join(CFLAGS)


def build(force: bool = True) -> str:
    """Compile the oracle into ``librrs_oracle.so`` next to this file."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", *CFLAGS, "-shared", "-fPIC", SRC, "-o", LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = ctypes.CDLL(LIB)
        i64, u64, i32, dbl = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_double
        p = ctypes.c_void_p
        L.o_philox4x64_10.argtypes = [p, p, p]
        L.o_uniform.argtypes = [u64]
        L.o_uniform.restype = dbl
        L.o_log.argtypes = [dbl]
        L.o_log.restype = dbl
        L.o_sincos_halfpi.argtypes = [dbl, p, p]
        L.o_gauss_pair.argtypes = [dbl, dbl, p, p]
        L.o_direction.argtypes = [u64, u64, u64, u64, i64, dbl, p, p]
        L.o_direction_ex.argtypes = [u64, u64, u64, u64, i64, dbl, p, p, ctypes.c_int,
                                     ctypes.c_int]
        L.o_area_cap_angle.argtypes = [dbl, dbl, i64, p, p]
        L.o_project.argtypes = [p, i64, i64, p, p, p]
        L.o_uni_halfspace.argtypes = [p, i64]
        L.o_uni_halfspace.restype = i64
        L.o_uni_projection.argtypes = [p, i64, p, p]
        L.o_uni_projection.restype = dbl
        L.o_uni_apd.argtypes = [p, i64, p, p]
        L.o_uni_apd.restype = dbl
        L.o_rrs_query.argtypes = [ctypes.c_int, p, i64, i64, p, u64, i64, i32, dbl, u64,
                                  p, p, p, p]
        L.o_rrs_depth.argtypes = [ctypes.c_int, p, i64, i64, p, i64, u64, i64, i32, dbl,
                                  u64, p, p, p, i32]
        L.o_rrs_depth_idx.argtypes = [ctypes.c_int, p, i64, i64, p, i64, p, i64, i32, dbl,
                                      u64, p, p, p, i32]
        L.o_rrs_depth_idx_mode.argtypes = [ctypes.c_int, p, i64, i64, p, i64, p, i64, i32,
                                           dbl, u64, p, p, p, i32, ctypes.c_int, ctypes.c_int]
        L.o_rrs_replay.argtypes = [ctypes.c_int, p, i64, i64, p, u64, i64, i32, dbl, u64, p, p]
        L.o_max_threads.restype = i32
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# Building blocks (exposed for the pin tests)
# --------------------------------------------------------------------------
def philox4x64_10(counter, key) -> np.ndarray:
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().o_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(word: int) -> float:
    return lib().o_uniform(int(word))


def log(x: float) -> float:
    return lib().o_log(float(x))


def sincos_halfpi(f: float):
    s = ctypes.c_double()
    c = ctypes.c_double()
    lib().o_sincos_halfpi(float(f), ctypes.byref(s), ctypes.byref(c))
    return s.value, c.value


def gauss_pair(u1: float, u2: float):
    a = ctypes.c_double()
    b = ctypes.c_double()
    lib().o_gauss_pair(float(u1), float(u2), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def direction(seed: int, q: int, l: int, j: int, d: int, phi: float, pole,
              first_cap: bool = False, area_cap: bool = False) -> np.ndarray:
    pole = _f64(pole)
    assert pole.shape == (d,)
    u = np.zeros(d, dtype=np.float64)
    if first_cap or area_cap:
        lib().o_direction_ex(int(seed), int(q), int(l), int(j), int(d), float(phi), _ptr(pole),
                             _ptr(u), 1 if first_cap else 0, 1 if area_cap else 0)
    else:
        lib().o_direction(int(seed), int(q), int(l), int(j), int(d), float(phi), _ptr(pole),
                          _ptr(u))
    return u


def area_cap_angle(u: float, phi: float, d: int):
    """(sin theta, cos theta) of the area-uniform cap angle for uniform u."""
    s = ctypes.c_double()
    c = ctypes.c_double()
    lib().o_area_cap_angle(float(u), float(phi), int(d), ctypes.byref(s), ctypes.byref(c))
    return s.value, c.value


def project(X, z, u) -> np.ndarray:
    X = _f64(X)
    n, d = X.shape
    z = _f64(z)
    u = _f64(u)
    t = np.zeros(n, dtype=np.float64)
    lib().o_project(_ptr(X), n, d, _ptr(z), _ptr(u), _ptr(t))
    return t


def uni_halfspace(t) -> int:
    t = _f64(t)
    return int(lib().o_uni_halfspace(_ptr(t), t.shape[0]))


def uni_projection(t):
    t = _f64(t)
    med = ctypes.c_double()
    mad = ctypes.c_double()
    D = lib().o_uni_projection(_ptr(t), t.shape[0], ctypes.byref(med), ctypes.byref(mad))
    return D, med.value, mad.value


def uni_apd(t):
    t = _f64(t)
    med = ctypes.c_double()
    madp = ctypes.c_double()
    D = lib().o_uni_apd(_ptr(t), t.shape[0], ctypes.byref(med), ctypes.byref(madp))
    return D, med.value, madp.value


# --------------------------------------------------------------------------
# RRS depth
# --------------------------------------------------------------------------
def rrs_query(notion: str, X, z, q: int, K: int, n_refine: int, cap_shrink: float,
              seed: int):
    """One query with its full trace: returns (depth, count, pole, trace) where
    trace[l] = (j*, improved, min value of refinement l)."""
    X = _f64(X)
    n, d = X.shape
    z = _f64(z)
    depth = ctypes.c_double()
    count = ctypes.c_int64()
    pole = np.zeros(d, dtype=np.float64)
    trace = np.zeros(3 * n_refine, dtype=np.int64)
    lib().o_rrs_query(NOTIONS[notion], _ptr(X), n, d, _ptr(z), int(q), int(K), int(n_refine),
                      float(cap_shrink), int(seed), ctypes.byref(depth), ctypes.byref(count),
                      _ptr(pole), _ptr(trace))
    tr = trace.reshape(n_refine, 3)
    vals = tr[:, 2].copy().view(np.float64)
    return depth.value, count.value, pole, [(int(a), bool(b), float(v))
                                            for a, b, v in zip(tr[:, 0], tr[:, 1], vals)]


def rrs_depth(notion: str, X, Z, K: int, n_refine: int, cap_shrink: float, seed: int,
              q0: int = 0, nthreads: int = 0, with_poles: bool = False):
    """Depth of every row of Z (query i keyed by stream index q0 + i).
    Returns depth (and counts for halfspace, poles if asked)."""
    X = _f64(X)
    Z = _f64(Z)
    n, d = X.shape
    nq = Z.shape[0]
    assert Z.shape[1] == d
    depth = np.zeros(nq, dtype=np.float64)
    count = np.zeros(nq, dtype=np.int64)
    poles = np.zeros((nq, d), dtype=np.float64) if with_poles else None
    lib().o_rrs_depth(NOTIONS[notion], _ptr(X), n, d, _ptr(Z), nq, int(q0), int(K),
                      int(n_refine), float(cap_shrink), int(seed), _ptr(depth), _ptr(count),
                      _ptr(poles) if with_poles else None, int(nthreads))
    out = {"depth": depth}
    if notion == "halfspace":
        out["count"] = count
    if with_poles:
        out["poles"] = poles
    return out


def rrs_depth_idx(notion: str, X, Z, qidx, K: int, n_refine: int, cap_shrink: float,
                  seed: int, nthreads: int = 0, with_poles: bool = False,
                  first_cap: bool = False, area_cap: bool = False):
    """Depth of every row of Z, row i keyed by stream index qidx[i].  first_cap:
    the first refinement draws from the pi/2 cap around e1 (Alg. S4) instead of
    the whole sphere; area_cap: cap directions uniform in area instead of in
    angle."""
    X = _f64(X)
    Z = _f64(Z)
    n, d = X.shape
    nq = Z.shape[0]
    q = np.ascontiguousarray(qidx, dtype=np.uint64)
    assert q.shape == (nq,) and Z.shape[1] == d
    depth = np.zeros(nq, dtype=np.float64)
    count = np.zeros(nq, dtype=np.int64)
    poles = np.zeros((nq, d), dtype=np.float64) if with_poles else None
    lib().o_rrs_depth_idx_mode(NOTIONS[notion], _ptr(X), n, d, _ptr(Z), nq, _ptr(q), int(K),
                               int(n_refine), float(cap_shrink), int(seed), _ptr(depth),
                               _ptr(count), _ptr(poles) if with_poles else None, int(nthreads),
                               1 if first_cap else 0, 1 if area_cap else 0)
    out = {"depth": depth}
    if notion == "halfspace":
        out["count"] = count
    if with_poles:
        out["poles"] = poles
    return out


def rrs_replay(notion: str, X, z, q: int, K: int, n_refine: int, cap_shrink: float, seed: int,
               traj) -> np.ndarray:
    """Exact depths along a given trajectory (rows of traj: chosen index,
    improved).  Returns [n_refine, 3]: exact minimum over the refinement's
    directions, exact depth of the chosen direction, first exact argmin."""
    X = _f64(X)
    n, d = X.shape
    z = _f64(z)
    tr = np.ascontiguousarray(np.asarray(traj, dtype=np.int64)[:, :2])
    t3 = np.zeros((n_refine, 3), dtype=np.int64)
    t3[:, :2] = tr
    out = np.zeros((n_refine, 3), dtype=np.float64)
    lib().o_rrs_replay(NOTIONS[notion], _ptr(X), n, d, _ptr(z), int(q), int(K), int(n_refine),
                       float(cap_shrink), int(seed), _ptr(t3), _ptr(out))
    return out


def mahalanobis_depth(X, Z) -> np.ndarray:
    """D_M(L) of the ranking study (Sec. "Center-outward ordering precision and
    depth benchmark"): (1 + (z - mu)' Sigma^-1 (z - mu))^-1 with mu the mean of
    X and Sigma its maximum-likelihood covariance (divisor n); the definition
    written out in binary64 numpy (mean, covariance, linear solve)."""
    X = _f64(X)
    Z = _f64(Z)
    mu = X.mean(axis=0)
    A = X - mu
    S = A.T @ A / X.shape[0]
    B = Z - mu
    q = np.sum(B * np.linalg.solve(S, B.T).T, axis=1)
    return 1.0 / (1.0 + q)


def max_threads() -> int:
    return int(lib().o_max_threads())
