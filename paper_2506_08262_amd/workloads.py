"""Seeded synthetic inputs for the depth workloads.

This module only draws data sets and queries (numpy ``default_rng``); it holds
none of the depth method's arithmetic, so both the GPU path's callers and the
oracle's callers can take their inputs from here.

Each workload mirrors the shapes, laws and hyper-parameters of the evaluation
configurations (all synthetic, as in the paper's own experiments):

* ``c1``  halfspace, X 1000x5 i.i.d. N(0,1), 100 queries of the same law,
          K=1000, r=10, alpha=0.5.
* ``c1b`` halfspace, X 200x2 N(0,I), 100 queries of the same law plus 10 far
          outside the hull, K=1000, r=10, alpha=0.5 (checked against exact
          depth in the plane).
* ``c2``  projection depth, X 10000x20 ~ N(0, S), S = G G^T / d (Wishart(d,I)/d),
          800 queries from N(0,S) and 200 multivariate Cauchy, K=5000, r=20,
          alpha=0.5.
* ``c3``  asymmetric projection depth, X 100000x50 = E R^T with E i.i.d.
          Exp(1) and R a Haar rotation, 10000 queries of the same law,
          K=10000, r=20, alpha=0.5.
* ``c5``  halfspace / projection, X 100000x100 from a 3-component Gaussian
          mixture (means N(0,I), covariances Wishart(d,I)/d), 500 queries,
          K=5000, r=25, alpha=0.6.
* ``c4``  serving stream (``c4_stream``): Poisson arrivals at 200 requests/s,
          halfspace or projection (1/2 each), each request with its own data
          set: n log-uniform in [1e3, 1e5], d uniform in {3..100}, N(0,I) or
          multivariate t(3) (1/2 each), 1..1000 queries of the same law,
          K in {1000, 5000, 10000}, r=10, alpha=0.5; seed_cfg 5.
* ``toeplitz`` the paper's experimental law N(0, T), T_ij = 2^-|i-j|.

``seed_cfg`` seeds numpy; the RRS direction stream is keyed separately by
``rrs_seed`` (0 everywhere unless a test asks otherwise).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = ["Workload", "make", "gaussian", "toeplitz_gaussian", "wishart_gaussian",
           "rotated_exponential", "gaussian_mixture", "student_t", "WORKLOADS", "c4_stream",
           "ServingRequest"]


@dataclass
class Workload:
    name: str
    notion: str
    X: np.ndarray
    Z: np.ndarray
    K: int
    n_refine: int
    cap_shrink: float
    rrs_seed: int = 0
    recipe: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def d(self) -> int:
        return int(self.X.shape[1])

    @property
    def nq(self) -> int:
        return int(self.Z.shape[0])

    @property
    def m_dirs(self) -> int:
        return -(-self.K // self.n_refine)

    @property
    def projections(self) -> int:
        """query x direction x point projections of one full run."""
        return self.nq * self.n_refine * self.m_dirs * self.n


def gaussian(rng, n, d):
    return rng.standard_normal((n, d))


def toeplitz_gaussian(rng, n, d):
    idx = np.arange(d)
    T = 2.0 ** (-np.abs(idx[:, None] - idx[None, :]))
    L = np.linalg.cholesky(T)
    return rng.standard_normal((n, d)) @ L.T


def wishart_factor(rng, d):
    """G with G G^T / d ~ Wishart(d, I) / d."""
    return rng.standard_normal((d, d)) / np.sqrt(d)


def wishart_gaussian(rng, n, d, G=None):
    G = wishart_factor(rng, d) if G is None else G
    return rng.standard_normal((n, d)) @ G.T, G


def multivariate_cauchy(rng, n, d, G):
    g = rng.standard_normal((n, d)) @ G.T
    w = np.abs(rng.standard_normal((n, 1)))
    return g / w


def haar_rotation(rng, d):
    A = rng.standard_normal((d, d))
    Q, R = np.linalg.qr(A)
    return Q * np.sign(np.diag(R))[None, :]


def rotated_exponential(rng, n, d, R=None):
    R = haar_rotation(rng, d) if R is None else R
    return rng.exponential(1.0, (n, d)) @ R.T, R


def gaussian_mixture(rng, n, d, comps=None, k=3):
    if comps is None:
        comps = [(rng.standard_normal(d), wishart_factor(rng, d)) for _ in range(k)]
    lab = rng.integers(0, len(comps), n)
    out = np.empty((n, d))
    for c, (mu, G) in enumerate(comps):
        sel = lab == c
        out[sel] = mu[None, :] + rng.standard_normal((int(sel.sum()), d)) @ G.T
    return out, comps


def student_t(rng, n, d, nu):
    g = rng.standard_normal((n, d))
    w = rng.chisquare(nu, (n, 1)) / nu
    return g / np.sqrt(w)


def _c1(scale=1.0):
    rng = np.random.default_rng(1)
    n, d, nq = 1000, 5, 100
    X = gaussian(rng, n, d)
    Z = gaussian(rng, nq, d)
    return Workload("c1", "halfspace", X, Z, 1000, 10, 0.5, 0,
                    "X 1000x5 iid N(0,1); Z 100 from the same law; seed_cfg 1")


def _c1b(scale=1.0):
    rng = np.random.default_rng(2)
    n, d = 200, 2
    X = gaussian(rng, n, d)
    Zin = gaussian(rng, 100, d)
    ang = rng.uniform(0, 2 * np.pi, 10)
    R = 10.0 * np.max(np.linalg.norm(X, axis=1))
    Zout = R * np.stack([np.cos(ang), np.sin(ang)], axis=1)
    Z = np.concatenate([Zin, Zout])
    return Workload("c1b", "halfspace", X, Z, 1000, 10, 0.5, 0,
                    "X 200x2 N(0,I); Z 100 same law + 10 at 10x max|x|; seed_cfg 2")


def _c2(scale=1.0):
    rng = np.random.default_rng(3)
    n, d = 10000, 20
    X, G = wishart_gaussian(rng, n, d)
    Zin, _ = wishart_gaussian(rng, 800, d, G)
    Zc = multivariate_cauchy(rng, 200, d, G)
    Z = np.concatenate([Zin, Zc])
    return Workload("c2", "projection", X, Z, 5000, 20, 0.5, 0,
                    "X 10000x20 N(0,GG^T/d); Z 800 same law + 200 multivariate Cauchy; "
                    "seed_cfg 3")


def _c3(scale=1.0):
    rng = np.random.default_rng(4)
    n, d, nq = 100000, 50, 10000
    X, R = rotated_exponential(rng, n, d)
    Z, _ = rotated_exponential(rng, nq, d, R)
    return Workload("c3", "apd", X, Z, 10000, 20, 0.5, 0,
                    "X 100000x50 = Exp(1) marginals x Haar rotation; Z 10000 same law; "
                    "seed_cfg 4")


def _c5(scale=1.0, notion="halfspace"):
    rng = np.random.default_rng(6)
    n, d, nq = 100000, 100, 500
    X, comps = gaussian_mixture(rng, n, d)
    Z, _ = gaussian_mixture(rng, nq, d, comps)
    return Workload("c5", notion, X, Z, 5000, 25, 0.6, 0,
                    "X 100000x100 3-component Gaussian mixture (means N(0,I), Wishart "
                    "covariances); Z 500 from the mixture; seed_cfg 6")


WORKLOADS = {"c1": _c1, "c1b": _c1b, "c2": _c2, "c3": _c3, "c5": _c5}


def make(name: str, **kw) -> Workload:
    return WORKLOADS[name](**kw)


def small(notion: str, n: int, d: int, nq: int, K: int, n_refine: int, cap_shrink: float,
          law: str = "gaussian", seed_cfg: int = 11, rrs_seed: int = 0) -> Workload:
    """A small workload of any shape for parity tests."""
    rng = np.random.default_rng(seed_cfg)
    if law == "gaussian":
        X = gaussian(rng, n, d)
        Z = gaussian(rng, nq, d)
    elif law == "toeplitz":
        X = toeplitz_gaussian(rng, n, d)
        Z = toeplitz_gaussian(rng, nq, d)
    elif law == "exponential":
        X, R = rotated_exponential(rng, n, d)
        Z, _ = rotated_exponential(rng, nq, d, R)
    elif law == "wishart_cauchy":
        X, G = wishart_gaussian(rng, n, d)
        nin = max(nq - nq // 5, 0)
        Zin, _ = wishart_gaussian(rng, nin, d, G)
        Z = np.concatenate([Zin, multivariate_cauchy(rng, nq - nin, d, G)])
    elif law == "mixture":
        X, comps = gaussian_mixture(rng, n, d)
        Z, _ = gaussian_mixture(rng, nq, d, comps)
    elif law == "integer":
        X = rng.integers(-50, 51, (n, d)).astype(np.float64)
        Z = rng.integers(-20, 21, (nq, d)).astype(np.float64)
    elif law.startswith("t") and law[1:].isdigit():
        # multivariate Student t with nu = int(law[1:]) degrees of freedom
        X = student_t(rng, n, d, float(law[1:]))
        Z = student_t(rng, nq, d, float(law[1:]))
    else:
        raise ValueError(law)
    return Workload(f"small-{law}", notion, np.ascontiguousarray(X), np.ascontiguousarray(Z),
                    K, n_refine, cap_shrink, rrs_seed,
                    f"{law} n={n} d={d} nq={nq} seed_cfg={seed_cfg}")


@dataclass
class ServingRequest:
    """One request of the serving stream: arrival time (s from the stream's
    start), its own data set and queries, and the RRS arguments."""
    arrival: float
    notion: str
    X: np.ndarray
    Z: np.ndarray
    K: int
    n_refine: int
    cap_shrink: float
    law: str

    @property
    def projections(self) -> int:
        m = -(-self.K // self.n_refine)
        return self.Z.shape[0] * self.n_refine * m * self.X.shape[0]


def c4_stream(n_requests: int, rate: float = 200.0, seed_cfg: int = 5,
              max_queries: int = 1000):
    """The first n_requests requests of the serving stream (see the module
    notes); max_queries caps the per-request query count below 1000 when a
    shorter run is wanted (the law of the other fields is unchanged)."""
    rng = np.random.default_rng(seed_cfg)
    t = 0.0
    out = []
    for _ in range(n_requests):
        t += rng.exponential(1.0 / rate)
        notion = "halfspace" if rng.random() < 0.5 else "projection"
        n = int(np.floor(10.0 ** rng.uniform(3.0, 5.0)))
        d = int(rng.integers(3, 101))
        law = "gaussian" if rng.random() < 0.5 else "t3"
        nq = int(rng.integers(1, min(1000, max_queries) + 1))
        K = int(rng.choice([1000, 5000, 10000]))
        if law == "gaussian":
            X, Z = gaussian(rng, n, d), gaussian(rng, nq, d)
        else:
            X, Z = student_t(rng, n, d, 3), student_t(rng, nq, d, 3)
        out.append(ServingRequest(t, notion, np.ascontiguousarray(X), np.ascontiguousarray(Z),
                                  K, 10, 0.5, law))
    return out
