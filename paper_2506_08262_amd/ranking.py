"""Center-outward ranking study: how well projection depth and asymmetric
projection depth order points of a known law, measured by rank correlation
with the law's density (Section "Center-outward ordering precision and depth
benchmark" of Leone, Mozharovskyi & Bounie, arXiv 2506.08262, Tables 4-5).

Set-up of that section: n points from N(0, Sigma) with the Toeplitz matrix
Sigma_ij = 2^-|i-j| (or a multivariate Student t with that scatter), depths of
randomly chosen points of the data set computed by RRS with 40 refinements,
100,000 directions and alpha = 0.9, then Spearman's rho and Kendall's tau of
each depth against the true density, beside the Mahalanobis depth with the
sample mean and the maximum-likelihood covariance.  The depths, the
Mahalanobis depth included, come from the library on the GPU; the density and
the correlations are evaluated here on the host (scipy).

    python -m paper_2506_08262_amd.ranking --dims 5 10 25 50 --queries 500
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def toeplitz_sigma(d: int) -> np.ndarray:
    """Sigma_ij = 2^-|i-j| (the covariance of the paper's Gaussian study)."""
    idx = np.arange(d)
    return 2.0 ** (-np.abs(idx[:, None] - idx[None, :]))


def sample(rng, n: int, d: int, law: str = "gaussian", nu: float = 0.0) -> np.ndarray:
    """n points of N(0, Sigma) or of the multivariate t with nu degrees of
    freedom and scatter Sigma (Gaussian vector over sqrt(chi2_nu / nu))."""
    L = np.linalg.cholesky(toeplitz_sigma(d))
    g = rng.standard_normal((n, d)) @ L.T
    if law == "gaussian":
        return g
    if law == "t":
        return g / np.sqrt(rng.chisquare(nu, (n, 1)) / nu)
    raise ValueError(f"unknown law {law!r}")


def true_logpdf(Z: np.ndarray, law: str = "gaussian", nu: float = 0.0) -> np.ndarray:
    """Log density of the generating law at the rows of Z."""
    from scipy import stats
    d = Z.shape[1]
    S = toeplitz_sigma(d)
    if law == "gaussian":
        return stats.multivariate_normal(mean=np.zeros(d), cov=S).logpdf(Z)
    return stats.multivariate_t(loc=np.zeros(d), shape=S, df=nu).logpdf(Z)


def rank_correlations(a: np.ndarray, b: np.ndarray) -> dict:
    """Spearman's rho and Kendall's tau (tau-b) of two score vectors."""
    from scipy import stats
    return {"spearman": float(stats.spearmanr(a, b).statistic),
            "kendall": float(stats.kendalltau(a, b).statistic)}


def study(d: int, n: int = 100_000, queries: int = 5000, K: int = 100_000, n_refine: int = 40,
          cap_shrink: float = 0.9, law: str = "gaussian", nu: float = 0.0, seed: int = 0,
          precision: str = "f32", device: str = "cuda:0", first_cap: bool = False,
          chunk: int = 500) -> dict:
    """One column of the study: depths D_P and D_AP and D_M(L) (all on the
    GPU) of `queries` points drawn from the n-point data set, correlated with
    the true density and with each other.  first_cap: refinement 1 draws in
    the half-angle pi/2 cap around e1 (Alg. S4) instead of on the sphere.
    The queries go to the library in calls of `chunk` rows, each with its
    stream offset, so the depths are those of a single call."""
    import torch

    from . import rrs

    rng = np.random.default_rng(seed)
    X = sample(rng, n, d, law, nu)
    pick = rng.choice(n, size=queries, replace=False)
    Z = X[pick]
    Xt = torch.from_numpy(X).to(device)
    Zt = torch.from_numpy(Z).to(device)
    out = {"d": d, "n": n, "queries": queries, "K": K, "n_refine": n_refine,
           "cap_shrink": cap_shrink, "law": law, "nu": nu, "precision": precision,
           "first_cap": first_cap}
    depths = {}
    for notion in ("projection", "apd"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        parts = []
        for q0 in range(0, queries, chunk):
            res = rrs.depth(notion, Xt, Zt[q0:q0 + chunk], K, n_refine, cap_shrink, seed,
                            precision=precision, first_cap=first_cap, query_offset=q0)
            parts.append(res["depth"])
            if queries > chunk:
                torch.cuda.synchronize()
                print(f"[ranking] {notion}: {min(q0 + chunk, queries)}/{queries} queries",
                      file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        depths[notion] = torch.cat(parts).cpu().numpy()
        print(f"[ranking] {law} nu={nu} d={d} {notion}: {sec:.1f} s", file=sys.stderr, flush=True)
        m = -(-K // n_refine)
        out[f"{notion}_seconds"] = sec
        out[f"{notion}_projections_per_s"] = queries * n_refine * m * n / sec
    logpdf = true_logpdf(Z, law, nu)
    dm = rrs.rrs_depth_mahalanobis(Xt, Zt).cpu().numpy()
    out["pdf_x_DP"] = rank_correlations(logpdf, depths["projection"])
    out["pdf_x_DAP"] = rank_correlations(logpdf, depths["apd"])
    out["pdf_x_DML"] = rank_correlations(logpdf, dm)
    out["DP_x_DAP"] = rank_correlations(depths["projection"], depths["apd"])
    return out


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--dims", type=int, nargs="*", default=[5, 10, 25, 50])
    ap.add_argument("--nus", type=float, nargs="*", default=[],
                    help="also the Student t laws with these degrees of freedom (d = 50)")
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--queries", type=int, default=500)
    ap.add_argument("--K", type=int, default=100_000)
    ap.add_argument("--n-refine", type=int, default=40)
    ap.add_argument("--cap-shrink", type=float, default=0.9)
    ap.add_argument("--precision", default="f32")
    ap.add_argument("--t-precision", default="f32",
                    help="precision form for the Student t laws (their heavy tails switch the "
                         "matrix-core forms' selects to per-point error bounds)")
    ap.add_argument("--first-cap", action="store_true",
                    help="refinement 1 in the pi/2 cap around e1 instead of on the sphere")
    ap.add_argument("--chunk", type=int, default=500,
                    help="queries per library call (stream offsets keep the depths of one call)")
    args = ap.parse_args(argv)
    runs = [("gaussian", 0.0, d) for d in args.dims] + [("t", nu, 50) for nu in args.nus]
    for law, nu, d in runs:
        r = study(d, args.n, args.queries, args.K, args.n_refine, args.cap_shrink, law, nu,
                  precision=args.precision if law == "gaussian" else args.t_precision,
                  first_cap=args.first_cap, chunk=args.chunk)
        print(json.dumps(r), flush=True)
        print(f"[ranking] {law} nu={nu} d={d} done", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
