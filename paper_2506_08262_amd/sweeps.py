"""Hyperparameter convergence sweeps of RRS projection depth (Section
"Hyperparameter fine-tuning" of Leone, Mozharovskyi & Bounie, arXiv
2506.08262: "Convergence and spherical cap shrinkage" and "Interdependence of
refinements and directions", with the supplementary figure for more
refinement counts).

Data: N(0, Sigma) with the Toeplitz Sigma_ij = 2^-|i-j|, or a multivariate
exponential law (independent Exp(1) marginals mixed by a seeded rotation).
Depths come from the library on the GPU (projection depth, binary32 matrix-core
form with binary64 recheck: results identical to the binary64 recipe).

alpha sweep:  a reference depth per point (the minimum over several runs with
  many directions and refinements), then the mean squared error of the depth
  against it over a grid of alpha, refinements and directions;
grid sweep:   for each dimension, the mean squared error of every
  (directions, refinements) pair against the lowest depth found for the point
  over the whole grid, and the fewest refinements that bring each point within
  1e-4.

    python -m paper_2506_08262_amd.sweeps alpha --n 50000 --d 50 --points 50
    python -m paper_2506_08262_amd.sweeps grid --n 10000 --dims 5 25 50 --points 50
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def toeplitz_gaussian(rng, n: int, d: int) -> np.ndarray:
    idx = np.arange(d)
    S = 2.0 ** (-np.abs(idx[:, None] - idx[None, :]))
    return rng.standard_normal((n, d)) @ np.linalg.cholesky(S).T


def rotated_exponential(rng, n: int, d: int) -> np.ndarray:
    Q, R = np.linalg.qr(rng.standard_normal((d, d)))
    Q = Q * np.sign(np.diag(R))
    return rng.exponential(1.0, (n, d)) @ Q.T


LAWS = {"gaussian": toeplitz_gaussian, "exponential": rotated_exponential}


def _depth(X, Z, K, r, alpha, seed, area_cap=False, precision="f32"):
    """Projection depth; refinements of 65536 or more directions (beyond the
    matrix-core forms' column index) run in binary64, which gives the same
    depths as the binary32 form with its binary64 recheck."""
    from . import rrs
    if precision != "f64" and -(-int(K) // int(r)) >= 65536:
        precision = "f64"
    return rrs.depth("projection", X, Z, int(K), int(r), float(alpha), int(seed),
                     precision=precision, area_cap=area_cap)["depth"].cpu().numpy()


def alpha_sweep(n=50_000, d=50, points=50, law="gaussian", ref_K=3_000_000, ref_r=100,
                ref_alpha=0.9, ref_runs=3, alphas=(0.6, 0.7, 0.8, 0.9),
                Ks=(200, 500, 1000, 2000, 5000, 10000, 20000, 50000, 90000), rs=(25, 30, 35),
                area_cap=False, seed=0, device="cuda:0"):
    """Mean squared error of projection depth against a reference minimum
    over a grid of cap shrinkage alpha, directions K and refinements r."""
    import torch
    rng = np.random.default_rng(seed)
    Xh = LAWS[law](rng, n, d)
    Zh = Xh[rng.choice(n, size=points, replace=False)]
    X = torch.from_numpy(Xh).to(device)
    Z = torch.from_numpy(Zh).to(device)
    t0 = time.perf_counter()
    ref = np.min([_depth(X, Z, ref_K, ref_r, ref_alpha, 1000 + i) for i in range(ref_runs)],
                 axis=0)
    out = {"mode": "alpha", "law": law, "n": n, "d": d, "points": points,
           "reference": {"K": ref_K, "r": ref_r, "alpha": ref_alpha, "runs": ref_runs,
                         "seconds": time.perf_counter() - t0},
           "area_cap": area_cap, "grid": []}
    print(f"[sweeps] reference done ({out['reference']['seconds']:.1f} s)", file=sys.stderr,
          flush=True)
    for r in rs:
        for a in alphas:
            for K in Ks:
                if K < r:
                    continue
                D = _depth(X, Z, K, r, a, 7, area_cap=area_cap)
                err = (D - ref) ** 2
                out["grid"].append({"r": r, "alpha": a, "K": K, "mse_mean": float(err.mean()),
                                    "mse_max": float(err.max()),
                                    "below_ref": int(np.count_nonzero(D < ref))})
            print(f"[sweeps] r={r} alpha={a} done", file=sys.stderr, flush=True)
    return out


def grid_sweep(n=10_000, dims=(5, 25, 50, 100), points=50, law="gaussian",
               Ks=(200, 1000, 5000, 20000, 100000), rs=(1, 5, 10, 25, 50, 100, 175),
               alpha=0.9, tol=1e-4, seed=0, device="cuda:0"):
    """Per dimension: depth for every (K, r) of the grid; the reference of a
    point is the lowest depth found for it; reported are the mean squared
    errors and, per K, the fewest refinements with every point within tol
    and the mean over points of their fewest refinements within tol."""
    import torch
    res = {"mode": "grid", "law": law, "n": n, "points": points, "alpha": alpha, "tol": tol,
           "dims": []}
    for d in dims:
        rng = np.random.default_rng(seed + d)
        Xh = LAWS[law](rng, n, d)
        Zh = Xh[rng.choice(n, size=points, replace=False)]
        X = torch.from_numpy(Xh).to(device)
        Z = torch.from_numpy(Zh).to(device)
        D = {}
        for K in Ks:
            for r in rs:
                if K < r:
                    continue
                D[(K, r)] = _depth(X, Z, K, r, alpha, 11)
        ref = np.min(np.stack(list(D.values())), axis=0)
        entry = {"d": d, "cells": []}
        for K in Ks:
            conv_all, first = None, np.full(points, np.nan)
            for r in rs:
                if (K, r) not in D:
                    continue
                err = (D[(K, r)] - ref) ** 2
                entry["cells"].append({"K": K, "r": r, "mse_mean": float(err.mean())})
                ok = err <= tol
                first = np.where(np.isnan(first) & ok, r, first)
                if conv_all is None and ok.all():
                    conv_all = r
            entry.setdefault("per_K", []).append(
                {"K": K, "min_r_all_points": conv_all,
                 "mean_min_r_converged": float(np.nanmean(first)) if np.any(~np.isnan(first))
                 else None, "converged_points": int(np.count_nonzero(~np.isnan(first)))})
        res["dims"].append(entry)
        print(f"[sweeps] d={d} done", file=sys.stderr, flush=True)
    return res


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="mode", required=True)
    a = sub.add_parser("alpha")
    a.add_argument("--n", type=int, default=50_000)
    a.add_argument("--d", type=int, default=50)
    a.add_argument("--points", type=int, default=50)
    a.add_argument("--law", default="gaussian", choices=sorted(LAWS))
    a.add_argument("--ref-K", type=int, default=3_000_000)
    a.add_argument("--ref-r", type=int, default=100)
    a.add_argument("--ref-runs", type=int, default=3)
    a.add_argument("--alphas", type=float, nargs="*", default=[0.6, 0.7, 0.8, 0.9])
    a.add_argument("--Ks", type=int, nargs="*",
                   default=[200, 500, 1000, 2000, 5000, 10000, 20000, 50000, 90000])
    a.add_argument("--rs", type=int, nargs="*", default=[25, 30, 35])
    a.add_argument("--area-cap", action="store_true")
    g = sub.add_parser("grid")
    g.add_argument("--n", type=int, default=10_000)
    g.add_argument("--dims", type=int, nargs="*", default=[5, 25, 50, 100])
    g.add_argument("--points", type=int, default=50)
    g.add_argument("--law", default="gaussian", choices=sorted(LAWS))
    g.add_argument("--Ks", type=int, nargs="*", default=[200, 1000, 5000, 20000, 100000])
    g.add_argument("--rs", type=int, nargs="*", default=[1, 5, 10, 25, 50, 100, 175])
    g.add_argument("--alpha", type=float, default=0.9)
    args = ap.parse_args(argv)
    if args.mode == "alpha":
        r = alpha_sweep(args.n, args.d, args.points, args.law, args.ref_K, args.ref_r, 0.9,
                        args.ref_runs, args.alphas, args.Ks, args.rs, args.area_cap)
    else:
        r = grid_sweep(args.n, args.dims, args.points, args.law, args.Ks, args.rs, args.alpha)
    print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
