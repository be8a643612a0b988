"""GPU Mahalanobis depth D_M(L) against the oracle's binary64 definition.
Both are binary64 but sum in different orders (the covariance over n points
in 4096-point chunks on the matrix cores); with the covariance condition
number kappa the relative difference is of order kappa n 2^-53, so the test
allows 1e-9 relative on the well-conditioned laws used here."""
import sys

import numpy as np
import pytest

import oracle
from paper_2506_08262_amd import ranking, rrs, workloads

pytestmark = pytest.mark.gpu

TOL = 1e-9


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("n,d,law", [(50, 1, "gaussian"), (777, 2, "gaussian"),
                                     (4097, 5, "exponential"), (10000, 17, "mixture"),
                                     (20001, 50, "toeplitz"), (100000, 150, "toeplitz")])
def test_maha_matches_oracle(n, d, law):
    _say("maha", n, d, law)
    if law == "toeplitz" and d > 50:
        rng = np.random.default_rng(d)
        X = ranking.sample(rng, n, d, "gaussian")
        Z = X[rng.choice(n, size=300, replace=False)]
    else:
        w = workloads.small("projection", n, d, 40, 10, 1, 0.5, law=law, seed_cfg=n + d)
        X, Z = w.X, w.Z
    got = rrs.rrs_depth_mahalanobis(X, Z)
    ref = oracle.mahalanobis_depth(X, Z)
    rel = np.abs(got - ref) / ref
    _say("  max rel", rel.max())
    assert rel.max() <= TOL


def test_maha_device_pointers_and_affine_invariance():
    import torch
    rng = np.random.default_rng(4)
    X = rng.standard_normal((3000, 4)) @ np.array([[1.0, 0, 0, 0], [0.3, 2.0, 0, 0],
                                                   [0, 0.1, 0.5, 0], [1.0, 0, 0, 1.0]])
    Z = rng.standard_normal((64, 4))
    dev = torch.device("cuda:0")
    got = rrs.rrs_depth_mahalanobis(torch.from_numpy(X).to(dev), torch.from_numpy(Z).to(dev))
    torch.cuda.synchronize()
    ref = oracle.mahalanobis_depth(X, Z)
    assert np.max(np.abs(got.cpu().numpy() - ref) / ref) <= TOL
    A = rng.standard_normal((4, 4)) + 3 * np.eye(4)
    b = rng.standard_normal(4)
    got2 = rrs.rrs_depth_mahalanobis(X @ A.T + b, Z @ A.T + b)
    assert np.max(np.abs(got2 - ref) / ref) <= 1e-8


def test_maha_rejects_singular_covariance():
    X = np.zeros((10, 3))
    X[:, 0] = np.arange(10.0)
    with pytest.raises(rrs.RRSError) as ei:
        rrs.rrs_depth_mahalanobis(X, np.zeros((2, 3)))
    assert ei.value.status == rrs.RRS_E_INVAL
