"""Pins of the oracle's Mahalanobis depth D_M(L) (mean, maximum-likelihood
covariance): closed forms of designs whose moments are known exactly, the
maximum at the mean, affine invariance, and the population value for a large
Gaussian sample."""
import numpy as np
import pytest

import oracle


def test_one_dimension_closed_form():
    # X = {0, 1, 2, 3}: mean 3/2, variance (9/4 + 1/4 + 1/4 + 9/4) / 4 = 5/4
    X = np.array([[0.0], [1.0], [2.0], [3.0]])
    Z = np.array([[0.0], [1.5], [4.0]])
    want = np.array([1.0 / (1.0 + 2.25 / 1.25), 1.0, 1.0 / (1.0 + 6.25 / 1.25)])
    assert np.allclose(oracle.mahalanobis_depth(X, Z), want, rtol=1e-15, atol=0)


@pytest.mark.parametrize("d,a", [(2, 1.0), (5, 3.0), (12, 0.25)])
def test_cross_design_closed_form(d, a):
    # the 2d points +-a e_i: mean 0, covariance (a^2 / d) I, so
    # D(z) = 1 / (1 + d |z|^2 / a^2)
    X = np.concatenate([a * np.eye(d), -a * np.eye(d)])
    rng = np.random.default_rng(d)
    Z = rng.standard_normal((7, d))
    want = 1.0 / (1.0 + d * np.sum(Z * Z, axis=1) / (a * a))
    assert np.allclose(oracle.mahalanobis_depth(X, Z), want, rtol=1e-13, atol=0)


def test_maximum_at_the_mean_and_affine_invariance():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((500, 3)) @ np.array([[2.0, 0, 0], [0.5, 1.0, 0], [0, 0.3, 0.7]])
    Z = rng.standard_normal((20, 3))
    D = oracle.mahalanobis_depth(X, Z)
    assert np.all((D > 0) & (D <= 1))
    assert abs(oracle.mahalanobis_depth(X, X.mean(axis=0, keepdims=True))[0] - 1.0) < 1e-12
    A = np.array([[1.0, 2.0, 0.0], [0.0, 1.0, -1.0], [3.0, 0.0, 1.0]])
    b = np.array([5.0, -2.0, 0.5])
    D2 = oracle.mahalanobis_depth(X @ A.T + b, Z @ A.T + b)
    assert np.allclose(D, D2, rtol=1e-9, atol=0)


def test_population_value_for_a_large_gaussian_sample():
    # N(0, S): D -> 1 / (1 + z' S^-1 z) with a sampling error O(n^-1/2)
    S = np.array([[2.0, 0.6], [0.6, 1.0]])
    rng = np.random.default_rng(9)
    X = rng.standard_normal((400_000, 2)) @ np.linalg.cholesky(S).T
    Z = np.array([[0.0, 0.0], [1.0, 1.0], [-2.0, 0.5]])
    Si = np.linalg.inv(S)
    want = 1.0 / (1.0 + np.einsum("ij,jk,ik->i", Z, Si, Z))
    assert np.allclose(oracle.mahalanobis_depth(X, Z), want, rtol=0, atol=0.01)
