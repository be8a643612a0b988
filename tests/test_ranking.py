"""Host-side pieces of the center-outward ranking study (density, rank
correlations), pinned against closed forms written out here."""
import math

import numpy as np
import pytest

from paper_2506_08262_amd import ranking


def test_toeplitz_sigma_entries():
    S = ranking.toeplitz_sigma(4)
    for i in range(4):
        for j in range(4):
            assert S[i, j] == 2.0 ** (-abs(i - j))


def test_gaussian_logpdf_matches_two_by_two_closed_form():
    Z = np.array([[0.0, 0.0], [1.0, -0.5], [2.0, 3.0]])
    # Sigma = [[1, 1/2], [1/2, 1]]: det 3/4, inverse (4/3) [[1, -1/2], [-1/2, 1]]
    q = (4.0 / 3.0) * (Z[:, 0] ** 2 - Z[:, 0] * Z[:, 1] + Z[:, 1] ** 2)
    ref = -0.5 * q - math.log(2.0 * math.pi) - 0.5 * math.log(0.75)
    assert np.allclose(ranking.true_logpdf(Z, "gaussian"), ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("nu", [1.0, 2.0, 5.0])
def test_student_t_logpdf_closed_form(nu):
    Z = np.array([[0.0, 0.0], [0.7, -1.2]])
    d = 2
    q = (4.0 / 3.0) * (Z[:, 0] ** 2 - Z[:, 0] * Z[:, 1] + Z[:, 1] ** 2)
    ref = (math.lgamma((nu + d) / 2) - math.lgamma(nu / 2) - (d / 2) * math.log(nu * math.pi)
           - 0.5 * math.log(0.75) - (nu + d) / 2 * np.log1p(q / nu))
    assert np.allclose(ranking.true_logpdf(Z, "t", nu), ref, rtol=0, atol=1e-12)


def test_rank_correlations_of_monotone_and_reversed_orders():
    a = np.arange(50.0)
    r = ranking.rank_correlations(a, a ** 3)
    assert abs(r["spearman"] - 1.0) < 1e-12 and abs(r["kendall"] - 1.0) < 1e-12
    r = ranking.rank_correlations(a, -a)
    assert abs(r["spearman"] + 1.0) < 1e-12 and abs(r["kendall"] + 1.0) < 1e-12
    # one swapped neighbour pair: tau = 1 - 2 / C(50, 2), rho = 1 - 6 * 2 / (50 (50^2 - 1))
    b = a.copy()
    b[[10, 11]] = b[[11, 10]]
    r = ranking.rank_correlations(a, b)
    assert abs(r["kendall"] - (1 - 2 / 1225)) < 1e-12
    assert abs(r["spearman"] - (1 - 12 / (50 * 2499))) < 1e-12


def test_samples_have_the_toeplitz_scatter():
    rng = np.random.default_rng(5)
    X = ranking.sample(rng, 200_000, 4, "gaussian")
    assert np.allclose(np.cov(X.T), ranking.toeplitz_sigma(4), atol=0.02)
    T = ranking.sample(rng, 200_000, 4, "t", 10.0)
    # the t law with nu degrees of freedom has covariance nu / (nu - 2) Sigma
    assert np.allclose(np.cov(T.T), 10.0 / 8.0 * ranking.toeplitz_sigma(4), atol=0.05)
