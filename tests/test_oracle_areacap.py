"""Pins of the oracle's area-uniform cap law (RRS_FLAG_AREA_CAP): the polar
angle theta of a point uniform on the cap {angle to the pole <= eps} of
S^(d-1) has density proportional to sin(theta)^(d-2) on [0, eps].  Checked
against closed forms (d = 2: uniform angle; d = 3: 1 - cos theta uniform),
against the numerically integrated distribution function for larger d, and
against rejection sampling from the uniform sphere; directions are unit
vectors inside the cap."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle


def _angles(d, phi, us):
    return np.array([math.atan2(*oracle.area_cap_angle(u, phi, d)) for u in us])


def test_d2_is_uniform_in_angle():
    us = (np.arange(400) + 0.5) / 400
    th = _angles(2, 0.7, us)
    assert np.allclose(th, us * 0.7 * math.pi / 2, rtol=0, atol=1e-12)


@pytest.mark.parametrize("phi", [0.99, 0.5, 0.05])
def test_d3_closed_form(phi):
    # d = 3: F(theta) = (1 - cos theta) / (1 - cos eps), so the sampled cosine
    # is the closed-form inverse at u
    eps = phi * math.pi / 2
    us = (np.arange(300) + 0.5) / 300
    for u in us:
        s, c = oracle.area_cap_angle(u, phi, 3)
        want = 1.0 - u * (1.0 - math.cos(eps))
        assert abs(c - want) < 1e-9
        assert abs(s * s + c * c - 1.0) < 1e-12


@pytest.mark.parametrize("d,phi", [(10, 0.3), (50, 0.6), (100, 0.2), (20, 0.9)])
def test_distribution_function_by_quadrature(d, phi):
    eps = phi * math.pi / 2
    tot = integrate.quad(lambda t: math.sin(t) ** (d - 2), 0.0, eps, epsabs=0, epsrel=1e-13)[0]
    for u in (0.01, 0.2, 0.5, 0.8, 0.99):
        th = math.atan2(*oracle.area_cap_angle(u, phi, d))
        F = integrate.quad(lambda t: math.sin(t) ** (d - 2), 0.0, th, epsabs=0, epsrel=1e-13)[0]
        assert abs(F / tot - u) < 1e-9, (d, phi, u, F / tot)


def test_matches_rejection_sampling_from_the_sphere():
    # uniform sphere points kept when within eps of e1: their angles follow
    # the area-uniform cap law
    d, phi = 4, 0.6
    eps = phi * math.pi / 2
    rng = np.random.default_rng(1)
    g = rng.standard_normal((400_000, d))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    ang = np.arccos(np.clip(g[:, 0], -1, 1))
    ref = ang[ang <= eps][:20000]
    mine = _angles(d, phi, rng.random(5000))
    assert stats.ks_2samp(mine, ref).pvalue > 1e-3


@pytest.mark.parametrize("d", [3, 7, 40])
def test_directions_are_unit_vectors_in_the_cap(d):
    rng = np.random.default_rng(d)
    pole = rng.standard_normal(d)
    pole /= np.linalg.norm(pole)
    phi = 0.25
    eps = phi * math.pi / 2
    for j in range(50):
        u = oracle.direction(5, 2, 3, j, d, phi, pole, area_cap=True)
        assert abs(np.dot(u, u) - 1.0) < 1e-13
        assert math.acos(min(1.0, float(np.dot(u, pole)))) <= eps + 1e-12
