"""GPU parity of the window select with per-point error bounds (the
matrix-core P / AP forms on heavy-tailed data): every point's approximation
carries its own bound alpha |a_i| + E instead of the largest point's, the
selects bin both ends of the points' intervals and rank the candidates
exactly, so depths, poles and traces stay identical to the binary64 oracle.
RRS_POINT_BOUNDS = 1 forces the mode on ordinary data as well."""
import sys

import numpy as np
import pytest

import oracle
from paper_2506_08262_amd import rrs, workloads

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _lib():
    oracle.build(force=False)
    rrs.load()
    yield
    rrs.rrs_release_workspace()


def _compare(notion, w, prec, q0=0):
    _say("point bounds parity", notion, prec, w.name, "n", w.n, "d", w.d, "nq", len(w.Z))
    got = rrs.depth(notion, w.X, w.Z, w.K, w.n_refine, w.cap_shrink, w.rrs_seed,
                    precision=prec, query_offset=q0, want_poles=True, want_trace=True)
    ref = oracle.rrs_depth(notion, w.X, w.Z, w.K, w.n_refine, w.cap_shrink, w.rrs_seed, q0=q0,
                           with_poles=True)
    assert np.array_equal(got["depth"], ref["depth"]), notion
    assert np.array_equal(got["poles"], ref["poles"])
    return got


def _fallback_fraction(notion, w, prec):
    rrs.rrs_profile_enable(True)
    rrs.depth(notion, w.X, w.Z, w.K, w.n_refine, w.cap_shrink, w.rrs_seed, precision=prec)
    fb = rrs.rrs_profile_counter("select_fallback")
    fast = rrs.rrs_profile_counter("select_fast")
    rrs.rrs_profile_enable(False)
    return fb / max(fb + fast, 1.0)


@pytest.mark.parametrize("prec", ["bf16", "f32"])
@pytest.mark.parametrize("notion", ["projection", "apd"])
@pytest.mark.parametrize("n,d,law", [(1000, 5, "gaussian"), (777, 7, "exponential"),
                                     (901, 3, "integer"), (20001, 4, "gaussian"),
                                     (640, 60, "mixture")])
def test_forced_point_bounds_parity(monkeypatch, prec, notion, n, d, law):
    monkeypatch.setenv("RRS_POINT_BOUNDS", "1")
    w = workloads.small(notion, n, d, 8, 180, 5, 0.5, law=law, seed_cfg=3 * n + d)
    _compare(notion, w, prec)


@pytest.mark.parametrize("notion", ["projection", "apd"])
@pytest.mark.parametrize("n", [1, 2, 3, 63, 513])
def test_forced_point_bounds_tiny_n(monkeypatch, notion, n):
    monkeypatch.setenv("RRS_POINT_BOUNDS", "1")
    w = workloads.small(notion, n, 4, 5, 60, 3, 0.5, law="gaussian", seed_cfg=n + 91)
    _compare(notion, w, "f32")


@pytest.mark.parametrize("prec", ["bf16", "f32"])
@pytest.mark.parametrize("notion", ["projection", "apd"])
@pytest.mark.parametrize("law,n", [("t1", 3000), ("t2", 3000), ("t1", 20001)])
def test_heavy_tails_parity(prec, notion, law, n):
    """Student t data with nu = 1, 2: the largest norm is far above the
    typical one, so the library picks per-point bounds by itself."""
    w = workloads.small(notion, n, 10, 8, 200, 5, 0.6, law=law, seed_cfg=n + 7)
    _compare(notion, w, prec)


@pytest.mark.parametrize("notion", ["projection", "apd"])
def test_heavy_tails_stay_off_the_fallback(monkeypatch, notion):
    """On Cauchy data (t, nu = 1) in the bfloat16 form the per-point bounds
    resolve nearly every order statistic in the window; the column-wide
    bound, set by the largest point, makes the windows overflow and the
    selects take the exact fallback (results are exact either way)."""
    w = workloads.small(notion, 20001, 10, 8, 120, 3, 0.6, law="t1", seed_cfg=5)
    monkeypatch.delenv("RRS_POINT_BOUNDS", raising=False)
    on = _fallback_fraction(notion, w, "bf16")
    monkeypatch.setenv("RRS_POINT_BOUNDS", "0")
    off = _fallback_fraction(notion, w, "bf16")
    _say(notion, "t1 select fallback: per-point", on, "column bound", off)
    assert on < 0.02
    assert off > 0.5
