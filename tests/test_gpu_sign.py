"""GPU parity of the persistent sign GEMM and cap culling (bfloat16 halfspace
form): counts, depths, poles and traces bit for bit against the oracle, over
shapes that hit every padded-K instantiation, ragged point counts, direction
counts that are not multiples of the 128-column tile, and data with exact
zeros (block recheck); culling on and off and the tile-per-workgroup GEMM
all give the same results."""
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


def _check(w, q0=0, **kw):
    _say("sign parity", w.name, "n", w.n, "d", w.d, "nq", w.nq, "K", w.K, "r", w.n_refine, kw)
    got = rrs.rrs_depth_halfspace(w.X, w.Z, w.K, w.n_refine, w.cap_shrink, w.rrs_seed,
                                  precision="bf16", query_offset=q0, want_poles=True,
                                  want_trace=True, **kw)
    ref = oracle.rrs_depth("halfspace", w.X, w.Z, w.K, w.n_refine, w.cap_shrink, w.rrs_seed,
                           q0=q0, with_poles=True)
    assert np.array_equal(got["count"], ref["count"])
    assert np.array_equal(got["depth"], ref["depth"])
    assert np.array_equal(got["poles"], ref["poles"])
    tr0 = oracle.rrs_query("halfspace", w.X, w.Z[0], q0, w.K, w.n_refine, w.cap_shrink,
                           w.rrs_seed)[3]
    assert [t[0] for t in tr0] == list(got["trace"][0][:, 0])
    return got


# padded K = d + 2 rounded up to 16: d = 2 -> 16 (one K step) ... d = 126 -> 128
@pytest.mark.parametrize("n,d,K,r,law", [
    (257, 2, 60, 3, "gaussian"),        # one K step; n just past a point tile
    (1025, 14, 258, 3, "mixture"),      # m = 86; n just past four point tiles
    (700, 15, 387, 3, "gaussian"),      # two K steps; m = 129 (two direction tiles)
    (3001, 30, 600, 6, "mixture"),      # m = 100
    (999, 46, 256, 2, "exponential"),   # m = 128 exactly
    (2000, 62, 400, 4, "toeplitz"),     # four K steps
    (1500, 78, 200, 2, "mixture"),      # five
    (1800, 94, 500, 5, "gaussian"),     # six
    (2500, 110, 300, 3, "mixture"),     # seven (the 1e5 x 100 workload's padding)
    (1300, 126, 200, 4, "gaussian"),    # eight
])
def test_sign_gemm_shapes(n, d, K, r, law, monkeypatch):
    # culling at every refinement l >= 2 (by default wide caps in many
    # dimensions skip it), so that the cull GEMM and the list-mode sign GEMM
    # run at every K padding
    monkeypatch.setenv("RRS_CULL_ANGLE", "1.5707963267948966")
    w = workloads.small("halfspace", n, d, 9, K, r, 0.6, law=law, seed_cfg=5 * n + d)
    _check(w)


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 255, 256, 511])
def test_sign_gemm_tiny_and_ragged(n):
    w = workloads.small("halfspace", n, 5, 7, 130, 4, 0.5, law="gaussian", seed_cfg=40 + n)
    _check(w)


def test_sign_gemm_single_direction_per_refinement():
    w = workloads.small("halfspace", 900, 6, 11, 7, 7, 0.5, law="mixture", seed_cfg=44)
    _check(w)


def test_exact_zeros_go_through_the_block_recheck():
    """Integer data with queries equal to data points and repeated points:
    many projections are exactly zero (both sides), so the sign GEMM hands
    whole tiles to the binary64 block recheck."""
    w = workloads.small("halfspace", 2000, 4, 16, 240, 6, 0.5, law="integer", seed_cfg=81)
    Z = w.Z.copy()
    Z[:8] = w.X[:8]
    w.Z = Z
    X = w.X.copy()
    X[500:700] = X[3]
    w.X = X
    rrs.rrs_profile_enable(True)
    _check(w)
    rechecked = rrs.rrs_profile_counter("recheck_pairs")
    rrs.rrs_profile_enable(False)
    assert rechecked > 0


def test_cull_and_gemm_choices_agree(monkeypatch):
    """Culling on (default) and off, and the tile-per-workgroup GEMM: same
    exact results; with culling the GEMM evaluates fewer pairs."""
    w = workloads.small("halfspace", 6000, 20, 12, 1200, 12, 0.6, law="mixture", seed_cfg=45)
    outs, pairs = {}, {}
    for mode, env in (("cull", {}), ("nocull", {"RRS_CULL": "0"}),
                      ("tiles", {"RRS_SIGN": "0"})):
        for k in ("RRS_CULL", "RRS_SIGN"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        rrs.rrs_profile_enable(True)
        outs[mode] = _check(w)
        pairs[mode] = rrs.rrs_profile_counter("gemm_pairs")
        rrs.rrs_profile_enable(False)
        _say(mode, "gemm pairs", pairs[mode])
    for mode in ("nocull", "tiles"):
        assert np.array_equal(outs[mode]["count"], outs["cull"]["count"])
        assert np.array_equal(outs[mode]["poles"], outs["cull"]["poles"])
    assert pairs["nocull"] == w.projections
    assert 0 < pairs["cull"] < pairs["nocull"]


def test_cull_angle_threshold_keeps_results(monkeypatch):
    """Culling only the refinements whose cap half-angle is below a
    threshold gives the same results."""
    w = workloads.small("halfspace", 4000, 12, 8, 600, 10, 0.5, law="gaussian", seed_cfg=46)
    monkeypatch.setenv("RRS_CULL_ANGLE", "0.1")
    _check(w, q0=3)


def test_large_query_batch_items():
    """Several hundred queries: the list-mode work list spans many queries
    with uneven lists."""
    w = workloads.small("halfspace", 5000, 8, 300, 200, 5, 0.6, law="mixture", seed_cfg=47)
    _check(w)


@pytest.mark.parametrize("words", [4096, 6144])
def test_queue_overflow_recounts_exactly(monkeypatch, words):
    """A recheck queue too small for the uncertain rows (one entry or none
    per wave segment, forced through the queue-size override) makes the
    refinement recount in binary64: the results are unchanged."""
    w = workloads.small("halfspace", 2000, 4, 16, 240, 6, 0.5, law="integer", seed_cfg=81)
    X = w.X.copy()
    X[500:900] = X[3]
    w.X = X
    Z = w.Z.copy()
    Z[:8] = w.X[:8]
    w.Z = Z
    monkeypatch.setenv("RRS_QUEUE_WORDS", str(words))
    _check(w)


@pytest.mark.parametrize("pct", ["0", "1000"])
def test_dense_or_list_choice_after_culling(monkeypatch, pct):
    """After culling, the device picks the dense GEMM over every point or the
    list-mode GEMM over the undecided points by their matrix-core work;
    forcing either (RRS_LIST_PCT 0: always dense, 1000: always lists) gives
    the same exact results."""
    w = workloads.small("halfspace", 5000, 24, 10, 900, 9, 0.6, law="mixture", seed_cfg=48)
    monkeypatch.setenv("RRS_LIST_PCT", pct)
    rrs.rrs_profile_enable(True)
    _check(w, q0=2)
    pairs = rrs.rrs_profile_counter("gemm_pairs")
    rrs.rrs_profile_enable(False)
    _say("list pct", pct, "gemm pairs", pairs, "of", w.projections)
    if pct == "0":
        assert pairs == w.projections
    else:
        assert pairs < w.projections
