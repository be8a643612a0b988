"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  In the F64 form every decision is exact, so counts,
poles, traces and depths must be bit-identical."""
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


# --------------------------------------------------------------------------
# a1: directions, bit for bit
# --------------------------------------------------------------------------
@pytest.mark.parametrize("d", [2, 3, 5, 7, 20, 33, 100])
def test_directions_sphere_bit_exact(d):
    _say("directions sphere d", d)
    m = 37
    got = rrs.rrs_debug_directions(d, m, 1, 1.0, 12345, 7, np.eye(d)[0])
    ref = np.array([oracle.direction(12345, 7, 1, j, d, 1.0, np.eye(d)[0]) for j in range(m)])
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6, 20, 51, 100])
@pytest.mark.parametrize("phi", [0.5, 3e-7])
def test_directions_cap_bit_exact(d, phi):
    _say("directions cap d", d, "phi", phi)
    rng = np.random.default_rng(d)
    for pole in (np.eye(d)[0], rng.standard_normal(d), -np.eye(d)[0]):
        pole = pole / np.linalg.norm(pole)
        m = 23
        got = rrs.rrs_debug_directions(d, m, 3, phi, 9, 11, pole)
        ref = np.array([oracle.direction(9, 11, 3, j, d, phi, pole) for j in range(m)])
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


def test_directions_many_bit_exact():
    # many stream positions: exercises sqrt / division / log / sin / cos over
    # a wide range of arguments
    _say("directions many")
    d, m = 9, 4000
    got = rrs.rrs_debug_directions(d, m, 1, 1.0, 3, 0, np.eye(d)[0])
    ref = np.array([oracle.direction(3, 0, 1, j, d, 1.0, np.eye(d)[0]) for j in range(m)])
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


# --------------------------------------------------------------------------
# Full RRS parity
# --------------------------------------------------------------------------
def _compare(notion, w, q0=0, nq=None, **kw):
    Z = w.Z if nq is None else w.Z[:nq]
    _say("parity", notion, w.name, "n", w.n, "d", w.d, "nq", len(Z), "K", w.K, "r", w.n_refine)
    got = rrs.depth(notion, w.X, Z, w.K, w.n_refine, w.cap_shrink, w.rrs_seed,
                    query_offset=q0, want_poles=True, want_trace=True, **kw)
    ref = oracle.rrs_depth(notion, w.X, Z, w.K, w.n_refine, w.cap_shrink, w.rrs_seed, q0=q0,
                           with_poles=True)
    assert np.array_equal(got["depth"], ref["depth"]), notion
    if notion == "halfspace":
        assert np.array_equal(got["count"], ref["count"])
    assert np.array_equal(got["poles"], ref["poles"])
    return got, ref


def test_c1_halfspace_full():
    w = workloads.make("c1")
    got, _ = _compare("halfspace", w)
    # trace agrees with the oracle's own per-refinement trace for a few queries
    for q in (0, 17, 99):
        _, _, _, tr = oracle.rrs_query("halfspace", w.X, w.Z[q], q, w.K, w.n_refine,
                                       w.cap_shrink, w.rrs_seed)
        g = got["trace"][q]
        assert [t[0] for t in tr] == list(g[:, 0])
        assert [int(t[1]) for t in tr] == list(g[:, 1])
        assert [int(t[2]) for t in tr] == list(g[:, 2])


def test_c1b_halfspace_plane_against_exact():
    from tests.test_oracle_pins import exact_halfspace_2d
    w = workloads.make("c1b")
    got, _ = _compare("halfspace", w)
    exact = np.array([exact_halfspace_2d(w.X, z) for z in w.Z])
    assert np.all(got["count"] >= exact)
    assert np.all(got["count"][100:] == 0)


@pytest.mark.parametrize("notion", ["projection", "apd"])
@pytest.mark.parametrize("n,d,law", [(1000, 5, "gaussian"), (777, 7, "exponential"),
                                     (1001, 3, "integer"), (2048, 20, "wishart_cauchy")])
def test_small_parity(notion, n, d, law):
    w = workloads.small(notion, n, d, 24, 300, 6, 0.5, law=law, seed_cfg=n + d)
    _compare(notion, w)


@pytest.mark.parametrize("notion", ["halfspace", "projection", "apd"])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 63, 513])
def test_tiny_and_ragged_n(notion, n):
    w = workloads.small(notion, n, 3, 5, 70, 3, 0.5, law="gaussian", seed_cfg=40 + n)
    _compare(notion, w)


@pytest.mark.parametrize("notion", ["halfspace", "projection", "apd"])
def test_ties_and_points_equal_to_queries(notion):
    w = workloads.small(notion, 300, 4, 16, 160, 4, 0.5, law="integer", seed_cfg=77)
    Z = w.Z.copy()
    Z[:6] = w.X[:6]
    w.Z = Z
    X = w.X.copy()
    X[100:140] = X[0]                  # many duplicated rows
    w.X = X
    _compare(notion, w)


@pytest.mark.parametrize("notion", ["projection", "apd"])
@pytest.mark.parametrize("n,law", [(16385, "gaussian"), (24001, "gaussian"),
                                   (40000, "integer"), (33333, "exponential")])
def test_select_streaming_long_columns(notion, n, law):
    # columns longer than the register-resident select holds: the streaming
    # select re-reads them from global memory
    w = workloads.small(notion, n, 3, 3, 32, 2, 0.5, law=law, seed_cfg=5 + n % 7)
    _compare(notion, w)


@pytest.mark.parametrize("notion", ["halfspace", "projection"])
def test_batching_and_query_offset_do_not_change_results(notion):
    w = workloads.small(notion, 600, 6, 40, 200, 5, 0.6, law="mixture", seed_cfg=3)
    full = rrs.depth(notion, w.X, w.Z, w.K, w.n_refine, w.cap_shrink, 1)["depth"]
    small = rrs.depth(notion, w.X, w.Z, w.K, w.n_refine, w.cap_shrink, 1,
                      workspace_limit=200_000)["depth"]
    assert np.array_equal(full, small)
    part = rrs.depth(notion, w.X, w.Z[13:29], w.K, w.n_refine, w.cap_shrink, 1,
                     query_offset=13)["depth"]
    assert np.array_equal(full[13:29], part)


def test_device_pointers_torch():
    import torch
    w = workloads.small("projection", 900, 5, 12, 120, 4, 0.5, seed_cfg=8)
    Xt = torch.from_numpy(w.X).cuda()
    Zt = torch.from_numpy(w.Z).cuda()
    got = rrs.rrs_depth_projection(Xt, Zt, w.K, w.n_refine, w.cap_shrink, 0)["depth"]
    host = rrs.rrs_depth_projection(w.X, w.Z, w.K, w.n_refine, w.cap_shrink, 0)["depth"]
    assert np.array_equal(got.cpu().numpy(), host)
    h = rrs.rrs_depth_halfspace(Xt, Zt, w.K, w.n_refine, w.cap_shrink, 0)
    hh = rrs.rrs_depth_halfspace(w.X, w.Z, w.K, w.n_refine, w.cap_shrink, 0)
    assert np.array_equal(h["count"].cpu().numpy(), hh["count"])


def test_c2_projection_full_size_sampled():
    """The projection-depth workload at full size in the benchmark's launch
    configuration (all 1000 queries in one call); sampled queries are
    recomputed by the oracle one by one."""
    w = workloads.make("c2")
    _say("c2 full size on GPU")
    got = rrs.rrs_depth_projection(w.X, w.Z, w.K, w.n_refine, w.cap_shrink, w.rrs_seed,
                                   want_poles=True)
    qs = np.array([0, 401, 799, 800, 999])
    _say("c2 oracle queries", qs)
    ref = oracle.rrs_depth_idx("projection", w.X, w.Z[qs], qs, w.K, w.n_refine, w.cap_shrink,
                               w.rrs_seed, with_poles=True)
    assert np.array_equal(got["depth"][qs], ref["depth"])
    assert np.array_equal(got["poles"][qs], ref["poles"])
    D = got["depth"]
    assert np.all((D > 0) & (D <= 1))
    # Cauchy queries (last 200) are far less central than in-law ones
    assert np.median(D[800:]) < np.median(D[:800])


def test_single_hip_runtime_in_process():
    import torch
    torch.zeros(1, device="cuda:0")
    rrs.load()
    libs = set()
    for line in open("/proc/self/maps"):
        if "libamdhip64" in line:
            libs.add(line.split()[-1])
    assert len(libs) == 1, libs


# --------------------------------------------------------------------------
# Halfspace depth on the matrix cores (bf16 split or binary32, each with a
# binary64 recheck of the uncertain signs): counts, poles and traces must be
# identical to the binary64 recipe.
# --------------------------------------------------------------------------
MFMA_EXACT = ["bf16", "f32"]


@pytest.mark.parametrize("prec", MFMA_EXACT)
def test_mfma_c1_halfspace(prec):
    w = workloads.make("c1")
    _compare("halfspace", w, precision=prec)


@pytest.mark.parametrize("prec", MFMA_EXACT)
@pytest.mark.parametrize("n,d,law", [(700, 2, "gaussian"), (1001, 3, "integer"),
                                     (1500, 7, "exponential"), (900, 33, "mixture"),
                                     (2100, 100, "toeplitz")])
def test_mfma_halfspace_parity(prec, n, d, law):
    w = workloads.small("halfspace", n, d, 20, 240, 6, 0.5, law=law, seed_cfg=n + 3 * d)
    _compare("halfspace", w, precision=prec)


@pytest.mark.parametrize("prec", MFMA_EXACT)
def test_mfma_halfspace_ties_and_far_queries(prec):
    w = workloads.small("halfspace", 300, 4, 16, 160, 4, 0.5, law="integer", seed_cfg=78)
    Z = w.Z.copy()
    Z[:6] = w.X[:6]
    Z[6] = 1e4
    w.Z = Z
    X = w.X.copy()
    X[100:140] = X[0]
    w.X = X
    _compare("halfspace", w, precision=prec)


@pytest.mark.parametrize("prec", MFMA_EXACT)
def test_mfma_matches_f64_on_c1b_and_offset_data(prec):
    w = workloads.make("c1b")
    _compare("halfspace", w, precision=prec)
    # data far from the origin: the centring by the mean keeps the margin small
    w2 = workloads.small("halfspace", 800, 5, 12, 200, 5, 0.6, law="gaussian", seed_cfg=9)
    w2.X = w2.X + 1e3
    w2.Z = w2.Z + 1e3
    _compare("halfspace", w2, precision=prec)


def test_f32_plain_halfspace_error_is_reported_and_small():
    """The plain binary32 form has no recheck: its counts are approximate.
    On C1 it must agree with the exact counts on almost every query, and it
    can only be off where projections sit within binary32 rounding of 0."""
    w = workloads.make("c1")
    exact = rrs.rrs_depth_halfspace(w.X, w.Z, w.K, w.n_refine, w.cap_shrink, w.rrs_seed)
    plain = rrs.rrs_depth_halfspace(w.X, w.Z, w.K, w.n_refine, w.cap_shrink, w.rrs_seed,
                                    precision="f32_plain")
    diff = np.abs(plain["count"] - exact["count"])
    _say("f32_plain vs f64 count mismatches:", int((diff > 0).sum()), "max", int(diff.max()))
    assert (diff == 0).mean() >= 0.9
    assert diff.max() <= 0.02 * w.n
    # a single refinement of sphere directions: the same directions, so each
    # count differs only through sign decisions within the rounding error
    one = dict(K=200, n_refine=1, cap_shrink=1.0)
    e1 = rrs.rrs_depth_halfspace(w.X, w.Z, one["K"], 1, 1.0, 5)["count"]
    p1 = rrs.rrs_depth_halfspace(w.X, w.Z, one["K"], 1, 1.0, 5, precision="f32_plain")["count"]
    assert np.abs(p1 - e1).max() <= 2


# --------------------------------------------------------------------------
# Projection / APD depth from matrix-core projections (binary32 s = a.u):
# the order statistics are made exact by recomputing their window in
# binary64, so depths, poles and traces are identical to the binary64 form.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec", MFMA_EXACT)
@pytest.mark.parametrize("notion", ["projection", "apd"])
@pytest.mark.parametrize("n,d,law", [(1000, 5, "gaussian"), (777, 7, "exponential"),
                                     (1200, 20, "wishart_cauchy"), (901, 3, "integer"),
                                     (640, 100, "mixture")])
def test_mfma_depth_parity(prec, notion, n, d, law):
    w = workloads.small(notion, n, d, 12, 240, 6, 0.5, law=law, seed_cfg=n + d)
    _compare(notion, w, precision=prec)


@pytest.mark.parametrize("prec", MFMA_EXACT)
@pytest.mark.parametrize("notion", ["projection", "apd"])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 63, 513, 6000, 8193, 10000, 16384, 20001])
def test_mfma_depth_tiny_ragged_and_long(prec, notion, n):
    w = workloads.small(notion, n, 4, 5, 60, 3, 0.5, law="gaussian", seed_cfg=n + 17)
    _compare(notion, w, precision=prec)


@pytest.mark.parametrize("prec", MFMA_EXACT)
@pytest.mark.parametrize("notion", ["projection", "apd"])
def test_mfma_depth_ties_offsets_and_far_queries(prec, notion):
    w = workloads.small(notion, 500, 4, 16, 160, 4, 0.5, law="integer", seed_cfg=79)
    Z = w.Z.copy()
    Z[:6] = w.X[:6]
    Z[6] = 1e4
    w.Z = Z
    X = w.X.copy()
    X[100:180] = X[0]
    w.X = X
    _compare(notion, w, precision=prec)
    w2 = workloads.small(notion, 900, 6, 8, 120, 4, 0.6, law="gaussian", seed_cfg=80)
    w2.X = w2.X + 1e3
    w2.Z = w2.Z + 1e3
    _compare(notion, w2, precision=prec)


@pytest.mark.parametrize("notion", ["projection", "apd"])
def test_f32_plain_depth_error_is_reported_and_small(notion):
    """Plain binary32 projections, no recheck: with one refinement (the same
    sphere directions in both forms) every depth is within a small relative
    error of the binary64 one; the full trajectory may differ and its error
    is reported."""
    w = workloads.make("c1")
    one = rrs.depth(notion, w.X, w.Z, 300, 1, 1.0, 2)["depth"]
    p1 = rrs.depth(notion, w.X, w.Z, 300, 1, 1.0, 2, precision="f32_plain")["depth"]
    rel = np.abs(p1 - one) / np.maximum(np.abs(one), 1e-300)
    _say(notion, "f32_plain single-refinement max rel err", float(rel.max()))
    assert rel.max() <= 1e-5
    full = rrs.depth(notion, w.X, w.Z, w.K, w.n_refine, w.cap_shrink, 0)["depth"]
    pf = rrs.depth(notion, w.X, w.Z, w.K, w.n_refine, w.cap_shrink, 0,
                   precision="f32_plain")["depth"]
    relf = np.abs(pf - full) / np.maximum(np.abs(full), 1e-300)
    _say(notion, "f32_plain full RRS: max rel err", float(relf.max()), "mean",
         float(relf.mean()), "exact queries", int((relf == 0).sum()), "of", len(relf))
    assert relf.max() <= 1e-2


def test_select_fast_path_dominates_on_centred_columns():
    """Queries at the centre of the data make the projection medians straddle
    zero; the bracketed select must still resolve almost every order
    statistic without the radix fallback (results are exact either way)."""
    w = workloads.small("projection", 4096, 8, 16, 400, 4, 0.5, law="gaussian", seed_cfg=12)
    w.Z = w.Z * 0.01
    rrs.rrs_profile_enable(True)
    got = rrs.rrs_depth_projection(w.X, w.Z, w.K, w.n_refine, w.cap_shrink, 0)["depth"]
    fast = rrs.rrs_profile_counter("select_fast")
    fb = rrs.rrs_profile_counter("select_fallback")
    rrs.rrs_profile_enable(False)
    ref = oracle.rrs_depth("projection", w.X, w.Z, w.K, w.n_refine, w.cap_shrink, 0)["depth"]
    assert np.array_equal(got, ref)
    assert fast > 0 and fb / (fast + fb) < 0.02, (fast, fb)


@pytest.mark.parametrize("notion", ["halfspace", "projection"])
@pytest.mark.parametrize("prec", MFMA_EXACT)
def test_gemm_variants_and_autotuner_agree(notion, prec, monkeypatch):
    """Every matrix-core GEMM variant (forced with RRS_TUNE=v+1) and the
    autotuner's own choice give the same exact results."""
    w = workloads.small(notion, 1700, 9, 10, 200, 4, 0.5, law="gaussian", seed_cfg=91)
    ref = oracle.rrs_depth(notion, w.X, w.Z, w.K, w.n_refine, w.cap_shrink, 0)
    pairs = w.projections
    for mode in ("1", "2", ""):
        monkeypatch.setenv("RRS_TUNE", mode)
        rrs.rrs_profile_enable(True)
        got = rrs.depth(notion, w.X, w.Z, w.K, w.n_refine, w.cap_shrink, 0, precision=prec)
        rechecked = rrs.rrs_profile_counter("recheck_pairs")
        fast = rrs.rrs_profile_counter("select_fast")
        fallback = rrs.rrs_profile_counter("select_fallback")
        rrs.rrs_profile_enable(False)
        assert np.array_equal(got["depth"], ref["depth"]), mode
        # a variant with wrong binary32 values would still be exact (everything
        # rechecked or sent to the exact fallback) but slow: both stay rare
        assert rechecked <= 0.02 * pairs, (mode, rechecked)
        assert fallback <= 0.05 * max(fast + fallback, 1), (mode, fast, fallback)


@pytest.mark.parametrize("notion,prec", [("halfspace", "bf16"), ("projection", "f32"),
                                         ("apd", "f64"), ("halfspace", "f64")])
def test_graph_replays_match_eager(notion, prec):
    """RRS_FLAG_GRAPH: the first call captures the device work, later calls
    replay it.  Every replay, with eager calls and host syncs between them,
    must give the eager result."""
    import torch
    w = workloads.small(notion, 2500, 6, 24, 300, 5, 0.5, law="gaussian", seed_cfg=93)
    dev = torch.device("cuda:0")
    X = torch.from_numpy(w.X).to(dev)
    Z = torch.from_numpy(w.Z).to(dev)
    s = torch.cuda.Stream()
    eager = rrs.depth(notion, X, Z, w.K, w.n_refine, w.cap_shrink, 4, precision=prec)
    ref = eager["depth"].cpu().numpy()
    for rep in range(4):
        with torch.cuda.stream(s):
            got = rrs.depth(notion, X, Z, w.K, w.n_refine, w.cap_shrink, 4, precision=prec,
                            stream=s, graph=True)
        torch.cuda.synchronize()
        assert np.array_equal(got["depth"].cpu().numpy(), ref), rep
        # eager work in between replays
        other = rrs.depth(notion, X, Z[:5], w.K, w.n_refine, w.cap_shrink, 9, precision=prec)
        torch.cuda.synchronize()
        assert other["depth"].shape[0] == 5
    oref = oracle.rrs_depth(notion, w.X, w.Z, w.K, w.n_refine, w.cap_shrink, 4)["depth"]
    assert np.array_equal(ref, oref)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("notion", ["projection", "apd"])
def test_select_recovers_when_samples_mislead(prec, notion):
    """The long-column selects sample 64 evenly spaced entries to bracket the
    rank; outliers planted exactly there make the bracket miss, and the
    select must recover (whole key range, then narrowing) with exact results."""
    n = 20001
    w = workloads.small(notion, n, 4, 4, 40, 2, 0.5, law="gaussian", seed_cfg=97)
    X = w.X.copy()
    pos = [((2 * t + 1) * n) // 128 for t in range(64)]
    X[pos] = 1e3 * np.sign(np.random.default_rng(5).standard_normal((64, 4)))
    w.X = X
    _compare(notion, w, precision=prec)


def _register_sample_rows(n):
    """Rows whose projections the register-resident selects take as their 64
    bracket samples: slot s of a group of g threads (one wave for n <= 8192,
    two up to 16384) reads register u = (2 (s // 8) + 1) V // 16 of thread
    64 (s // (64 // w)) + s % (64 // w), entry thread + g u."""
    if n <= 64 * 128:
        waves, g = 1, 64
        v = next(b for b in (8, 16, 32, 64, 96, 128) if n <= 64 * b)
    else:
        waves, g = 2, 128
        v = next(b for b in (80, 128) if n <= 128 * b)
    per = 64 // waves
    rows = []
    for slot in range(64):
        tid = 64 * (slot // per) + slot % per
        rows.append(tid + g * (((2 * (slot >> 3) + 1) * v) // 16))
    return [r for r in rows if r < n]


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("notion", ["projection", "apd"])
@pytest.mark.parametrize("n", [6000, 10000])
def test_register_select_recovers_when_samples_mislead(prec, notion, n):
    """Outliers planted on the rows the register-resident selects sample make
    their bracket useless; the column must fall through to the streamed
    select of the same kernel and still give the exact depths."""
    w = workloads.small(notion, n, 4, 4, 40, 2, 0.5, law="gaussian", seed_cfg=98)
    X = w.X.copy()
    rows = _register_sample_rows(n)
    X[rows] = 1e3 * np.sign(np.random.default_rng(6).standard_normal((len(rows), 4)))
    w.X = X
    _compare(notion, w, precision=prec)


@pytest.mark.parametrize("parts", [2, 4])
@pytest.mark.parametrize("notion,prec", [("halfspace", "f64"), ("halfspace", "bf16"),
                                         ("projection", "f64"), ("projection", "f32"),
                                         ("apd", "bf16")])
def test_two_stream_split_matches_oracle(monkeypatch, notion, prec, parts):
    """Large calls run their queries in parts on separate streams; forced on a
    small call with an odd number of queries and a query offset, every output
    (depths, counts, poles, traces) must equal the oracle's and the unsplit
    call's."""
    w = workloads.small(notion, 900, 5, 7, 150, 4, 0.5, law="gaussian", seed_cfg=101)
    monkeypatch.setenv("RRS_SPLIT_PARTS", str(parts))
    monkeypatch.setenv("RRS_SPLIT_WORK", "1e30")
    one = rrs.depth(notion, w.X, w.Z, w.K, w.n_refine, w.cap_shrink, w.rrs_seed,
                    query_offset=3, want_poles=True, want_trace=True, precision=prec)
    monkeypatch.setenv("RRS_SPLIT_WORK", "1")
    got, _ = _compare(notion, w, q0=3, precision=prec)
    for key in ("depth", "poles", "trace") + (("count",) if notion == "halfspace" else ()):
        assert np.array_equal(got[key], one[key]), key
