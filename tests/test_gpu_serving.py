"""Serving context on the GPU: resident data sets, admission by memory,
continuously batched requests.  Every request's result must be identical to
the same request run alone through the synchronous entry points (and those
are bit-identical to the oracle, see test_gpu_parity)."""
import sys
import time

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


def _mix():
    """Three data sets and a mix of requests over them (notion, precision,
    query counts, K and r differ)."""
    sets = [workloads.small("halfspace", 3000, 5, 40, 600, 6, 0.5, law="gaussian", seed_cfg=31),
            workloads.small("projection", 2000, 12, 30, 400, 5, 0.6, law="toeplitz", seed_cfg=32),
            workloads.small("apd", 5000, 3, 25, 300, 4, 0.5, law="exponential", seed_cfg=33)]
    reqs = []
    rng = np.random.default_rng(7)
    for k in range(14):
        si = k % 3
        w = sets[si]
        notion = ["halfspace", "projection", "apd"][(k + si) % 3]
        prec = "bf16" if (notion == "halfspace" and k % 2 == 0) else "f64"
        nq = int(rng.integers(1, len(w.Z) + 1))
        q0 = int(rng.integers(0, 1000))
        K = int(rng.choice([120, 250, 400]))
        r = int(rng.choice([2, 3, 5]))
        reqs.append(dict(set=si, notion=notion, precision=prec, Z=w.Z[:nq], K=K, r=r,
                         alpha=0.5, seed=k, q0=q0))
    return sets, reqs


def _alone(w, q):
    return rrs.depth(q["notion"], w.X, q["Z"], q["K"], q["r"], q["alpha"], q["seed"],
                     precision=q["precision"], query_offset=q["q0"])


def test_results_identical_alone_and_in_the_mix():
    sets, reqs = _mix()
    with rrs.Context(slots=4, hbm_budget=4 << 30) as ctx:
        dss = [ctx.put(w.X) for w in sets]
        handles = [ctx.submit(dss[q["set"]], q["notion"], q["Z"], q["K"], q["r"], q["alpha"],
                              q["seed"], precision=q["precision"], query_offset=q["q0"])
                   for q in reqs]
        outs = [h.wait(timeout=120) for h in handles]
        st = ctx.stats()
        _say("stats", st)
        assert st["completed"] == len(reqs) and st["failed"] == 0
        assert st["bytes_peak"] <= st["budget"]
    overlap = 0
    for q, out in zip(reqs, outs):
        ref = _alone(sets[q["set"]], q)
        assert np.array_equal(out["depth"], ref["depth"]), q["notion"]
        if q["notion"] == "halfspace":
            assert np.array_equal(out["count"], ref["count"])
        info = out["info"]
        assert info["submit_s"] <= info["admit_s"] <= info["done_s"]
    infos = sorted((o["info"] for o in outs), key=lambda i: i["admit_s"])
    for a, b in zip(infos, infos[1:]):
        overlap += b["admit_s"] < a["done_s"]
    _say("overlapping admissions:", overlap)
    assert overlap > 0, "requests never overlapped on the device"


def test_mix_against_oracle_on_one_request():
    w = workloads.small("projection", 1500, 6, 8, 200, 4, 0.5, law="gaussian", seed_cfg=41)
    with rrs.Context(slots=2, hbm_budget=1 << 30) as ctx:
        ds = ctx.put(w.X)
        a = ctx.submit(ds, "projection", w.Z, w.K, w.n_refine, w.cap_shrink, 3, query_offset=11)
        b = ctx.submit(ds, "apd", w.Z[:3], w.K, w.n_refine, w.cap_shrink, 4)
        ra, rb = a.wait(60), b.wait(60)
    ref = oracle.rrs_depth("projection", w.X, w.Z, w.K, w.n_refine, w.cap_shrink, 3, q0=11)
    assert np.array_equal(ra["depth"], ref["depth"])
    refb = oracle.rrs_depth("apd", w.X, w.Z[:3], w.K, w.n_refine, w.cap_shrink, 4)
    assert np.array_equal(rb["depth"], refb["depth"])


def test_admission_by_memory_serialises_when_budget_is_tight():
    """A budget that holds one request at a time: requests still all finish
    with identical results, one after the other."""
    w = workloads.small("projection", 4000, 8, 20, 400, 4, 0.5, law="gaussian", seed_cfg=42)
    # one request: Z + outputs + T (m * n * 8 per query, batched to the limit)
    limit = 8 << 20
    # data set ~0.5 MB, one request ~6.4 MB (two queries per batch): two
    # requests never fit 10 MiB together
    with rrs.Context(slots=4, hbm_budget=10 << 20, request_ws_limit=limit) as ctx:
        ds = ctx.put(w.X)
        hs = [ctx.submit(ds, "projection", w.Z, w.K, w.n_refine, w.cap_shrink, s)
              for s in range(4)]
        outs = [h.wait(120) for h in hs]
        st = ctx.stats()
    assert st["bytes_peak"] <= st["budget"]
    infos = sorted((o["info"] for o in outs), key=lambda i: i["admit_s"])
    for a, b in zip(infos, infos[1:]):
        assert b["admit_s"] >= a["done_s"] - 1e-3
    for s, o in enumerate(outs):
        ref = rrs.rrs_depth_projection(w.X, w.Z, w.K, w.n_refine, w.cap_shrink, s)
        assert np.array_equal(o["depth"], ref["depth"])


def test_request_larger_than_budget_is_rejected_at_submit():
    w = workloads.small("projection", 3000, 4, 4, 100, 2, 0.5, seed_cfg=43)
    with rrs.Context(slots=1, hbm_budget=1 << 20) as ctx:
        ds = ctx.put(w.X)
        with pytest.raises(rrs.RRSError) as ei:
            ctx.submit(ds, "projection", w.Z, 20000, 2, 0.5, 0)
        assert ei.value.status == rrs.RRS_E_NOMEM


def test_wait_timeout_then_result_and_cancel_on_destroy():
    w = workloads.small("halfspace", 20000, 10, 64, 2000, 4, 0.5, seed_cfg=44)
    ctx = rrs.Context(slots=1, hbm_budget=2 << 30)
    ds = ctx.put(w.X)
    first = ctx.submit(ds, "halfspace", w.Z, w.K, w.n_refine, w.cap_shrink, 0)
    with pytest.raises(rrs.RRSError) as ei:
        first.wait(timeout=0.0)
    assert ei.value.status == rrs.RRS_E_BUSY
    queued = [ctx.submit(ds, "halfspace", w.Z, w.K, w.n_refine, w.cap_shrink, s)
              for s in range(1, 6)]
    got = first.wait(120)
    ref = rrs.rrs_depth_halfspace(w.X, w.Z, w.K, w.n_refine, w.cap_shrink, 0)
    assert np.array_equal(got["count"], ref["count"])
    ctx.close()
    statuses = []
    for q in queued:
        try:
            q.wait(60)
            statuses.append(rrs.RRS_OK)
        except rrs.RRSError as e:
            statuses.append(e.status)
    assert set(statuses) <= {rrs.RRS_OK, rrs.RRS_E_CANCELLED}
    _say("after destroy:", statuses)


def test_dataset_release_while_requests_are_in_flight():
    w = workloads.small("apd", 3000, 5, 16, 300, 3, 0.5, law="exponential", seed_cfg=45)
    with rrs.Context(slots=2, hbm_budget=1 << 30) as ctx:
        ds = ctx.put(w.X)
        hs = [ctx.submit(ds, "apd", w.Z, w.K, w.n_refine, w.cap_shrink, s) for s in range(3)]
        ds.release()
        with pytest.raises(rrs.RRSError):
            ctx.submit(ds, "apd", w.Z, w.K, w.n_refine, w.cap_shrink, 0)   # released handle
        outs = [h.wait(120) for h in hs]
        time.sleep(0.05)
        st = ctx.stats()
    assert st["datasets"] == 0
    for s, o in enumerate(outs):
        ref = rrs.rrs_depth_apd(w.X, w.Z, w.K, w.n_refine, w.cap_shrink, s)
        assert np.array_equal(o["depth"], ref["depth"])
