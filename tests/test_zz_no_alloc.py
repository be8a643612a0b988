"""rrs_depth_halfspace_noalloc (static device scratch, no allocation inside
the call) against rrs_depth_halfspace on the same device inputs: depth,
count, poles and trace bit for bit, for two calls in a row on one stream,
the second with a smaller input (the scratch keeps the first call's
contents), in every precision form; plus its argument checks."""
import sys

import numpy as np
import pytest

from paper_2506_08262_amd import rrs, workloads

pytestmark = pytest.mark.gpu

CASES = [  # (n, d, queries, K, n_refine, cap_shrink, law, seed_cfg)
    (3001, 7, 13, 300, 5, 0.5, "mixture", 21),
    (700, 4, 5, 120, 3, 0.6, "gaussian", 22),
]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("prec", ["f64", "bf16", "f32"])
def test_noalloc_matches_halfspace_twice(prec):
    import torch
    rrs.load()
    dev = torch.device("cuda:0")
    for (n, d, nq, K, r, a, law, sc) in CASES:
        _say("noalloc case", prec, n, d, nq, K, r, a, law)
        w = workloads.small("halfspace", n, d, nq, K, r, a, law=law, seed_cfg=sc)
        X = torch.from_numpy(w.X).to(dev)
        Z = torch.from_numpy(w.Z).to(dev)
        ref = rrs.rrs_depth_halfspace(X, Z, K, r, a, 3, precision=prec, query_offset=5,
                                      want_poles=True, want_trace=True)
        out = {"depth": torch.full((nq,), float("nan"), dtype=torch.float64, device=dev),
               "count": torch.full((nq,), -1, dtype=torch.int64, device=dev),
               "poles": torch.full((nq, d), float("nan"), dtype=torch.float64, device=dev),
               "trace": torch.full((nq, r, 3), -1, dtype=torch.int64, device=dev)}
        torch.cuda.synchronize()
        got = rrs.rrs_depth_halfspace_noalloc(X, Z, K, r, a, 3, precision=prec, query_offset=5,
                                              out=out)
        torch.cuda.synchronize()
        for key in ("depth", "count", "poles", "trace"):
            g = got[key].cpu().numpy()
            e = ref[key].cpu().numpy()
            assert np.array_equal(g, e), (prec, n, key)


def test_noalloc_query_batches_under_workspace_limit():
    """A small workspace limit forces several query batches through the
    scratch; results stay identical."""
    import torch
    dev = torch.device("cuda:0")
    w = workloads.small("halfspace", 2000, 5, 24, 200, 4, 0.5, law="gaussian", seed_cfg=23)
    X = torch.from_numpy(w.X).to(dev)
    Z = torch.from_numpy(w.Z).to(dev)
    ref = rrs.rrs_depth_halfspace(X, Z, 200, 4, 0.5, 0, precision="bf16")
    got = rrs.rrs_depth_halfspace_noalloc(X, Z, 200, 4, 0.5, 0, precision="bf16",
                                          workspace_limit=12 << 20)
    torch.cuda.synchronize()
    assert np.array_equal(got["count"].cpu().numpy(), ref["count"].cpu().numpy())
    assert np.array_equal(got["depth"].cpu().numpy(), ref["depth"].cpu().numpy())


def test_noalloc_rejects_host_pointers_and_oversize():
    import ctypes

    import torch
    L = rrs.load()
    X = np.zeros((10, 3))
    Z = np.zeros((2, 3))
    dep = np.zeros(2)
    o = rrs.rrs_opts()
    st = L.rrs_depth_halfspace_noalloc(X.ctypes.data_as(ctypes.c_void_p), 10, 3,
                                       Z.ctypes.data_as(ctypes.c_void_p), 2, 10, 2, 0.5, 0,
                                       dep.ctypes.data_as(ctypes.c_void_p), None,
                                       ctypes.byref(o))
    assert st == rrs.RRS_E_INVAL
    # a data set whose prepared transpose alone exceeds the scratch
    dev = torch.device("cuda:0")
    Xb = torch.zeros((1 << 20, 40), dtype=torch.float64, device=dev)
    Zb = torch.zeros((1, 40), dtype=torch.float64, device=dev)
    with pytest.raises(rrs.RRSError) as ei:
        rrs.rrs_depth_halfspace_noalloc(Xb, Zb, 10, 2, 0.5, 0)
    assert ei.value.status == rrs.RRS_E_NOMEM
