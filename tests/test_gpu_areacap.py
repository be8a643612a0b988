"""RRS_FLAG_AREA_CAP (cap directions uniform in area): GPU results
bit-identical to the oracle's with the same law, every notion, binary64 and
matrix-core forms."""
import numpy as np
import pytest

import oracle
from paper_2506_08262_amd import rrs, workloads

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("notion,prec", [("halfspace", "f64"), ("halfspace", "bf16"),
                                         ("projection", "f32"), ("apd", "f64"),
                                         ("apd", "bf16")])
def test_area_cap_parity(notion, prec):
    first = False
    w = workloads.small(notion, 2000, 9, 10, 240, 6, 0.8, law="gaussian", seed_cfg=34)
    got = rrs.depth(notion, w.X, w.Z, w.K, w.n_refine, w.cap_shrink, 5, precision=prec,
                    want_poles=True, first_cap=first, area_cap=True)
    ref = oracle.rrs_depth_idx(notion, w.X, w.Z, np.arange(len(w.Z)), w.K, w.n_refine,
                               w.cap_shrink, 5, with_poles=True, first_cap=first, area_cap=True)
    assert np.array_equal(got["depth"], ref["depth"])
    assert np.array_equal(got["poles"], ref["poles"])
