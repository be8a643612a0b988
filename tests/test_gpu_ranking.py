"""Center-outward ranking study on the GPU at a small size: the depths order
the points of a Toeplitz Gaussian like its density does, and the depths of the
study are the oracle's."""
import numpy as np
import pytest
import torch

import oracle
from paper_2506_08262_amd import ranking, rrs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_small_ranking_study(prec):
    r = ranking.study(5, n=4000, queries=150, K=2000, n_refine=10, cap_shrink=0.9,
                      precision=prec)
    print("ranking", prec, r, flush=True)
    assert r["pdf_x_DP"]["spearman"] > 0.98 and r["pdf_x_DP"]["kendall"] > 0.85
    assert r["pdf_x_DAP"]["spearman"] > 0.95
    assert r["pdf_x_DML"]["spearman"] > 0.99


def test_ranking_study_depths_match_the_oracle():
    rng = np.random.default_rng(0)
    X = ranking.sample(rng, 3000, 5, "t", 2.0)
    Z = X[rng.choice(3000, size=4, replace=False)]
    for notion in ("projection", "apd"):
        got = rrs.depth(notion, torch.from_numpy(X).cuda(), torch.from_numpy(Z).cuda(), 400, 8,
                        0.9, 0, precision="f32")["depth"].cpu().numpy()
        ref = oracle.rrs_depth(notion, X, Z, 400, 8, 0.9, 0)["depth"]
        assert np.array_equal(got, ref), notion


def test_chunked_study_equals_one_call():
    """The study hands its queries to the library in chunks with their stream
    offsets: the depths and correlations equal those of a single call."""
    one = ranking.study(5, n=3000, queries=60, K=600, n_refine=6, cap_shrink=0.9,
                        precision="f32", chunk=60)
    parts = ranking.study(5, n=3000, queries=60, K=600, n_refine=6, cap_shrink=0.9,
                          precision="f32", chunk=17)
    for key in ("pdf_x_DP", "pdf_x_DAP", "DP_x_DAP"):
        assert one[key] == parts[key], key
