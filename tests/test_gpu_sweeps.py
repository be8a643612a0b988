"""The convergence sweeps run end to end on the GPU at a small size, and more
directions bring the depths closer to the reference minimum."""
import numpy as np
import pytest

from paper_2506_08262_amd import sweeps

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("area_cap", [False, True])
def test_alpha_sweep_small(area_cap):
    r = sweeps.alpha_sweep(n=3000, d=6, points=8, ref_K=40000, ref_r=40, ref_runs=2,
                           alphas=(0.6, 0.9), Ks=(100, 3000), rs=(10,), area_cap=area_cap)
    cells = {(c["alpha"], c["K"]): c for c in r["grid"]}
    assert len(cells) == 4
    for c in r["grid"]:
        assert c["mse_mean"] >= 0.0 and c["mse_max"] >= c["mse_mean"]
    # more directions: no larger mean error (the depth is a minimum over them)
    for a in (0.6, 0.9):
        assert cells[(a, 3000)]["mse_mean"] <= cells[(a, 100)]["mse_mean"] + 1e-12


def test_grid_sweep_small():
    r = sweeps.grid_sweep(n=2000, dims=(3, 8), points=6, Ks=(100, 2000), rs=(1, 5, 20))
    assert [e["d"] for e in r["dims"]] == [3, 8]
    for e in r["dims"]:
        assert min(c["mse_mean"] for c in e["cells"]) >= 0.0
        assert all(p["converged_points"] <= 6 for p in e["per_K"])
