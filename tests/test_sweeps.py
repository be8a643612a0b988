"""Host logic of the convergence sweep driver (no GPU)."""
import numpy as np

from paper_2506_08262_amd import rrs, sweeps


def test_refinements_beyond_the_matrix_core_column_range_run_in_binary64(monkeypatch):
    """The matrix-core forms index at most 65535 directions per refinement;
    the driver runs larger refinements in binary64 (same depths) and leaves
    the others in the requested form."""
    seen = []

    class _Host:
        def cpu(self):
            return self

        def numpy(self):
            return np.zeros(1)

    def fake_depth(notion, X, Z, K, r, alpha, seed, precision="f64", area_cap=False):
        seen.append((notion, K, r, precision))
        return {"depth": _Host()}

    monkeypatch.setattr(rrs, "depth", fake_depth)
    for K, r in ((100000, 1), (100000, 2), (65535, 1), (65536, 1), (200, 175)):
        sweeps._depth(None, None, K, r, 0.9, 11)
    assert seen == [("projection", 100000, 1, "f64"), ("projection", 100000, 2, "f32"),
                    ("projection", 65535, 1, "f32"), ("projection", 65536, 1, "f64"),
                    ("projection", 200, 175, "f32")]


def test_laws_have_the_requested_shape_and_are_seeded():
    for law in sweeps.LAWS.values():
        a = law(np.random.default_rng(3), 500, 7)
        b = law(np.random.default_rng(3), 500, 7)
        assert a.shape == (500, 7) and a.dtype == np.float64
        assert np.array_equal(a, b)
