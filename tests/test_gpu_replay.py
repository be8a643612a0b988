"""Replay protocol for the plain binary32 form (approximate projections, no
recheck).  Its trajectory may leave the binary64 one as soon as a binary32
order statistic moves a refinement's argmin, so its final depth is not
compared with the oracle's directly.  Instead the oracle follows the GPU's
own trajectory (its chosen direction and improvement flag per refinement)
and computes the exact depth of every direction of every refinement; per
refinement, the GPU's minimum must be within 1e-6 relative of the exact
minimum over the same directions, and the exact depth of the direction the
GPU chose must be within 1e-6 relative of that minimum.  Refinements where
two directions' exact depths lie within 1e-6 of each other (near ties) are
counted and printed."""
import sys

import numpy as np
import pytest

import oracle
from paper_2506_08262_amd import rrs, workloads

pytestmark = pytest.mark.gpu

TOL = 1e-6


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _lib():
    oracle.build(force=False)
    rrs.load()
    yield
    rrs.rrs_release_workspace()


def _replay(notion, w, nq):
    Z = w.Z[:nq]
    got = rrs.depth(notion, w.X, Z, w.K, w.n_refine, w.cap_shrink, w.rrs_seed,
                    precision="f32_plain", want_trace=True)
    worst_min, worst_pick, steps = 0.0, 0.0, 0
    for i in range(nq):
        tr = got["trace"][i]
        gvals = tr[:, 2].copy().view(np.float64)
        ex = oracle.rrs_replay(notion, w.X, Z[i], i, w.K, w.n_refine, w.cap_shrink,
                               w.rrs_seed, tr)
        emin, epick = ex[:, 0], ex[:, 1]
        scale = np.maximum(np.abs(emin), 1e-300)
        rmin = np.abs(gvals - emin) / scale
        rpick = np.abs(epick - emin) / scale
        worst_min = max(worst_min, float(rmin.max()))
        worst_pick = max(worst_pick, float(rpick.max()))
        steps += w.n_refine
        assert rmin.max() <= TOL, (i, rmin.max())
        assert rpick.max() <= TOL, (i, rpick.max())
        # the final depth is the smallest improving minimum of the trajectory
        imp = tr[:, 1].astype(bool)
        final = min([1.0] + [float(v) for v, b in zip(gvals, imp) if b])
        assert got["depth"][i] == final
    _say(notion, w.name, "refinements", steps, "max rel |gpu min - exact min|", worst_min,
         "max rel |exact(gpu pick) - exact min|", worst_pick)


@pytest.mark.parametrize("notion", ["projection", "apd"])
def test_plain_f32_replay_small(notion):
    w = workloads.small(notion, 3000, 8, 10, 400, 8, 0.5, law="wishart_cauchy", seed_cfg=61)
    _replay(notion, w, 10)


@pytest.mark.parametrize("notion", ["projection", "apd"])
def test_plain_f32_replay_config_shape(notion):
    """The 10,000 x 20 Wishart/Cauchy workload's data, K = 5000 and r = 20 as
    configured, on queries from both the Gaussian and the Cauchy part."""
    w = workloads.make("c2")
    idx = np.array([0, 1, 2, 900, 901])
    w.Z = w.Z[idx]
    _replay(notion, w, len(idx))
