"""GPU: group-dependent characteristic grids (groups swept on grids of their
own spacing, advanced together as one batch) against the oracle run of each
group range on its own grid, and the grey closures of the whole problem
(lc_grey_closures_dims) against the oracle's."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import closures as oc, solve as osolve
from tests.parity_util import err_E, err_F, err_f

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lcmod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_11998_amd import driver, lc
    return lc, driver


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-5)])
def test_group_ranges_on_their_own_grids(lcmod, prec, tol):
    lc, driver = lcmod
    rng = np.random.default_rng(41)
    nx, ny = 12, 9
    Ts = [rng.uniform(0.01, 1.0, nx * ny) for _ in range(2)]
    prob = W.make_problem(nx, ny, 1.2, 0.9, 8, 2, 6, 0.001, 20.0, 0.05, 2.0, Ts, name="split")
    parts = [(0, 2, 0.06), (2, 6, 0.025)]
    gs = driver.GroupSplitSolver(prob, parts, prec=prec)
    gs.reset()
    gs.step(2)
    got = gs.moments()
    refs = []
    for (g0, g1, h), sub in zip(parts, gs.subs):
        _say(f"groups {g0}:{g1} on spacing {h}")
        r = osolve.run(sub)["steps"][-1]
        refs.append(r)
        c = W.C_LIGHT
        assert err_E(got["E"][g0:g1], r["E"]) <= tol
        assert err_F(got["F"][g0:g1], r["F"], r["E"], c) <= tol
        assert err_f(got["f"][g0:g1], r["f"], r["E"]) <= tol
    E = np.concatenate([r["E"] for r in refs])
    F = np.concatenate([r["F"] for r in refs])
    f = np.concatenate([r["f"] for r in refs])
    ref = oc.grey_closures(E, F, f, prob.kappa[1], prob.planck[1])
    out = gs.grey_closures(1)
    rows = range(oc.N_GREY) if prec == 0 else [oc.NAMES.index(n) for n in ("E", "kappa_E", "kappa_B", "fE_xx",
                                                                             "fE_yy", "fE_zz")]
    for r in rows:
        scale = np.abs(ref[r]).max()
        assert np.all(np.abs(out[r] - ref[r]) <= tol * (np.abs(ref[r]) + scale)), oc.NAMES[r]
