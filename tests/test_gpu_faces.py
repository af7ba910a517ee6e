"""GPU: interior-face moments of eq. (16) (lc_sweep_points +
lc_face_moments) against the oracle, for both grid constructions, both
precisions and more groups than a bundle holds; and the plain sweep's
results are unchanged by storing the upwind intensities."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import faces as OF, rays as R, sweep as OS
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


def _problem(nx, ny, G, n_pol=2, steps=2, seed=31, h_moc=0.04):
    rng = np.random.default_rng(seed)
    Ts = [rng.uniform(0.01, 1.0, nx * ny) for _ in range(steps)]
    return W.make_problem(nx, ny, nx * 0.1, ny * 0.1, 8, n_pol, G, 0.001, 20.0, h_moc, 2.0, Ts, name="faces")


def _oracle_faces(prob, mode):
    g = R.build(prob.nx, prob.ny, prob.lx, prob.ly, prob.phi, prob.h_moc, mode)
    st = OS.initial_state(g, prob.n_pol, prob.state0)
    pts = None
    for t in range(prob.steps):
        pts = np.zeros_like(st)
        st, _ = OS.sweep(g, prob.mu, prob.kappa[t], prob.planck[t], prob.c_dt, st, prob.I_in, points=pts)
    return OF.face_moments(g, prob.phi, prob.mu, prob.omega, pts, W.C_LIGHT)


@pytest.mark.parametrize("nx,ny,G,n_pol,mode,prec", [
    (9, 7, 5, 2, 0, 0), (9, 7, 5, 2, 0, 1), (8, 6, 3, 4, 1, 0), (8, 6, 3, 4, 1, 1),
    (6, 5, 70, 2, 0, 0), (1, 6, 4, 2, 0, 0), (7, 1, 4, 3, 0, 1)])
def test_face_moments_match_oracle(lcmod, nx, ny, G, n_pol, mode, prec):
    lc, driver = lcmod
    prob = _problem(nx, ny, G, n_pol=n_pol)
    _say(f"faces {nx}x{ny} G={G} P={n_pol} mode={mode} prec={prec}")
    s = driver.Solver(prob, prec=prec, mode=mode)
    s.enable_faces()
    s.reset()
    s.step_faces(prob.steps)
    got = s.face_moments()
    E, F, f = _oracle_faces(prob, mode)
    tol = 1e-12 if prec == 0 else 1e-5
    if E.shape[1] == 0:
        assert got["E"].shape == E.shape
        return
    eE, eF, ef = err_E(got["E"], E), err_F(got["F"], F, E, W.C_LIGHT), err_f(got["f"], f, E)
    _say(f"  E {eE:.2e} F {eF:.2e} f {ef:.2e}")
    assert eE <= tol and eF <= tol and ef <= tol


def test_storing_upwind_intensities_leaves_the_sweep_unchanged(lcmod):
    lc, driver = lcmod
    prob = _problem(10, 8, 6)
    a = driver.Solver(prob, prec=lc.LC_F32)
    b = driver.Solver(prob, prec=lc.LC_F32)
    b.enable_faces()
    a.reset()
    b.reset()
    a.step(2, graph=False)
    b.step_faces(2)
    ma, mb = a.moments(), b.moments()
    for k in ("E", "F", "f", "bnd"):
        assert np.array_equal(ma[k], mb[k]), k
    assert np.array_equal(a.state_canonical(), b.state_canonical())
    assert np.array_equal(a.exits(), b.exits())
