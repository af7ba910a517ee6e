"""GPU: lc_state_import, the inverse of lc_state_export.

* float64 and float32 states survive export -> import -> export unchanged,
  and a run resumed from the imported buffer gives the moments and state of
  the uninterrupted run bit for bit;
* a float32 state imported into a float64 plan of the same grid gives, with
  the float64 moment gather, the float32 run's moments within 1e-5 (the
  difference is the float32 gather's rounding alone)."""
import sys

import numpy as np
import pytest

import workloads as W
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


def _problem(steps=3):
    rng = np.random.default_rng(77)
    nx, ny = 24, 18
    Ts = [rng.uniform(0.01, 1.0, nx * ny) for _ in range(steps)]
    return W.make_problem(nx, ny, 2.4, 1.8, 12, 4, 7, 0.001, 20.0, 0.04, 2.0, Ts, name="st")


@pytest.mark.parametrize("prec", [0, 1])
def test_import_round_trip_and_resume(lcmod, prec):
    import torch
    lc, driver = lcmod
    prob = _problem()
    _say(f"case state import prec={prec}")
    full = driver.Solver(prob, prec=prec)
    full.reset()
    full.step(3, graph=False)
    ref = full.moments()
    ref_state = full.state_canonical()

    s = driver.Solver(prob, prec=prec, rays=full.rays)
    s.reset()
    s.step(2, graph=False)
    canon = torch.empty(s.plan.n_state, dtype=torch.float64, device="cuda")
    lc.lc_state_export(s.plan, s.state[s.cur], canon)
    other = s.plan.new_state().zero_()
    lc.lc_state_import(s.plan, canon, other)
    again = torch.empty_like(canon)
    lc.lc_state_export(s.plan, other, again)
    torch.cuda.synchronize()
    assert torch.equal(canon, again)
    # resume from the imported buffer
    s.state[s.cur] = other
    s.step(1, graph=False)
    got = s.moments()
    for k in ("E", "F", "f", "bnd"):
        assert np.array_equal(got[k], ref[k]), k
    assert np.array_equal(s.state_canonical(), ref_state)


def test_float32_state_in_a_float64_plan(lcmod):
    import torch
    lc, driver = lcmod
    prob = _problem(steps=1)
    s32 = driver.Solver(prob, prec=lc.LC_F32)
    s32.reset()
    s32.step(1, graph=False)
    m32 = s32.moments()
    s64 = driver.Solver(prob, prec=lc.LC_F64, rays=s32.rays)
    canon = torch.empty(s32.plan.n_state, dtype=torch.float64, device="cuda")
    lc.lc_state_export(s32.plan, s32.state[s32.cur], canon)
    st = s64.plan.new_state()
    lc.lc_state_import(s64.plan, canon, st)
    lc.lc_moments(s64.plan, st, s64.c, s64.E, s64.F, s64.f)
    m = s64.moments()
    c = W.C_LIGHT
    e = (err_E(m32["E"], m["E"]), err_F(m32["F"], m["F"], m["E"], c), err_f(m32["f"], m["f"], m["E"]))
    _say(f"  float32 gather vs float64 gather of the same state: E {e[0]:.2e} F {e[1]:.2e} f {e[2]:.2e}")
    assert max(e) <= 1e-5
