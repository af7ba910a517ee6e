"""GPU: the process-wide test and debug settings.

* lc_set_validation: with it on, a sweep or a step whose kappa, planck or
  I_in holds a value that is not finite or is negative fails with LC_ERR_ARG
  naming the array and the first such index, before any launch; valid
  inputs give the same results bit for bit as with it off.
* lc_set_alloc_limit: allocations above the limit fail as an exhausted
  device would -- plan, batch and low-order handle creation return
  LC_ERR_ALLOC and free what they had -- and everything works again once
  the limit is lifted."""
import sys

import numpy as np
import pytest

import workloads as W

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


def _sweep(lc, s, kappa, planck, I_in):
    lc.lc_sweep(s.plan, kappa, planck, s.prob.c_dt, s.state[0], s.state[1], I_in, s.I_exit)


def test_validation_rejects_bad_inputs(lcmod):
    import torch
    lc, driver = lcmod
    prob = W.config(0)
    s = driver.Solver(prob, prec=lc.LC_F64)
    _say("case validation mode on the 16x16 workload")
    kap, pla = s.kappa[0].reshape(-1).clone(), s.planck[0].reshape(-1).clone()
    s.reset()
    _sweep(lc, s, kap, pla, s.I_in)
    ref = s.state[1].clone()
    try:
        lc.lc_set_validation(True)
        s.reset()
        _sweep(lc, s, kap, pla, s.I_in)
        assert torch.equal(s.state[1], ref)
        for name, arr, idx, val in (("kappa", kap, 77, float("nan")), ("planck", pla, 5, -1.0),
                                    ("I_in", s.I_in, 123, float("inf"))):
            bad = arr.clone().reshape(-1)
            bad[idx] = val
            args = {"kappa": kap, "planck": pla, "I_in": s.I_in.reshape(-1)}
            args[name] = bad
            with pytest.raises(lc.LcError) as e:
                _sweep(lc, s, args["kappa"], args["planck"], args["I_in"])
            assert e.value.status == lc.LC_ERR_ARG and f"{name}[{idx}]" in str(e.value), str(e.value)
        bad = kap.clone()
        bad[-1] = float("nan")
        with pytest.raises(lc.LcError) as e:
            lc.lc_step(s.plan, 1, bad, pla, prob.c_dt, s.c, s.state[0], s.state[1], s.I_in, s.I_exit, s.E, s.F, s.f,
                       s.bnd)
        assert e.value.status == lc.LC_ERR_ARG and f"kappa[{kap.numel() - 1}]" in str(e.value)
    finally:
        lc.lc_set_validation(False)
    bad = kap.clone()
    bad[0] = -1.0
    _sweep(lc, s, bad, pla, s.I_in)                  # not checked when off
    torch.cuda.synchronize()


def test_alloc_limit_forces_clean_errors(lcmod):
    import torch
    lc, driver = lcmod
    prob = W.config(0)
    rays = lc.lc_build_rays(prob.nx, prob.ny, prob.lx, prob.ly, prob.phi, prob.mu, prob.omega, prob.h_moc)
    _say("case allocation limit")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    try:
        lc.lc_set_alloc_limit(4096)
        for make in (lambda: lc.Plan(rays, prob.G, lc.LC_F64), lambda: lc.Loqd(16, 16, 6.0, 6.0, 4)):
            with pytest.raises(lc.LcError) as e:
                make()
            assert e.value.status == lc.LC_ERR_ALLOC
    finally:
        lc.lc_set_alloc_limit(0)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] >= free0 - (64 << 20)    # nothing of the failed calls stays allocated
    plan = lc.Plan(rays, prob.G, lc.LC_F64)                     # and creation works again
    h = lc.Loqd(16, 16, 6.0, 6.0, 4)
    del plan, h
