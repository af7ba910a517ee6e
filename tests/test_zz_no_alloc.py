"""GPU: lc_sweep_noalloc (the sweep with its scratch in the library's static
device array) against lc_sweep, through the C ABI: the new state (header
and values) and the exit intensities bit for bit, for calls in a row on one
device -- a larger problem, then a smaller one, in float32 and in float64 --
and the refusal of a plan whose scratch exceeds the array."""
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


def _problem(nx, ny, n_az, n_pol, G, seed):
    rng = np.random.default_rng(seed)
    T = rng.uniform(0.01, 1.0, nx * ny)
    p = W.make_problem(nx, ny, nx * 0.1, ny * 0.1, n_az, n_pol, G, 0.001, 20.0, 0.04, 2.0, [T], name=f"n{seed}")
    p.I_in = rng.uniform(0.0, 0.3, p.I_in.shape)
    p.state0 = W.group_planck(p.edges, rng.uniform(0.005, 0.5, nx * ny))
    return p


def _both(lc, driver, prob, prec):
    """One sweep from the problem's initial state with lc_sweep and with
    lc_sweep_noalloc into zeroed buffers; returns both states and exits."""
    import torch
    s = driver.Solver(prob, prec=prec)
    s.reset()
    out = []
    for fn in (lc.lc_sweep, lc.lc_sweep_noalloc):
        st = s.plan.new_state().zero_()
        ex = torch.zeros_like(s.I_exit)
        fn(s.plan, s.kappa.view(-1), s.planck.view(-1), prob.c_dt, s.state[0], st, s.I_in, ex)
        out.append((st, ex))
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("prec", [1, 0])
def test_noalloc_sweep_equals_sweep_on_calls_in_a_row(lcmod, prec):
    import torch
    lc, driver = lcmod
    big = _problem(40, 30, 12, 2, 17, 1)
    small = _problem(12, 10, 8, 3, 3, 2)
    for prob in (big, small):
        _say(f"case no-alloc sweep prec={prec}: {prob.nx}x{prob.ny} G={prob.G} M={prob.M}")
        (sa, ea), (sb, eb) = _both(lc, driver, prob, prec)
        assert torch.equal(sa, sb), "state differs"
        assert torch.equal(ea, eb), "exit intensities differ"
        assert float(ea.abs().max()) > 0.0


def test_noalloc_sweep_refuses_a_plan_beyond_the_scratch(lcmod):
    import torch
    lc, driver = lcmod
    nx = ny = 33
    G = 4096                        # 33 * 33 * 4096 float64 records of 16 bytes > 64 MiB
    phi, mu, om = W.product_quadrature(4, 1)
    rays = lc.lc_build_rays(nx, ny, 3.3, 3.3, phi, mu, om, 0.05)
    plan = lc.Plan(rays, G, lc.LC_F64)
    kap = torch.ones(G * nx * ny, dtype=torch.float64, device="cuda")
    a, b = plan.new_state().zero_(), plan.new_state().zero_()
    I_in = torch.zeros(plan.n_in, dtype=torch.float64, device="cuda")
    with pytest.raises(lc.LcError) as e:
        lc.lc_sweep_noalloc(plan, kap, kap, 1.0, a, b, I_in)
    assert e.value.status == lc.LC_ERR_ARG
    assert "static scratch" in str(e.value)
