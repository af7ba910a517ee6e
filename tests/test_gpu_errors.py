"""GPU: the argument checks that need a live plan or batch return their
documented status, leave lc_last_error() describing the failure, launch
nothing, and leave the handle usable (a valid call afterwards gives the same
result as one on a fresh handle)."""
import ctypes as C
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_11998_amd import driver, lc
    rng = np.random.default_rng(7)
    Ts = [rng.uniform(0.01, 1.0, 8 * 6) for _ in range(2)]
    prob = W.make_problem(8, 6, 0.8, 0.6, 8, 2, 3, 0.001, 20.0, 0.05, 2.0, Ts, name="err")
    s = driver.Solver(prob, prec=lc.LC_F32)
    return lc, driver, s


def _p(t):
    return None if t is None else t.data_ptr()


def _expect(lc, status, want, needle):
    assert status == want, (status, lc._lib.lc_last_error())
    msg = lc._lib.lc_last_error().decode()
    assert needle in msg, msg


def test_plan_create_rejects_group_count_and_precision(env):
    lc, driver, s = env
    h = C.c_void_p()
    _say("plan_create: G 0, G 4097, precision 7")
    _expect(lc, lc._lib.lc_plan_create(s.rays.handle, 0, lc.LC_F32, C.byref(h)), lc.LC_ERR_ARG, "G must be")
    _expect(lc, lc._lib.lc_plan_create(s.rays.handle, 4097, lc.LC_F32, C.byref(h)), lc.LC_ERR_ARG, "G must be")
    _expect(lc, lc._lib.lc_plan_create(s.rays.handle, 3, 7, C.byref(h)), lc.LC_ERR_ARG, "precision")
    _expect(lc, lc._lib.lc_plan_create(s.rays.handle, 3, lc.LC_F32, None), lc.LC_ERR_ARG, "out")


def test_tuning_rejects_out_of_range_values_and_keeps_the_old_setting(env):
    lc, driver, s = env
    lc.lc_plan_set_tuning(s.plan, 4, 2)
    for u, e, needle in [(3, 2, "sweep_unroll"), (32, 2, "sweep_unroll"), (0, 2, "sweep_unroll"),
                         (4, 0, "moments_entries"), (4, 5, "moments_entries")]:
        _say(f"set_tuning {u} {e}")
        t = lc.lc_tuning_t(u, e)
        _expect(lc, lc._lib.lc_plan_set_tuning(s.plan.handle, C.byref(t)), lc.LC_ERR_ARG, needle)
        assert lc.lc_plan_get_tuning(s.plan) == dict(sweep_unroll=4, moments_entries=2)
    _expect(lc, lc._lib.lc_plan_set_tuning(s.plan.handle, None), lc.LC_ERR_ARG, "tuning")
    # 16-step chunks: float32 only
    p64 = lc.Plan(s.rays, 3, lc.LC_F64)
    t = lc.lc_tuning_t(16, 2)
    _expect(lc, lc._lib.lc_plan_set_tuning(p64.handle, C.byref(t)), lc.LC_ERR_ARG, "sweep_unroll 16")
    lc.lc_plan_set_tuning(s.plan, 16, 2)
    assert lc.lc_plan_get_tuning(s.plan) == dict(sweep_unroll=16, moments_entries=2)


def test_sweep_moments_and_step_reject_bad_arguments(env):
    lc, driver, s = env
    L = lc._lib
    pl = s.plan.handle
    a, b = s.state
    k, B, Iin, Iex = _p(s.kappa), _p(s.planck), _p(s.I_in), _p(s.I_exit)
    _say("sweep: null kappa, aliased states, c_dt <= 0, c_dt nan")
    _expect(lc, L.lc_sweep(pl, None, B, 2.0, _p(a), _p(b), Iin, Iex, None), lc.LC_ERR_ARG, "NULL")
    _expect(lc, L.lc_sweep(pl, k, B, 2.0, _p(a), _p(a), Iin, Iex, None), lc.LC_ERR_ARG, "distinct")
    _expect(lc, L.lc_sweep(pl, k, B, 0.0, _p(a), _p(b), Iin, Iex, None), lc.LC_ERR_ARG, "c_dt")
    _expect(lc, L.lc_sweep(pl, k, B, float("nan"), _p(a), _p(b), Iin, Iex, None), lc.LC_ERR_ARG, "c_dt")
    _say("moments: null state, c <= 0, boundary factors without I_exit")
    E, F, f, bnd = _p(s.E), _p(s.F), _p(s.f), _p(s.bnd)
    _expect(lc, L.lc_moments(pl, None, Iex, Iin, 1.0, E, F, f, bnd, None), lc.LC_ERR_ARG, "state")
    _expect(lc, L.lc_moments(pl, _p(a), Iex, Iin, -1.0, E, F, f, bnd, None), lc.LC_ERR_ARG, "c must")
    _expect(lc, L.lc_moments(pl, _p(a), None, Iin, 1.0, E, F, f, bnd, None), lc.LC_ERR_ARG, "I_exit")
    _say("step: n_steps 0, aliased states, negative stride, c 0, boundary factors without I_exit")
    args = dict(n=1, stride=0, cdt=2.0, c=1.0, sa=_p(a), sb=_p(b), iex=Iex, bnd=bnd)

    def step(**kw):
        q = dict(args, **kw)
        return L.lc_step(pl, q["n"], k, B, q["stride"], q["cdt"], q["c"], q["sa"], q["sb"], Iin, q["iex"],
                         E, F, f, q["bnd"], None)
    _expect(lc, step(n=0), lc.LC_ERR_ARG, "n_steps")
    _expect(lc, step(sb=_p(a)), lc.LC_ERR_ARG, "distinct")
    _expect(lc, step(stride=-1), lc.LC_ERR_ARG, "material_stride")
    _expect(lc, step(c=0.0), lc.LC_ERR_ARG, "c_dt and c")
    _expect(lc, step(iex=None), lc.LC_ERR_ARG, "I_exit")
    _say("grey closures: null output")
    _expect(lc, L.lc_grey_closures(pl, E, F, f, k, B, None, None), lc.LC_ERR_ARG, "out")


def test_plan_still_works_after_rejected_calls(env):
    """After the rejected calls above, the plan gives the same result as a
    fresh one."""
    lc, driver, s = env
    lc.lc_plan_set_tuning(s.plan, 2, 3)
    s.reset()
    s.step(2)
    fresh = driver.Solver(s.prob, prec=lc.LC_F32)
    lc.lc_plan_set_tuning(fresh.plan, 2, 3)
    fresh.reset()
    fresh.step(2)
    m0, m1 = s.moments(), fresh.moments()
    for key in ("E", "F", "f", "bnd"):
        assert np.array_equal(m0[key], m1[key])


def test_batch_rejects_bad_problem_sets(env):
    import torch
    lc, driver, s = env
    s64 = driver.Solver(s.prob, prec=lc.LC_F64)

    def prob_of(sv, **kw):
        d = dict(plan=sv.plan.handle, kappa=_p(sv.kappa), planck=_p(sv.planck), material_stride=0, c_dt=2.0,
                 state_a=_p(sv.state[0]), state_b=_p(sv.state[1]), I_in=_p(sv.I_in), I_exit=_p(sv.I_exit),
                 E=_p(sv.E), F=_p(sv.F), f=_p(sv.f), bnd=_p(sv.bnd))
        d.update(kw)
        return lc.lc_problem_t(**d)

    def create(*ps):
        arr = (lc.lc_problem_t * len(ps))(*ps)
        h = C.c_void_p()
        return lc._lib.lc_batch_create(len(ps), arr, C.byref(h)), h

    _say("batch_create: empty, missing I_exit, aliased states, c_dt 0, negative stride, mixed precision")
    h = C.c_void_p()
    _expect(lc, lc._lib.lc_batch_create(0, None, C.byref(h)), lc.LC_ERR_ARG, "at least one")
    _expect(lc, create(prob_of(s, I_exit=None))[0], lc.LC_ERR_ARG, "problem 0")
    _expect(lc, create(prob_of(s), prob_of(s, state_b=_p(s.state[0])))[0], lc.LC_ERR_ARG, "problem 1")
    _expect(lc, create(prob_of(s, c_dt=0.0))[0], lc.LC_ERR_ARG, "c_dt")
    _expect(lc, create(prob_of(s, material_stride=-3))[0], lc.LC_ERR_ARG, "material_stride")
    _expect(lc, create(prob_of(s), prob_of(s64))[0], lc.LC_ERR_ARG, "one precision")
    s.reset()
    st, h = create(prob_of(s))
    assert st == lc.LC_OK
    try:
        _say("batch_step: n_steps 0, c nan")
        _expect(lc, lc._lib.lc_batch_step(h, 0, 1.0, None), lc.LC_ERR_ARG, "n_steps")
        _expect(lc, lc._lib.lc_batch_step(h, 1, float("nan"), None), lc.LC_ERR_ARG, "c must")
        assert lc._lib.lc_batch_step(h, 1, 1.0, None) == lc.LC_OK
        torch.cuda.synchronize()
    finally:
        assert lc._lib.lc_batch_free(h) == lc.LC_OK
