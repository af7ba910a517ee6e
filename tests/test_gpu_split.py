"""GPU: the split sweep (traversals cut into chunks whose affine transfer maps
are composed by a scan, lc_plan_set_split) against the oracle, and against
the whole-traversal sweep: bit-identical while a traversal has at most two
chunks (the first two chunks round exactly as the whole sweep), within a few
rounding steps beyond."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import rays as orays
from tests.test_gpu_parity import TOL32, TOL64, _compare_full, _custom_problem

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


def _longest(prob, mode=0):
    g = orays.build(prob.nx, prob.ny, prob.lx, prob.ly, prob.phi, prob.h_moc, mode)
    return max(len(c) for pr in g.pairs for c in pr.cells)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("chunk", [4, 8, 12])
def test_split_sweep_matches_oracle(lcmod, prec, chunk):
    lc, driver = lcmod
    prob = _custom_problem(nx=20, ny=14, lx=2.0, ly=1.4, n_az=8, G=5, h_moc=0.03, steps=2)
    _compare_full(lc, driver, prob, prec, TOL64 if prec == 0 else TOL32, split=chunk)


@pytest.mark.parametrize("case", ["config0", "many_groups", "odd_polar", "thin", "tubes", "eager"])
def test_split_sweep_cases(lcmod, case):
    lc, driver = lcmod
    mode, graph, prec = 0, True, 0
    if case == "config0":
        prob, prec = W.config(0), 1
    elif case == "many_groups":
        prob = _custom_problem(nx=10, ny=9, lx=1.0, ly=0.9, n_az=4, G=70, h_moc=0.05, steps=2)
    elif case == "odd_polar":
        prob = _custom_problem(mu=[-0.6, 0.2, 0.7], w=[0.3, 0.4, 0.3], n_az=8, G=3, steps=2)
    elif case == "thin":
        prob = _custom_problem(nx=9, ny=1, lx=1.8, ly=0.2, n_az=8, G=2, h_moc=0.02, steps=1)
    elif case == "tubes":
        prob, mode = _custom_problem(nx=8, ny=6, lx=0.8, ly=0.6, n_az=8, G=3, h_moc=0.04, steps=2), 1
    else:
        prob, graph, prec = _custom_problem(n_az=8, G=4, steps=2), False, 1
    _compare_full(lc, driver, prob, prec, TOL64 if prec == 0 else TOL32, graph=graph, mode=mode, split=4)


@pytest.mark.parametrize("prec", [0, 1])
def test_split_against_whole_traversals(lcmod, prec):
    lc, driver = lcmod
    prob = _custom_problem(nx=24, ny=18, lx=2.4, ly=1.8, n_az=8, G=6, h_moc=0.03, steps=2)
    Lmax = _longest(prob)
    ref = driver.Solver(prob, prec=prec)
    ref.reset()
    ref.step(2)
    mr = ref.moments()
    for chunk, exact in ((((Lmax + 1) // 2 + 3) // 4 * 4, True), (4 * ((Lmax + 15) // 16), False), (4, False)):
        _say(f"chunk {chunk} (longest characteristic {Lmax}) prec={prec}")
        s = driver.Solver(prob, prec=prec, split=chunk)
        s.reset()
        s.step(2)
        m = s.moments()
        st, ex = s.state_canonical(), s.exits()
        if exact:
            for k in ("E", "F", "f", "bnd"):
                assert np.array_equal(m[k], mr[k]), k
            assert np.array_equal(st, ref.state_canonical())
            assert np.array_equal(ex, ref.exits())
        else:
            rt = 1e-13 if prec == 0 else 2e-6
            sr = ref.state_canonical()
            assert np.max(np.abs(st - sr)) <= rt * np.max(np.abs(sr))
            assert np.allclose(m["E"], mr["E"], rtol=rt, atol=0)


def test_split_graph_replays_equal_eager_and_switch_off(lcmod):
    lc, driver = lcmod
    prob = _custom_problem(nx=16, ny=12, lx=1.6, ly=1.2, n_az=8, G=4, h_moc=0.03, steps=2)
    a = driver.Solver(prob, prec=lc.LC_F32, split=8)
    b = driver.Solver(prob, prec=lc.LC_F32, split=8)
    a.reset()
    a.step(2, graph=True)
    b.reset()
    b.step(2, graph=False)
    for _ in range(3):                  # replays of the captured graph, eager work between them
        a.reset()
        a.step(2, graph=True)
        assert np.array_equal(a.state_canonical(), b.state_canonical())
        assert np.array_equal(a.exits(), b.exits())
        ma, mb = a.moments(), b.moments()
        for k in ("E", "F", "f", "bnd"):
            assert np.array_equal(ma[k], mb[k]), k
    # turning the split off gives the whole-traversal sweep again
    lc.lc_plan_set_split(a.plan, 0)
    c = driver.Solver(prob, prec=lc.LC_F32)
    for s in (a, c):
        s.reset()
        s.step(2)
    assert np.array_equal(a.state_canonical(), c.state_canonical())


def test_split_argument_errors(lcmod):
    lc, driver = lcmod
    prob = _custom_problem(nx=6, ny=5, lx=0.6, ly=0.5, n_az=4, G=2, steps=1)
    s = driver.Solver(prob)
    for bad in (-4, 3, 6, (1 << 24) + 4):
        with pytest.raises(lc.LcError) as e:
            lc.lc_plan_set_split(s.plan, bad)
        assert e.value.status == lc.LC_ERR_ARG
    lc.lc_plan_set_split(s.plan, 1 << 24)
    lc.lc_plan_set_split(s.plan, 0)


def test_tuner_choice_is_cached_with_the_split(lcmod, tmp_path):
    """The tuner's choice (split chunk length included) is stored and
    restored from its cache; results with the restored setting equal those
    right after tuning."""
    lc, driver = lcmod
    from paper_2305_11998_amd import tune
    prob = _custom_problem(nx=12, ny=10, lx=1.2, ly=1.0, n_az=8, G=2, h_moc=0.02, steps=1)
    cache = str(tmp_path / "tune.json")
    a = driver.Solver(prob, prec=lc.LC_F32)
    ta = tune.tune(a, reps=1, cache=cache)
    assert not ta["cached"] and ta["split"] in tune.SPLIT_CANDIDATES
    assert set(ta["split_ms"]) == {str(c) for c in tune.SPLIT_CANDIDATES}
    b = driver.Solver(prob, prec=lc.LC_F32)
    tb = tune.tune(b, reps=1, cache=cache)
    assert tb["cached"] and tb["split"] == ta["split"] and tb["sweep_unroll"] == ta["sweep_unroll"]
    assert tb["sweep_capped"] == ta["sweep_capped"] and ta["sweep_capped"] in (0, 1)
    for s in (a, b):
        s.reset()
        s.step(1)
    assert np.array_equal(a.state_canonical(), b.state_canonical())
    assert np.array_equal(a.moments()["E"], b.moments()["E"])
