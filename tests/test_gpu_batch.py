"""GPU: the batched form (one persistent launch per phase over many uneven
problems) against the single-problem path and against the oracle."""
import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle import rays as orays, solve as osolve
from tests.parity_util import err_E, err_F, err_f, err_rel

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


def _mixed_problems(steps=2):
    out = []
    specs = [(12, 10, 8, 2, 3), (20, 20, 12, 4, 5), (7, 16, 8, 3, 1), (24, 8, 16, 2, 8), (16, 16, 4, 1, 2)]
    for j, (nx, ny, n_az, n_pol, G) in enumerate(specs):
        rng = np.random.default_rng(100 + j)
        Ts = [rng.uniform(0.01, 1.0, nx * ny) for _ in range(steps)]
        prob = W.make_problem(nx, ny, nx * 0.1, ny * 0.1, n_az, n_pol, G, 0.001, 20.0, 0.03, 2.0, Ts,
                              name=f"m{j}")
        out.append(prob)
    return out


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_equals_single_problem_runs(lcmod, prec):
    lc, driver = lcmod
    probs = _mixed_problems()
    _say(f"batch of {len(probs)} mixed problems, prec {prec}")
    bs = driver.BatchSolver(probs, prec=prec)
    bs.reset()
    bs.step(2)
    for p, sb in zip(probs, bs.solvers):
        s = driver.Solver(p, prec=prec)
        s.reset()
        s.step(2)
        mb, ms = sb.moments(), s.moments()
        for k in ("E", "F", "f", "bnd"):
            assert np.array_equal(mb[k], ms[k]), (p.name, k, np.abs(mb[k] - ms[k]).max())
        assert np.array_equal(sb.state_canonical(), s.state_canonical())


def test_batch_against_oracle(lcmod):
    lc, driver = lcmod
    probs = _mixed_problems()
    bs = driver.BatchSolver(probs, prec=lc.LC_F64)
    bs.reset()
    bs.step(2)
    for p, sb in zip(probs, bs.solvers):
        _say(f"oracle {p.name}")
        ref = osolve.run(p)["steps"][-1]
        got = sb.moments()
        c = W.C_LIGHT
        assert err_E(got["E"], ref["E"]) <= 1e-12
        assert err_F(got["F"], ref["F"], ref["E"], c) <= 1e-12
        assert err_f(got["f"], ref["f"], ref["E"]) <= 1e-12
        for q in range(4):
            assert err_rel(got["bnd"][..., q], ref["bnd"][..., q]) <= 1e-11


def test_batch_repeated_steps_are_deterministic(lcmod):
    lc, driver = lcmod
    probs = _mixed_problems(steps=1)
    outs = []
    for _ in range(2):
        bs = driver.BatchSolver(probs, prec=lc.LC_F32, static_material=True)
        bs.reset()
        bs.step(3)
        outs.append([s.moments()["E"] for s in bs.solvers])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_full_batched_workload_sampled(lcmod):
    """The 64-problem batched workload, one step in float32, three members
    checked on sampled cells against the oracle (1e-5)."""
    lc, driver = lcmod
    probs = W.batch_problems(steps=1)
    _say("64-problem batch: building")
    bs = driver.BatchSolver(probs, prec=lc.LC_F32)
    bs.reset()
    bs.step(1)
    rng = np.random.default_rng(5)
    members = [int(i) for i in rng.choice(len(probs), 3, replace=False)]
    for q in members:
        p, s = probs[q], bs.solvers[q]
        got = s.moments()
        cells = np.concatenate([rng.choice(p.cells, 4, replace=False), [0, p.cells - 1]])
        _say(f"  member {q}: {p.nx}^2 G={p.G} M={p.M}")
        g = orays.build(p.nx, p.ny, p.lx, p.ly, p.phi, p.h_moc, only_cells=cells)
        ref = osolve.run_sampled(p, g, cells)["steps"][-1]
        c = W.C_LIGHT
        eE = err_E(got["E"][:, cells], ref["E"])
        eF = err_F(got["F"][:, :, cells], ref["F"], ref["E"], c)
        ef = err_f(got["f"][:, :, cells], ref["f"], ref["E"])
        _say(f"    E {eE:.2e} F {eF:.2e} f {ef:.2e}")
        assert eE <= 1e-5 and eF <= 1e-5 and ef <= 1e-5


def test_batch_graph_replays_equal_eager_phases(lcmod):
    """Every replay of the captured step graph, with eager work (state
    resets) between replays, gives the result of the eager, profiled path
    bit for bit."""
    import torch
    lc, driver = lcmod
    probs = _mixed_problems(steps=1)
    bs = driver.BatchSolver(probs, prec=lc.LC_F32, static_material=True)
    lc.lc_batch_profile(bs.batch, True)
    bs.reset()
    bs.step(2)
    torch.cuda.synchronize()
    lc.lc_batch_profile_read(bs.batch)
    lc.lc_batch_profile(bs.batch, False)
    ref = [(s.moments(), s.state_canonical()) for s in bs.solvers]
    for rep in range(3):
        _say(f"graph replay {rep}")
        bs.reset()
        bs.step(2)
        torch.cuda.synchronize()
        for (m0, st0), s in zip(ref, bs.solvers):
            m = s.moments()
            for k in ("E", "F", "f", "bnd"):
                assert np.array_equal(m[k], m0[k])
            assert np.array_equal(s.state_canonical(), st0)


def test_batch_with_more_than_64_groups(lcmod):
    """A member with G > 64 beside small-G members: batch equals the
    single-problem runs bit for bit."""
    lc, driver = lcmod
    specs = [(9, 7, 8, 2, 70), (12, 10, 8, 2, 5)]
    probs = []
    for j, (nx, ny, n_az, n_pol, G) in enumerate(specs):
        rng = np.random.default_rng(300 + j)
        Ts = [rng.uniform(0.01, 1.0, nx * ny) for _ in range(2)]
        probs.append(W.make_problem(nx, ny, nx * 0.1, ny * 0.1, n_az, n_pol, G, 0.001, 20.0, 0.03, 2.0, Ts,
                                    name=f"g{j}"))
    for prec in (0, 1):
        bs = driver.BatchSolver(probs, prec=prec)
        bs.reset()
        bs.step(2)
        for p, sb in zip(probs, bs.solvers):
            s = driver.Solver(p, prec=prec)
            s.reset()
            s.step(2)
            mb, ms = sb.moments(), s.moments()
            for k in ("E", "F", "f", "bnd"):
                assert np.array_equal(mb[k], ms[k]), (p.name, k)


def test_batch_polar_bound_eight(lcmod):
    """Members with 8 and 5 polar angles share the polar-bound-8 launches;
    batch equals the single-problem runs bit for bit."""
    lc, driver = lcmod
    probs = []
    for j, (nx, ny, n_pol, G) in enumerate([(10, 8, 8, 6), (8, 9, 5, 3), (12, 6, 2, 4)]):
        rng = np.random.default_rng(400 + j)
        Ts = [rng.uniform(0.01, 1.0, nx * ny) for _ in range(2)]
        probs.append(W.make_problem(nx, ny, nx * 0.1, ny * 0.1, 8, n_pol, G, 0.001, 20.0, 0.03, 2.0, Ts,
                                    name=f"p{j}"))
    for prec in (0, 1):
        bs = driver.BatchSolver(probs, prec=prec)
        bs.reset()
        bs.step(2)
        for p, sb in zip(probs, bs.solvers):
            s = driver.Solver(p, prec=prec)
            s.reset()
            s.step(2)
            mb, ms = sb.moments(), s.moments()
            for k in ("E", "F", "f", "bnd"):
                assert np.array_equal(mb[k], ms[k]), (p.name, k)
            assert np.array_equal(sb.state_canonical(), s.state_canonical())
