"""GPU: the batched form (one persistent launch per phase over many uneven
problems) against the single-problem path and against the oracle."""
import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle import rays as orays, solve as osolve
from tests import oracle_pool
from tests.parity_util import bnd_errors, bnd_worst, err_E, err_F, err_f, err_rel, sample_cells, sample_faces

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
        eb, ebc = bnd_errors(got["bnd"], ref["bnd"], floor=0.0)
        assert eb <= 1e-12 and ebc <= 1e-12


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


@pytest.mark.timeout(900)
def test_full_batched_workload_sampled(lcmod):
    """The 64-problem batched workload in float32, checked after 1 and after 3
    steps against the oracle (1e-5) on four members (the largest, the
    smallest and two at random): 16 cells each (corners, domain edges, both
    sides of moment-tile edges, random ones) and 8 boundary faces each (the
    corner faces and faces that grazing directions leave empty)."""
    lc, driver = lcmod
    steps = 3
    probs = W.batch_problems(steps=steps)
    _say("64-problem batch: building")
    bs = driver.BatchSolver(probs, prec=lc.LC_F32)
    cost = [p.cells * p.G * p.M for p in probs]
    rng = np.random.default_rng(5)
    members = [int(np.argmax(cost)), int(np.argmin(cost))]
    members += [int(i) for i in rng.choice([j for j in range(len(probs)) if j not in members], 2, replace=False)]
    samples = {q: (sample_cells(probs[q].nx, probs[q].ny, 16, q), sample_faces(probs[q], 8, q)[0]) for q in members}
    got = {}
    for n in (1, steps):
        bs.reset()
        bs.step(n)
        for q in members:
            m = bs.solvers[q].moments()
            cells, faces = samples[q]
            got[(q, n)] = dict(E=m["E"][:, cells], F=m["F"][:, :, cells], f=m["f"][:, :, cells],
                               bnd=m["bnd"][:, faces])
    del bs
    jobs, owner = [], []
    for q in members:
        cells, faces = samples[q]
        nblk = 4
        for cb, fb in zip(oracle_pool.blocks(cells, nblk), oracle_pool.blocks(faces, nblk)):
            jobs.append((("batch", q, steps), cb, fb))
            owner.append(q)
    _say(f"  oracle: {len(jobs)} blocks on {oracle_pool.workers()} processes")
    res = oracle_pool.run_blocks(jobs)
    c = W.C_LIGHT
    for q in members:
        p = probs[q]
        rs = [r for r, o in zip(res, owner) if o == q]
        for n in (1, steps):
            ref = {k: np.concatenate([r[n - 1][k] for r in rs], axis=-1) for k in ("E", "F", "f")}
            ref_b = np.concatenate([r[n - 1]["bnd"] for r in rs], axis=1)
            g = got[(q, n)]
            eE = err_E(g["E"], ref["E"])
            eF = err_F(g["F"], ref["F"], ref["E"], c)
            ef = err_f(g["f"], ref["f"], ref["E"])
            eb, ebc = bnd_errors(g["bnd"], ref_b)
            _say(f"  member {q} ({p.nx}^2 G={p.G} M={p.M}) after {n} steps: E {eE:.2e} F {eF:.2e} f {ef:.2e} "
                 f"bnd {eb:.2e} / C,f_b {ebc:.2e}; largest C difference {bnd_worst(g['bnd'], ref_b)}")
            assert eE <= 1e-5 and eF <= 1e-5 and ef <= 1e-5
            assert eb <= 1e-5 and ebc <= 1e-5


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
