"""GPU parity: the HIP library (through the C ABI) against the CPU oracle, on
the same seeded inputs.  FP64 path: 1e-12 (relative, floored metrics);
float32 path: 1e-5 in the same metrics.  Integer geometry is bit-exact."""
import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle import moments as om_, rays as orays, solve as osolve, sweep as osweep
from tests.parity_util import (FLOOR, bnd_errors, bnd_worst, err_E, err_F, err_f, err_rel, mask_of,
                               sample_cells, sample_faces)

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


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


def _custom_problem(nx=32, ny=24, lx=3.2, ly=2.4, n_az=12, mu=None, w=None, G=5, h_moc=0.04,
                    steps=2, seed=11):
    rng = np.random.default_rng(seed)
    phi, mu0, om = W.product_quadrature(n_az, 3)
    if mu is not None:
        mu = np.asarray(mu, float)
        w = np.asarray(w, float) / np.sum(w) * 2.0
        om = np.repeat(np.full(n_az, 2 * math.pi / n_az), len(mu)) * np.tile(w, n_az)
    else:
        mu = mu0
    edges = W.group_edges(G, 0.001, 20.0)
    Ts = [rng.uniform(0.01, 1.0, nx * ny) for _ in range(steps)]
    kap = [W.fc_opacity(W.group_midpoints(edges), T) for T in Ts]
    B = [W.group_planck(edges, T) for T in Ts]
    I_in = rng.uniform(0.0, 0.3, (2 * (nx + ny), len(om), G))
    s0 = W.group_planck(edges, rng.uniform(0.005, 0.5, nx * ny))
    return W.Problem(nx, ny, lx, ly, phi, mu, om, edges, h_moc, 1.7, kap, B, I_in, s0, Ts, "custom")


def _oracle_full(prob, steps=None, mode=0):
    return osolve.run(prob, steps=steps, mode=mode)


def _compare_full(lc, driver, prob, prec, tol, graph=True, check_state=True, mode=0, split=0):
    _say(f"case {prob.name}: {prob.nx}x{prob.ny} G={prob.G} M={prob.M} prec={prec} steps={prob.steps} mode={mode}"
         f" split={split}")
    ref = _oracle_full(prob, mode=mode)
    s = driver.Solver(prob, prec=prec, mode=mode, split=split)
    s.reset()
    s.step(prob.steps, graph=graph)
    got = s.moments()
    v = s.moment_views()
    assert np.array_equal(v["E"][:, 0].cpu().numpy(), got["E"])
    assert np.array_equal(v["F"].cpu().numpy(), got["F"]) and np.array_equal(v["f"].cpu().numpy(), got["f"])
    r = ref["steps"][-1]
    c = W.C_LIGHT
    eE = err_E(got["E"], r["E"])
    eF = err_F(got["F"], r["F"], r["E"], c)
    ef = err_f(got["f"], r["f"], r["E"])
    bref = r["bnd"]
    eb, ebc = bnd_errors(got["bnd"], bref, floor=0.0 if prec == 0 else FLOOR)
    msg = f"  E {eE:.2e}  F {eF:.2e}  f {ef:.2e}  bnd {eb:.2e} / C,f_b {ebc:.2e}"
    if check_state:
        st = s.state_canonical()
        assert st.shape == ref["state"].shape
        est = err_rel(st, ref["state"])
        ex_ref = np.concatenate([e.transpose(1, 0, 2, 3) for e in ref["exits"]])
        eex = err_rel(s.exits(), ex_ref)
        msg += f"  state {est:.2e}  exits {eex:.2e}"
    _say(msg)
    assert eE <= tol and eF <= tol and ef <= tol
    assert eb <= tol and ebc <= tol
    if check_state:
        assert est <= tol and eex <= tol
    return s, ref


def test_geometry_matches_oracle(lcmod):
    lc, driver = lcmod
    for prob in (W.config(0), _custom_problem(), _custom_problem(nx=7, ny=1, lx=2.1, ly=0.3, h_moc=0.05)):
        _say(f"geometry {prob.nx}x{prob.ny} n_az={prob.n_az}")
        g = orays.build(prob.nx, prob.ny, prob.lx, prob.ly, prob.phi, prob.h_moc)
        r = lc.lc_build_rays(prob.nx, prob.ny, prob.lx, prob.ly, prob.phi, prob.mu, prob.omega, prob.h_moc)
        ro, so, ce, ln, wd, fc = lc.lc_rays_export(r)
        ray_off, seg_off, cell, length, w = g.flat()
        assert np.array_equal(ro, ray_off)
        assert np.array_equal(so, seg_off)
        assert np.array_equal(ce, cell)
        assert np.allclose(ln, length, rtol=1e-13, atol=1e-15 * prob.lx)
        assert np.allclose(wd, w, rtol=1e-15)
        faces = np.concatenate([np.stack([p.entry_face, p.exit_face], 1) for p in g.pairs])
        assert np.array_equal(fc, faces)


@pytest.mark.parametrize("shape", [(16, 16, 6.0, 6.0, 0.05), (20, 12, 2.0, 1.2, 0.02), (5, 9, 1.0, 1.8, 0.07)])
def test_geometry_tube_mode_matches_oracle(lcmod, shape):
    """The paper's vertex-avoiding, width-halving construction built on the
    GPU (sorted vertex projections) against the oracle's."""
    lc, driver = lcmod
    nx, ny, lx, ly, h = shape
    phi, mu, om = W.product_quadrature(16, 2)
    _say(f"tube geometry {nx}x{ny} h_moc={h}")
    g = orays.build(nx, ny, lx, ly, phi, h, orays.TUBES)
    r = lc.lc_build_rays(nx, ny, lx, ly, phi, mu, om, h, lc.LC_RAYS_TUBES)
    ro, so, ce, ln, wd, fc = lc.lc_rays_export(r)
    ray_off, seg_off, cell, length, w = g.flat()
    assert np.array_equal(ro, ray_off)
    assert np.array_equal(so, seg_off)
    assert np.array_equal(ce, cell)
    assert np.allclose(ln, length, rtol=1e-12, atol=1e-14 * lx)
    assert np.allclose(wd, w, rtol=1e-13, atol=0)
    # traced area per cell and direction equals the cell area (exact construction)
    area = (lx / nx) * (ly / ny)
    for a in range(len(ro) - 1):
        traced = np.zeros(nx * ny)
        for k in range(ro[a], ro[a + 1]):
            np.add.at(traced, ce[so[k]:so[k + 1]], ln[so[k]:so[k + 1]] * wd[k])
        assert np.allclose(traced, area, rtol=1e-11)


@pytest.mark.parametrize("prec", [0, 1])
def test_tube_mode_full_parity(lcmod, prec):
    lc, driver = lcmod
    prob = _custom_problem(nx=12, ny=10, lx=1.2, ly=1.0, n_az=8, G=3, h_moc=0.04, steps=2)
    _compare_full(lc, driver, prob, prec, TOL64 if prec == 0 else TOL32, mode=lc.LC_RAYS_TUBES)


def test_config0_fp64(lcmod):
    lc, driver = lcmod
    _compare_full(lc, driver, W.config(0), lc.LC_F64, TOL64)


def test_config0_fp32(lcmod):
    lc, driver = lcmod
    _compare_full(lc, driver, W.config(0), lc.LC_F32, TOL32)


@pytest.mark.parametrize("prec", [0, 1])
def test_multitile_ragged_two_steps(lcmod, prec):
    lc, driver = lcmod
    tol = TOL64 if prec == 0 else TOL32
    _compare_full(lc, driver, _custom_problem(), prec, tol)


def test_asymmetric_polar_set_and_eager_path(lcmod):
    lc, driver = lcmod
    prob = _custom_problem(mu=[-0.6, 0.2, 0.7, 0.85], w=[0.3, 0.4, 0.2, 0.1], n_az=8, G=3, steps=2)
    _compare_full(lc, driver, prob, lc.LC_F64, TOL64, graph=False)


@pytest.mark.parametrize("shape", [(1, 1, 1.0, 1.0), (1, 7, 0.2, 1.4), (9, 2, 1.8, 0.4)])
def test_degenerate_grids(lcmod, shape):
    lc, driver = lcmod
    nx, ny, lx, ly = shape
    prob = _custom_problem(nx=nx, ny=ny, lx=lx, ly=ly, n_az=4, G=1, h_moc=0.03, steps=1)
    _compare_full(lc, driver, prob, lc.LC_F64, TOL64)


def test_single_polar_angle(lcmod):
    lc, driver = lcmod
    prob = _custom_problem(mu=[0.0], w=[1.0], n_az=8, G=2, steps=1)
    _compare_full(lc, driver, prob, lc.LC_F64, TOL64)


def test_graph_equals_eager_and_is_deterministic(lcmod):
    lc, driver = lcmod
    prob = _custom_problem(steps=3)
    out = []
    for graph in (True, False, True):
        s = driver.Solver(prob, prec=lc.LC_F32)
        s.reset()
        s.step(3, graph=graph)
        out.append((s.moments(), s.state_canonical()))
    for m, st in out[1:]:
        for k in ("E", "F", "f", "bnd"):
            assert np.array_equal(m[k], out[0][0][k])
        assert np.array_equal(st, out[0][1])


@pytest.mark.parametrize("prec,mode,h_moc,n_pol", [(1, 0, 0.04, 3), (1, 1, 0.04, 3), (0, 0, 0.015, 3),
                                                  (1, 0, 0.04, 4), (0, 0, 0.04, 2)])
def test_tuning_settings_give_identical_results(lcmod, prec, mode, h_moc, n_pol):
    """Every launch tuning gives bit-identical moments, boundary factors and
    state.  Tube grids and fine spacing make (cell, pair) lists longer than the
    moment kernel's pipelined slots, so its tail loop is covered too.  Three
    polar angles run the sweep with per-angle branches, 2 and 4 (symmetric
    Gauss-Legendre sets) the branch-free form; 16-step chunks exist in
    float32 only."""
    lc, driver = lcmod
    mu = w = None
    if n_pol != 3:
        mu, w = np.polynomial.legendre.leggauss(n_pol)
    prob = _custom_problem(h_moc=h_moc, steps=2, mu=mu, w=w)
    s = driver.Solver(prob, prec=prec, mode=mode)
    ro, so, ce, _, _, _ = lc.lc_rays_export(s.rays)
    longest = max(int(np.bincount(ce[so[ro[a]]:so[ro[a + 1]]]).max()) for a in range(len(ro) - 1))
    _say(f"  longest (cell, pair) list: {longest}")
    if mode == 1 or h_moc < 0.02:
        assert longest > 4                      # the tail loop runs
    out = []
    settings = [(2, 3), (1, 1), (4, 2), (2, 4), (1, 3), (8, 2)] + ([(16, 1), (16, 3)] if prec == 1 else [])
    for u, e in settings:
        _say(f"case tuning prec={prec} mode={mode} h_moc={h_moc}: unroll {u} entries {e}")
        lc.lc_plan_set_tuning(s.plan, u, e)
        s.reset()
        s.step(2, graph=False)
        out.append((s.moments(), s.state_canonical()))
    for m, st in out[1:]:
        for k in ("E", "F", "f", "bnd"):
            assert np.array_equal(m[k], out[0][0][k])
        assert np.array_equal(st, out[0][1])


def test_sweep_residency_gives_identical_results(lcmod):
    """The residency cap of the sweep changes occupancy only."""
    lc, driver = lcmod
    prob = _custom_problem(G=7, steps=2)
    outs = []
    for capped in (1, 0):
        s = driver.Solver(prob, prec=lc.LC_F32)
        lc.lc_plan_set_sweep_residency(s.plan, capped)
        s.reset()
        s.step(2)
        m = s.moments()
        outs.append((s.state_canonical(), s.exits(), m["E"], m["F"], m["f"], m["bnd"]))
        assert lc._lib.lc_plan_set_sweep_residency(s.plan.handle, 2) == lc.LC_ERR_ARG
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("G,prec", [(66, 0), (100, 0), (100, 1), (260, 1)])
def test_many_groups_span_three_bundles(lcmod, G, prec):
    """G > 64: a characteristic's groups can span three 64-lane bundles (the
    moment gather then looks up each lane's bundle).  G = 260 also exceeds
    the block size of the float32 prologue's group maxima."""
    lc, driver = lcmod
    prob = _custom_problem(nx=9, ny=7, lx=0.9, ly=0.7, n_az=8, G=G, h_moc=0.04, steps=1)
    _compare_full(lc, driver, prob, prec, TOL64 if prec == 0 else TOL32)


@pytest.mark.parametrize("n_pol,prec", [(8, 0), (8, 1), (5, 1), (6, 0), (6, 1)])
def test_polar_counts_above_four(lcmod, n_pol, prec):
    """P = 8 (whole-vector state accesses of 8 values), P = 5 (element
    accesses) and P = 6 (pairs of values per access, the polar count of the
    512^2 workload) against the oracle."""
    lc, driver = lcmod
    mu, w = np.polynomial.legendre.leggauss(n_pol)
    prob = _custom_problem(nx=10, ny=8, lx=1.0, ly=0.8, n_az=8, mu=mu, w=w, G=6, h_moc=0.04, steps=2)
    _compare_full(lc, driver, prob, prec, TOL64 if prec == 0 else TOL32)


@pytest.mark.parametrize("cfg,prec,split", [(1, 0, 0), (2, 0, 0), (2, 1, 0), (1, 1, 256), (1, 0, 32)])
def test_full_size_sampled_cells(lcmod, cfg, prec, split):
    """Full-size workloads: 64 sampled cells (the corners, every domain edge,
    both sides of moment-tile edges, the rest at random) and 16 boundary
    faces (the corner faces and faces that grazing directions leave empty)
    against the oracle, which sweeps only the characteristics reaching those
    samples (exact, since characteristics evolve independently under
    prescribed material data).  The 128^2 problem also runs as the split
    sweep (chunks of 256 steps are what the tuner picks for it in float32)."""
    lc, driver = lcmod
    prob = W.config(cfg)
    tol = TOL64 if prec == 0 else TOL32
    _say(f"config {cfg} prec {prec} split {split}: GPU run")
    s = driver.Solver(prob, prec=prec, split=split)
    s.reset()
    s.step(prob.steps)
    got = s.moments()
    cells = sample_cells(prob.nx, prob.ny, 64, cfg)
    faces, _ = sample_faces(prob, 16, cfg)
    _say(f"  oracle on {len(cells)} cells and {len(faces)} boundary faces")
    g = orays.build(prob.nx, prob.ny, prob.lx, prob.ly, prob.phi, prob.h_moc, only_cells=cells,
                    only_faces=faces)
    ref = osolve.run_sampled(prob, g, cells, faces=faces)["steps"][-1]
    c = W.C_LIGHT
    eE = err_E(got["E"][:, cells], ref["E"])
    eF = err_F(got["F"][:, :, cells], ref["F"], ref["E"], c)
    ef = err_f(got["f"][:, :, cells], ref["f"], ref["E"])
    eb, ebc = bnd_errors(got["bnd"][:, faces], ref["bnd"], floor=0.0 if prec == 0 else FLOOR)
    _say(f"  E {eE:.2e}  F {eF:.2e}  f {ef:.2e}  bnd {eb:.2e} / C,f_b {ebc:.2e}; largest C difference "
         f"(g, face, C, C_ref, Phi+_ref, group max Phi+_ref) = {bnd_worst(got['bnd'][:, faces], ref['bnd'])}")
    assert eE <= tol and eF <= tol and ef <= tol
    assert eb <= tol and ebc <= tol
    # realisability over the whole field, where the group's intensity has not
    # underflowed (the error metrics use the same floor)
    E, F, f = got["E"], got["F"], got["f"]
    assert np.all(E >= 0)
    m = mask_of(E)
    Fn = np.hypot(F[:, 0], F[:, 1])
    assert np.all(Fn[m] <= c * E[m] * (1 + 1e-6))
    assert np.allclose((f[:, 0] + f[:, 2] + f[:, 3])[m], 1.0, atol=1e-6 if prec else 1e-12)


@pytest.mark.parametrize("prec", [0, 1])
def test_grazing_boundary_faces_worked_case(lcmod, prec):
    """The 3 x 2 grid on which the empty-face stand-in was worked by hand
    (one polar angle, azimuths 0.15 and 1.2 rad, spacing 0.6): GPU against
    the oracle, element by element."""
    import json
    import os
    lc, driver = lcmod
    from tests.test_oracle_sampled import GOLDEN, _grazing_problem
    prob = _grazing_problem(json.load(open(GOLDEN)))
    _compare_full(lc, driver, prob, prec, TOL64 if prec == 0 else TOL32)
