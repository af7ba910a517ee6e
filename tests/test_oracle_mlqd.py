"""CPU pins of the Fleck-Cummings material and of one time step of the
multilevel method (oracle/material.py, oracle/mlqd.py).

* group Planck functions: the groups of a spectrum [0, inf) sum to
  a_R c T^4 / 4 pi (closed form); the Rayleigh-Jeans end of the integral
  against its Taylor series; an independent series/tail evaluation;
* opacity: its two temperature limits;
* the MLQD step: radiative equilibrium is kept exactly, energy is conserved
  at convergence, the grey solution equals the sum of the group solutions
  at convergence, and the converged temperature satisfies the energy
  balance with the averages of its own opacities."""
import math
import warnings

import numpy as np
import pytest

import workloads as W
from oracle import loqd, material, mlqd, rays, sweep

C, A_R = W.C_LIGHT, W.A_RAD


def test_open_groups_sum_to_the_total():
    T = np.array([0.001, 0.01, 0.3, 1.0, 3.0])
    edges = W.open_group_edges(9, 0.05, 40.0)
    B = material.group_planck(edges, T, A_R, C)
    total = A_R * C * T ** 4 / (4 * math.pi)
    assert np.allclose(B.sum(0), total, rtol=1e-13)
    assert np.all(B >= 0)


def test_planck_integral_small_argument():
    # x^3/(e^x - 1) = x^2 - x^3/2 + x^4/12 - x^6/720 + x^8/30240 - ...
    for x in (1e-3, 1e-2, 0.1):
        series = x ** 3 / 3 - x ** 4 / 8 + x ** 5 / 60 - x ** 7 / 5040 + x ** 9 / 272160
        assert math.isclose(material.planck_integral(0.0, x), series, rel_tol=1e-12)
    assert math.isclose(material.planck_integral(0.0, math.inf), math.pi ** 4 / 15, rel_tol=1e-13)


def test_group_planck_against_series_and_tails():
    """The quadrature against the Bernoulli series / exponential tails
    that generate the workloads' inputs (two independent evaluations)."""
    T = np.array([0.002, 0.05, 0.7, 2.0])
    for edges in (W.group_edges(12, 0.001, 30.0), W.open_group_edges(17, 0.3, 30.0)):
        a = material.group_planck(edges, T, A_R, C)
        b = W.group_planck(edges, T)
        scale = np.maximum(b, 1e-300)
        big = b > 1e-200 * b.max(0)[None, :]
        assert np.max(np.abs(a - b)[big] / scale[big]) <= 1e-11


def test_fc_opacity_limits():
    nu = np.array([0.1, 1.0, 10.0])
    cold = material.fc_opacity(nu, np.array([1e-6]))[:, 0]
    assert np.allclose(cold, 27.0 / nu ** 3, rtol=1e-15)
    hot = material.fc_opacity(nu, np.array([1e6]))[:, 0]
    assert np.allclose(hot, 27.0 / (nu ** 2 * 1e6), rtol=1e-5)


def _small_fc(h_mat=1.5, h_moc=0.3, n_az=8, n_pol=2, G=4):
    return W.fc_mlqd(h_mat, h_moc, n_az, n_pol, G, nu_lo=0.3, nu_hi=30.0)


def _start(p):
    g = rays.build(p.nx, p.ny, p.lx, p.ly, p.phi, p.h_moc)
    st = sweep.initial_state(g, p.n_pol, p.state0)
    E0, F0 = mlqd.initial_low_order(p, C)
    return g, st, np.full(p.cells, p.T0), E0, F0


def test_mlqd_keeps_radiative_equilibrium():
    """Uniform T, the intensity of every direction and group at the Planck
    function of T inside and entering through every face: one step changes
    nothing."""
    p = _small_fc()
    Teq = 0.35
    B = material.group_planck(p.edges, np.array([Teq]), A_R, C)[:, 0]
    nb = 2 * (p.nx + p.ny)
    p.I_in = np.broadcast_to(B[None, None, :], (nb, len(p.omega), p.G)).copy()
    p.state0 = np.repeat(B[:, None], p.cells, axis=1)
    g, st, _, _, F0 = _start(p)
    E0 = np.repeat((4 * math.pi * B / C)[:, None], p.cells, axis=1)
    T0 = np.full(p.cells, Teq)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        r = mlqd.outer_step(g, p, st, T0, E0, F0, C, A_R, eps=1e-12)
    assert r["outer"] <= 2
    assert np.allclose(r["T"], Teq, rtol=1e-12)
    assert np.allclose(r["E_cell"], E0, rtol=1e-11)
    assert np.allclose(r["E_face"], 4 * math.pi * B[:, None] / C, rtol=1e-11)
    assert np.max(np.abs(r["F_face"])) <= 1e-11 * C * E0.max()
    assert np.allclose(r["state"], sweep.initial_state(g, p.n_pol, p.state0), rtol=1e-12)


@pytest.fixture(scope="module")
def fc_step():
    p = _small_fc()
    g, st, T0, E0, F0 = _start(p)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        r1 = mlqd.outer_step(g, p, st, T0, E0, F0, C, A_R, eps=1e-11)
        r2 = mlqd.outer_step(g, p, r1["state"], r1["T"], r1["E_cell"], r1["F_face"], C, A_R, eps=1e-11)
    return p, (T0, E0, F0), r1, r2


def _boundary_inflow(p, F_face):
    nx, ny = p.nx, p.ny
    hx, hy = p.lx / nx, p.ly / ny
    nint = loqd.n_interior(nx, ny)
    sgn = np.concatenate([-np.ones(ny), np.ones(ny), -np.ones(nx), np.ones(nx)])
    lens = np.concatenate([np.full(ny, hy), np.full(ny, hy), np.full(nx, hx), np.full(nx, hx)])
    return -(p.c_dt / C) * np.sum(sgn * F_face.sum(0)[nint:] * lens)


def test_mlqd_step_conserves_energy(fc_step):
    p, (T0, E0, F0), r1, r2 = fc_step
    hx, hy = p.lx / p.nx, p.ly / p.ny
    for (Tp, Ep), r in (((T0, E0), r1), ((r1["T"], r1["E_cell"]), r2)):
        assert r["changes"][0] <= 1e-11 and r["changes"][1] <= 1e-11
        gained = np.sum(p.c_v * (r["T"] - Tp) + (r["E_cell"] - Ep).sum(0)) * hx * hy
        inflow = _boundary_inflow(p, r["F_face"])
        assert inflow > 0
        assert math.isclose(gained, inflow, rel_tol=1e-8)
    assert r2["T"].max() > r1["T"].max() > 10 * p.T0      # the wave has come in


def test_mlqd_grey_is_the_sum_of_groups_at_convergence(fc_step):
    p, _, r1, r2 = fc_step
    for r in (r1, r2):
        summed = r["E_cell"].sum(0)
        assert np.max(np.abs(summed - r["E_grey"])) <= 1e-9 * np.max(summed)


def test_mlqd_temperature_satisfies_its_energy_balance(fc_step):
    """c_v (T - T^{n-1})/dt = sum_g (c kappa_g(T) E_g - 4 pi kappa_g(T) B_g(T))
    with the converged multigroup E_g (the multigroup form of eq. (6))."""
    p, (T0, _, _), r1, r2 = fc_step
    for Tp, r in ((T0, r1), (r1["T"], r2)):
        T = r["T"]
        kap = material.fc_opacity(p.nu, T)
        B = material.group_planck(p.edges, T, A_R, C)
        rhs = (C * kap * r["E_cell"] - 4 * math.pi * kap * B).sum(0)
        lhs = p.c_v * (T - Tp) / (p.c_dt / C)
        scale = np.max((4 * math.pi * kap * B).sum(0))
        assert np.max(np.abs(lhs - rhs)) <= 1e-8 * scale


def _small_step(monkeypatch=None, max_outer=60, max_inner=1000):
    p = _small_fc()
    g, st, T0, E0, F0 = _start(p)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        r = mlqd.outer_step(g, p, st, T0, E0, F0, C, A_R, eps=1e-11, max_outer=max_outer, max_inner=max_inner)
    return p, (T0, E0), r


def _defects(p, prev, r):
    T0, E0 = prev
    hx, hy = p.lx / p.nx, p.ly / p.ny
    gained = np.sum(p.c_v * (r["T"] - T0) + (r["E_cell"] - E0).sum(0)) * hx * hy
    inflow = _boundary_inflow(p, r["F_face"])
    kap = material.fc_opacity(p.nu, r["T"])
    B = material.group_planck(p.edges, r["T"], A_R, C)
    rhs = (C * kap * r["E_cell"] - 4 * math.pi * kap * B).sum(0)
    lhs = p.c_v * (r["T"] - T0) / (p.c_dt / C)
    meb = np.max(np.abs(lhs - rhs)) / np.max((4 * math.pi * kap * B).sum(0))
    return abs(gained - inflow) / abs(inflow), meb


def test_planted_mistakes_in_the_step_are_caught(monkeypatch):
    """The pins of the step fail for plausible mistakes in its composition:
    the grey problem given the current temperature instead of T^{n-1}, and
    a multigroup solve that sees a slightly different opacity than the grey
    coefficients."""
    p, prev, r = _small_step()
    good = _defects(p, prev, r)
    assert good[0] <= 1e-8 and good[1] <= 1e-8
    real_low = mlqd.low_order
    monkeypatch.setattr(mlqd, "low_order", lambda prob, T_start, T_prev, *a, **k: real_low(prob, T_start, T_start,
                                                                                          *a, **k))
    p, prev, r = _small_step(max_outer=8, max_inner=60)
    assert max(_defects(p, prev, r)) > 1e-6
    monkeypatch.setattr(mlqd, "low_order", real_low)
    real_solve = loqd.solve
    monkeypatch.setattr(loqd, "solve", lambda nx, ny, lx, ly, c, c_dt, kappa, *a: real_solve(nx, ny, lx, ly, c, c_dt,
                                                                                          kappa * (1 + 1e-6), *a))
    p, prev, r = _small_step(max_outer=20, max_inner=200)
    assert _defects(p, prev, r)[1] > 1e-8
