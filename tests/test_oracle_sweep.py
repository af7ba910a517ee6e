"""Pins for the oracle's sweep (paper eq. (10)-(13)): closed-form solutions in
a uniform absorber, the exact segment-average weight alpha, the integrated
segment balance, independent ODE integration on tiny grids, linearity, and the
backward-Euler recurrence in an infinite uniform medium."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import workloads as W
from oracle import moments, rays, solve, sweep


def _uniform_problem(n=6, n_az=8, n_pol=2, G=3, kappa=(0.3, 2.0, 40.0), B=(1.0, 0.5, 2.0),
                     c_dt=3.0, h_moc=0.15, L=2.0):
    phi, mu, om = W.product_quadrature(n_az, n_pol)
    cells = n * n
    kap = np.repeat(np.array(kappa)[:, None], cells, 1)
    Bg = np.repeat(np.array(B)[:, None], cells, 1)
    g = rays.build(n, n, L, L, phi, h_moc)
    return phi, mu, om, kap, Bg, g


def test_alpha_matches_high_precision():
    import mpmath as mp
    mp.mp.dps = 50
    taus = np.concatenate([np.geomspace(1e-9, 1e3, 300), [0.0999999, 0.1, 0.1000001]])
    got = sweep.alpha_of_tau(taus)
    for t, a in zip(taus, got):
        t_ = mp.mpf(t)
        ref = 1 / t_ - mp.exp(-t_) / (1 - mp.exp(-t_))
        # the closed form cancels by a factor ~2/tau: <= ~20 ulp at tau >= 0.1
        assert abs(a - float(ref)) <= 5e-15 * float(ref), (t, a, ref)
    assert sweep.alpha_of_tau(np.array([0.0]))[0] == 0.5


def test_alpha_gives_exact_segment_average():
    # alpha I_in + (1 - alpha) I_out equals the mean of the exact solution of
    # dI/ds + kt I = Q over the segment (constant source)
    from scipy.integrate import quad
    for kt, Q, I0, L in ((0.7, 2.0, 5.0, 0.3), (20.0, 1.0, 0.0, 0.05), (1e-3, 3.0, 1.0, 0.2)):
        S = Q / kt
        exact = lambda s: I0 * math.exp(-kt * s) - S * math.expm1(-kt * s)
        mean = quad(exact, 0, L, epsabs=0, epsrel=1e-13)[0] / L
        I_out, I_bar = sweep.segment_step(np.array(I0), np.array(kt), np.array(Q), np.array(L), 1.0)
        assert abs(I_out - exact(L)) <= 1e-14 * max(abs(exact(L)), 1)
        assert abs(I_bar - mean) <= 1e-13 * abs(mean)


def test_segment_balance():
    # integrating the ODE over a segment: I_in - I_out = tau (I_bar - Q/kt)
    rng = np.random.default_rng(5)
    n = 2000
    I = rng.uniform(0, 3, n); kt = 10 ** rng.uniform(-4, 4, n); Q = rng.uniform(0, 5, n) * kt
    L = rng.uniform(1e-4, 0.3, n); sz = rng.uniform(0.2, 1.0, n)
    I_out, I_bar = sweep.segment_step(I, kt, Q, L, sz)
    tau = kt * L / sz
    lhs = I - I_out
    rhs = tau * (I_bar - Q / kt)
    assert np.all(np.abs(lhs - rhs) <= 1e-12 * (np.abs(I) + np.abs(I_out) + tau * Q / kt))
    assert np.all(I_bar >= np.minimum(I, I_out) - 1e-15)
    assert np.all(I_bar <= np.maximum(I, I_out) + 1e-15)


def test_uniform_absorber_exit_and_segment_averages():
    """kappa, B uniform and previous intensity = B give S = B on every
    segment: I_exit = B + (I_in - B) exp(-kt chord / sin zeta) and each
    segment average is B + (I_s - B)(1 - e^-tau)/tau."""
    phi, mu, om, kap, Bg, g = _uniform_problem()
    c_dt = 3.0
    G = kap.shape[0]
    M = len(om)
    nb = 4 * 6
    rng = np.random.default_rng(1)
    I_in = rng.uniform(0, 4, (nb, M, G))
    st0 = sweep.initial_state(g, len(mu), Bg)
    st, exits = sweep.sweep(g, mu, kap, Bg, c_dt, st0, I_in)
    kt = kap[:, 0] + 1 / c_dt
    sz = np.sqrt(1 - mu ** 2)
    for a, pr in enumerate(g.pairs):
        for d in (0, 1):
            fin = pr.entry_face if d == 0 else pr.exit_face
            for k in range(pr.K):
                L = pr.lens[k].sum()
                for p in range(len(mu)):
                    m = sweep.direction_index(a, d, p, g.n_az, len(mu))
                    ref = Bg[:, 0] + (I_in[fin[k], m] - Bg[:, 0]) * np.exp(-kt * L / sz[p])
                    assert np.allclose(exits[a][d, k, p], ref, rtol=1e-14, atol=0)
                    # segment averages along the ray
                    lens = pr.lens[k] if d == 0 else pr.lens[k][::-1]
                    Is = I_in[fin[k], m].copy()
                    j0 = pr.seg_base + int(pr.nseg[:k].sum())
                    js = np.arange(j0, j0 + len(lens))
                    js = js if d == 0 else js[::-1]
                    for ln, j in zip(lens, js):
                        tau = kt * ln / sz[p]
                        ref_bar = Bg[:, 0] + (Is - Bg[:, 0]) * (-np.expm1(-tau)) / tau
                        assert np.allclose(st[j, d, p], ref_bar, rtol=1e-13, atol=0)
                        Is = Bg[:, 0] + (Is - Bg[:, 0]) * np.exp(-tau)


def _ode_segment(I0, kt, Q, L, sz):
    """Integrate dI/du = (Q - kt I)/sin(zeta) and its running integral."""
    f = lambda u, y: [(Q - kt * y[0]) / sz, y[0]]
    r = solve_ivp(f, (0.0, L), [I0, 0.0], method="DOP853", rtol=1e-12, atol=1e-14)
    return r.y[0, -1], r.y[1, -1] / L


@pytest.mark.parametrize("nx,ny", [(2, 2), (3, 2)])
def test_tiny_grid_against_ode_integration(nx, ny):
    """Every segment of every characteristic of a tiny grid with random
    cell data, previous-step intensities and boundary data, integrated
    segment by segment with an adaptive ODE solver."""
    rng = np.random.default_rng(nx * 10 + ny)
    lx, ly = 1.0, 0.8
    phi, mu, om = W.product_quadrature(4, 2)
    G = 2
    kap = rng.uniform(0.2, 6.0, (G, nx * ny))
    Bg = rng.uniform(0.1, 2.0, (G, nx * ny))
    c_dt = 0.7
    g = rays.build(nx, ny, lx, ly, phi, 0.2)
    I_in = rng.uniform(0, 3, (2 * (nx + ny), len(om), G))
    st0 = rng.uniform(0, 2, (g.n_seg, 2, len(mu), G))
    st, exits = sweep.sweep(g, mu, kap, Bg, c_dt, st0, I_in)
    sz = np.sqrt(1 - mu ** 2)
    for a, pr in enumerate(g.pairs):
        for d in (0, 1):
            fin = pr.entry_face if d == 0 else pr.exit_face
            for k in range(pr.K):
                j0 = pr.seg_base + int(pr.nseg[:k].sum())
                order = range(len(pr.cells[k])) if d == 0 else range(len(pr.cells[k]) - 1, -1, -1)
                for p in range(len(mu)):
                    m = sweep.direction_index(a, d, p, g.n_az, len(mu))
                    for gg in range(G):
                        I = I_in[fin[k], m, gg]
                        for s in order:
                            i = pr.cells[k][s]
                            kt = kap[gg, i] + 1 / c_dt
                            Q = kap[gg, i] * Bg[gg, i] + st0[j0 + s, d, p, gg] / c_dt
                            I, mean = _ode_segment(I, kt, Q, pr.lens[k][s], sz[p])
                            assert abs(st[j0 + s, d, p, gg] - mean) <= 1e-9 * abs(mean)
                        assert abs(exits[a][d, k, p, gg] - I) <= 1e-9 * abs(I)


def test_linearity_and_power_of_two_scaling():
    p = W.config(0)
    g = solve.build_grid(p)
    st0 = sweep.initial_state(g, p.n_pol, p.state0)
    st1, ex1 = sweep.sweep(g, p.mu, p.kappa[0], p.planck[0], p.c_dt, st0, p.I_in)
    # scaling every source (boundary, emission, previous step) by 2^-7
    s = 2.0 ** -7
    st2, ex2 = sweep.sweep(g, p.mu, p.kappa[0], p.planck[0] * s, p.c_dt, st0 * s, p.I_in * s)
    assert np.array_equal(st2, st1 * s)
    # superposition of two source sets
    rng = np.random.default_rng(3)
    Ia = rng.uniform(0, 1, p.I_in.shape)
    sta, _ = sweep.sweep(g, p.mu, p.kappa[0], p.planck[0], p.c_dt, st0, Ia)
    stb, _ = sweep.sweep(g, p.mu, p.kappa[0], 0 * p.planck[0], p.c_dt, 0 * st0, p.I_in)
    stab, _ = sweep.sweep(g, p.mu, p.kappa[0], p.planck[0], p.c_dt, st0, Ia + p.I_in)
    assert np.allclose(stab, sta + stb, rtol=1e-13, atol=1e-300)


def test_backward_euler_recurrence_in_uniform_medium():
    """Uniform medium with every incoming intensity set to the step's
    spatially uniform solution S^n = (kappa B + X^{n-1}/(c dt))/kt: the
    solution stays uniform and X^n = B + (X^0 - B) r^n, r = 1/(c dt kt)."""
    phi, mu, om, kap, Bg, g = _uniform_problem(G=3)
    c_dt = 1.5
    X0 = np.array([0.2, 3.0, 1.0])
    st = sweep.initial_state(g, len(mu), np.repeat(X0[:, None], 36, 1))
    kt = kap[:, 0] + 1 / c_dt
    r = 1 / (c_dt * kt)
    X = X0.copy()
    for n in range(1, 4):
        S = (kap[:, 0] * Bg[:, 0] + X / c_dt) / kt
        I_in = np.broadcast_to(S, (24, len(om), 3)).copy()
        st, exits = sweep.sweep(g, mu, kap, Bg, c_dt, st, I_in)
        X = S
        ref = Bg[:, 0] + (X0 - Bg[:, 0]) * r ** n
        assert np.allclose(X, ref, rtol=1e-14)
        assert np.allclose(st, ref[None, None, None, :], rtol=1e-13)
        E, F, f = moments.cell_moments(g, phi, mu, om, st, W.C_LIGHT)
        assert np.allclose(E, 4 * math.pi * ref[:, None] / W.C_LIGHT, rtol=1e-13)
