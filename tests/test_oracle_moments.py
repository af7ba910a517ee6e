"""Pins for the oracle's moments (paper eq. (7), (14)-(16)) and boundary
factors: single-direction indicators, isotropic equilibrium with the
closed-form half-range factor, mirror symmetry, realisability, and agreement
with the literal eq. (15) for the paper's own characteristic grid."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import moments, rays, solve, sweep


def _omega(phi, mu, a, p):
    sz = math.sqrt(1 - mu[p] ** 2)
    return np.array([sz * math.cos(phi[a]), sz * math.sin(phi[a]), mu[p]])


def test_single_direction_indicator_cells():
    nx, ny, L = 5, 4, 2.0
    phi, mu, om = W.product_quadrature(8, 2)
    g = rays.build(nx, ny, L, 1.6, phi, 0.1)
    n_pol = len(mu)
    for a in range(len(g.pairs)):
        for d in (0, 1):
            for p in range(n_pol):
                st = np.zeros((g.n_seg, 2, n_pol, 1))
                pr = g.pairs[a]
                st[pr.seg_base:pr.seg_base + int(pr.nseg.sum()), d, p, 0] = 1.0
                E, F, f = moments.cell_moments(g, phi, mu, om, st, 1.0)
                az = a + d * (len(phi) // 2)
                m = az * n_pol + p
                Om = _omega(phi, mu, az, p)
                assert np.allclose(E, om[m], rtol=1e-14)
                assert np.allclose(F[0, 0], om[m] * Om[0], rtol=1e-13, atol=1e-15)
                assert np.allclose(F[0, 1], om[m] * Om[1], rtol=1e-13, atol=1e-15)
                ref = [Om[0] * Om[0], Om[0] * Om[1], Om[1] * Om[1], Om[2] * Om[2]]
                for q in range(4):
                    assert np.allclose(f[0, q], ref[q], rtol=1e-13, atol=1e-15)


def test_single_direction_indicator_boundary():
    nx, ny, L = 4, 3, 1.0
    phi, mu, om = W.product_quadrature(8, 2)
    g = rays.build(nx, ny, L, 0.75, phi, 0.05)
    n_pol, M = len(mu), len(om)
    nb = 2 * (nx + ny)
    normals = W.boundary_faces(nx, ny)
    for a in range(len(g.pairs)):
        for d in (0, 1):
            for p in range(n_pol):
                az = a + d * (len(phi) // 2)
                m = az * n_pol + p
                Om = _omega(phi, mu, az, p)
                exits = [np.zeros((2, pr.K, n_pol, 1)) for pr in g.pairs]
                exits[a][d, :, p, 0] = 1.0
                I_in = np.zeros((nb, M, 1))
                I_in[:, m, 0] = 2.0           # read only where m is incoming
                bnd = moments.boundary_factors(g, phi, mu, om, exits, I_in)[0]
                for b in range(nb):
                    odn = Om[0] * normals[b, 0] + Om[1] * normals[b, 1]
                    if odn > 0:
                        assert np.allclose(bnd[b, :4], [om[m], om[m] * odn, 0, 0], rtol=1e-13, atol=1e-16)
                        assert abs(bnd[b, 4] - odn) < 1e-13
                        I = 1.0
                    else:
                        assert np.allclose(bnd[b, :4], [0, 0, 2 * om[m], 2 * om[m] * -odn], rtol=1e-13, atol=1e-16)
                        I = 2.0
                    ref = [Om[0] * Om[0], Om[0] * Om[1], Om[1] * Om[1]]
                    assert np.allclose(bnd[b, 5:], ref, rtol=1e-12, atol=1e-15)


def _linear_field_case(unweighted=False):
    nx, ny, lx, ly = 4, 3, 1.0, 0.75
    phi, mu, om = W.product_quadrature(8, 2)
    g = rays.build(nx, ny, lx, ly, phi, 0.05, rays.TUBES)
    if unweighted:                                       # planted mistake: plain mean of the exits
        for pr in g.pairs:
            pr.w = np.ones_like(pr.w)
    return nx, ny, lx, ly, phi, mu, om, g


def _linear_field_check(nx, ny, lx, ly, phi, mu, om, g):
    """Largest relative deviation of Phi+, J+ and C from the closed form."""
    n_pol, M, half = len(mu), len(om), len(phi) // 2
    nb = 2 * (nx + ny)
    normals = W.boundary_faces(nx, ny)
    centres = rays.face_centres(nx, ny, lx, ly)
    V0 = 10.0
    slope = lambda m: 0.5 + 0.25 * m                     # a different field for every direction
    exits = []
    for a, pr in enumerate(g.pairs):
        e = np.zeros((2, pr.K, n_pol, 1))
        for d in (0, 1):
            for p in range(n_pol):
                e[d, :, p, 0] = V0 + slope((a + d * half) * n_pol + p) * pr.v
        exits.append(e)
    bnd = moments.boundary_factors(g, phi, mu, om, exits, np.zeros((nb, M, 1)))[0]
    worst = 0.0
    for b in range(nb):
        Pp = Jp = 0.0
        for a, pr in enumerate(g.pairs):
            vb = -centres[b, 0] * pr.s + centres[b, 1] * pr.c
            for d in (0, 1):
                for p in range(n_pol):
                    m = (a + d * half) * n_pol + p
                    Om = _omega(phi, mu, a + d * half, p)
                    odn = Om[0] * normals[b, 0] + Om[1] * normals[b, 1]
                    if odn > 0:
                        I = V0 + slope(m) * vb
                        Pp += om[m] * I
                        Jp += om[m] * odn * I
        assert bnd[b, 2] == 0.0 and bnd[b, 3] == 0.0
        worst = max(worst, abs(bnd[b, 0] / Pp - 1), abs(bnd[b, 1] / Jp - 1), abs(bnd[b, 4] / (Jp / Pp) - 1))
    return worst


def test_boundary_exit_means_of_a_linear_field_on_the_papers_grid():
    """On the vertex-avoiding grid the characteristics leaving through a
    boundary face tile the face's projection exactly, so an exit intensity
    linear in the characteristic coordinate v = -x sin(phi) + y cos(phi) has
    the width-weighted mean of its value at the face centre: Phi+, J+ and
    C = J+/Phi+ then follow in closed form for a mix of directions whose
    fields differ (reading R4/R5: width-weighted mean within a direction,
    then the sum over directions).  A plain mean of the exits fails it."""
    assert _linear_field_check(*_linear_field_case()) < 1e-12
    assert _linear_field_check(*_linear_field_case(unweighted=True)) > 1e-6


def _c_iso(n_az, mu_w):
    """Half-range factor for an isotropic intensity, closed form for the
    product set: (sum_p w_p sin zeta_p / sum_p w_p) x (mean of |cos| over the
    outgoing half of the azimuths), with the azimuth sum evaluated as a
    finite trigonometric sum: sum_{a<n/2} sin((a+1/2) 2 pi/n) = 1/sin(pi/n)."""
    mu, w = mu_w
    polar = (w * np.sqrt(1 - mu ** 2)).sum() / w.sum()
    azim = (1.0 / math.sin(math.pi / n_az)) / (n_az / 2)
    return polar * azim


@pytest.mark.parametrize("n_az,n_pol", [(16, 2), (32, 4), (12, 6)])
def test_isotropic_equilibrium(n_az, n_pol):
    n, L = 6, 1.8
    phi, mu, om = W.product_quadrature(n_az, n_pol)
    G = 2
    Bv = np.array([0.7, 2.5])
    kap = np.repeat(np.array([0.4, 30.0])[:, None], n * n, 1)
    Bg = np.repeat(Bv[:, None], n * n, 1)
    g = rays.build(n, n, L, L, phi, 0.08)
    I_in = np.broadcast_to(Bv, (4 * n, len(om), G)).copy()
    st0 = sweep.initial_state(g, n_pol, Bg)
    st, exits = sweep.sweep(g, mu, kap, Bg, 3.0, st0, I_in)
    assert np.allclose(st, Bv[None, None, None, :], rtol=1e-14)
    c = W.C_LIGHT
    E, F, f = moments.cell_moments(g, phi, mu, om, st, c)
    assert np.allclose(E, 4 * math.pi * Bv[:, None] / c, rtol=1e-13)
    assert np.all(np.abs(F) <= 1e-13 * c * E[:, None, :])
    assert np.allclose(f[:, [0, 2, 3]], 1 / 3, rtol=1e-13)
    assert np.all(np.abs(f[:, 1]) < 1e-14)
    bnd = moments.boundary_factors(g, phi, mu, om, exits, I_in)
    mu_w = np.polynomial.legendre.leggauss(n_pol)
    ci = _c_iso(n_az, mu_w)
    assert np.allclose(bnd[:, :, 4], ci, rtol=1e-13)
    assert np.allclose(bnd[:, :, 0], 2 * math.pi * Bv[:, None], rtol=1e-13)
    assert np.allclose(bnd[:, :, 5], 1 / 3, rtol=1e-13)
    assert np.allclose(bnd[:, :, 7], 1 / 3, rtol=1e-13)


def test_c_iso_matches_quoted_values():
    # half-range factors of the four quadratures used by the workloads
    for (n_az, n_pol), ref in (((16, 2), 0.523152925072), ((32, 2), 0.520633800745),
                               ((32, 4), 0.503826907973), ((48, 6), 0.501334315012)):
        assert abs(_c_iso(n_az, np.polynomial.legendre.leggauss(n_pol)) - ref) < 1e-11


def test_mirror_symmetry():
    """A problem symmetric under y -> L - y has E, F_x, f_xx, f_yy, f_zz
    symmetric and F_y, f_xy antisymmetric, and bottom/top boundary factors
    that mirror each other."""
    n, L = 8, 2.0
    phi, mu, om = W.product_quadrature(16, 2)
    edges = W.group_edges(3, 0.01, 5.0)
    rng = np.random.default_rng(7)
    T = rng.uniform(0.05, 1.0, (n, n))
    T = 0.5 * (T + T[::-1, :])                     # T(x, y) = T(x, L - y)
    T = T.ravel()
    kap = W.fc_opacity(W.group_midpoints(edges), T)
    Bg = W.group_planck(edges, T)
    I_in = W.inflow_left_planck(n, n, phi, mu, edges, 1.0)
    g = rays.build(n, n, L, L, phi, L / n / 3)
    st0 = sweep.initial_state(g, len(mu), np.repeat(W.group_planck(edges, np.array([0.01])), n * n, 1))
    st, exits = sweep.sweep(g, mu, kap, Bg, 3.0, st0, I_in)
    E, F, f = moments.cell_moments(g, phi, mu, om, st, W.C_LIGHT)
    mir = lambda X: X.reshape(X.shape[:-1] + (n, n))[..., ::-1, :].reshape(X.shape)
    tol = 1e-11
    assert np.allclose(E, mir(E), rtol=tol, atol=0)
    assert np.allclose(F[:, 0], mir(F[:, 0]), rtol=tol, atol=1e-12 * np.abs(F).max())
    assert np.allclose(F[:, 1], -mir(F[:, 1]), rtol=tol, atol=1e-12 * np.abs(F).max())
    for q, sgn in ((0, 1), (1, -1), (2, 1), (3, 1)):
        assert np.allclose(f[:, q], sgn * mir(f[:, q]), rtol=1e-10, atol=1e-12)
    bnd = moments.boundary_factors(g, phi, mu, om, exits, I_in)
    bot = bnd[:, 2 * n:3 * n]
    top = bnd[:, 3 * n:4 * n]
    assert np.allclose(bot[..., [0, 1, 2, 3, 4, 5, 7]], top[..., [0, 1, 2, 3, 4, 5, 7]], rtol=1e-10)
    assert np.allclose(bot[..., 6], -top[..., 6], rtol=1e-10, atol=1e-14)
    left = bnd[:, :n]
    assert np.allclose(left, left[:, ::-1] * np.array([1, 1, 1, 1, 1, 1, -1, 1]), rtol=1e-10, atol=1e-14)


def test_realisability_on_workload():
    p = W.config(0)
    r = solve.run(p)
    st = r["state"]
    assert np.all(st >= 0)
    E, F, f = (r["steps"][0][k] for k in ("E", "F", "f"))
    Fn = np.hypot(F[:, 0], F[:, 1])
    assert np.all(Fn <= W.C_LIGHT * E * (1 + 1e-12))
    tr = f[:, 0] + f[:, 2] + f[:, 3]
    assert np.allclose(tr, 1.0, atol=1e-13)
    # 2x2 in-plane block is positive semi-definite
    det = f[:, 0] * f[:, 2] - f[:, 1] ** 2
    assert np.all(f[:, 0] >= 0) and np.all(f[:, 2] >= 0) and np.all(det >= -1e-14)


def test_per_direction_normalisation_equals_literal_form_on_paper_grid():
    """With the vertex-avoiding construction the traced area of each
    direction equals the cell area, so the per-direction normalised tensor
    equals the literal eq. (15) (one normalisation over all directions)."""
    n, L = 6, 1.2
    phi, mu, om = W.product_quadrature(8, 2)
    edges = W.group_edges(2, 0.01, 3.0)
    T = np.random.default_rng(2).uniform(0.05, 1.0, n * n)
    kap = W.fc_opacity(W.group_midpoints(edges), T)
    Bg = W.group_planck(edges, T)
    I_in = W.inflow_left_planck(n, n, phi, mu, edges, 1.0)
    g = rays.build(n, n, L, L, phi, 0.05, rays.TUBES)
    st0 = sweep.initial_state(g, len(mu), Bg * 0.3)
    st, _ = sweep.sweep(g, mu, kap, Bg, 3.0, st0, I_in)
    E, F, f = moments.cell_moments(g, phi, mu, om, st, 1.0)
    # literal eq. (15): sums over all (m, k, s) in C(i, m)
    num = np.zeros((2, n * n)); den = np.zeros((2, n * n))
    for a, pr in enumerate(g.pairs):
        j = pr.seg_base
        for k in range(pr.K):
            for cell, ln in zip(pr.cells[k], pr.lens[k]):
                A = ln * pr.w[k]
                for d in (0, 1):
                    for p in range(len(mu)):
                        az = a + d * (len(phi) // 2)
                        m = az * len(mu) + p
                        Om = _omega(phi, mu, az, p)
                        num[:, cell] += om[m] * A * Om[0] * Om[0] * st[j, d, p]
                        den[:, cell] += om[m] * A * st[j, d, p]
                j += 1
    assert np.allclose(f[:, 0], num / den, rtol=1e-12)
