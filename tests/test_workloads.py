"""Pins for the seeded input generators: quadrature moments, the group Planck
function against its closed-form total and against direct quadrature, and the
Fleck-Cummings problem data of the paper's results section."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("n_az,n_pol", [(16, 2), (32, 2), (32, 4), (48, 6), (8, 3)])
def test_quadrature_moments(n_az, n_pol):
    phi, mu, om = W.product_quadrature(n_az, n_pol)
    sz = np.sqrt(1 - mu ** 2)
    ox = np.outer(np.cos(phi), sz).ravel()
    oy = np.outer(np.sin(phi), sz).ravel()
    oz = np.tile(mu, n_az)
    assert abs(om.sum() - 4 * math.pi) < 1e-13
    for o in (ox, oy, oz):
        assert abs((om * o).sum()) < 1e-13
    for a, b, ref in ((ox, ox, 4 * math.pi / 3), (oy, oy, 4 * math.pi / 3),
                      (oz, oz, 4 * math.pi / 3), (ox, oy, 0.0), (ox, oz, 0.0)):
        assert abs((om * a * b).sum() - ref) < 1e-13
    # opposite azimuths are exactly pi apart and mu pairs are mirror images
    assert np.allclose(phi[n_az // 2:] - phi[:n_az // 2], math.pi, atol=1e-14)
    assert np.array_equal(mu, -mu[::-1])


def test_planck_total_closed_form():
    # sum over groups that cover (0, inf) = a_R c T^4 / (4 pi)
    for T in (0.001, 0.03, 1.0, 2.5):
        edges = np.concatenate([[0.0], np.geomspace(1e-6 * T, 60 * T, 200), [1e4 * T]])
        Bg = W.group_planck(edges, np.array([T]))[:, 0]
        ref = W.A_RAD * W.C_LIGHT * T ** 4 / (4 * math.pi)
        assert abs(Bg.sum() / ref - 1.0) < 1e-13


def _mp_planck(mp, x1, x2):
    """int_{x1}^{x2} x^3/(e^x - 1) dx by tanh-sinh quadrature; above x = 1 in
    the variable t = exp(-(x - x1)), where the integrand is smooth."""
    if x2 <= 1:
        return mp.quad(lambda x: x ** 3 / mp.expm1(x), [x1, x2])
    lo = x1
    acc = mp.mpf(0)
    if x1 < 1:
        acc += mp.quad(lambda x: x ** 3 / mp.expm1(x), [x1, 1])
        lo = mp.mpf(1)

    def g(t):
        x = lo - mp.log(t)
        return x ** 3 * mp.exp(-lo) / (-mp.expm1(-x))
    return acc + mp.quad(g, [mp.exp(-(x2 - lo)), 1])


def test_planck_groups_vs_quadrature():
    import mpmath as mp
    mp.mp.dps = 40
    edges = W.group_edges(17, 0.001, 30.0)
    for T in (0.001, 0.05, 1.0):
        Bg = W.group_planck(edges, np.array([T]))[:, 0]
        pref = mp.mpf(W.A_RAD * W.C_LIGHT / (4 * math.pi)) * mp.mpf(T) ** 4 * 15 / mp.pi ** 4
        for g in range(17):
            x1, x2 = mp.mpf(edges[g]) / T, mp.mpf(edges[g + 1]) / T
            ref = float(pref * _mp_planck(mp, x1, x2))
            if ref > 1e-300:
                assert abs(Bg[g] - ref) <= 1e-12 * ref, (T, g, Bg[g], ref)
            else:
                assert Bg[g] <= 1e-290
    # an integration by scipy's adaptive quadrature agrees too (different method)
    T = 0.3
    Bg = W.group_planck(edges, np.array([T]))[:, 0]
    pref = W.A_RAD * W.C_LIGHT * T ** 4 / (4 * math.pi) * 15 / math.pi ** 4
    for g in range(17):
        val, _ = integrate.quad(lambda x: x ** 3 / math.expm1(x), edges[g] / T,
                                edges[g + 1] / T, epsabs=0, epsrel=1e-13)
        assert abs(Bg[g] - pref * val) <= 1e-12 * pref * val


def test_planck_integral_matches_mpmath():
    import mpmath as mp
    mp.mp.dps = 40
    for x in (1e-4, 0.3, 1.9999, 2.0, 2.5, 7.0, 31.0, 120.0):
        ref = mp.quad(lambda t: t ** 3 / mp.expm1(t), [0, x])
        got = W.planck_integral_0x(np.array([x]))[0]
        assert abs(got - float(ref)) <= 2e-15 * float(ref)


def test_fleck_cummings_data_match_paper():
    fc = json.load(open(os.path.join(GOLDEN, "fleck_cummings.json")))
    p = W.config(0)
    assert (p.lx, p.ly) == tuple(fc["domain_cm"])
    # opacity law 27 / nu^3 (1 - exp(-nu/T))
    nu, T = np.array([0.5, 3.0]), np.array([0.2, 1.0])
    k = W.fc_opacity(nu, T)
    ref = fc["opacity_coefficient"] * nu[:, None] ** fc["opacity_nu_power"] * \
        (1 - np.exp(-nu[:, None] / T[None, :]))
    assert np.allclose(k, ref, rtol=1e-15)
    # inflow: 1 keV Planckian on the x = 0 face for Omega_x > 0 only
    Bin = W.group_planck(p.edges, np.array([fc["T_in_keV"]]))[:, 0]
    ny = p.ny
    for a, ph in enumerate(p.phi):
        for q in range(p.n_pol):
            m = a * p.n_pol + q
            if math.cos(ph) > 0:
                assert np.array_equal(p.I_in[:ny, m, :], np.broadcast_to(Bin, (ny, p.G)))
            assert not p.I_in[ny:, m, :].any()
    # initial segment intensity is B_g(T0)
    B0 = W.group_planck(p.edges, np.array([fc["T0_keV"]]))[:, 0]
    assert np.array_equal(p.state0[:, 0], B0)


def test_configs_are_seeded_and_sized():
    a, b = W.config(0), W.config(0)
    assert np.array_equal(a.T[0], b.T[0])
    assert a.G == 4 and a.M == 32 and a.nx == 16 and a.h_moc == 0.05
    specs = W.batch_spec(64)
    assert len(specs) == 64
    assert {s[0] for s in specs} <= {32, 64, 128, 256}
    assert {s[1] for s in specs} <= {8, 17, 51}
    assert {s[2] for s in specs} <= {16, 64, 128}
