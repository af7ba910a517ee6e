"""Pins of the grey-closure oracle (eq. (8)-(9) and the Planck mean of (5a)):
a two-group example worked by hand, closed forms for group-independent
opacities, the identity the grey momentum equation relies on, invariances
and the 0/0 readings."""
import json
import os

import numpy as np
import pytest

from oracle import closures as C

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "grey_closures_two_group.json")
IDX = {n: i for i, n in enumerate(C.NAMES)}


def _random(G, cells, seed):
    rng = np.random.default_rng(seed)
    E = rng.uniform(0.1, 2.0, (G, cells))
    F = rng.uniform(-1.0, 1.0, (G, 2, cells)) * E[:, None, :]
    fxx = rng.uniform(0.1, 0.6, (G, cells))
    fyy = rng.uniform(0.1, 0.6, (G, cells)) * (1 - fxx)
    f = np.stack([fxx, rng.uniform(-0.1, 0.1, (G, cells)), fyy, 1 - fxx - fyy], axis=1)
    kap = rng.uniform(0.5, 50.0, (G, cells))
    B = rng.uniform(0.0, 3.0, (G, cells))
    return E, F, f, kap, B


def test_two_group_example_worked_by_hand():
    """Values in the fixture were worked out by hand from the definitions
    (the fractions are written beside each value there)."""
    gold = json.load(open(GOLDEN))
    inp = gold["input"]
    got = C.grey_closures(np.array(inp["E"])[:, None], np.array(inp["F"])[:, :, None],
                          np.array(inp["f"])[:, :, None], np.array(inp["kappa"])[:, None],
                          np.array(inp["planck"])[:, None])[:, 0]
    for name, v in gold["expected"].items():
        assert abs(got[IDX[name]] - v) <= 1e-14 * max(1.0, abs(v)), (name, got[IDX[name]], v)


def test_group_independent_opacity():
    """kappa_g = kappa for every g: every average is kappa and eta = 0."""
    E, F, f, kap, B = _random(7, 50, 1)
    k = np.linspace(0.3, 9.0, 50)
    kap = np.broadcast_to(k, E.shape)
    out = C.grey_closures(E, F, f, kap, B)
    for name in ("kappa_E", "kappa_B", "KR_xx", "KR_yy"):
        assert np.allclose(out[IDX[name]], k, rtol=1e-14)
    assert np.allclose(out[IDX["eta_x"]], 0.0, atol=1e-13)
    assert np.allclose(out[IDX["eta_y"]], 0.0, atol=1e-13)


def test_single_group_reduces_to_the_group_values():
    E, F, f, kap, B = _random(1, 30, 2)
    out = C.grey_closures(E, F, f, kap, B)
    assert np.array_equal(out[IDX["E"]], E[0])
    assert np.allclose(out[IDX["kappa_E"]], kap[0], rtol=1e-15)
    for c, n in enumerate(("fE_xx", "fE_xy", "fE_yy", "fE_zz")):
        assert np.allclose(out[IDX[n]], f[0, c], rtol=1e-15, atol=1e-17)
    assert np.allclose(out[IDX["eta_x"]], 0.0, atol=1e-13 * kap.max())


def test_grey_momentum_reproduces_the_group_sum():
    """sum_g kappa_g F_g = K_R F + eta E: the grey momentum equation's
    absorption terms equal the sum of the multigroup ones."""
    E, F, f, kap, B = _random(9, 40, 3)
    out = C.grey_closures(E, F, f, kap, B)
    for a, (kr, eta, fn) in enumerate((("KR_xx", "eta_x", "Fx"), ("KR_yy", "eta_y", "Fy"))):
        lhs = np.sum(kap * F[:, a], axis=0)
        rhs = out[IDX[kr]] * out[IDX[fn]] + out[IDX[eta]] * out[IDX["E"]]
        assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12 * np.abs(lhs).max())


def test_grey_energy_terms_reproduce_the_group_sums():
    """<kappa>_E E = sum_g kappa_g E_g and <kappa>_B sum_g B_g =
    sum_g kappa_g B_g; the grey Eddington tensor times E is sum f_g E_g."""
    E, F, f, kap, B = _random(6, 40, 4)
    out = C.grey_closures(E, F, f, kap, B)
    assert np.allclose(out[IDX["kappa_E"]] * out[IDX["E"]], np.sum(kap * E, axis=0), rtol=1e-13)
    assert np.allclose(out[IDX["kappa_B"]] * B.sum(axis=0), np.sum(kap * B, axis=0), rtol=1e-13)
    for c, n in enumerate(("fE_xx", "fE_xy", "fE_yy", "fE_zz")):
        assert np.allclose(out[IDX[n]] * out[IDX["E"]], np.sum(f[:, c] * E, axis=0), rtol=1e-12, atol=1e-14)


def test_trace_and_invariances():
    E, F, f, kap, B = _random(5, 30, 5)
    out = C.grey_closures(E, F, f, kap, B)
    tr = out[IDX["fE_xx"]] + out[IDX["fE_yy"]] + out[IDX["fE_zz"]]
    assert np.allclose(tr, 1.0, atol=1e-14)
    # scaling the radiation field and the sources leaves every average alone
    s = 2.0 ** 7
    out2 = C.grey_closures(E * s, F * s, f, kap, B * 3.0)
    for n in C.NAMES[3:]:
        assert np.allclose(out2[IDX[n]], out[IDX[n]], rtol=1e-13, atol=1e-15), n
    # the group order does not matter beyond rounding
    perm = np.random.default_rng(6).permutation(E.shape[0])
    out3 = C.grey_closures(E[perm], F[perm], f[perm], kap[perm], B[perm])
    for r in range(C.N_GREY):
        assert np.allclose(out3[r], out[r], rtol=1e-13, atol=1e-13 * np.abs(out[r]).max()), C.NAMES[r]


def test_zero_over_zero_readings():
    E, F, f, kap, B = _random(4, 6, 7)
    E[:, 0] = 0.0
    F[:, :, 0] = 0.0                       # no radiation in cell 0
    B[:, 1] = 0.0                          # no emission in cell 1
    F[:, 0, 2] = 0.0                       # no x flux in cell 2
    E[:, 3] = 0.0
    F[:, :, 3] = 0.0
    B[:, 3] = 0.0                          # nothing at all in cell 3
    out = C.grey_closures(E, F, f, kap, B)
    kB0 = np.sum(kap[:, 0] * B[:, 0]) / np.sum(B[:, 0])
    assert out[IDX["kappa_E"], 0] == pytest.approx(kB0, rel=1e-14)
    assert out[IDX["KR_xx"], 0] == pytest.approx(kB0, rel=1e-14)
    assert out[IDX["eta_x"], 0] == 0.0 and out[IDX["eta_y"], 0] == 0.0
    assert tuple(out[IDX[n], 0] for n in ("fE_xx", "fE_xy", "fE_yy", "fE_zz")) == (1 / 3, 0.0, 1 / 3, 1 / 3)
    assert out[IDX["kappa_B"], 1] == out[IDX["kappa_E"], 1]
    assert out[IDX["KR_xx"], 2] == out[IDX["kappa_E"], 2]
    assert out[IDX["kappa_E"], 3] == pytest.approx(kap[:, 3].mean(), rel=1e-14)
    assert np.all(np.isfinite(out))
