"""GPU: multilevel (MLQD) time steps on the Fleck-Cummings material
(lc_mlqd_material, lc_mlqd_step) against the oracle (oracle/material.py,
oracle/mlqd.py), and properties of the library's steps at a larger size.

Tolerances.  The material functions are closed-form evaluations: opacity
to 1e-14 relative, group Planck functions (series and tails in the
library, adaptive quadrature in the oracle) to 1e-11 relative wherever B_g
is above 1e-200 of the group sum.  A time step is an iteration to a
fixed point that both sides stop once the temperature changes by at most
eps = 1e-11 between iterations; with contraction factors up to about 0.8
each side sits within a few eps of the fixed point in T, and the
intensities of groups in the Wien tail of a cold cell move by (nu/T) dT/T,
up to a few hundred times more; the low-order solves add their residual
(1e-13 at the end) times the condition number.  T, E and F (normwise per
group) and the transport state are compared at 1e-8."""
import math
import sys
import warnings

import numpy as np
import pytest

import workloads as W
from oracle import loqd as OL, material as OMAT, mlqd as OMQ, rays as OR, sweep as OS
from tests.parity_util import err_rel

pytestmark = pytest.mark.gpu

C, A_R = W.C_LIGHT, W.A_RAD
TOL = 1e-8


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


def _fc(h_mat=1.0, h_moc=0.1, n_az=8, n_pol=2, G=6):
    return W.fc_mlqd(h_mat, h_moc, n_az, n_pol, G, nu_lo=0.3, nu_hi=30.0)


def test_material_matches_the_oracle(lcmod):
    import torch
    lc, driver = lcmod
    p = _fc(h_mat=0.2, h_moc=0.05, G=17)                 # 30 x 30 cells: four blocks, ragged
    _say(f"case fc material {p.nx}x{p.ny} G={p.G}")
    s = driver.MlqdSolver(p)
    rng = np.random.default_rng(5)
    Tu = 10.0 ** rng.uniform(-3, 0.5, 60)
    T = Tu[rng.integers(0, 60, p.cells)]
    G, N = p.G, p.cells
    kap = torch.zeros(G * N, dtype=torch.float64, device="cuda")
    pla = torch.zeros(G * N, dtype=torch.float64, device="cuda")
    lc.lc_mlqd_material(s.h, torch.from_numpy(T).cuda(), kap, pla)
    kap, pla = kap.cpu().numpy().reshape(G, N), pla.cpu().numpy().reshape(G, N)
    rk = OMAT.fc_opacity(p.nu, T)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        rb = OMAT.group_planck(p.edges, T, A_R, C)
    ek = np.max(np.abs(kap - rk) / rk)
    big = rb > 1e-200 * rb.sum(0)[None, :]
    eb = np.max(np.abs(pla - rb)[big] / rb[big])
    _say(f"  opacity {ek:.2e}  Planck {eb:.2e}")
    assert ek <= 1e-14 and eb <= 1e-11
    assert np.all(pla[~big] <= 1e-199 * rb.sum(0)[None, :].repeat(G, 0)[~big])


def _oracle_steps(p, steps, eps, mode=OR.UNIFORM):
    g = OR.build(p.nx, p.ny, p.lx, p.ly, p.phi, p.h_moc, mode=mode)
    st = OS.initial_state(g, p.n_pol, p.state0)
    E0, F0 = OMQ.initial_low_order(p, C)
    T = np.full(p.cells, p.T0)
    out = []
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        for _ in range(steps):
            r = OMQ.outer_step(g, p, st, T, E0, F0, C, A_R, eps=eps)
            out.append(r)
            st, T, E0, F0 = r["state"], r["T"], r["E_cell"], r["F_face"]
    return out


def _normwise(a, b):
    a, b = np.atleast_2d(a), np.atleast_2d(b)
    return max(float(np.max(np.abs(x - y)) / np.max(np.abs(y))) for x, y in zip(a, b))


def test_mlqd_steps_match_the_oracle(lcmod):
    lc, driver = lcmod
    p = _fc()
    eps = 1e-11
    _say(f"case fc mlqd {p.nx}x{p.ny} G={p.G} M={len(p.omega)}, 2 steps, eps {eps}")
    ref = _oracle_steps(p, 2, eps)
    s = driver.MlqdSolver(p, eps=eps)
    s.reset()
    for n in range(2):
        s.step(1)
        got = s.solution()
        r = ref[n]
        outer, inner, ch = s.history[-1]
        e = dict(T=_normwise(got["T"], r["T"]), E_cell=_normwise(got["E_cell"], r["E_cell"]),
                 E_face=_normwise(got["E_face"], r["E_face"]), F_face=_normwise(got["F_face"], r["F_face"]),
                 E_grey=_normwise(got["E_grey"], r["E_grey"]), state=err_rel(s.state_canonical(), r["state"]))
        _say(f"  step {n}: outer {outer} (oracle {r['outer']}), inner {inner} (oracle {r['inner']}); "
             + " ".join(f"{k} {v:.2e}" for k, v in e.items()))
        assert abs(outer - r["outer"]) <= 1
        assert max(e.values()) <= TOL


def test_mlqd_keeps_radiative_equilibrium(lcmod):
    import torch
    lc, driver = lcmod
    p = _fc(h_mat=1.5, h_moc=0.3, G=4)
    Teq = 0.35
    B = OMAT.group_planck(p.edges, np.array([Teq]), A_R, C)[:, 0]
    nb = 2 * (p.nx + p.ny)
    p.I_in = np.broadcast_to(B[None, None, :], (nb, len(p.omega), p.G)).copy()
    p.state0 = np.repeat(B[:, None], p.cells, axis=1)
    p.T0 = Teq
    _say("case fc mlqd equilibrium 4x4")
    s = driver.MlqdSolver(p)
    s.reset()
    st0 = s.state_canonical()
    s.step(1)
    got = s.solution()
    assert s.history[-1][0] <= 2
    assert np.allclose(got["T"], Teq, rtol=1e-12)
    assert np.allclose(got["E_cell"], (4 * math.pi * B / C)[:, None], rtol=1e-11)
    assert np.max(np.abs(got["F_face"])) <= 1e-11 * 4 * math.pi * B.sum()
    assert np.allclose(s.state_canonical(), st0, rtol=1e-12)


def _boundary_inflow(p, F_face):
    nx, ny = p.nx, p.ny
    hx, hy = p.lx / nx, p.ly / ny
    nint = OL.n_interior(nx, ny)
    sgn = np.concatenate([-np.ones(ny), np.ones(ny), -np.ones(nx), np.ones(nx)])
    lens = np.concatenate([np.full(ny, hy), np.full(ny, hy), np.full(nx, hx), np.full(nx, hx)])
    return -(p.c_dt / C) * np.sum(sgn * F_face.sum(0)[nint:] * lens)


@pytest.mark.parametrize("h_mat,h_moc", [(0.3, 0.02), (0.15, 0.001)])
def test_mlqd_steps_conserve_energy_at_the_papers_counts(lcmod, h_mat, h_moc):
    """The paper's counts: 17 groups, 144 directions, on 20 x 20 cells and on
    its finest grid (40 x 40 cells of 0.15 cm crossed by characteristics
    1e-3 cm apart: 5.5 million segments), three steps: each conserves
    energy, its grey energy is the sum of the group energies, and its
    temperature satisfies the multigroup energy balance with its own
    opacities and Planck functions."""
    lc, driver = lcmod
    p = W.fc_mlqd(h_mat, h_moc, 36, 4, 17, nu_lo=0.3, nu_hi=30.0)
    _say(f"case fc mlqd {p.nx}x{p.ny} G={p.G} M={len(p.omega)} h_moc={p.h_moc}, 3 steps")
    s = driver.MlqdSolver(p, eps=1e-11)
    s.reset()
    prev = dict(T=np.full(p.cells, p.T0), E_cell=4 * math.pi * p.state0 / C)
    hx, hy = p.lx / p.nx, p.ly / p.ny
    for n in range(3):
        s.step(1)
        got = s.solution()
        outer, inner, ch = s.history[-1]
        gained = np.sum(p.c_v * (got["T"] - prev["T"]) + (got["E_cell"] - prev["E_cell"]).sum(0)) * hx * hy
        inflow = _boundary_inflow(p, got["F_face"])
        summed = got["E_cell"].sum(0)
        grey = np.max(np.abs(summed - got["E_grey"])) / np.max(summed)
        T = got["T"]
        kap = OMAT.fc_opacity(p.nu, T)
        B = W.group_planck(p.edges, T)
        rhs = (C * kap * got["E_cell"] - 4 * math.pi * kap * B).sum(0)
        lhs = p.c_v * (T - prev["T"]) / (p.c_dt / C)
        meb = np.max(np.abs(lhs - rhs)) / np.max((4 * math.pi * kap * B).sum(0))
        _say(f"  step {n}: outer {outer} inner {inner} changes {ch[0]:.1e} {ch[1]:.1e}; T max {T.max():.4f}; "
             f"energy gained {gained:.6e} inflow {inflow:.6e}; grey-sum {grey:.1e}; balance {meb:.1e}")
        assert math.isclose(gained, inflow, rel_tol=1e-8)
        assert grey <= 1e-9 and meb <= 1e-8
        prev = got


def test_mlqd_reports_non_convergence_and_refuses_float32(lcmod):
    lc, driver = lcmod
    p = _fc(h_mat=1.5, h_moc=0.3, G=4)
    s = driver.MlqdSolver(p, eps=1e-12, max_outer=1)
    s.reset()
    with pytest.raises(lc.LcError) as e:
        s.step(1)
    assert e.value.status == lc.LC_ERR_UNSUPPORTED
    with pytest.raises(lc.LcError) as e:
        driver.MlqdSolver(p, prec=lc.LC_F32)
    assert e.value.status == lc.LC_ERR_UNSUPPORTED


def test_mlqd_acceleration_keeps_the_fixed_point(lcmod):
    """Plain inner passes (depth 0) and Anderson mixing (depth 3) reach the
    same step result within the iteration tolerance, the mixing in fewer
    passes."""
    lc, driver = lcmod
    p = _fc()
    _say("case fc mlqd 6x6: plain vs accelerated inner iterations, 2 steps")
    out = {}
    for depth in (0, 3):
        s = driver.MlqdSolver(p, eps=1e-11, depth=depth)
        s.reset()
        s.step(2)
        out[depth] = (s.solution(), sum(h[1] for h in s.history))
    a, b = out[0][0], out[3][0]
    e = max(_normwise(a[k], b[k]) for k in ("T", "E_cell", "E_face", "F_face"))
    _say(f"  inner passes: plain {out[0][1]}, accelerated {out[3][1]}; difference {e:.2e}")
    assert out[3][1] < out[0][1] and e <= TOL



def test_mlqd_steps_repeat_bit_for_bit(lcmod):
    """A step's results depend on its arguments alone: the same steps run
    again from reset() on the same handle, on a fresh handle, and with the
    transport gathers whole instead of split over azimuth pairs give the same
    bits and the same iteration counts."""
    lc, driver = lcmod
    p = _fc(h_mat=0.6, h_moc=0.02, G=6)
    _say(f"case fc mlqd {p.nx}x{p.ny} G={p.G} h_moc {p.h_moc}: repeated steps")
    runs = []
    a = driver.MlqdSolver(p, eps=1e-11)
    assert lc.lc_plan_get_moment_split(a.plan) == 3
    b = driver.MlqdSolver(p, eps=1e-11)
    lc.lc_plan_set_moment_split(b.plan, 0)
    for s in (a, a, b):
        s.reset()
        s.step(2)
        runs.append((s.solution(), [tuple(h[:2]) for h in s.history]))
    for sol, hist in runs[1:]:
        assert hist == runs[0][1]
        for k in sol:
            assert np.array_equal(sol[k], runs[0][0][k]), k
    _say(f"  iterations {runs[0][1]}")


def test_mlqd_steps_match_the_oracle_on_the_papers_grid(lcmod):
    """The vertex-avoiding, width-halving characteristic grid (the paper's
    construction), 5 x 5 cells of 1.2 cm, h_moc = 0.15 cm: two steps against
    the oracle's, as on the equally spaced grid."""
    lc, driver = lcmod
    p = _fc(h_mat=1.2, h_moc=0.15, G=5)
    eps = 1e-11
    _say(f"case fc mlqd {p.nx}x{p.ny} G={p.G} tube grid, 2 steps, eps {eps}")
    ref = _oracle_steps(p, 2, eps, mode=OR.TUBES)
    rays = lc.lc_build_rays(p.nx, p.ny, p.lx, p.ly, p.phi, p.mu, p.omega, p.h_moc, lc.LC_RAYS_TUBES)
    s = driver.MlqdSolver(p, rays=rays, eps=eps)
    s.reset()
    for n in range(2):
        s.step(1)
        got = s.solution()
        r = ref[n]
        outer, inner, ch = s.history[-1]
        e = dict(T=_normwise(got["T"], r["T"]), E_cell=_normwise(got["E_cell"], r["E_cell"]),
                 F_face=_normwise(got["F_face"], r["F_face"]), state=err_rel(s.state_canonical(), r["state"]))
        _say(f"  step {n}: outer {outer} (oracle {r['outer']}), inner {inner} (oracle {r['inner']}); "
             + " ".join(f"{k} {v:.2e}" for k, v in e.items()))
        assert abs(outer - r["outer"]) <= 1
        assert max(e.values()) <= TOL
