"""GPU: the multigroup LOQD solve (lc_loqd_solve, eq. (4) for one
backward-Euler step) against the oracle's sparse direct solve of the same
finite-volume scheme (oracle/loqd.py), on the same inputs.

The GPU solves the face system by BiCGSTAB to a relative residual of 1e-13
and the oracle solves it directly, so the two differ by the iteration's
error, bounded by the system's condition number times the residual (about
1e4 x 1e-13 on these grids).  Comparisons are normwise per group --
max |x - x_ref| / max |x_ref| over the cells, the faces and the face fluxes --
at 1e-9.  Cases: random coefficients (several groups, ragged grids, more
than one reduction block), the smooth manufactured solution of the oracle's
convergence pin, an optically thin worst case, closures from the oracle's
own transport solve on the 16 x 16 workload fed to both, and the whole chain
on the GPU (sweep with face intensities, moments, LOQD) against the whole
chain in the oracle."""
import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle import faces as OF, loqd as OL, moments as OM, rays as OR, solve as OSV, sweep as OS

pytestmark = pytest.mark.gpu

TOL = 1e-9


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


def _gpu_layouts(nx, ny, f_cell, f_face, bc):
    """Oracle-side closures -> the library's layouts: f_cell [G][3][cells] ->
    [cells][4][G]; interior f_face [G][3][faces] -> [interior][4][G]; boundary
    tensors and (C, Phi^-, J^-) -> bnd [G][nb][8]."""
    G, _, N = f_cell.shape
    nint = OL.n_interior(nx, ny)
    nb = 2 * (nx + ny)
    fc = np.full((N, 4, G), 1.0 / 3.0)
    fc[:, :3, :] = f_cell.transpose(2, 1, 0)
    ff = np.full((max(nint, 1), 4, G), 1.0 / 3.0)
    ff[:nint, :3, :] = f_face[:, :, :nint].transpose(2, 1, 0)
    bnd = np.zeros((G, nb, 8))
    bnd[:, :, 4] = bc[:, :, 0]
    bnd[:, :, 2] = bc[:, :, 1]
    bnd[:, :, 3] = bc[:, :, 2]
    bnd[:, :, 5:8] = f_face[:, :, nint:].transpose(0, 2, 1)
    return fc, ff, bnd


def _gpu_solve(lc, nx, ny, lx, ly, c, c_dt, kappa, planck, E_prev, F_prev, f_cell, f_face, bc, rtol=1e-13,
               max_iter=20000, solver=0):
    import torch
    G = kappa.shape[0]
    fc, ff, bnd = _gpu_layouts(nx, ny, f_cell, f_face, bc)
    h = lc.Loqd(nx, ny, lx, ly, G)
    lc.lc_loqd_set_solver(h, solver)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    Ec = torch.zeros(G * h.cells, dtype=torch.float64, device="cuda")
    Ef = torch.zeros(G * h.nf, dtype=torch.float64, device="cuda")
    Ff = torch.zeros(G * h.nf, dtype=torch.float64, device="cuda")
    it, res = lc.lc_loqd_solve(h, c, c_dt, d(kappa), d(planck), d(E_prev), d(F_prev), d(fc), d(ff), d(bnd),
                               Ec, Ef, Ff, rtol=rtol, max_iter=max_iter)
    out = (Ec.cpu().numpy().reshape(G, -1), Ef.cpu().numpy().reshape(G, -1), Ff.cpu().numpy().reshape(G, -1))
    return out, it, res


def _compare(got, ref, what):
    assert len(got) == len(ref)
    names = ("E_cell", "E_face", "F_face") if len(got) == 3 else ("T", "E_cell", "E_face", "F_face")
    worst = 0.0
    for name, a, b in zip(names, got, ref, strict=True):
        for g in range(a.shape[0]):
            scale = np.max(np.abs(b[g]))
            if scale == 0.0:
                assert np.max(np.abs(a[g])) == 0.0
                continue
            worst = max(worst, float(np.max(np.abs(a[g] - b[g])) / scale))
    _say(f"  {what}: worst normwise difference {worst:.2e}")
    assert worst <= TOL
    return worst


def _random_groups(nx, ny, lx, ly, G, seed, thin=False):
    rng = np.random.default_rng(seed)
    N, nf = nx * ny, OL.n_faces(nx, ny)
    nb = 2 * (nx + ny)
    c, c_dt = 299.792458, 3.0
    scale = 10.0 ** rng.uniform(-3, 3, G)[:, None]
    kappa = np.zeros((G, N)) if thin else 10.0 ** rng.uniform(-2, 3, (G, N))
    planck = rng.uniform(0, 1, (G, N)) * scale
    E_prev = rng.uniform(0, 1, (G, N)) * scale * 4 * math.pi / c
    F_prev = rng.uniform(-0.3, 0.3, (G, nf)) * scale

    def tensors(n):
        a = rng.uniform(0.15, 0.6, (G, n))
        dd = rng.uniform(0.15, 0.6, (G, n))
        b = rng.uniform(-0.5, 0.5, (G, n)) * np.sqrt(a * dd)
        return np.stack([a, b, dd], axis=1)
    bc = np.stack([rng.uniform(0.3, 0.7, (G, nb)), rng.uniform(0, 1, (G, nb)) * scale,
                   rng.uniform(0, 0.5, (G, nb)) * scale], axis=2)
    return (nx, ny, lx, ly, c, c_dt, kappa, planck, E_prev, F_prev, tensors(N), tensors(nf), bc)


@pytest.mark.parametrize("solver", [1, 2])
@pytest.mark.parametrize("shape", [(7, 5, 1.4, 0.7, 3), (33, 20, 3.3, 1.0, 5), (1, 6, 0.2, 1.2, 2), (9, 1, 0.9, 0.1, 2)])
def test_loqd_random_coefficients(lcmod, shape, solver):
    lc, _ = lcmod
    nx, ny, lx, ly, G = shape
    args = _random_groups(nx, ny, lx, ly, G, seed=nx * 31 + ny)
    _say(f"case loqd random {nx}x{ny} G={G} solver {solver}")
    ref = OL.solve(*args)
    got, it, res = _gpu_solve(lc, *args, solver=solver)
    _say(f"  {it} iterations, residuals {np.max(res):.1e}")
    _compare(got, ref, "random")


def test_loqd_thin_worst_case(lcmod):
    """kappa = 0 (only 1/(c dt) attenuates): the most diffusive system."""
    lc, _ = lcmod
    args = _random_groups(48, 40, 6.0, 5.0, 2, seed=5, thin=True)
    _say("case loqd thin 48x40 G=2")
    ref = OL.solve(*args)
    got, it, res = _gpu_solve(lc, *args)
    _say(f"  {it} iterations, residuals {np.max(res):.1e}")
    _compare(got, ref, "thin")


def test_loqd_manufactured_solution(lcmod):
    lc, _ = lcmod
    from tests.test_oracle_loqd import _manufactured_case
    args, exact, _ = _manufactured_case(32)
    nx, ny, lx, ly, c, c_dt, kap, planck, E_prev, F_prev, f_cell, f_face, bc = args
    stack = (nx, ny, lx, ly, c, c_dt, kap[None], planck[None], E_prev[None], F_prev[None], f_cell[None],
             f_face[None], bc[None])
    _say("case loqd manufactured 32x32")
    ref = OL.solve(*stack)
    got, it, res = _gpu_solve(lc, *stack)
    _compare(got, ref, "manufactured")
    # and the GPU solution approximates the exact one to the scheme's accuracy
    assert np.sqrt(np.mean((got[0][0] - exact[0]) ** 2)) < 1e-4


def _oracle_transport_closures(prob):
    """Cell, interior-face and boundary closures of one step of the oracle's
    transport solve (with the upwind-face intensities of the sweep)."""
    g = OR.build(prob.nx, prob.ny, prob.lx, prob.ly, prob.phi, prob.h_moc)
    st = OS.initial_state(g, prob.n_pol, prob.state0)
    pts = np.zeros_like(st)
    st, exits = OS.sweep(g, prob.mu, prob.kappa[0], prob.planck[0], prob.c_dt, st, prob.I_in, points=pts)
    E, F, f = OM.cell_moments(g, prob.phi, prob.mu, prob.omega, st, W.C_LIGHT)
    bnd = OM.boundary_factors(g, prob.phi, prob.mu, prob.omega, exits, prob.I_in)
    Ef, Ff, ff = OF.face_moments(g, prob.phi, prob.mu, prob.omega, pts, W.C_LIGHT)
    return E, f, ff, bnd


def _loqd_inputs(prob):
    c = W.C_LIGHT
    G, N = prob.G, prob.cells
    nf = OL.n_faces(prob.nx, prob.ny)
    E_prev = 4 * math.pi * prob.state0 / c                 # E^{n-1} of the isotropic initial intensity
    return c, prob.c_dt, prob.kappa[0], prob.planck[0], E_prev, np.zeros((G, nf))


def test_loqd_with_oracle_transport_closures(lcmod):
    lc, _ = lcmod
    prob = W.config(0)
    _say("case loqd on oracle transport closures, 16x16 G=4")
    E_tr, f, ff, bnd = _oracle_transport_closures(prob)
    f_cell, f_face, bc = OL.closures_from_transport(prob.nx, prob.ny, f, ff, bnd)
    c, c_dt, kap, pla, E_prev, F_prev = _loqd_inputs(prob)
    args = (prob.nx, prob.ny, prob.lx, prob.ly, c, c_dt, kap, pla, E_prev, F_prev, f_cell, f_face, bc)
    ref = OL.solve(*args)
    got, it, res = _gpu_solve(lc, *args)
    _compare(got, ref, "oracle closures")
    # the low-order solution is consistent with the transport's energy density
    gE = got[0].sum(0)
    tE = E_tr.sum(0)
    _say(f"  grey E: LOQD vs transport max relative difference {np.max(np.abs(gE - tE) / tE):.2e}")


def test_loqd_whole_chain_on_gpu(lcmod):
    """Sweep storing face intensities, cell and face moments, boundary factors
    and the LOQD solve all in the library, from the problem's inputs only,
    against the same chain in the oracle."""
    import torch
    lc, driver = lcmod
    prob = W.config(0)
    _say("case loqd whole chain 16x16 G=4")
    s = driver.Solver(prob, prec=lc.LC_F64)
    s.enable_faces()
    s.reset()
    s.step_faces(1)
    G, N = prob.G, prob.cells
    h = lc.Loqd(prob.nx, prob.ny, prob.lx, prob.ly, G)
    c, c_dt, kap, pla, E_prev, F_prev = _loqd_inputs(prob)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    Ec = torch.zeros(G * N, dtype=torch.float64, device="cuda")
    Ef = torch.zeros(G * h.nf, dtype=torch.float64, device="cuda")
    Ff = torch.zeros(G * h.nf, dtype=torch.float64, device="cuda")
    lc.lc_loqd_solve(h, c, c_dt, s.kappa[0].reshape(-1), s.planck[0].reshape(-1), d(E_prev), d(F_prev), s.f,
                     s.ff, s.bnd, Ec, Ef, Ff)
    got = (Ec.cpu().numpy().reshape(G, -1), Ef.cpu().numpy().reshape(G, -1), Ff.cpu().numpy().reshape(G, -1))
    _, f, ff, bnd = _oracle_transport_closures(prob)
    f_cell, f_face, bc = OL.closures_from_transport(prob.nx, prob.ny, f, ff, bnd)
    ref = OL.solve(prob.nx, prob.ny, prob.lx, prob.ly, c, c_dt, kap, pla, E_prev, F_prev, f_cell, f_face, bc)
    _compare(got, ref, "whole chain")


def test_loqd_is_deterministic_and_reports_non_convergence(lcmod):
    lc, _ = lcmod
    args = _random_groups(20, 16, 2.0, 1.6, 3, seed=9)
    a, _, _ = _gpu_solve(lc, *args)
    b, _, _ = _gpu_solve(lc, *args)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    with pytest.raises(lc.LcError) as e:
        _gpu_solve(lc, *args, rtol=1e-15, max_iter=1)
    assert e.value.status == lc.LC_ERR_UNSUPPORTED


# ---------------------------------------------------------------------------
# general form and the effective grey equations, eq. (5)
# ---------------------------------------------------------------------------

def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _gpu_general(lc, nx, ny, lx, ly, c, c_dt, sigma, source, k_side, eta_side, F_prev, f_cell, f_face, bc):
    """Arrays with a leading group axis, oracle layouts (k_side [G][cells][4])."""
    import torch
    G = sigma.shape[0]
    h = lc.Loqd(nx, ny, lx, ly, G)
    Ec = torch.zeros(G * h.cells, dtype=torch.float64, device="cuda")
    Ef = torch.zeros(G * h.nf, dtype=torch.float64, device="cuda")
    Ff = torch.zeros(G * h.nf, dtype=torch.float64, device="cuda")
    it, res = lc.lc_loqd_solve_general(h, c, c_dt, _dev(sigma), _dev(source), _dev(k_side.transpose(0, 2, 1)),
                                       _dev(eta_side.transpose(0, 2, 1)), _dev(F_prev), _dev(f_cell), _dev(f_face),
                                       _dev(bc), Ec, Ef, Ff)
    return (Ec.cpu().numpy().reshape(G, -1), Ef.cpu().numpy().reshape(G, -1), Ff.cpu().numpy().reshape(G, -1))


def test_loqd_general_form(lcmod):
    """Side-dependent k and non-zero eta (the shape of the grey equations)."""
    lc, _ = lcmod
    rng = np.random.default_rng(12)
    nx, ny, lx, ly, G = 17, 11, 1.7, 1.1, 2
    N, nf, nb = nx * ny, OL.n_faces(nx, ny), 2 * (nx + ny)
    c, c_dt = 299.792458, 0.6
    sigma = c * 10.0 ** rng.uniform(0, 2, (G, N))
    source = rng.uniform(0, 100, (G, N))
    k_side = 10.0 ** rng.uniform(0, 2, (G, N, 4))
    eta_side = rng.uniform(-0.5, 0.5, (G, N, 4)) * k_side
    F_prev = rng.uniform(-0.3, 0.3, (G, nf))

    def tensors(n):
        a = rng.uniform(0.15, 0.6, (G, n)); dd = rng.uniform(0.15, 0.6, (G, n))
        return np.stack([a, rng.uniform(-0.5, 0.5, (G, n)) * np.sqrt(a * dd), dd], axis=1)
    fc, ff = tensors(N), tensors(nf)
    bc = np.stack([rng.uniform(0.3, 0.7, (G, nb)), rng.uniform(0, 1, (G, nb)), rng.uniform(0, 0.5, (G, nb))], axis=2)
    _say("case loqd general form 17x11 G=2")
    got = _gpu_general(lc, nx, ny, lx, ly, c, c_dt, sigma, source, k_side, eta_side, F_prev, fc, ff, bc)
    ref = [np.stack(x) for x in zip(*[OL.solve_general(nx, ny, lx, ly, c, c_dt, sigma[g], source[g], k_side[g],
                                                       eta_side[g], F_prev[g], fc[g], ff[g], bc[g])
                                      for g in range(G)])]
    _compare(got, ref, "general form")


def _gpu_grey_coefficients(lc, nx, ny, lx, ly, c, c_dt, kappa, planck, E_prev, F_prev, f_cell, f_face, bc, sol):
    """The library's grey coefficients from a multigroup solution `sol`
    (E_cell, E_face, F_face [G][...]), returned in the oracle's layouts."""
    import torch
    G = kappa.shape[0]
    h = lc.Loqd(nx, ny, lx, ly, G)
    fc, ff, bnd = _gpu_layouts(nx, ny, f_cell, f_face, bc)
    N, nf, nb = h.cells, h.nf, h.nb
    z = lambda n: torch.zeros(n, dtype=torch.float64, device="cuda")
    out = dict(sigma=z(N), source=z(N), E_prev=z(N), k_side=z(4 * N), eta_side=z(4 * N), F_prev=z(nf),
               f_cell=z(3 * N), f_face=z(3 * nf), bc=z(3 * nb), kappa_E=z(N), kappa_B=z(N))
    lc.lc_loqd_grey_coefficients(h, c, c_dt, _dev(kappa), _dev(planck), _dev(E_prev), _dev(F_prev), _dev(fc),
                                 _dev(ff), _dev(bnd), _dev(sol[0]), _dev(sol[1]), _dev(sol[2]), out)
    o = {k: v.cpu().numpy() for k, v in out.items()}
    return dict(sigma=o["sigma"], source=o["source"], E_prev=o["E_prev"], k_side=o["k_side"].reshape(4, N).T,
                eta_side=o["eta_side"].reshape(4, N).T, F_prev=o["F_prev"], f_cell=o["f_cell"].reshape(3, N),
                f_face=o["f_face"].reshape(3, nf), bc=o["bc"].reshape(nb, 3), kappa_E=o["kappa_E"],
                kappa_B=o["kappa_B"])


def test_grey_coefficients_and_solve_match_the_oracle(lcmod):
    """From one multigroup solution (the oracle's), the library's grey
    coefficients equal the oracle's, and the grey solves agree."""
    lc, _ = lcmod
    from tests.test_oracle_loqd import _multigroup_case
    args = _multigroup_case(G=5, nx=14, ny=9, lx=2.8, ly=1.8, seed=31)
    nx, ny, lx, ly, c, c_dt, kappa, planck, E_prev, F_prev, f_cell, f_face, bc = args
    _say("case grey coefficients 14x9 G=5")
    sol = OL.solve(*args)
    ref = OL.grey_coefficients(nx, ny, c, c_dt, kappa, planck, E_prev, F_prev, f_cell, f_face, bc, *sol)
    got = _gpu_grey_coefficients(lc, *args, sol)
    for k in ref:
        scale = np.max(np.abs(ref[k])) or 1.0
        d = np.max(np.abs(got[k] - ref[k])) / scale
        assert d <= 1e-13, (k, d)
    g1 = lambda a: a[None]
    gs = _gpu_general(lc, nx, ny, lx, ly, c, c_dt, g1(got["sigma"]), g1(got["source"]), g1(got["k_side"]),
                      g1(got["eta_side"]), g1(got["F_prev"]), g1(got["f_cell"]), g1(got["f_face"]), g1(got["bc"]))
    rs = OL.solve_grey(nx, ny, lx, ly, c, c_dt, ref)
    _compare(gs, [g1(x) for x in rs], "grey solve")


def test_grey_equals_the_sum_of_the_groups_on_the_gpu(lcmod):
    """The whole low-order chain in the library -- multigroup solve, grey
    coefficients, grey solve -- on closures of the transport sweep of the
    16 x 16 workload (sweep, moments and face moments in the library too):
    the grey solution is the sum of the group solutions (1e-9 normwise), and
    agrees with the same chain in the oracle."""
    import torch
    lc, driver = lcmod
    prob = W.config(0)
    _say("case grey chain 16x16 G=4")
    s = driver.Solver(prob, prec=lc.LC_F64)
    s.enable_faces()
    s.reset()
    s.step_faces(1)
    G, N = prob.G, prob.cells
    c, c_dt, kap, pla, E_prev, F_prev = _loqd_inputs(prob)
    h = lc.Loqd(prob.nx, prob.ny, prob.lx, prob.ly, G)
    z = lambda n: torch.zeros(n, dtype=torch.float64, device="cuda")
    Ec, Ef, Ff = z(G * N), z(G * h.nf), z(G * h.nf)
    kd, pd, epd, fpd = s.kappa[0].reshape(-1), s.planck[0].reshape(-1), _dev(E_prev), _dev(F_prev)
    lc.lc_loqd_solve(h, c, c_dt, kd, pd, epd, fpd, s.f, s.ff, s.bnd, Ec, Ef, Ff)
    out = dict(sigma=z(N), source=z(N), E_prev=z(N), k_side=z(4 * N), eta_side=z(4 * N), F_prev=z(h.nf),
               f_cell=z(3 * N), f_face=z(3 * h.nf), bc=z(3 * h.nb))
    lc.lc_loqd_grey_coefficients(h, c, c_dt, kd, pd, epd, fpd, s.f, s.ff, s.bnd, Ec, Ef, Ff, out)
    hg = lc.Loqd(prob.nx, prob.ny, prob.lx, prob.ly, 1)
    gE, gEf, gF = z(N), z(hg.nf), z(hg.nf)
    lc.lc_loqd_solve_general(hg, c, c_dt, out["sigma"], out["source"], out["k_side"], out["eta_side"],
                             out["F_prev"], out["f_cell"], out["f_face"], out["bc"], gE, gEf, gF)
    grey = (gE.cpu().numpy()[None], gEf.cpu().numpy()[None], gF.cpu().numpy()[None])
    summed = tuple(x.cpu().numpy().reshape(G, -1).sum(0)[None] for x in (Ec, Ef, Ff))
    _compare(grey, summed, "grey vs sum of groups (library)")
    # the oracle's chain
    _, f, ff, bnd = _oracle_transport_closures(prob)
    f_cell, f_face, bc = OL.closures_from_transport(prob.nx, prob.ny, f, ff, bnd)
    oargs = (prob.nx, prob.ny, prob.lx, prob.ly, c, c_dt, kap, pla, E_prev, F_prev, f_cell, f_face, bc)
    osol = OL.solve(*oargs)
    ocoef = OL.grey_coefficients(prob.nx, prob.ny, c, c_dt, kap, pla, E_prev, F_prev, f_cell, f_face, bc, *osol)
    oref = OL.solve_grey(prob.nx, prob.ny, prob.lx, prob.ly, c, c_dt, ocoef)
    _compare(grey, tuple(x[None] for x in oref), "grey chain vs oracle")


# ---------------------------------------------------------------------------
# the grey problem with the energy balance, eq. (5)-(6)
# ---------------------------------------------------------------------------

def _gpu_meb(lc, geo, coefs, T_prev, c_v, a_R, newton_tol=1e-11, max_newton=50):
    """lc_loqd_grey_meb over independent grey problems (one per entry of
    coefs, oracle layouts), T starting at T_prev.  Returns (T, E_cell,
    E_face, F_face) [problems][...] and the Newton iterations."""
    import torch
    nx, ny, lx, ly, c, c_dt = geo
    G = len(coefs)
    h = lc.Loqd(nx, ny, lx, ly, G)
    st = lambda key, f=(lambda a: a): _dev(np.stack([f(cf[key]) for cf in coefs]))
    z = lambda n: torch.zeros(n, dtype=torch.float64, device="cuda")
    T = _dev(np.stack(T_prev))
    Ec, Ef, Ff = z(G * h.cells), z(G * h.nf), z(G * h.nf)
    nit, it, res = lc.lc_loqd_grey_meb(h, c, c_dt, st("kappa_E"), st("kappa_B"), st("E_prev"),
                                       st("k_side", lambda a: a.T), st("eta_side", lambda a: a.T), st("F_prev"),
                                       st("f_cell"), st("f_face"), st("bc"), _dev(np.stack(T_prev)), c_v, a_R, T,
                                       Ec, Ef, Ff, newton_tol=newton_tol, max_newton=max_newton)
    out = tuple(x.cpu().numpy().reshape(G, -1) for x in (T, Ec, Ef, Ff))
    return out, nit


def test_grey_meb_matches_the_oracle(lcmod):
    """Grey coefficients of a multigroup solution on a 33 x 20 grid (several
    reduction blocks, ragged tail), T^{n-1} in [0.05, 0.8] keV: T, E and F
    of the library's Newton iteration against the oracle's, 1e-9 normwise,
    and energy conserved by the library's solution."""
    lc, _ = lcmod
    from tests.test_oracle_loqd import A_R, C_V, _grey_meb_case, energy_defects
    geo, coef, Ts = _grey_meb_case(seed=51, nx=33, ny=20, lx=3.3, ly=2.0)
    _say("case grey energy balance 33x20")
    ref = OL.solve_grey_meb(*geo, coef, Ts, C_V, A_R, tol=1e-12)
    got, nit = _gpu_meb(lc, geo, [coef], [Ts], C_V, A_R)
    _say(f"  Newton iterations: library {nit}, oracle {ref[4]}")
    assert abs(nit - ref[4]) <= 1
    _compare(got, tuple(x[None] for x in ref[:4]), "grey energy balance")
    gained, inflow, meb = energy_defects(geo, coef, Ts, got[0][0], got[1][0], got[3][0], C_V, A_R)
    _say(f"  energy gained {gained:.6e} vs boundary inflow {inflow:.6e}; energy-balance residual {meb:.1e}")
    assert math.isclose(gained, inflow, rel_tol=1e-8) and meb <= 1e-9


def test_grey_meb_independent_problems(lcmod):
    """Three problems in one handle (G = 3), one of them starting far from
    its solution, each against its own oracle solve."""
    lc, _ = lcmod
    from tests.test_oracle_loqd import A_R, C_V, _grey_meb_case
    cases = [_grey_meb_case(seed=s, nx=14, ny=9, lx=1.4, ly=0.9) for s in (61, 62, 63)]
    geo = cases[0][0]
    coefs = [cs[1] for cs in cases]
    T_prev = [cs[2] for cs in cases]
    T_prev[2] = np.full_like(T_prev[2], 0.001)           # cold matter under the inflow
    _say("case grey energy balance 14x9, three problems")
    got, nit = _gpu_meb(lc, geo, coefs, T_prev, C_V, A_R)
    for g in range(3):
        ref = OL.solve_grey_meb(*geo, coefs[g], T_prev[g], C_V, A_R, tol=1e-12)
        _compare(tuple(x[g:g + 1] for x in got), tuple(x[None] for x in ref[:4]), f"problem {g}")


def test_grey_meb_whole_chain(lcmod):
    """Transport sweep, moments, multigroup LOQD, grey coefficients and the
    grey problem with the energy balance all in the library on the 16 x 16
    workload (c_v = 0.5917 a_R keV^-3 material), against the same chain in
    the oracle; the library's result conserves energy."""
    import torch
    lc, driver = lcmod
    from tests.test_oracle_loqd import A_R, C_V, energy_defects
    prob = W.config(0)
    _say("case grey energy balance whole chain 16x16 G=4")
    s = driver.Solver(prob, prec=lc.LC_F64)
    s.enable_faces()
    s.reset()
    s.step_faces(1)
    G, N = prob.G, prob.cells
    c, c_dt, kap, pla, E_prev, F_prev = _loqd_inputs(prob)
    h = lc.Loqd(prob.nx, prob.ny, prob.lx, prob.ly, G)
    z = lambda n: torch.zeros(n, dtype=torch.float64, device="cuda")
    Ec, Ef, Ff = z(G * N), z(G * h.nf), z(G * h.nf)
    kd, pd, epd, fpd = s.kappa[0].reshape(-1), s.planck[0].reshape(-1), _dev(E_prev), _dev(F_prev)
    lc.lc_loqd_solve(h, c, c_dt, kd, pd, epd, fpd, s.f, s.ff, s.bnd, Ec, Ef, Ff)
    out = dict(sigma=z(N), source=z(N), E_prev=z(N), k_side=z(4 * N), eta_side=z(4 * N), F_prev=z(h.nf),
               f_cell=z(3 * N), f_face=z(3 * h.nf), bc=z(3 * h.nb), kappa_E=z(N), kappa_B=z(N))
    lc.lc_loqd_grey_coefficients(h, c, c_dt, kd, pd, epd, fpd, s.f, s.ff, s.bnd, Ec, Ef, Ff, out)
    hg = lc.Loqd(prob.nx, prob.ny, prob.lx, prob.ly, 1)
    Ts = np.asarray(prob.T[0], dtype=np.float64)
    T = _dev(Ts)
    gE, gEf, gF = z(N), z(hg.nf), z(hg.nf)
    nit, _, _ = lc.lc_loqd_grey_meb(hg, c, c_dt, out["kappa_E"], out["kappa_B"], out["E_prev"], out["k_side"],
                                    out["eta_side"], out["F_prev"], out["f_cell"], out["f_face"], out["bc"],
                                    _dev(Ts), C_V, A_R, T, gE, gEf, gF, newton_tol=1e-11)
    got = tuple(x.cpu().numpy()[None] for x in (T, gE, gEf, gF))
    # the oracle's chain
    _, f, ff, bnd = _oracle_transport_closures(prob)
    f_cell, f_face, bc = OL.closures_from_transport(prob.nx, prob.ny, f, ff, bnd)
    osol = OL.solve(prob.nx, prob.ny, prob.lx, prob.ly, c, c_dt, kap, pla, E_prev, F_prev, f_cell, f_face, bc)
    ocoef = OL.grey_coefficients(prob.nx, prob.ny, c, c_dt, kap, pla, E_prev, F_prev, f_cell, f_face, bc, *osol)
    geo = (prob.nx, prob.ny, prob.lx, prob.ly, c, c_dt)
    ref = OL.solve_grey_meb(*geo, ocoef, Ts, C_V, A_R, tol=1e-12)
    _say(f"  Newton iterations: library {nit}, oracle {ref[4]}")
    _compare(got, tuple(x[None] for x in ref[:4]), "grey energy balance chain")
    gained, inflow, meb = energy_defects(geo, ocoef, Ts, got[0][0], got[1][0], got[3][0], C_V, A_R)
    _say(f"  energy gained {gained:.6e} vs boundary inflow {inflow:.6e}; energy-balance residual {meb:.1e}")
    assert math.isclose(gained, inflow, rel_tol=1e-8) and meb <= 1e-9


def test_grey_meb_is_deterministic_and_reports_non_convergence(lcmod):
    lc, _ = lcmod
    from tests.test_oracle_loqd import A_R, C_V, _grey_meb_case
    geo, coef, Ts = _grey_meb_case(seed=71, nx=12, ny=7, lx=1.2, ly=0.7)
    a, _ = _gpu_meb(lc, geo, [coef], [Ts], C_V, A_R)
    b, _ = _gpu_meb(lc, geo, [coef], [Ts], C_V, A_R)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    with pytest.raises(lc.LcError) as e:
        _gpu_meb(lc, geo, [coef], [Ts], C_V, A_R, newton_tol=0.0, max_newton=1)
    assert e.value.status == lc.LC_ERR_UNSUPPORTED


def test_loqd_warm_start(lcmod):
    """A second solve started from the first's solution: the same result
    within rtol, in fewer iterations."""
    import torch
    lc, _ = lcmod
    args = _random_groups(33, 20, 3.3, 1.0, 5, seed=21)
    nx, ny, lx, ly, c, c_dt, kappa, planck, E_prev, F_prev, f_cell, f_face, bc = args
    G = kappa.shape[0]
    fc, ff, bnd = _gpu_layouts(nx, ny, f_cell, f_face, bc)
    h = lc.Loqd(nx, ny, lx, ly, G)
    z = lambda n: torch.zeros(n, dtype=torch.float64, device="cuda")
    Ec, Ef, Ff = z(G * h.cells), z(G * h.nf), z(G * h.nf)
    ins = [_dev(a) for a in (kappa, planck, E_prev, F_prev, fc, ff, bnd)]
    it0, _ = lc.lc_loqd_solve(h, c, c_dt, *ins, Ec, Ef, Ff)
    cold = (Ec.cpu().numpy().reshape(G, -1), Ef.cpu().numpy().reshape(G, -1), Ff.cpu().numpy().reshape(G, -1))
    lc.lc_loqd_set_warm_start(h, True)
    it1, res = lc.lc_loqd_solve(h, c, c_dt, *ins, Ec, Ef, Ff)
    warm = (Ec.cpu().numpy().reshape(G, -1), Ef.cpu().numpy().reshape(G, -1), Ff.cpu().numpy().reshape(G, -1))
    _say(f"case loqd warm start: iterations cold {it0}, warm {it1}")
    assert it1 < it0 and np.all(res <= 1e-13)
    _compare(warm, cold, "warm vs cold")



@pytest.mark.parametrize("nx,ny", [(50, 45), (70, 60)])
def test_loqd_mid_size_one_workgroup_form(lcmod, nx, ny):
    """Face systems of 4,595 and 8,530 faces: above the register form's
    4096, below the one-workgroup limit -- the form that keeps its vectors
    in global memory (16 and 32 rows a thread) -- against the oracle."""
    lc, _ = lcmod
    nf = OL.n_faces(nx, ny)
    assert 4096 < nf <= 16384
    args = _random_groups(nx, ny, nx * 0.1, ny * 0.1, 2, seed=nx + ny)
    _say(f"case loqd random {nx}x{ny} G=2 ({nf} faces, one workgroup, vectors in global memory)")
    ref = OL.solve(*args)
    got, it, res = _gpu_solve(lc, *args)
    _say(f"  {it} iterations, residuals {np.max(res):.1e}")
    _compare(got, ref, "mid-size")


def test_loqd_register_form_at_its_largest(lcmod):
    """45 x 44 cells, 4,049 faces: eight rows a thread, the register form's
    largest systems, whose products, r^ and inverse diagonal take about
    130 KB of LDS -- against the oracle."""
    lc, _ = lcmod
    nx, ny = 45, 44
    nf = OL.n_faces(nx, ny)
    assert 3584 < nf <= 4096
    args = _random_groups(nx, ny, nx * 0.1, ny * 0.1, 2, seed=89)
    _say(f"case loqd random {nx}x{ny} G=2 ({nf} faces, one workgroup, 8 rows a thread)")
    ref = OL.solve(*args)
    got, it, res = _gpu_solve(lc, *args)
    _say(f"  {it} iterations, residuals {np.max(res):.1e}")
    _compare(got, ref, "largest register form")


def test_loqd_large_system_takes_the_block_path(lcmod):
    """A face system above the one-workgroup size (95 x 90 cells, 17,285
    faces) through the automatic choice, against the oracle."""
    lc, _ = lcmod
    args = _random_groups(95, 90, 6.0, 5.7, 1, seed=95)
    _say("case loqd random 95x90 G=1 (automatic: block path)")
    assert OL.n_faces(95, 90) > 16384
    ref = OL.solve(*args)
    got, it, res = _gpu_solve(lc, *args)
    _say(f"  {it} iterations, residuals {np.max(res):.1e}")
    _compare(got, ref, "large")



@pytest.mark.parametrize("nx", [40, 30])
def test_loqd_at_the_study_size(lcmod, nx):
    """The multigroup solve at the size of the paper's finest material grid
    (40 x 40 cells, 17 groups; and 30 x 30, whose 1,860 faces take the
    4-row register form) with physically shaped data: the Fleck-Cummings
    opacity and Planck functions of a temperature front, closures of the
    random-tensor kind, against the oracle's direct solve."""
    lc, _ = lcmod
    from oracle import material as OMAT
    ny = nx
    h = 6.0 / nx
    rng = np.random.default_rng(404)
    x = (np.arange(nx) + 0.5) * h
    T = np.tile(np.where(x < 1.5, 0.8, 0.002) + 0.05 * rng.random(nx), ny)
    p = W.fc_mlqd(h, 0.05, 8, 2, 17, nu_lo=0.3, nu_hi=30.0)
    kappa = OMAT.fc_opacity(p.nu, T)
    planck = W.group_planck(p.edges, T)
    args = list(_random_groups(nx, ny, 6.0, 6.0, 17, seed=41))
    args[6], args[7] = kappa, planck
    args[8] = 4 * math.pi * planck / W.C_LIGHT
    _say(f"case loqd {nx}x{ny} G=17 Fleck-Cummings material ({OL.n_faces(nx, ny)} faces)")
    ref = OL.solve(*args)
    got, it, res = _gpu_solve(lc, *args)
    _say(f"  {it} iterations, residuals {np.max(res):.1e}")
    _compare(got, ref, "study size")
