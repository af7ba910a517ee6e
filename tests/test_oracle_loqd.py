"""Pins of the LOQD oracle (oracle/loqd.py): the finite-volume reading of the
multigroup low-order equations, eq. (4), for one backward-Euler step.

* A linear energy density with constant coefficients (anisotropic Eddington
  tensor with a cross term, a previous-step flux, unequal cell sides) is
  reproduced exactly in the cells and on the faces, flux included.
* A smooth manufactured solution with varying opacity and Eddington tensor
  (sources derived symbolically) converges at second order in cells and
  face fluxes.
* Isotropic equilibrium with the quadrature's own boundary factors stays in
  equilibrium: E = 4 pi B / c, F = 0.
* Every cell balances with the returned fluxes, both cells next to a face
  give it the same flux, and the sources equal the outflow over the
  boundary (conservation).
* With opacities up to 1e8 per cm the solution equals a dense solve of the
  system with the cell unknowns eliminated by hand (full accuracy in
  optically thick cells).
* Planted mistakes (cross-term sign, cell tensor on the face, previous-step
  flux dropped, boundary-condition sign) fail the pins."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import loqd


def _faces_geometry(nx, ny, lx, ly):
    """Centre, normal axis (0 = x, 1 = y) and the two end points of every face
    in the all-face numbering."""
    hx, hy = lx / nx, ly / ny
    nf = loqd.n_faces(nx, ny)
    cen = np.zeros((nf, 2))
    axis = np.zeros(nf, dtype=int)
    cf = loqd.cell_faces(nx, ny)
    for iy in range(ny):
        for ix in range(nx):
            L, R, B, T = cf[iy * nx + ix]
            x0, x1, y0, y1 = ix * hx, (ix + 1) * hx, iy * hy, (iy + 1) * hy
            cen[L] = (x0, (y0 + y1) / 2); cen[R] = (x1, (y0 + y1) / 2)
            cen[B] = ((x0 + x1) / 2, y0); cen[T] = ((x0 + x1) / 2, y1)
            axis[B] = axis[T] = 1
    return cen, axis


def _outward_sign(nx, ny):
    """+1 where a boundary face's outward normal points along +axis."""
    nb = 2 * (nx + ny)
    s = np.ones(nb)
    s[:ny] = -1.0                         # x = 0
    s[2 * ny:2 * ny + nx] = -1.0          # y = 0
    return s


# ---------------------------------------------------------------------------
# linear fields are exact
# ---------------------------------------------------------------------------

def _linear_case(nx=6, ny=4, lx=1.2, ly=1.0):
    c, c_dt, kap = 3.0, 0.5, 2.0
    kt = kap + 1.0 / c_dt
    a0, bx, by = 2.0, 0.7, -0.4
    T = np.array([[0.40, 0.12], [0.12, 0.35]])
    Fp = np.array([0.3, -0.2])
    gradE = np.array([bx, by])
    F = (Fp / c_dt - c * T @ gradE) / kt                     # constant flux
    N = nx * ny
    hx, hy = lx / nx, ly / ny
    xc = (np.arange(nx) + 0.5) * hx
    yc = (np.arange(ny) + 0.5) * hy
    X, Y = np.meshgrid(xc, yc)
    Ec = (a0 + bx * X + by * Y).ravel()
    S = c * kt * Ec                                          # div F = 0
    E_prev = 0.5 * Ec
    planck = (S - c * E_prev / c_dt) / (4 * math.pi * kap)
    cen, axis = _faces_geometry(nx, ny, lx, ly)
    nf = len(axis)
    Ef = a0 + bx * cen[:, 0] + by * cen[:, 1]
    F_face = F[axis]
    F_prev = Fp[axis]
    f_cell = np.array([np.full(N, T[0, 0]), np.full(N, T[0, 1]), np.full(N, T[1, 1])])
    f_face = np.array([np.full(nf, T[0, 0]), np.full(nf, T[0, 1]), np.full(nf, T[1, 1])])
    nint = loqd.n_interior(nx, ny)
    sgn = _outward_sign(nx, ny)
    nb = 2 * (nx + ny)
    C = 0.45 + 0.05 * np.cos(np.arange(nb))
    Pm = 0.3 + 0.1 * np.sin(np.arange(nb))
    nF = sgn * F_face[nint:]
    Jm = C * (c * Ef[nint:] - Pm) - nF                       # the boundary condition holds exactly
    bc = np.stack([C, Pm, Jm], axis=1)
    args = (nx, ny, lx, ly, c, c_dt, np.full(N, kap), planck, E_prev, F_prev, f_cell, f_face, bc)
    return args, (Ec, Ef, F_face)


def test_linear_field_is_reproduced_exactly():
    args, (Ec, Ef, Ff) = _linear_case()
    e, ef, ff = loqd.solve_group(*args)
    assert np.allclose(e, Ec, rtol=1e-12, atol=0)
    assert np.allclose(ef, Ef, rtol=1e-12, atol=0)
    assert np.allclose(ff, Ff, rtol=1e-11, atol=1e-12)


# ---------------------------------------------------------------------------
# second-order convergence on a smooth manufactured solution
# ---------------------------------------------------------------------------

def _manufactured():
    import sympy as S
    x, y = S.symbols("x y")
    c, c_dt = 2.0, 0.8
    E = 1 + 0.5 * S.sin(2 * x + 0.3) * S.cos(1.5 * y) + 0.2 * x * y
    kap = 1.5 + 0.8 * S.sin(x + 2 * y) ** 2
    kt = kap + 1 / c_dt
    fxx = S.Rational(1, 3) + 0.1 * S.cos(x) * S.sin(y)
    fyy = S.Rational(1, 3) - 0.05 * S.sin(2 * x)
    fxy = 0.08 * S.sin(x + y)
    Fpx = 0.2 * S.cos(y) * x
    Fpy = -0.1 * S.sin(x) + 0.05
    Fx = (Fpx / c_dt - c * (S.diff(fxx * E, x) + S.diff(fxy * E, y))) / kt
    Fy = (Fpy / c_dt - c * (S.diff(fxy * E, x) + S.diff(fyy * E, y))) / kt
    src = c * kt * E + S.diff(Fx, x) + S.diff(Fy, y)
    f = {k: S.lambdify((x, y), v, "numpy") for k, v in dict(E=E, kap=kap, fxx=fxx, fyy=fyy, fxy=fxy, Fpx=Fpx,
                                                            Fpy=Fpy, Fx=Fx, Fy=Fy, src=src).items()}
    return f, c, c_dt


def _gl(n=4):
    t, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (t + 1.0), 0.5 * w


def _cell_avg(fn, nx, ny, lx, ly):
    hx, hy = lx / nx, ly / ny
    t, w = _gl()
    out = np.zeros(nx * ny)
    for iy in range(ny):
        for ix in range(nx):
            X, Y = np.meshgrid(ix * hx + t * hx, iy * hy + t * hy)
            out[iy * nx + ix] = np.sum(np.outer(w, w) * np.broadcast_to(fn(X, Y), X.shape))
    return out


def _face_avg(fn, nx, ny, lx, ly):
    hx, hy = lx / nx, ly / ny
    cen, axis = _faces_geometry(nx, ny, lx, ly)
    t, w = _gl()
    out = np.zeros(len(axis))
    for f in range(len(axis)):
        if axis[f] == 0:
            xs, ys = np.full_like(t, cen[f, 0]), cen[f, 1] - hy / 2 + t * hy
        else:
            xs, ys = cen[f, 0] - hx / 2 + t * hx, np.full_like(t, cen[f, 1])
        out[f] = np.sum(w * np.broadcast_to(fn(xs, ys), xs.shape))
    return out


def _manufactured_case(n, lx=1.0, ly=0.8):
    f, c, c_dt = _manufactured()
    nx = ny = n
    avg = lambda k: _cell_avg(f[k], nx, ny, lx, ly)
    favg = lambda k: _face_avg(f[k], nx, ny, lx, ly)
    _, axis = _faces_geometry(nx, ny, lx, ly)
    kap = avg("kap")
    Ec = avg("E")
    S = avg("src")
    E_prev = S * c_dt / c                                   # the whole source through E^{n-1}
    planck = np.zeros_like(Ec)
    f_cell = np.array([avg("fxx"), avg("fxy"), avg("fyy")])
    f_face = np.array([favg("fxx"), favg("fxy"), favg("fyy")])
    F_prev = np.where(axis == 0, favg("Fpx"), favg("Fpy"))
    F_face = np.where(axis == 0, favg("Fx"), favg("Fy"))
    Ef = favg("E")
    nint = loqd.n_interior(nx, ny)
    sgn = _outward_sign(nx, ny)
    C = np.full(2 * (nx + ny), 0.5)
    Pm = np.zeros(2 * (nx + ny))
    Jm = C * c * Ef[nint:] - sgn * F_face[nint:]
    bc = np.stack([C, Pm, Jm], axis=1)
    args = (nx, ny, lx, ly, c, c_dt, kap, planck, E_prev, F_prev, f_cell, f_face, bc)
    return args, (Ec, Ef, F_face), lx * ly / (nx * ny)


def _errors(n):
    args, (Ec, Ef, Ff), area = _manufactured_case(n)
    e, ef, ff = loqd.solve_group(*args)
    return (math.sqrt(np.sum((e - Ec) ** 2) * area), float(np.max(np.abs(ff - Ff))))


def test_second_order_convergence_on_a_manufactured_solution():
    errs = [_errors(n) for n in (8, 16, 32)]
    rates_E = [math.log2(a[0] / b[0]) for a, b in zip(errs, errs[1:])]
    rates_F = [math.log2(a[1] / b[1]) for a, b in zip(errs, errs[1:])]
    assert all(r > 1.8 for r in rates_E), (errs, rates_E)
    assert rates_F[-1] > 1.5, (errs, rates_F)
    assert errs[-1][0] < 1e-3


# ---------------------------------------------------------------------------
# isotropic equilibrium
# ---------------------------------------------------------------------------

def test_isotropic_equilibrium_is_kept():
    nx, ny, lx, ly = 5, 3, 1.0, 0.6
    c, c_dt = 299.792458, 3.0
    phi, mu, om = W.product_quadrature(16, 2)
    ox = (np.cos(phi)[:, None] * np.sqrt(1 - mu ** 2)[None, :]).ravel()
    oy = (np.sin(phi)[:, None] * np.sqrt(1 - mu ** 2)[None, :]).ravel()
    normals = W.boundary_faces(nx, ny)
    Bv = 0.37
    N = nx * ny
    nf = loqd.n_faces(nx, ny)
    bc = []
    for n in normals:
        dn = ox * n[0] + oy * n[1]
        out, inn = dn > 0, dn < 0
        C_iso = np.sum(om[out] * dn[out]) / np.sum(om[out])
        bc.append((C_iso, np.sum(om[inn]) * Bv, np.sum(om[inn] * np.abs(dn[inn])) * Bv))
    bc = np.array(bc)
    third = np.full((3, N), 1 / 3); third[1] = 0.0
    thirdf = np.full((3, nf), 1 / 3); thirdf[1] = 0.0
    kap = np.linspace(0.5, 3.0, N)
    e, ef, ff = loqd.solve_group(nx, ny, lx, ly, c, c_dt, kap, np.full(N, Bv), np.full(N, 4 * math.pi * Bv / c),
                                 np.zeros(nf), third, thirdf, bc)
    E0 = 4 * math.pi * Bv / c
    assert np.allclose(e, E0, rtol=1e-13) and np.allclose(ef, E0, rtol=1e-13)
    assert np.max(np.abs(ff)) < 1e-12 * c * E0


# ---------------------------------------------------------------------------
# conservation
# ---------------------------------------------------------------------------

def _random_case(nx=7, ny=5, lx=1.4, ly=0.7, seed=3):
    rng = np.random.default_rng(seed)
    N, nf = nx * ny, loqd.n_faces(nx, ny)
    c, c_dt = 5.0, 0.7
    kap = rng.uniform(0.1, 10.0, N)
    planck = rng.uniform(0.0, 1.0, N)
    E_prev = rng.uniform(0.0, 1.0, N)
    F_prev = rng.uniform(-0.5, 0.5, nf)

    def tensors(n):
        a = rng.uniform(0.15, 0.6, n)
        d = rng.uniform(0.15, 0.6, n)
        b = rng.uniform(-0.5, 0.5, n) * np.sqrt(a * d)
        return np.array([a, b, d])
    bc = np.stack([rng.uniform(0.3, 0.7, 2 * (nx + ny)), rng.uniform(0, 1, 2 * (nx + ny)),
                   rng.uniform(0, 0.5, 2 * (nx + ny))], axis=1)
    return (nx, ny, lx, ly, c, c_dt, kap, planck, E_prev, F_prev, tensors(N), tensors(nf), bc)


def test_discrete_conservation():
    args = _random_case()
    nx, ny, lx, ly, c, c_dt, kap, planck, E_prev, F_prev, f_cell, f_face, bc = args
    e, ef, ff = loqd.solve_group(*args)
    hx, hy = lx / nx, ly / ny
    kt = kap + 1.0 / c_dt
    src = 4 * math.pi * kap * planck + c * E_prev / c_dt
    cf = loqd.cell_faces(nx, ny)
    L, R, B, T = cf.T
    div = (ff[R] - ff[L]) / hx + (ff[T] - ff[B]) / hy
    assert np.allclose(c * kt * e + div, src, rtol=1e-11, atol=1e-12 * np.max(src))
    # the other cell next to each interior face gives the same flux
    _, _, k_side, eta_side = loqd.multigroup_coefficients(c, c_dt, kap, planck, E_prev)
    q = loqd._Group(nx, ny, lx, ly, c, c_dt, k_side, eta_side, F_prev, f_cell, f_face)
    x = np.concatenate([e, ef])
    lo, hi, _ = loqd.face_cells(nx, ny)
    for fidx in range(loqd.n_interior(nx, ny)):
        terms, const = loqd.half_cell_flux(q, hi[fidx], fidx)
        other = sum(v * x[col] for col, v in terms) + const
        assert abs(other - ff[fidx]) <= 1e-10 * (1 + abs(ff[fidx]))
    # sources = absorption + outflow through the boundary
    nint = loqd.n_interior(nx, ny)
    sgn = _outward_sign(nx, ny)
    lens = np.concatenate([np.full(ny, hy), np.full(ny, hy), np.full(nx, hx), np.full(nx, hx)])
    outflow = np.sum(sgn * ff[nint:] * lens)
    assert math.isclose(np.sum((src - c * kt * e) * hx * hy), outflow, rel_tol=1e-10, abs_tol=1e-12)
    # and the boundary condition holds
    C, Pm, Jm = bc.T
    assert np.allclose(sgn * ff[nint:], C * (c * ef[nint:] - Pm) - Jm, rtol=1e-10, atol=1e-12)


# ---------------------------------------------------------------------------
# accuracy with optically thick cells
# ---------------------------------------------------------------------------

def test_thick_cells_keep_full_accuracy():
    """Opacities from 0.1 to 1e8 per cm (the Fleck-Cummings law at 1 eV gives
    such values in the lowest groups): the oracle's solution equals a dense
    solve of the system with the cell unknowns eliminated by hand (each cell
    equation holds only E_i and its own faces), to 1e-12 normwise.  An
    unscaled direct solve of the full system is off by about 1e-3 here."""
    import scipy.sparse.linalg as spla
    args = list(_random_case(nx=12, ny=9, lx=1.2, ly=0.9, seed=8))
    rng = np.random.default_rng(8)
    args[6] = 10.0 ** rng.uniform(-1, 8, 12 * 9)
    args[5] = 3.0
    args[4] = 299.792458
    e, ef, ff = loqd.solve_group(*args)
    A, b, q = loqd.assemble_group(*args)
    N = q.N
    Ad = A.toarray()
    assert np.count_nonzero(Ad[:N, :N] - np.diag(np.diag(Ad[:N, :N]))) == 0
    dc = np.diag(Ad[:N, :N])
    S = Ad[N:, N:] - Ad[N:, :N] @ (Ad[:N, N:] / dc[:, None])
    xf = np.linalg.solve(S, b[N:] - Ad[N:, :N] @ (b[:N] / dc))
    xc = (b[:N] - Ad[:N, N:] @ xf) / dc
    ref = np.concatenate([xc, xf])
    got = np.concatenate([e, ef])
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    plain = spla.spsolve(A.tocsc(), b)
    assert np.max(np.abs(plain - ref)) > 1e3 * np.max(np.abs(got - ref))   # the scaling matters here


# ---------------------------------------------------------------------------
# planted mistakes
# ---------------------------------------------------------------------------

_orig_flux = loqd.half_cell_flux


def _cross_sign_flipped(q, i, face):
    terms, const = _orig_flux(q, i, face)
    return terms[:2] + [(col, -v) for col, v in terms[2:]], const


def _cell_tensor_on_face(q, i, face):
    terms, const = _orig_flux(q, i, face)
    L, R, B, T = q.cf[i]
    out = []
    for col, v in terms[:2]:
        if col >= q.N and col - q.N in (L, R):
            v = v * q.fxx[i] / q.gxx[col - q.N]
        elif col >= q.N and col - q.N in (B, T) and face in (B, T):
            v = v * q.fyy[i] / q.gyy[col - q.N]
        out.append((col, v))
    return out + terms[2:], const


def _no_previous_flux(q, i, face):
    terms, _ = _orig_flux(q, i, face)
    return terms, 0.0


@pytest.mark.parametrize("bad", [_cross_sign_flipped, _cell_tensor_on_face, _no_previous_flux])
def test_planted_flux_mistakes_are_caught(monkeypatch, bad):
    monkeypatch.setattr(loqd, "half_cell_flux", bad)
    caught = 0
    for pin in (test_linear_field_is_reproduced_exactly, test_second_order_convergence_on_a_manufactured_solution):
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught >= 1


def test_planted_boundary_mistake_is_caught(monkeypatch):
    monkeypatch.setattr(loqd, "boundary_condition", lambda C, Pm, Jm, c: (C * c, -C * Pm + Jm))
    with pytest.raises(AssertionError):
        test_linear_field_is_reproduced_exactly()


# ---------------------------------------------------------------------------
# effective grey equations, eq. (5): consistency with the multigroup scheme
# ---------------------------------------------------------------------------

def _multigroup_case(G=4, nx=9, ny=7, lx=1.8, ly=1.4, seed=21):
    rng = np.random.default_rng(seed)
    N, nf = nx * ny, loqd.n_faces(nx, ny)
    nb = 2 * (nx + ny)
    c, c_dt = 299.792458, 0.6
    kappa = 10.0 ** rng.uniform(-1, 4, (G, N))
    planck = rng.uniform(0, 1, (G, N)) * 10.0 ** rng.uniform(-3, 0, (G, 1))
    E_prev = rng.uniform(0, 1, (G, N)) * 4 * math.pi / c * 10.0 ** rng.uniform(-3, 0, (G, 1))
    F_prev = rng.uniform(-0.3, 0.3, (G, nf))

    def tensors(n):
        a = rng.uniform(0.15, 0.6, (G, n))
        dd = rng.uniform(0.15, 0.6, (G, n))
        b = rng.uniform(-0.5, 0.5, (G, n)) * np.sqrt(a * dd)
        return np.stack([a, b, dd], axis=1)
    bc = np.stack([rng.uniform(0.3, 0.7, (G, nb)), rng.uniform(0, 1, (G, nb)), rng.uniform(0, 0.5, (G, nb))], axis=2)
    return (nx, ny, lx, ly, c, c_dt, kappa, planck, E_prev, F_prev, tensors(N), tensors(nf), bc)


@pytest.mark.parametrize("seed", [21, 22])
def test_grey_solution_is_the_sum_of_the_group_solutions(seed):
    """With closures from the multigroup solution the grey scheme, eq. (5),
    reproduces sum_g E_g in cells and on faces and sum_g F_g on faces (the
    paper's algebraic consistency of the two schemes)."""
    args = _multigroup_case(seed=seed)
    nx, ny, lx, ly, c, c_dt, kappa, planck, E_prev, F_prev, f_cell, f_face, bc = args
    Ec, Ef, Ff = loqd.solve(*args)
    coef = loqd.grey_coefficients(nx, ny, c, c_dt, kappa, planck, E_prev, F_prev, f_cell, f_face, bc, Ec, Ef, Ff)
    e, ef, ff = loqd.solve_grey(nx, ny, lx, ly, c, c_dt, coef)
    for got, want in ((e, Ec.sum(0)), (ef, Ef.sum(0)), (ff, Ff.sum(0))):
        assert np.max(np.abs(got - want)) <= 1e-10 * np.max(np.abs(want))


def test_grey_closures_special_cases_and_a_face_by_hand():
    """Group-independent opacity: K_R = kappa and eta = 0 on every side.  A
    two-group face worked by hand: kappa = (1, 3), F = (2, -1), E_f = 4:
    K_R = (1*2 + 3*1)/3 = 5/3, eta = ((1 - 5/3) 2 + (3 - 5/3)(-1)) / 4 = -2/3."""
    args = list(_multigroup_case(G=3, seed=5))
    nx, ny = args[0], args[1]
    args[6] = np.repeat(args[6][:1], 3, axis=0)               # the same opacity in every group
    Ec, Ef, Ff = loqd.solve(*args)
    coef = loqd.grey_coefficients(nx, ny, args[4], args[5], args[6], args[7], args[8], args[9], args[10],
                                  args[11], args[12], Ec, Ef, Ff)
    assert np.allclose(coef["k_side"], (args[6][0] + 1 / args[5])[:, None], rtol=1e-13)
    assert np.max(np.abs(coef["eta_side"])) <= 1e-12 * np.max(args[6]) * np.max(np.abs(Ff)) / np.min(np.abs(Ef.sum(0)))
    # the hand-worked face: a 1 x 1 grid, two groups, face L of the cell
    nf = loqd.n_faces(1, 1)
    kap = np.array([[1.0], [3.0]])
    Fface = np.zeros((2, nf)); Fface[:, 0] = (2.0, -1.0)
    Eface = np.ones((2, nf)); Eface[:, 0] = (1.5, 2.5)
    coef = loqd.grey_coefficients(1, 1, 1.0, 1.0, kap, np.ones((2, 1)), np.zeros((2, 1)), np.zeros((2, nf)),
                                  np.full((2, 3, 1), 1 / 3), np.full((2, 3, nf), 1 / 3), np.full((2, 4, 3), 0.5),
                                  np.ones((2, 1)), Eface, Fface)
    assert math.isclose(coef["k_side"][0, 0], 5 / 3 + 1.0, rel_tol=1e-14)
    assert math.isclose(coef["eta_side"][0, 0], -2 / 3, rel_tol=1e-14)


def _eta_on_cell_energy(nx, ny, c, c_dt, kappa, planck, E_prev, F_prev, f_cell, f_face, bc, E_cell, E_face,
                        F_face):
    # mistake: eta formed with the cell's grey E instead of the face's
    coef = _orig_grey(nx, ny, c, c_dt, kappa, planck, E_prev, F_prev, f_cell, f_face, bc, E_cell, E_face, F_face)
    cf = loqd.cell_faces(nx, ny)
    Ef, E = E_face.sum(0), E_cell.sum(0)
    coef["eta_side"] = coef["eta_side"] * Ef[cf] / E[:, None]
    return coef


_orig_grey = loqd.grey_coefficients


def test_planted_grey_mistake_is_caught(monkeypatch):
    monkeypatch.setattr(loqd, "grey_coefficients", _eta_on_cell_energy)
    with pytest.raises(AssertionError):
        test_grey_solution_is_the_sum_of_the_group_solutions(21)


# ---------------------------------------------------------------------------
# effective grey problem with the energy balance, eq. (5)-(6)
# ---------------------------------------------------------------------------

A_R = W.A_RAD
C_V = 0.5917 * A_R          # eps = c_v T with c_v = 0.5917 a_R (1 keV)^3


def _grey_meb_case(seed=41, nx=10, ny=8, lx=1.0, ly=0.8):
    """Grey coefficients from a multigroup solution of physically shaped
    data (Fleck-Cummings opacity and group Planck functions of a random
    temperature field, inflow at x = 0)."""
    rng = np.random.default_rng(seed)
    Ts = rng.uniform(0.05, 0.8, nx * ny)
    p = W.make_problem(nx, ny, lx, ly, 8, 2, 5, 0.001, 20.0, 0.05, 0.6, [Ts], name="meb")
    c = W.C_LIGHT
    nf = loqd.n_faces(nx, ny)
    E_prev = 4 * math.pi * p.planck[0] / c
    F_prev = np.zeros((p.G, nf))
    G, N = p.G, nx * ny
    f_cell = np.zeros((G, 3, N)); f_cell[:, 0] = f_cell[:, 2] = 1 / 3
    f_face = np.zeros((G, 3, nf)); f_face[:, 0] = f_face[:, 2] = 1 / 3
    nb = 2 * (nx + ny)
    bc = np.zeros((G, nb, 3)); bc[:, :, 0] = 0.5
    bc[:, :ny, 1] = 2 * math.pi * W.group_planck(p.edges, np.array([1.0]))[:, 0][:, None]   # x = 0: Phi^-
    bc[:, :ny, 2] = 0.5 * bc[:, :ny, 1]                                                     # J^- = Phi^-/2
    args = (nx, ny, lx, ly, c, p.c_dt, p.kappa[0], p.planck[0], E_prev, F_prev, f_cell, f_face, bc)
    sol = loqd.solve(*args)
    coef = loqd.grey_coefficients(nx, ny, c, p.c_dt, p.kappa[0], p.planck[0], E_prev, F_prev, f_cell, f_face, bc,
                                  *sol)
    return (nx, ny, lx, ly, c, p.c_dt), coef, Ts


def energy_defects(geo, coef, T_prev, T, E, F, c_v, a_R):
    """(energy gained by matter and radiation over the step, energy that
    crossed the boundary in it, the largest cell residual of the energy
    balance relative to c_v T / dt) of a solution of the grey problem."""
    nx, ny, lx, ly, c, c_dt = geo
    dt = c_dt / c
    hx, hy = lx / nx, ly / ny
    gained = np.sum(c_v * (T - T_prev) + (E - coef["E_prev"])) * hx * hy
    nint = loqd.n_interior(nx, ny)
    sgn = np.concatenate([-np.ones(ny), np.ones(ny), -np.ones(nx), np.ones(nx)])
    lens = np.concatenate([np.full(ny, hy), np.full(ny, hy), np.full(nx, hx), np.full(nx, hx)])
    inflow = -dt * np.sum(sgn * F[nint:] * lens)
    meb = c_v * (T - T_prev) / dt - (c * coef["kappa_E"] * E - c * coef["kappa_B"] * a_R * T ** 4)
    return gained, inflow, np.max(np.abs(meb)) / np.max(np.abs(c_v * T / dt))


def test_grey_energy_balance_conserves_energy():
    """Summed over the cells, the change of material plus radiation energy
    over the step equals the energy that crosses the boundary (discrete
    balance and energy balance add up exactly once Newton has converged)."""
    geo, coef, Ts = _grey_meb_case()
    nx, ny, lx, ly, c, c_dt = geo
    T, E, Ef, F, it = loqd.solve_grey_meb(*geo, coef, Ts, C_V, A_R)
    assert it < 20
    gained, inflow, meb = energy_defects(geo, coef, Ts, T, E, F, C_V, A_R)
    assert math.isclose(gained, inflow, rel_tol=1e-9, abs_tol=1e-12 * np.sum(C_V * T) * geo[2] * geo[3] / Ts.size)
    # and the energy balance of every cell holds with the converged T
    assert meb <= 1e-9


def test_grey_energy_balance_keeps_equilibrium():
    """Uniform temperature, radiation in equilibrium with it, and an
    isotropic equilibrium boundary: nothing changes."""
    nx, ny, lx, ly = 6, 5, 1.2, 1.0
    c, c_dt, Teq = W.C_LIGHT, 0.6, 0.37
    N, nf, nb = nx * ny, loqd.n_faces(nx, ny), 2 * (nx + ny)
    Eeq = A_R * Teq ** 4
    kap = np.linspace(0.5, 20.0, N)
    coef = dict(kappa_E=kap, kappa_B=kap, E_prev=np.full(N, Eeq), k_side=np.repeat((kap + 1 / c_dt)[:, None], 4, 1),
                eta_side=np.zeros((N, 4)), F_prev=np.zeros(nf), f_cell=np.array([np.full(N, 1 / 3), np.zeros(N),
                                                                                  np.full(N, 1 / 3)]),
                f_face=np.array([np.full(nf, 1 / 3), np.zeros(nf), np.full(nf, 1 / 3)]),
                bc=np.stack([np.full(nb, 0.5), np.full(nb, c * Eeq / 2), np.full(nb, c * Eeq / 4)], axis=1))
    T, E, Ef, F, it = loqd.solve_grey_meb(nx, ny, lx, ly, c, c_dt, coef, np.full(N, Teq), C_V, A_R)
    assert np.allclose(T, Teq, rtol=1e-13) and np.allclose(E, Eeq, rtol=1e-12) and np.allclose(Ef, Eeq, rtol=1e-12)
    assert np.max(np.abs(F)) <= 1e-12 * c * Eeq


def test_grey_energy_balance_with_infinite_heat_capacity():
    """c_v -> infinity: the temperature cannot move, and E is the solution
    of the grey equations with the emission of the fixed temperature."""
    geo, coef, Ts = _grey_meb_case(seed=43)
    nx, ny, lx, ly, c, c_dt = geo
    T, E, Ef, F, it = loqd.solve_grey_meb(*geo, coef, Ts, 1e30, A_R)
    assert np.allclose(T, Ts, rtol=1e-12)
    source = c * coef["E_prev"] / c_dt + c * coef["kappa_B"] * A_R * Ts ** 4
    e, ef, ff = loqd.solve_general(nx, ny, lx, ly, c, c_dt, coef["sigma"], source, coef["k_side"],
                                   coef["eta_side"], coef["F_prev"], coef["f_cell"], coef["f_face"], coef["bc"])
    assert np.allclose(E, e, rtol=1e-10) and np.allclose(F, ff, rtol=1e-9, atol=1e-12 * np.max(np.abs(ff)))


def test_newton_converges_quadratically():
    geo, coef, Ts = _grey_meb_case(seed=44)
    changes = []
    T = Ts.copy()
    for k in range(1, 7):
        Tk, *_ = loqd.solve_grey_meb(*geo, coef, Ts, C_V, A_R, T_start=Ts, max_newton=k, tol=0.0)
        changes.append(np.max(np.abs(Tk - T) / np.abs(Tk)))
        T = Tk
    # successive changes fall quadratically once in the basin (a Newton
    # step with a wrong derivative falls only linearly)
    for a, b in zip(changes[1:4], changes[2:5]):
        assert b <= 4 * a * a
    assert changes[5] < 1e-14
