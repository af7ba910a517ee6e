"""Multigroup low-order quasidiffusion (LOQD) equations of the paper's
multilevel method, eq. (4), for one backward-Euler time step on the material
grid, closed by the Eddington tensors of the transport sweep (eq. (7), (15)
for cells, (16) for faces) and the half-range boundary factor C.

TEST INFRASTRUCTURE ONLY: plain Python + scipy's sparse direct solver (on
the row-scaled system); the HIP library never imports it.

Time-discrete equations (backward Euler, kappa_t = kappa + 1/(c dt)):
    c kappa_t E + div F = 4 pi kappa B + E^{n-1}/dt                   (4a)
    kappa_t F + c div(f E) = F^{n-1}/(c dt)                          (4b)

The paper discretises them with a second-order finite-volume scheme that it
cites but does not print.  Reading (the scheme implemented here):

* unknowns per group: the cell averages E_i and the face averages E_f on
  every face (interior and boundary); the normal face fluxes F_f (the x
  component on x-faces, y on y-faces) follow from them;
* (4a) integrated over cell i of size hx x hy:
    c kappa_t,i E_i + (F_R - F_L)/hx + (F_T - F_B)/hy = 4 pi kappa_i B_i + E^{n-1}_i/dt;
* (4b), x component, integrated over each half of the cell next to an
  x-face, with the half-cell average of kappa_t F_x taken as kappa_t,i times
  the face value and f E taken as the cell tensor times E_i at the centre,
  the face tensor times E_f on the face, and the y-face averages of the
  cell on the half-cell's top and bottom:
    kappa_t,i (hx/2) F_R = -c (f_xx,R E_R - f_xx,i E_i)
                           - c hx/(2 hy) (f_xy,T E_T - f_xy,B E_B) + (hx/2) F^{n-1}_R/(c dt)
    kappa_t,i (hx/2) F_L = -c (f_xx,i E_i - f_xx,L E_L)
                           - c hx/(2 hy) (f_xy,T E_T - f_xy,B E_B) + (hx/2) F^{n-1}_L/(c dt)
  and alike for the y component on y-faces (f_yy, and f_xy on the cell's
  x-faces);
* an interior face has one flux: the relations of its two cells give the
  same F_f (one equation per interior face);
* a boundary face with outward normal n closes with the exact QD boundary
  condition n.F = C (c E_f - Phi^-) - J^-, where C = J^+/Phi^+ is the
  half-range factor and Phi^-, J^- are the incoming half-range moments of
  the boundary intensity (all three from the transport's boundary factors).

Face numbering (shared with the library by this written convention only):
interior x-faces (x = ix hx, 1 <= ix < nx) of row iy are iy (nx-1) + ix - 1;
interior y-faces (y = iy hy, 1 <= iy < ny) of column ix follow at
(nx-1) ny + (iy-1) nx + ix; then the boundary faces in their own order
([0, ny) x = 0, [ny, 2ny) x = lx, [2ny, 2ny+nx) y = 0, then y = ly) offset
by the interior count.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def n_interior(nx, ny):
    return (nx - 1) * ny + nx * (ny - 1)


def n_faces(nx, ny):
    return n_interior(nx, ny) + 2 * (nx + ny)


def cell_faces(nx, ny):
    """Faces (L, R, B, T) of every cell in the all-face numbering: [cells][4]."""
    nint = n_interior(nx, ny)
    out = np.zeros((nx * ny, 4), dtype=np.int64)
    for iy in range(ny):
        for ix in range(nx):
            i = iy * nx + ix
            L = iy * (nx - 1) + ix - 1 if ix > 0 else nint + iy
            R = iy * (nx - 1) + ix if ix < nx - 1 else nint + ny + iy
            B = (nx - 1) * ny + (iy - 1) * nx + ix if iy > 0 else nint + 2 * ny + ix
            T = (nx - 1) * ny + iy * nx + ix if iy < ny - 1 else nint + 2 * ny + nx + ix
            out[i] = (L, R, B, T)
    return out


def face_cells(nx, ny):
    """For every face: (cell on the low side, cell on the high side) along its
    normal axis, -1 outside the domain, and whether it is an x-face."""
    nf = n_faces(nx, ny)
    lo = np.full(nf, -1, dtype=np.int64)
    hi = np.full(nf, -1, dtype=np.int64)
    is_x = np.zeros(nf, dtype=bool)
    cf = cell_faces(nx, ny)
    for i in range(nx * ny):
        L, R, B, T = cf[i]
        hi[L] = i; lo[R] = i; hi[B] = i; lo[T] = i
        is_x[L] = is_x[R] = True
    return lo, hi, is_x


SIDES = ("L", "R", "B", "T")


class _Group:
    """Per-group data of one solve (plain attribute bag).  k_side and
    eta_side ([cells][4], sides L, R, B, T) are the coefficients of the
    flux and of the face energy density in the half-cell relations; the
    multigroup equations have k = kappa_t of the cell and eta = 0."""

    def __init__(self, nx, ny, lx, ly, c, c_dt, k_side, eta_side, F_prev, f_cell, f_face):
        self.nx, self.ny = nx, ny
        self.hx, self.hy = lx / nx, ly / ny
        self.N = nx * ny
        self.c, self.c_dt = c, c_dt
        self.k_side = k_side
        self.eta_side = eta_side
        self.F_prev = F_prev
        self.fxx, self.fxy, self.fyy = f_cell
        self.gxx, self.gxy, self.gyy = f_face
        self.cf = cell_faces(nx, ny)


def half_cell_flux(q, i, face):
    """The first-moment relation of cell i on the half of the cell next to one
    of its faces,
        k (h/2) F_face = -c ((f E)_high - (f E)_low) - c h/(2 h_t) (mixed term)
                         - (h/2) eta E_face + (h/2) F^{n-1}_face / (c dt),
    solved for that face's normal flux: F_face = sum coef * x[col] + const,
    with columns 0..N-1 the cell unknowns and N + f the face unknowns.
    Returns ([(col, coef)], const)."""
    c, N = q.c, q.N
    L, R, B, T = q.cf[i]
    side = (L, R, B, T).index(face)
    if face in (L, R):
        h = q.hx
        a = q.k_side[i, side] * h / 2.0
        cross = [(N + T, -c * q.hx / (2 * q.hy) * q.gxy[T] / a), (N + B, c * q.hx / (2 * q.hy) * q.gxy[B] / a)]
        if face == R:
            terms = [(N + R, -c * q.gxx[R] / a), (i, c * q.fxx[i] / a)]
        else:
            terms = [(i, -c * q.fxx[i] / a), (N + L, c * q.gxx[L] / a)]
    else:
        h = q.hy
        a = q.k_side[i, side] * h / 2.0
        cross = [(N + R, -c * q.hy / (2 * q.hx) * q.gxy[R] / a), (N + L, c * q.hy / (2 * q.hx) * q.gxy[L] / a)]
        if face == T:
            terms = [(N + T, -c * q.gyy[T] / a), (i, c * q.fyy[i] / a)]
        else:
            terms = [(i, -c * q.fyy[i] / a), (N + B, c * q.gyy[B] / a)]
    eta = [(N + face, -(h / 2.0) * q.eta_side[i, side] / a)] if q.eta_side[i, side] != 0.0 else []
    return terms + cross + eta, (h / 2.0) * q.F_prev[face] / q.c_dt / a


def boundary_condition(C, Phi_in, J_in, c):
    """n.F = C (c E_f - Phi^-) - J^- as (coefficient of E_f, constant)."""
    return C * c, -C * Phi_in - J_in


def assemble_general(nx, ny, lx, ly, c, c_dt, sigma, source, k_side, eta_side, F_prev, f_cell, f_face, bc):
    """The linear system of one group of the low-order scheme in general
    form: cell balances sigma_i E_i + div F = source_i, half-cell relations
    with side coefficients k_side and eta_side, one flux per interior face,
    boundary condition from bc.  Returns (A [n][n] sparse, rhs [n], data),
    n = cells + faces, cell unknowns first."""
    q = _Group(nx, ny, lx, ly, c, c_dt, k_side, eta_side, F_prev, f_cell, f_face)
    N = q.N
    nf = n_faces(nx, ny)
    nint = n_interior(nx, ny)
    lo, hi, _ = face_cells(nx, ny)
    rows, cols, vals = [], [], []
    rhs = np.zeros(N + nf)

    def add(r, terms, scale):
        for col, v in terms:
            rows.append(r); cols.append(col); vals.append(scale * v)

    # cell balances: sigma_i E_i + (F_R - F_L)/hx + (F_T - F_B)/hy = source_i
    for i in range(N):
        L, R, B, T = q.cf[i]
        add(i, [(i, sigma[i])], 1.0)
        rhs[i] = source[i]
        for face, sgn, h in ((R, 1.0, q.hx), (L, -1.0, q.hx), (T, 1.0, q.hy), (B, -1.0, q.hy)):
            terms, const = half_cell_flux(q, i, face)
            add(i, terms, sgn / h)
            rhs[i] -= sgn / h * const
    # face equations
    for f in range(nf):
        r = N + f
        if lo[f] >= 0 and hi[f] >= 0:               # one flux from both sides
            t1, c1 = half_cell_flux(q, lo[f], f)
            t2, c2 = half_cell_flux(q, hi[f], f)
            add(r, t1, 1.0)
            add(r, t2, -1.0)
            rhs[r] = c2 - c1
        else:                                      # n.F from the cell equals the boundary condition
            C, Pm, Jm = bc[f - nint]
            i = lo[f] if lo[f] >= 0 else hi[f]
            sgn = 1.0 if lo[f] >= 0 else -1.0      # n = +axis when the cell lies below the face
            t1, c1 = half_cell_flux(q, i, f)
            ce, cc = boundary_condition(C, Pm, Jm, c)
            add(r, t1, sgn)
            add(r, [(N + f, -ce)], 1.0)
            rhs[r] = cc - sgn * c1
    A = sp.csr_matrix((vals, (rows, cols)), shape=(N + nf, N + nf))
    return A, rhs, q


def multigroup_coefficients(c, c_dt, kappa, planck, E_prev):
    """sigma, source, k_side, eta_side of one group of eq. (4):
    sigma = c kappa_t, source = 4 pi kappa B + E^{n-1}/dt, k = kappa_t on
    every side, eta = 0."""
    kt = kappa + 1.0 / c_dt
    sigma = c * kt
    source = 4.0 * np.pi * kappa * planck + c * E_prev / c_dt
    k_side = np.repeat(kt[:, None], 4, axis=1)
    return sigma, source, k_side, np.zeros_like(k_side)


def assemble_group(nx, ny, lx, ly, c, c_dt, kappa, planck, E_prev, F_prev, f_cell, f_face, bc):
    """The linear system of one group of eq. (4)."""
    sigma, source, k_side, eta_side = multigroup_coefficients(c, c_dt, kappa, planck, E_prev)
    return assemble_general(nx, ny, lx, ly, c, c_dt, sigma, source, k_side, eta_side, F_prev, f_cell, f_face, bc)


def solve_assembled(nx, ny, A, rhs, q):
    """Direct solve of an assembled system, then the face fluxes.

    Each equation is divided by its largest coefficient before the direct
    solve.  The solution is unchanged, but in optically thick cells the
    balance rows (of order c kappa_t) would otherwise dwarf the face rows
    (of order c / (kappa_t h)) and leave the solve with few correct digits."""
    N = q.N
    nf = n_faces(nx, ny)
    lo, hi, _ = face_cells(nx, ny)
    scale = 1.0 / abs(A).max(axis=1).toarray().ravel()
    x = spla.spsolve((sp.diags(scale) @ A).tocsc(), scale * rhs)
    E_cell, E_face = x[:N], x[N:]
    F_face = np.zeros(nf)
    for f in range(nf):
        i = lo[f] if lo[f] >= 0 else hi[f]
        terms, const = half_cell_flux(q, i, f)
        F_face[f] = sum(v * x[col] for col, v in terms) + const
    return E_cell, E_face, F_face


def solve_group(nx, ny, lx, ly, c, c_dt, kappa, planck, E_prev, F_prev, f_cell, f_face, bc):
    """One group of eq. (4).  kappa, planck, E_prev: [cells]; F_prev: [faces]
    normal flux of the previous step (x component on x-faces, y on y-faces);
    f_cell: [3][cells] and f_face: [3][faces] Eddington tensor entries
    (xx, xy, yy); bc: [nb][3] = (C, Phi^-, J^-) per boundary face.
    Returns (E_cell [cells], E_face [faces], F_face [faces])."""
    A, rhs, q = assemble_group(nx, ny, lx, ly, c, c_dt, kappa, planck, E_prev, F_prev, f_cell, f_face, bc)
    return solve_assembled(nx, ny, A, rhs, q)


def solve_general(nx, ny, lx, ly, c, c_dt, sigma, source, k_side, eta_side, F_prev, f_cell, f_face, bc):
    """One group of the scheme in general form (see assemble_general)."""
    A, rhs, q = assemble_general(nx, ny, lx, ly, c, c_dt, sigma, source, k_side, eta_side, F_prev, f_cell,
                                 f_face, bc)
    return solve_assembled(nx, ny, A, rhs, q)


def solve(nx, ny, lx, ly, c, c_dt, kappa, planck, E_prev, F_prev, f_cell, f_face, bc):
    """All groups: kappa, planck, E_prev [G][cells]; F_prev [G][faces];
    f_cell [G][3][cells]; f_face [G][3][faces]; bc [G][nb][3].  Returns
    E_cell [G][cells], E_face [G][faces], F_face [G][faces]."""
    G = kappa.shape[0]
    out = [solve_group(nx, ny, lx, ly, c, c_dt, kappa[g], planck[g], E_prev[g], F_prev[g], f_cell[g],
                       f_face[g], bc[g]) for g in range(G)]
    return tuple(np.stack([o[k] for o in out]) for k in range(3))


def closures_from_transport(nx, ny, E_cellmajor_f, face_f, bnd):
    """Arrange the transport's outputs as the solver's closures:
    cell tensors from the cell moments f [G][4][cells] (xx, xy, yy, zz),
    interior face tensors from the face moments f [G][4][interior faces],
    boundary face tensors and (C, Phi^-, J^-) from the boundary factors
    [G][nb][8] (Phi+, J+, Phi-, J-, C, fxx, fxy, fyy).  Returns
    (f_cell [G][3][cells], f_face [G][3][faces], bc [G][nb][3])."""
    f_cell = E_cellmajor_f[:, [0, 1, 2], :]
    f_face = np.concatenate([face_f[:, [0, 1, 2], :], bnd[:, :, 5:8].transpose(0, 2, 1)], axis=2)
    bc = bnd[:, :, [4, 2, 3]]
    return f_cell, f_face, bc


# ---------------------------------------------------------------------------
# effective grey low-order equations, eq. (5)
# ---------------------------------------------------------------------------

def grey_coefficients(nx, ny, c, c_dt, kappa, planck, E_prev, F_prev, f_cell, f_face, bc, E_cell, E_face,
                      F_face):
    """Coefficients of the effective grey equations, eq. (5), in the general
    form of the scheme, from a multigroup solution of eq. (4) on the same
    grid (its cell and face energy densities and face fluxes).

    The paper makes the grey scheme algebraically consistent with the
    multigroup one.  Reading: the spectrum averages of eq. (8)-(9) are taken
    where the scheme uses them --
      cell balance: <kappa>_E and <kappa>_B of the cell (with a_R T^4 read
        as (4 pi / c) sum_g B_g), so sigma E = sum_g c kappa_t,g E_g;
      half-cell relation of cell i at face f: K_R = sum_g kappa_g,i |F_g,f| /
        sum_g |F_g,f| (the normal flux component of the face) and
        eta = sum_g (kappa_g,i - K_R) F_g,f / E_f with the face's grey E, so
        K_R F_f + eta E_f = sum_g kappa_g,i F_g,f;
      Eddington tensor: <f>_E of the cell with cell energies, of the face
        with face energies;
      boundary: C = sum_g C_g E_g,f / E_f and the incoming part
        J^- = sum_g (C_g Phi^-_g + J^-_g) (Phi^- = 0), the sum of the group
        conditions.
    Summed over the groups the multigroup equations then are the grey ones,
    so the grey solution is the sum of the group solutions.  Zero (not
    negative: the scheme is not positivity preserving) denominators: <kappa>_E -> <kappa>_B -> the mean of kappa_g; K_R ->
    <kappa>_E; eta = 0; <f> = 1/3 on the diagonal; C -> mean of C_g.

    Inputs as for solve() plus E_cell [G][cells], E_face [G][faces],
    F_face [G][faces].  Returns a dict with sigma, source [cells], k_side,
    eta_side [cells][4], F_prev [faces], f_cell [3][cells], f_face
    [3][faces], bc [nb][3], E_prev [cells], kappa_E and kappa_B [cells]."""
    G, N = kappa.shape
    nf = n_faces(nx, ny)
    nint = n_interior(nx, ny)
    cf = cell_faces(nx, ny)
    E = E_cell.sum(0)
    Ef = E_face.sum(0)
    mean_k = kappa.mean(0)
    sB = planck.sum(0)
    kB_num = (kappa * planck).sum(0)
    kE_num = (kappa * E_cell).sum(0)
    kB = np.where(sB != 0, kB_num / np.where(sB != 0, sB, 1.0), np.nan)
    kE = np.where(E != 0, kE_num / np.where(E != 0, E, 1.0), np.where(np.isnan(kB), mean_k, kB))
    kB = np.where(np.isnan(kB), kE, kB)
    sigma = c * (kE + 1.0 / c_dt)
    source = 4.0 * np.pi * kB * sB + c * E_prev.sum(0) / c_dt
    k_side = np.zeros((N, 4))
    eta_side = np.zeros((N, 4))
    for i in range(N):
        for s in range(4):
            f = cf[i, s]
            Fg = F_face[:, f]
            aF = np.abs(Fg).sum()
            K = (kappa[:, i] * np.abs(Fg)).sum() / aF if aF > 0 else kE[i]
            k_side[i, s] = K + 1.0 / c_dt
            eta_side[i, s] = ((kappa[:, i] - K) * Fg).sum() / Ef[f] if Ef[f] != 0 else 0.0

    def spectrum_tensor(ft, Eg, Et):
        out = np.empty((3, Eg.shape[1]))
        for q, dflt in zip(range(3), (1 / 3, 0.0, 1 / 3)):
            num = (ft[:, q, :] * Eg).sum(0)
            out[q] = np.where(Et != 0, num / np.where(Et != 0, Et, 1.0), dflt)
        return out
    f_cell_g = spectrum_tensor(f_cell, E_cell, E)
    f_face_g = spectrum_tensor(f_face, E_face, Ef)
    Eb = E_face[:, nint:]
    Ebt = Eb.sum(0)
    C = np.where(Ebt != 0, (bc[:, :, 0] * Eb).sum(0) / np.where(Ebt != 0, Ebt, 1.0), bc[:, :, 0].mean(0))
    Jm = (bc[:, :, 0] * bc[:, :, 1] + bc[:, :, 2]).sum(0)
    bc_g = np.stack([C, np.zeros_like(C), Jm], axis=1)
    return dict(sigma=sigma, source=source, k_side=k_side, eta_side=eta_side, F_prev=F_prev.sum(0),
                f_cell=f_cell_g, f_face=f_face_g, bc=bc_g, E_prev=E_prev.sum(0), kappa_E=kE, kappa_B=kB)


def solve_grey(nx, ny, lx, ly, c, c_dt, coef):
    """The grey equations with the coefficients of grey_coefficients()."""
    return solve_general(nx, ny, lx, ly, c, c_dt, coef["sigma"], coef["source"], coef["k_side"],
                         coef["eta_side"], coef["F_prev"], coef["f_cell"], coef["f_face"], coef["bc"])



def solve_grey_meb(nx, ny, lx, ly, c, c_dt, coef, T_prev, c_v, a_R, T_start=None, tol=1e-13, max_newton=50):
    """The effective grey problem: eq. (5) coupled to the grey energy
    balance, eq. (6), with material energy eps = c_v T, over one
    backward-Euler step:
        c_v (T - T^{n-1}) / dt = c <kappa>_E E - c <kappa>_B a_R T^4,
        c (<kappa>_E + 1/(c dt)) E + div F = c <kappa>_B a_R T^4 + E^{n-1}/dt,
    with the spectrum averages and the rest of the grey coefficients held
    fixed (coef from grey_coefficients).  Newton iteration on T: a_R T^4 is
    linearised about the iterate T_k, the energy balance then gives
    T = alpha + beta E in every cell, which turns the emission into an
    absorption and a source of the grey equations; each iteration solves
    them and updates T, until max |T_{k+1} - T_k| / T_{k+1} <= tol.
    Returns (T, E_cell, E_face, F_face, iterations)."""
    kE, kB = coef["kappa_E"], coef["kappa_B"]
    cv_dt = c_v * c / c_dt                       # c_v / dt
    T = np.array(T_prev if T_start is None else T_start, dtype=np.float64)
    base = c * coef["E_prev"] / c_dt
    for it in range(1, max_newton + 1):
        A = a_R * T ** 4
        D = 4.0 * a_R * T ** 3
        den = cv_dt + c * kB * D
        beta = c * kE / den
        alpha = (cv_dt * T_prev - c * kB * (A - D * T)) / den
        sigma = c * (kE + 1.0 / c_dt) - c * kB * D * beta
        source = base + c * kB * (A + D * (alpha - T))
        Ec, Ef, Ff = solve_general(nx, ny, lx, ly, c, c_dt, sigma, source, coef["k_side"], coef["eta_side"],
                                   coef["F_prev"], coef["f_cell"], coef["f_face"], coef["bc"])
        T_new = alpha + beta * Ec
        change = np.max(np.abs(T_new - T) / np.abs(T_new))
        T = T_new
        if change <= tol:
            break
    return T, Ec, Ef, Ff, it
