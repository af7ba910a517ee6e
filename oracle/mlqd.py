"""One time step of the multilevel quasidiffusion (MLQD) method on the
Fleck-Cummings problem: the paper's composition of

  1. the transport equation by the method of long characteristics,
     eq. (10)-(13), giving the Eddington tensors of the cells (eq. (7),
     (15)), of the faces (eq. (16)) and the boundary factors;
  2. the multigroup LOQD equations, eq. (4), closed by them;
  3. the effective grey problem, eq. (5)-(6), closed by the spectrum
     averages of eq. (8)-(9),

repeated (outer iterations) with the opacities and Planck functions of the
newest temperature until the temperature and the grey energy density stop
changing.

TEST INFRASTRUCTURE ONLY: plain composition of the other oracle modules.

Iterations (T^(0) = T^{n-1}).  Outer (transport) iteration s: sweep from
the state of step n-1 with kappa_g, B_g of T^(s); closures.  Then inner
(low-order) iterations l, with those closures held fixed, T^(s,0) = T^(s):
kappa_g, B_g of T^(s,l); multigroup LOQD with E_g^{n-1}, F_g^{n-1}; grey
coefficients; grey problem (Newton, started at T^(s,l)) -> T^(s,l+1), E;
until max_i |T^(s,l+1) - T^(s,l)| / T^(s,l+1) <= eps.  T^(s+1) is the last
inner iterate; the step ends when max_i |T^(s+1) - T^(s)| / T^(s+1) <= eps
and max |E^(s+1) - E^(s)| / max |E^(s+1)| <= eps (E: the grey cell energy).
The step's results are those of the last iterations: T, the multigroup
E_g, F_g (the next step's E^{n-1}, F^{n-1}) and the transport state (the
next step's I^{n-1}).
"""
from __future__ import annotations

import numpy as np

from . import faces, loqd, material, moments, sweep


def low_order(prob, T_start, T_prev, E_prev, F_prev, f_cell, f_face, bc, c, a_R, eps, max_inner, depth=3):
    """Inner iterations with fixed closures: the fixed point T = Phi(T) of
    one pass (material of T, multigroup solve, grey coefficients, grey
    problem), with Anderson mixing of depth `depth` (0: plain iteration) on
    x = log T: with the map g(x) = log Phi(e^x) and residual r = g(x) - x,
    the next x is g(x) - dG gamma, gamma minimising |r - dF gamma| over
    the last `depth` differences dF of residuals and dG of map values.  The
    iteration stops when max_i |Phi(T)_i - T_i| / Phi(T)_i <= eps.  Returns
    (Phi(T) of the last pass, its multigroup (E_cell, E_face, F_face), its
    grey E, passes, last change)."""
    nx, ny, lx, ly = prob.nx, prob.ny, prob.lx, prob.ly
    x = np.log(np.asarray(T_start, dtype=np.float64))
    dF, dG = [], []
    r_prev = g_prev = None
    for l in range(1, max_inner + 1):
        T = np.exp(x)
        kappa = material.fc_opacity(prob.nu, T)
        planck = material.group_planck(prob.edges, T, a_R, c)
        mg = loqd.solve(nx, ny, lx, ly, c, prob.c_dt, kappa, planck, E_prev, F_prev, f_cell, f_face, bc)
        coef = loqd.grey_coefficients(nx, ny, c, prob.c_dt, kappa, planck, E_prev, F_prev, f_cell, f_face, bc, *mg)
        T_new, E, _, _, _ = loqd.solve_grey_meb(nx, ny, lx, ly, c, prob.c_dt, coef, T_prev, prob.c_v, a_R,
                                                T_start=T, tol=min(eps, 1e-13))
        change = float(np.max(np.abs(T_new - T) / np.abs(T_new)))
        if change <= eps:
            break
        g = np.log(T_new)
        r = g - x
        if r_prev is not None and depth > 0:
            dF.append(r - r_prev)
            dG.append(g - g_prev)
            del dF[:-depth], dG[:-depth]
        r_prev, g_prev = r, g
        if dF:
            gamma = np.linalg.lstsq(np.column_stack(dF), r, rcond=None)[0]
            x = g - np.column_stack(dG) @ gamma
        else:
            x = g
    return T_new, mg, E, l, change


def outer_step(grid, prob, state_prev, T_prev, E_prev, F_prev, c, a_R, eps=1e-12, max_outer=60, max_inner=1000,
               depth=3):
    """prob: an object with nx, ny, lx, ly, phi, mu, omega, edges, nu,
    c_dt, c_v, I_in (the Fleck-Cummings builder's fields).  state_prev is the
    transport state of step n-1, T_prev [cells], E_prev [G][cells], F_prev
    [G][faces] the low-order solution of step n-1.  Returns a dict with T,
    E_cell, E_face, F_face (multigroup), E_grey, state, outer and inner
    (total) iterations and the last outer changes (dT, dE)."""
    nx, ny = prob.nx, prob.ny
    T = np.array(T_prev, dtype=np.float64)
    E_old = None
    inner = 0
    for s in range(1, max_outer + 1):
        kappa = material.fc_opacity(prob.nu, T)
        planck = material.group_planck(prob.edges, T, a_R, c)
        points = np.zeros_like(state_prev)
        state, exits = sweep.sweep(grid, prob.mu, kappa, planck, prob.c_dt, state_prev, prob.I_in, points=points)
        _, _, f = moments.cell_moments(grid, prob.phi, prob.mu, prob.omega, state, c)
        bnd = moments.boundary_factors(grid, prob.phi, prob.mu, prob.omega, exits, prob.I_in)
        _, _, ff = faces.face_moments(grid, prob.phi, prob.mu, prob.omega, points, c)
        f_cell, f_face, bc = loqd.closures_from_transport(nx, ny, f, ff, bnd)
        T_new, mg, E, l, _ = low_order(prob, T, T_prev, E_prev, F_prev, f_cell, f_face, bc, c, a_R, eps, max_inner,
                                       depth)
        inner += l
        dT = float(np.max(np.abs(T_new - T) / np.abs(T_new)))
        dE = np.inf if E_old is None else float(np.max(np.abs(E - E_old)) / np.max(np.abs(E)))
        T, E_old = T_new, E
        if dT <= eps and dE <= eps:
            break
    return dict(T=T, E_cell=mg[0], E_face=mg[1], F_face=mg[2], E_grey=E, state=state, outer=s, inner=inner,
                changes=(dT, dE))


def initial_low_order(prob, c):
    """E_g^0 = 4 pi B_g(T^0) / c in every cell (the isotropic initial
    intensity) and F^0 = 0 on every face."""
    E0 = 4.0 * np.pi * prob.state0 / c
    return E0, np.zeros((prob.G, loqd.n_faces(prob.nx, prob.ny)))
