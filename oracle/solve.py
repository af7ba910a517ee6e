"""Time loop of the transport step with prescribed material data (backward
Euler, paper eq. (10)-(11); initial intensity from eq. (2)).

Each step n sweeps with kappa^n, B^n and the previous step's segment-average
intensities, then forms the cell moments and the boundary factors.  The
material temperature is prescribed per step (the energy balance is not part
of the transport step).
"""
from __future__ import annotations

import numpy as np

from . import moments, rays, sweep


def build_grid(prob, mode=rays.UNIFORM):
    return rays.build(prob.nx, prob.ny, prob.lx, prob.ly, prob.phi, prob.h_moc, mode)


def run(prob, grid=None, steps=None, c=None, mode=rays.UNIFORM):
    """Full solve.  Returns a dict with the final state, exit intensities and
    per-step moments (E, F, f, bnd)."""
    from workloads import C_LIGHT
    c = C_LIGHT if c is None else c
    grid = build_grid(prob, mode) if grid is None else grid
    n = prob.steps if steps is None else steps
    st = sweep.initial_state(grid, prob.n_pol, prob.state0)
    hist = []
    exits = None
    for t in range(n):
        st, exits = sweep.sweep(grid, prob.mu, prob.kappa[t], prob.planck[t],
                                prob.c_dt, st, prob.I_in)
        E, F, f = moments.cell_moments(grid, prob.phi, prob.mu, prob.omega, st, c)
        bnd = moments.boundary_factors(grid, prob.phi, prob.mu, prob.omega, exits,
                                       prob.I_in)
        hist.append(dict(E=E, F=F, f=f, bnd=bnd))
    return dict(grid=grid, state=st, exits=exits, steps=hist)


def run_sampled(prob, grid, cells, steps=None, c=None, faces=None):
    """Moments of a sample of cells (and boundary factors of a sample of
    boundary faces) at any problem size.

    ``grid`` is the characteristic grid restricted to the characteristics
    that reach the samples (``rays.build(..., only_cells=cells,
    only_faces=faces)``).  Under prescribed material data each
    characteristic evolves independently of the others: its segment states
    depend only on its own previous states, the material data and the
    boundary intensity of the face it enters through.  So the plain time loop
    of ``run`` over that subset gives, step by step, the same segment states
    as over the whole grid, and the sampled cells' and faces' moments follow
    from the characteristics reaching them.

    Returns per step a dict {E [G][n], F [G][2][n], f [G][4][n]} over the
    sampled cells, in the order of ``cells``, and ``bnd`` [G][n_faces][8]
    when ``faces`` is given; plus the grid, final state and exits (for
    segment-level comparisons)."""
    from workloads import C_LIGHT
    c = C_LIGHT if c is None else c
    n = prob.steps if steps is None else steps
    cells = np.asarray(cells, dtype=np.int64)
    st = sweep.initial_state(grid, prob.n_pol, prob.state0)
    hist = []
    exits = None
    for t in range(n):
        st, exits = sweep.sweep(grid, prob.mu, prob.kappa[t], prob.planck[t],
                                prob.c_dt, st, prob.I_in)
        E, F, f = moments.cell_moments(grid, prob.phi, prob.mu, prob.omega, st, c, cells=cells)
        h = dict(E=E, F=F, f=f)
        if faces is not None:
            h["bnd"] = moments.boundary_factors(grid, prob.phi, prob.mu, prob.omega, exits,
                                                prob.I_in, faces=faces)
        hist.append(h)
    return dict(grid=grid, state=st, exits=exits, steps=hist)
