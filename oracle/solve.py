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


def rays_through_cells(grid, cells):
    """Per pair, the characteristics that cross any of the given cells."""
    cells = set(int(c) for c in cells)
    out = []
    for pr in grid.pairs:
        out.append(np.array([k for k in range(pr.K)
                             if cells.intersection(pr.cells[k].tolist())],
                            dtype=np.int64))
    return out


def run_sampled(prob, grid, cells, steps=None, c=None):
    """Cell moments for a sample of cells only, at any problem size: each
    characteristic evolves independently of the others (material data are
    prescribed), so sweeping only the characteristics that cross the sampled
    cells over all steps gives those cells' moments exactly.

    Returns per step a dict {E, F, f} of arrays [G][n_sample] (and [G][2]/[4]
    components) in the order of ``cells``, plus the swept rays per pair and
    their final segment rows (for segment-level comparisons)."""
    from workloads import C_LIGHT
    c = C_LIGHT if c is None else c
    n = prob.steps if steps is None else steps
    cells = np.asarray(cells, dtype=np.int64)
    sel = rays_through_cells(grid, cells)
    n_pol = prob.n_pol
    local = []
    for a, pr in enumerate(grid.pairs):
        ks = sel[a]
        X = prob.state0
        rows = []
        for k in ks:
            rows.append(np.broadcast_to(X[:, pr.cells[k]].T[:, None, None, :],
                                        (len(pr.cells[k]), 2, n_pol, X.shape[0])))
        local.append(np.concatenate(rows).copy() if rows else None)
    hist = []
    for t in range(n):
        Iim = np.zeros((len(cells), prob.M, prob.G))
        out_j = []
        for a, pr in enumerate(grid.pairs):
            ks = sel[a]
            if len(ks) == 0:
                raise ValueError("a sampled cell is crossed by no characteristic")
            j, rows, _, _ = sweep.sweep_pair(grid, a, prob.mu, prob.kappa[t],
                                             prob.planck[t], prob.c_dt, local[a],
                                             prob.I_in, rays=ks, local_state=True)
            local[a] = rows
            out_j.append(j)
            # area-weighted per-direction averages for the sampled cells
            cs = np.concatenate([pr.cells[k] for k in ks])
            As = np.concatenate([pr.lens[k] * pr.w[k] for k in ks])
            for q, cell in enumerate(cells):
                mask = cs == cell
                A = As[mask]
                for d in (0, 1):
                    for p in range(n_pol):
                        m = sweep.direction_index(a, d, p, grid.n_az, n_pol)
                        Iim[q, m, :] = (A[:, None] * rows[mask, d, p, :]).sum(0) / A.sum()
        E, F, f = moments._moments_from_averages(Iim, prob.phi, prob.mu, prob.omega, c)
        hist.append(dict(E=E, F=F, f=f))
    return dict(steps=hist, rays=sel, rows=local, j=out_j)
