"""Angular moments of the sweep solution (paper, eq. (7), (14)-(16), and the
boundary factors that close the low-order equations).

Cell moments, per group g and material cell i:
    I_{i,m}  = sum_{(k,s) in C(i,m)} A_{k,s} I_bar_{k,s} / sum_{C(i,m)} A_{k,s},
               A_{k,s} = l_{k,s} w_k                                      (14)
    Phi      = sum_m omega_m I_{i,m}            (E = Phi / c)
    F        = sum_m omega_m Omega_m I_{i,m}    (x, y components)
    T        = sum_m omega_m Omega_m Omega_m I_{i,m}  (xx, xy, yy, zz)
    f        = T / Phi                                                  (7), (15)

Reading: eq. (15) weights each direction's segments by their areas over the
sum of all directions; because the traced area sum_{C(i,m)} A equals the cell
area only for the paper's vertex-avoiding construction, each direction is
normalised by its own traced area before the angular sum.  Both agree exactly
for that construction; the per-direction form keeps f = 1/3 for an isotropic
intensity with evenly spaced characteristics too.

Boundary factors, per boundary face b and group g, with
I_{b,m} = width-weighted mean exit intensity of the characteristics leaving
through b (Omega_m . n_b > 0), or the given incoming I_in[b, m] otherwise:
    Phi+ = sum_out omega I,  J+ = sum_out omega (Omega.n) I,
    Phi- = sum_in  omega I,  J- = sum_in  omega |Omega.n| I,
    C    = J+ / Phi+,
    f_b  = sum_m omega Omega Omega I / sum_m omega I   (xx, xy, yy; eq. (16)
           read per direction as for the cells).
If no characteristic leaves through b in direction m, the one whose exit
point is nearest to the face centre is used (ties: lower k).  Where Phi (or
Phi+) is zero, f = 1/3 on the diagonal and C = its isotropic value.
The boundary factor C is named but not written out in the paper, so the
definition above is a reading.  Its evaluation is pinned (the isotropic
closed form, single-direction indicators, and a field linear in the
characteristic coordinate on the vertex-avoiding grid, whose width-weighted
exit means are the face-centre values); against the paper itself, which
prints no value of C, parity is unpinned.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .rays import face_centres
from .sweep import direction_index

N_BND = 8   # Phi+, J+, Phi-, J-, C, fxx, fxy, fyy


def directions(phi, mu):
    """Omega_m = (sin zeta cos phi, sin zeta sin phi, mu) for m = a*P + p."""
    phi = np.asarray(phi)
    mu = np.asarray(mu)
    sz = np.sqrt(1.0 - mu ** 2)
    ox = (np.cos(phi)[:, None] * sz[None, :]).ravel()
    oy = (np.sin(phi)[:, None] * sz[None, :]).ravel()
    oz = np.tile(mu, len(phi))
    return ox, oy, oz


def cell_direction_averages(grid, n_pol, state, cells=None):
    """I_{i,m,g} for all cells (or only the listed ones, in their order),
    directions and groups: [cells][M][G].  Every returned cell must be
    crossed by a characteristic of every azimuth pair."""
    n_cells = grid.nx * grid.ny
    rows_out = np.arange(n_cells) if cells is None else np.asarray(cells, dtype=np.int64)
    G = state.shape[-1]
    out = np.zeros((len(rows_out), grid.n_az * n_pol, G))
    for a, pr in enumerate(grid.pairs):
        js, cs, As = [], [], []
        j = pr.seg_base
        for k in range(pr.K):
            n = len(pr.cells[k])
            js.append(np.arange(j, j + n)); cs.append(pr.cells[k])
            As.append(pr.lens[k] * pr.w[k])
            j += n
        js = (np.concatenate(js) - pr.seg_base) if js else np.zeros(0, dtype=np.int64)
        cs = np.concatenate(cs) if cs else np.zeros(0, dtype=np.int64)
        As = np.concatenate(As) if As else np.zeros(0)
        traced = np.bincount(cs, weights=As, minlength=n_cells)
        if np.any(traced[rows_out] <= 0.0):
            raise ValueError(f"pair {a}: some cell is crossed by no characteristic")
        Wm = sp.csr_matrix((As / np.where(traced > 0.0, traced, 1.0)[cs], (cs, js)),
                           shape=(n_cells, int(pr.nseg.sum())))[rows_out]
        rows = state[pr.seg_base:pr.seg_base + int(pr.nseg.sum())]
        for d in (0, 1):
            for p in range(n_pol):
                m = direction_index(a, d, p, grid.n_az, n_pol)
                out[:, m, :] = Wm @ rows[:, d, p, :]
    return out


def cell_moments(grid, phi, mu, omega, state, c, cells=None):
    """E [G][cells], F [G][2][cells], f [G][4][cells] (xx, xy, yy, zz); with
    ``cells``, only those cells, in their order."""
    n_pol = len(mu)
    Iim = cell_direction_averages(grid, n_pol, state, cells)    # [cells][M][G]
    return _moments_from_averages(Iim, phi, mu, omega, c)


def _moments_from_averages(Iim, phi, mu, omega, c):
    ox, oy, oz = directions(phi, mu)
    w = np.asarray(omega)
    Phi = np.einsum('m,imG->Gi', w, Iim)
    Fx = np.einsum('m,imG->Gi', w * ox, Iim)
    Fy = np.einsum('m,imG->Gi', w * oy, Iim)
    Txx = np.einsum('m,imG->Gi', w * ox * ox, Iim)
    Txy = np.einsum('m,imG->Gi', w * ox * oy, Iim)
    Tyy = np.einsum('m,imG->Gi', w * oy * oy, Iim)
    Tzz = np.einsum('m,imG->Gi', w * oz * oz, Iim)
    E = Phi / c
    F = np.stack([Fx, Fy], axis=1)
    zero = Phi == 0.0
    safe = np.where(zero, 1.0, Phi)
    f = np.stack([np.where(zero, 1 / 3, Txx / safe), np.where(zero, 0.0, Txy / safe),
                  np.where(zero, 1 / 3, Tyy / safe), np.where(zero, 1 / 3, Tzz / safe)],
                 axis=1)
    return E, F, f


def face_normals(nx, ny):
    n = np.zeros((2 * (nx + ny), 2))
    n[:ny] = (-1, 0); n[ny:2 * ny] = (1, 0)
    n[2 * ny:2 * ny + nx] = (0, -1); n[2 * ny + nx:] = (0, 1)
    return n


def boundary_intensities(grid, mu, exits, I_in, faces=None):
    """I_{b,m,g}: [nb][M][G] (outgoing: width-weighted exit mean; incoming:
    I_in) and the outgoing mask [nb][M].  With ``faces``, only those faces'
    outgoing entries are formed (the others keep I_in and a False mask)."""
    nx, ny = grid.nx, grid.ny
    nb = 2 * (nx + ny)
    n_pol = len(mu)
    M = grid.n_az * n_pol
    G = I_in.shape[-1]
    centres = face_centres(nx, ny, grid.lx, grid.ly)
    normals = face_normals(nx, ny)
    Ib = np.array(I_in, dtype=np.float64, copy=True)
    out_mask = np.zeros((nb, M), dtype=bool)
    for a, pr in enumerate(grid.pairs):
        for d in (0, 1):
            sign = 1.0 if d == 0 else -1.0
            dirn = sign * np.array([pr.c, pr.s])
            fexit = pr.exit_face if d == 0 else pr.entry_face
            pexit = pr.exit_pt if d == 0 else pr.entry_pt
            for b in (range(nb) if faces is None else faces):
                if normals[b] @ dirn <= 0.0:
                    continue
                sel = np.nonzero(fexit == b)[0]
                if len(sel) == 0:
                    dist = np.hypot(pexit[:, 0] - centres[b, 0], pexit[:, 1] - centres[b, 1])
                    sel = np.array([int(np.argmin(dist))])
                wk = pr.w[sel]
                for p in range(n_pol):
                    m = direction_index(a, d, p, grid.n_az, n_pol)
                    Ib[b, m, :] = (wk[:, None] * exits[a][d, sel, p, :]).sum(0) / wk.sum()
                    out_mask[b, m] = True
    return Ib, out_mask


def boundary_factors(grid, phi, mu, omega, exits, I_in, faces=None):
    """[G][nb][8]: Phi+, J+, Phi-, J-, C, fxx, fxy, fyy per boundary face;
    with ``faces``, [G][len(faces)][8] for those faces only."""
    Ib, out_mask = boundary_intensities(grid, mu, exits, I_in, faces)
    nb, M, G = Ib.shape
    sel = np.arange(nb) if faces is None else np.asarray(faces, dtype=np.int64)
    ox, oy, oz = directions(phi, mu)
    w = np.asarray(omega)
    normals = face_normals(grid.nx, grid.ny)
    res = np.zeros((G, len(sel), 8))
    for q, b in enumerate(sel):
        odn = ox * normals[b, 0] + oy * normals[b, 1]           # Omega . n
        o = out_mask[b]
        i = ~o
        Pp = (w[o, None] * Ib[b, o]).sum(0)
        Jp = ((w * odn)[o, None] * Ib[b, o]).sum(0)
        Pm = (w[i, None] * Ib[b, i]).sum(0)
        Jm = ((w * np.abs(odn))[i, None] * Ib[b, i]).sum(0)
        c_iso = (w * odn)[o].sum() / w[o].sum()
        C = np.where(Pp > 0.0, Jp / np.where(Pp > 0.0, Pp, 1.0), c_iso)
        S = (w[:, None] * Ib[b]).sum(0)
        Sxx = ((w * ox * ox)[:, None] * Ib[b]).sum(0)
        Sxy = ((w * ox * oy)[:, None] * Ib[b]).sum(0)
        Syy = ((w * oy * oy)[:, None] * Ib[b]).sum(0)
        z = S == 0.0
        Ss = np.where(z, 1.0, S)
        res[:, q, 0], res[:, q, 1], res[:, q, 2], res[:, q, 3] = Pp, Jp, Pm, Jm
        res[:, q, 4] = C
        res[:, q, 5] = np.where(z, 1 / 3, Sxx / Ss)
        res[:, q, 6] = np.where(z, 0.0, Sxy / Ss)
        res[:, q, 7] = np.where(z, 1 / 3, Syy / Ss)
    return res
