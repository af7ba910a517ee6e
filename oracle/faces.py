"""Face-average moments and Eddington tensor on the interior faces of the
material grid (paper, eq. (16) with the set F(f, m) of characteristic
segments whose upwind face lies on face f).  TEST INFRASTRUCTURE ONLY.

Faces: x-faces (x = ix * hx, 1 <= ix <= nx - 1, row iy) are numbered
iy * (nx - 1) + (ix - 1); y-faces (y = iy * hy, 1 <= iy <= ny - 1, column ix)
follow them, numbered (nx - 1) * ny + (iy - 1) * nx + ix.

A characteristic crosses an interior face where two consecutive segments
lie in cells that share that face.  In the forward traversal (d = 0) the
crossing is the upwind face of the later segment; in the reverse traversal
(d = 1) it is the upwind face of the earlier one.  The intensity there is the
point intensity I_{k,s} entering that segment.  A step between diagonal
neighbours (a passage through a vertex) crosses no face interior and is left
out.

Per face f, group g and direction m:
    I_{f,m} = sum_{k in F(f,m)} w_k I_{k,s} / sum_{k in F(f,m)} w_k,
read per direction as for the boundary faces (the width sum over a face is
proportional to |n . Omega_m|, so the literal weights of eq. (16) would
not give 1/3 for an isotropic intensity); a direction no characteristic
crosses the face in contributes nothing.  Then
    Phi_f = sum_m omega_m I_{f,m},  E_f = Phi_f / c,
    F_f = sum_m omega_m Omega_m I_{f,m},
    f_f = sum_m omega_m Omega_m Omega_m I_{f,m} / Phi_f   (xx, xy, yy, zz),
with f_f = 1/3 on the diagonal where Phi_f = 0.
"""
from __future__ import annotations

import numpy as np

from .moments import _moments_from_averages
from .sweep import direction_index


def n_faces(nx, ny):
    return (nx - 1) * ny + nx * (ny - 1)


def face_of_step(nx, ny, c0, c1):
    """Interior face shared by cells c0 and c1, or -1 (not neighbours)."""
    iy0, ix0 = divmod(int(c0), nx)
    iy1, ix1 = divmod(int(c1), nx)
    if iy0 == iy1 and abs(ix0 - ix1) == 1:
        return iy0 * (nx - 1) + min(ix0, ix1)
    if ix0 == ix1 and abs(iy0 - iy1) == 1:
        return (nx - 1) * ny + min(iy0, iy1) * nx + ix0
    return -1


def crossings(grid):
    """Per pair: arrays (face, k, j_after, j_before) of the interior-face
    crossings, j the global indices of the segments after and before the
    crossing in forward order."""
    out = []
    for pr in grid.pairs:
        f_, k_, ja, jb = [], [], [], []
        j = pr.seg_base
        for k in range(pr.K):
            cells = pr.cells[k]
            for s in range(1, len(cells)):
                f = face_of_step(grid.nx, grid.ny, cells[s - 1], cells[s])
                if f >= 0:
                    f_.append(f); k_.append(k); ja.append(j + s); jb.append(j + s - 1)
            j += len(cells)
        out.append(tuple(np.asarray(x, dtype=np.int64) for x in (f_, k_, ja, jb)))
    return out


def face_direction_averages(grid, n_pol, points):
    """I_{f,m,g} for every interior face: [faces][M][G]."""
    nf = n_faces(grid.nx, grid.ny)
    G = points.shape[-1]
    out = np.zeros((nf, grid.n_az * n_pol, G))
    for a, (pr, (fs, ks, ja, jb)) in enumerate(zip(grid.pairs, crossings(grid))):
        w = pr.w[ks]
        wsum = np.bincount(fs, weights=w, minlength=nf)
        has = wsum > 0.0
        for d in (0, 1):
            src = points[ja, 0] if d == 0 else points[jb, 1]          # [n][P][G]
            for p in range(n_pol):
                m = direction_index(a, d, p, grid.n_az, n_pol)
                acc = np.zeros((nf, G))
                np.add.at(acc, fs, w[:, None] * src[:, p, :])
                out[has, m, :] = acc[has] / wsum[has, None]
    return out


def face_moments(grid, phi, mu, omega, points, c):
    """E [G][faces], F [G][2][faces], f [G][4][faces] on the interior faces."""
    Ifm = face_direction_averages(grid, len(mu), points)
    return _moments_from_averages(Ifm, phi, mu, omega, c)
