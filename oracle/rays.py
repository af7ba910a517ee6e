"""Characteristic grid of the method of long characteristics (paper, section
"Method of Long Characteristics / Ray-Tracing Scheme": the (u, v)
characteristic coordinates with e_u along Omega, the K_m characteristics per
direction, segment lengths, segment areas eq. (14), and the construction of
the grid of characteristics in the paragraph after eq. (16)).

Conventions (shared with the HIP library only through this written
specification, never through code):

* material grid: nx x ny uniform cells on [0, lx] x [0, ly], cell
  i = iy * nx + ix;
* directions come in azimuth pairs: pair a < n_az/2 holds azimuth a (forward,
  d = 0) and azimuth a + n_az/2 = a + pi (reverse, d = 1), which share one set
  of characteristics traversed in opposite orders;
* for pair a, with (c, s) = (cos phi_a, sin phi_a), a point is
  r = u (c, s) + v (-s, c); characteristics are the lines v = v_k, ordered by
  v ascending; segments are listed in the forward (+u) order;
* the segment length is the in-plane (projected) length l = u_exit - u_entry;
  the 3D path length in direction m is l / sin(zeta_m);
* grid-line crossings closer than TOL_REL * min(hx, hy) to each other or to
  the ends of the characteristic are merged (a passage through a vertex gives
  no zero-length segment);
* a characteristic entering or leaving through a domain corner is assigned to
  the x = const face;
* global segment index j runs over pairs a, then characteristics k, then
  segments s (forward order).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

TOL_REL = 1e-12
UNIFORM, TUBES = 0, 1


@dataclass
class PairRays:
    """Characteristics of one azimuth pair."""
    phi: float
    c: float
    s: float
    v: np.ndarray            # [K] centreline offsets
    w: np.ndarray            # [K] widths
    cells: list              # K int arrays (forward order)
    lens: list               # K float arrays (forward order)
    entry_face: np.ndarray   # [K] boundary face where the forward traversal enters
    exit_face: np.ndarray    # [K] boundary face where it leaves
    entry_pt: np.ndarray     # [K][2]
    exit_pt: np.ndarray      # [K][2]
    seg_base: int = 0        # global index of this pair's first segment

    @property
    def K(self):
        return len(self.v)

    @property
    def nseg(self):
        return np.array([len(c) for c in self.cells], dtype=np.int64)


@dataclass
class CharGrid:
    nx: int
    ny: int
    lx: float
    ly: float
    n_az: int
    h_moc: float
    mode: int
    pairs: list

    @property
    def hx(self):
        return self.lx / self.nx

    @property
    def hy(self):
        return self.ly / self.ny

    @property
    def n_seg(self):
        return sum(int(p.nseg.sum()) for p in self.pairs)

    @property
    def n_rays(self):
        return sum(p.K for p in self.pairs)

    def flat(self):
        """Canonical flat geometry: (ray_off per pair [n_pairs+1],
        seg_off per ray [n_rays+1], cell[n_seg], len[n_seg], w[n_rays])."""
        ray_off = np.cumsum([0] + [p.K for p in self.pairs])
        nseg = np.concatenate([p.nseg for p in self.pairs])
        seg_off = np.concatenate([[0], np.cumsum(nseg)])
        cell = np.concatenate([np.concatenate(p.cells) for p in self.pairs])
        ln = np.concatenate([np.concatenate(p.lens) for p in self.pairs])
        w = np.concatenate([p.w for p in self.pairs])
        return ray_off, seg_off, cell, ln, w


def _face_index(nx, ny, lx, ly, x, y, on_x_face, x_side_right):
    hx, hy = lx / nx, ly / ny
    if on_x_face:
        iy = min(max(int(math.floor(y / hy)), 0), ny - 1)
        return (ny + iy) if x_side_right else iy
    ix = min(max(int(math.floor(x / hx)), 0), nx - 1)
    return (2 * ny + nx + ix) if x_side_right else (2 * ny + ix)


def endpoints(nx, ny, lx, ly, c, s, v):
    """Where the characteristic v = const of direction (c, s) enters and
    leaves the domain: (u_in, u_out, entry_face, exit_face, entry_pt,
    exit_pt) of the forward (+u) traversal, or None when the line misses the
    domain (or only grazes it)."""
    hx, hy = lx / nx, ly / ny
    tol = TOL_REL * min(hx, hy)
    # u-interval inside 0 <= x <= lx and 0 <= y <= ly
    ux = sorted(((0.0 + v * s) / c, (lx + v * s) / c))
    uy = sorted(((0.0 - v * c) / s, (ly - v * c) / s))
    u_in = max(ux[0], uy[0])
    u_out = min(ux[1], uy[1])
    if u_out - u_in <= tol:
        return None
    in_on_x = ux[0] >= uy[0]          # tie (corner): x face
    out_on_x = ux[1] <= uy[1]
    x_in, y_in = u_in * c - v * s, u_in * s + v * c
    x_out, y_out = u_out * c - v * s, u_out * s + v * c
    if in_on_x:
        f_in = _face_index(nx, ny, lx, ly, x_in, y_in, True, c < 0)
    else:
        f_in = _face_index(nx, ny, lx, ly, x_in, y_in, False, s < 0)
    if out_on_x:
        f_out = _face_index(nx, ny, lx, ly, x_out, y_out, True, c > 0)
    else:
        f_out = _face_index(nx, ny, lx, ly, x_out, y_out, False, s > 0)
    return u_in, u_out, f_in, f_out, (x_in, y_in), (x_out, y_out)


def trace_characteristic(nx, ny, lx, ly, c, s, v):
    """Cut the characteristic v = const of direction (c, s) into segments.

    All crossings with the interior grid lines x = i hx and y = j hy are
    collected, sorted and merged; each consecutive pair of points is one
    segment whose cell is found from its midpoint.  Returns
    (cells, lens, entry_face, exit_face, entry_pt, exit_pt) or None when the
    line misses the domain.
    """
    hx, hy = lx / nx, ly / ny
    tol = TOL_REL * min(hx, hy)
    ends = endpoints(nx, ny, lx, ly, c, s, v)
    if ends is None:
        return None
    u_in, u_out, f_in, f_out, (x_in, y_in), (x_out, y_out) = ends

    cross = [(i * hx + v * s) / c for i in range(1, nx)]
    cross += [(j * hy - v * c) / s for j in range(1, ny)]
    cross = sorted(u for u in cross if u_in + tol < u < u_out - tol)
    pts = [u_in]
    for u in cross:
        if u - pts[-1] > tol:
            pts.append(u)
    pts.append(u_out)
    cells, lens = [], []
    for u0, u1 in zip(pts[:-1], pts[1:]):
        um = 0.5 * (u0 + u1)
        xm, ym = um * c - v * s, um * s + v * c
        ix = min(max(int(math.floor(xm / hx)), 0), nx - 1)
        iy = min(max(int(math.floor(ym / hy)), 0), ny - 1)
        cells.append(iy * nx + ix)
        lens.append(u1 - u0)
    return (np.array(cells, dtype=np.int64), np.array(lens), f_in, f_out,
            (x_in, y_in), (x_out, y_out))


def _v_range(lx, ly, c, s):
    vs = [-x * s + y * c for x, y in ((0, 0), (lx, 0), (0, ly), (lx, ly))]
    return min(vs), max(vs)


def uniform_offsets(lx, ly, c, s, h_moc):
    """Equal widths delta = W / ceil(W / h_moc) tiling the projected width W;
    centrelines at v_min + (k + 1/2) delta."""
    vmin, vmax = _v_range(lx, ly, c, s)
    W = vmax - vmin
    K = int(math.ceil(W / h_moc * (1.0 - 1e-12)))
    K = max(K, 1)
    delta = W / K
    v = np.array([vmin + (k + 0.5) * delta for k in range(K)])
    return v, np.full(K, delta)


def tube_offsets(nx, ny, lx, ly, c, s, h_moc):
    """The paper's construction: an initial set of characteristics that never
    pass over a vertex (the gaps between the sorted projections of all grid
    vertices onto the v axis), each halved into equal parts until no width
    exceeds h_moc."""
    hx, hy = lx / nx, ly / ny
    proj = sorted(-(i * hx) * s + (j * hy) * c
                  for i in range(nx + 1) for j in range(ny + 1))
    vmin, vmax = proj[0], proj[-1]
    tol = TOL_REL * (vmax - vmin)
    distinct = [proj[0]]
    for p in proj[1:]:
        if p - distinct[-1] > tol:
            distinct.append(p)
    distinct[-1] = vmax
    v, w = [], []
    for lo, hi in zip(distinct[:-1], distinct[1:]):
        width = hi - lo
        parts = 1
        while width / parts > h_moc:
            parts *= 2
        sub = width / parts
        for q in range(parts):
            v.append(lo + (q + 0.5) * sub)
            w.append(sub)
    return np.array(v), np.array(w)


def _crossing(v, nx, ny, lx, ly, c, s, cells):
    """Offsets v (sorted) of the characteristics that cross any of the given
    cells: a line v = const crosses a convex cell iff v lies strictly inside
    the cell's projected extent."""
    hx, hy = lx / nx, ly / ny
    keep = np.zeros(len(v), dtype=bool)
    for cell in cells:
        ix, iy = int(cell) % nx, int(cell) // nx
        cv = [-(x * hx) * s + (y * hy) * c for x in (ix, ix + 1) for y in (iy, iy + 1)]
        keep |= (v > min(cv)) & (v < max(cv))
    return keep


def face_centres(nx, ny, lx, ly):
    """Centres [nb][2] of the boundary faces, numbered [0, ny) x = 0 (row iy),
    [ny, 2ny) x = lx, [2ny, 2ny + nx) y = 0 (column ix), then y = ly."""
    hx, hy = lx / nx, ly / ny
    yc = (np.arange(ny) + 0.5) * hy
    xc = (np.arange(nx) + 0.5) * hx
    return np.concatenate([
        np.stack([np.zeros(ny), yc], 1), np.stack([np.full(ny, lx), yc], 1),
        np.stack([xc, np.zeros(nx)], 1), np.stack([xc, np.full(nx, ly)], 1)])


def _leaving(v, nx, ny, lx, ly, c, s, faces):
    """Offsets of the characteristics whose values on the given boundary
    faces enter the boundary factors: those that enter or leave the domain
    through one of the faces, and, per face and traversal, every one whose
    exit point lies nearest the face's centre (the stand-in for a face that
    no characteristic of the direction leaves through)."""
    ends = [endpoints(nx, ny, lx, ly, c, s, vv) for vv in v]
    inside = np.array([e is not None for e in ends])
    keep = np.zeros(len(v), dtype=bool)
    if not inside.any():
        return keep
    idx = np.nonzero(inside)[0]
    f_in = np.array([ends[k][2] for k in idx])
    f_out = np.array([ends[k][3] for k in idx])
    p_in = np.array([ends[k][4] for k in idx])
    p_out = np.array([ends[k][5] for k in idx])
    centres = face_centres(nx, ny, lx, ly)
    for b in faces:
        keep[idx[(f_in == b) | (f_out == b)]] = True
        for pts in (p_out, p_in):                 # exits of d = 0 and d = 1
            dist = np.hypot(pts[:, 0] - centres[b, 0], pts[:, 1] - centres[b, 1])
            keep[idx[dist == dist.min()]] = True
    return keep


def build(nx, ny, lx, ly, phi, h_moc, mode=UNIFORM, only_cells=None, only_faces=None) -> CharGrid:
    """Characteristic grid for every azimuth pair of the quadrature.

    With ``only_cells`` and/or ``only_faces`` only a subset of the
    characteristics is traced: those crossing the given cells (enough for
    their cell moments, which involve no other characteristic) and those
    whose exit values enter the boundary factors of the given boundary faces.
    Characteristics keep their order (v ascending) and widths."""
    n_az = len(phi)
    if n_az % 2:
        raise ValueError("azimuths must come in opposite pairs")
    pairs = []
    base = 0
    for a in range(n_az // 2):
        ph = float(phi[a])
        if abs(float(phi[a + n_az // 2]) - (ph + math.pi)) > 1e-12:
            raise ValueError("azimuth a + n_az/2 must equal azimuth a + pi")
        c, s = math.cos(ph), math.sin(ph)
        if abs(c) < 1e-12 or abs(s) < 1e-12:
            raise ValueError("directions parallel to a grid axis are not supported")
        if mode == UNIFORM:
            v, w = uniform_offsets(lx, ly, c, s, h_moc)
        else:
            v, w = tube_offsets(nx, ny, lx, ly, c, s, h_moc)
        if only_cells is not None or only_faces is not None:
            keep = np.zeros(len(v), dtype=bool)
            if only_cells is not None:
                keep |= _crossing(v, nx, ny, lx, ly, c, s, only_cells)
            if only_faces is not None:
                keep |= _leaving(v, nx, ny, lx, ly, c, s, only_faces)
            v, w = v[keep], w[keep]
        cells, lens, fi, fo, pi, po, vk, wk = [], [], [], [], [], [], [], []
        for vv, ww in zip(v, w):
            r = trace_characteristic(nx, ny, lx, ly, c, s, vv)
            if r is None:
                continue
            cells.append(r[0]); lens.append(r[1])
            fi.append(r[2]); fo.append(r[3]); pi.append(r[4]); po.append(r[5])
            vk.append(vv); wk.append(ww)
        pr = PairRays(ph, c, s, np.array(vk), np.array(wk), cells, lens,
                      np.array(fi, dtype=np.int64), np.array(fo, dtype=np.int64),
                      np.array(pi).reshape(-1, 2), np.array(po).reshape(-1, 2), base)
        base += int(pr.nseg.sum())
        pairs.append(pr)
    return CharGrid(nx, ny, lx, ly, n_az, h_moc, mode, pairs)


def cell_sets(grid: CharGrid):
    """C(i, m) of eq. (15) for every pair: per pair a list of
    (global segment j, cell i, area A = l w) over all segments, in
    (k, s) order."""
    out = []
    for p in grid.pairs:
        js, cs, As = [], [], []
        j = p.seg_base
        for k in range(p.K):
            for cell, ln in zip(p.cells[k], p.lens[k]):
                js.append(j); cs.append(int(cell)); As.append(ln * p.w[k])
                j += 1
        out.append((np.array(js), np.array(cs), np.array(As)))
    return out
