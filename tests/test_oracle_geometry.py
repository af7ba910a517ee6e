"""Pins for the oracle's characteristic grid (paper: segment lengths between
cell-boundary crossings, widths w_k, segment areas eq. (14), and the
vertex-avoiding, width-halving construction that follows eq. (16))."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import rays

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def chord(lx, ly, c, s, v):
    """Length of the line v = const inside the rectangle, from the clip
    interval (plain geometry, independent of the segment cutting)."""
    ux = sorted(((v * s) / c, (lx + v * s) / c))
    uy = sorted(((-v * c) / s, (ly - v * c) / s))
    return max(0.0, min(ux[1], uy[1]) - max(ux[0], uy[0]))


def sampled_segments(nx, ny, lx, ly, c, s, v, n=400_001):
    """Brute force: sample the line densely, label each sample by its cell
    and count runs -- an independent way to get the cell sequence and
    approximate lengths."""
    hx, hy = lx / nx, ly / ny
    ux = sorted(((v * s) / c, (lx + v * s) / c))
    uy = sorted(((-v * c) / s, (ly - v * c) / s))
    u0, u1 = max(ux[0], uy[0]), min(ux[1], uy[1])
    u = u0 + (np.arange(n) + 0.5) / n * (u1 - u0)
    x, y = u * c - v * s, u * s + v * c
    cell = np.clip(np.floor(y / hy), 0, ny - 1).astype(int) * nx + \
        np.clip(np.floor(x / hx), 0, nx - 1).astype(int)
    brk = np.nonzero(np.diff(cell))[0]
    starts = np.concatenate([[0], brk + 1])
    ends = np.concatenate([brk + 1, [n]])
    return cell[starts], (ends - starts) / n * (u1 - u0)


@pytest.mark.parametrize("nx,ny,lx,ly,phi", [(1, 1, 1.0, 1.0, 0.3), (2, 2, 2.0, 2.0, 0.7),
                                             (3, 2, 1.5, 1.2, 2.1), (4, 4, 6.0, 6.0, 4.0),
                                             (5, 3, 2.0, 3.0, 5.5)])
def test_segments_vs_dense_sampling(nx, ny, lx, ly, phi):
    c, s = math.cos(phi), math.sin(phi)
    v, w = rays.uniform_offsets(lx, ly, c, s, min(lx / nx, ly / ny) / 3)
    for vv in v:
        r = rays.trace_characteristic(nx, ny, lx, ly, c, s, vv)
        cells_ref, lens_ref = sampled_segments(nx, ny, lx, ly, c, s, vv)
        # runs shorter than the sampling pitch may be missed by sampling
        L = chord(lx, ly, c, s, vv)
        keep = r[1] > 4 * L / 400_001
        assert np.array_equal(r[0][keep], cells_ref)
        assert np.allclose(r[1][keep], lens_ref, atol=2 * L / 400_001)
        assert abs(r[1].sum() - L) <= 1e-13 * max(lx, ly)


def test_segment_points_lie_on_grid_lines():
    nx, ny, lx, ly = 7, 5, 3.5, 2.0
    hx, hy = lx / nx, ly / ny
    for phi in np.linspace(0.1, 2 * math.pi - 0.1, 13):
        c, s = math.cos(phi), math.sin(phi)
        if min(abs(c), abs(s)) < 1e-3:
            continue
        v, _ = rays.uniform_offsets(lx, ly, c, s, 0.07)
        for vv in v[::7]:
            cells, lens, fi, fo, pin, pout = rays.trace_characteristic(nx, ny, lx, ly, c, s, vv)
            assert np.all(lens > 0)
            u = np.cumsum(np.concatenate([[0.0], lens]))
            x = pin[0] + u * c
            y = pin[1] + u * s
            for q in range(1, len(u) - 1):       # interior points: on a grid line
                dx = abs(x[q] / hx - round(x[q] / hx))
                dy = abs(y[q] / hy - round(y[q] / hy))
                assert min(dx, dy) < 1e-9
            for q in range(len(cells)):          # each segment's midpoint in its cell
                xm, ym = 0.5 * (x[q] + x[q + 1]), 0.5 * (y[q] + y[q + 1])
                assert cells[q] == int(ym // hy) * nx + int(xm // hx)
            # faces are the boundary faces that hold the end points
            nb = W.boundary_faces(nx, ny)
            for f, (px, py) in ((fi, pin), (fo, pout)):
                assert 0 <= f < len(nb)
                if f < 2 * ny:
                    assert abs(px - (0 if f < ny else lx)) < 1e-12
                    assert int(min(py // hy, ny - 1)) == f % ny
                else:
                    assert abs(py - (0 if f < 2 * ny + nx else ly)) < 1e-12
                    assert int(min(px // hx, nx - 1)) == (f - 2 * ny) % nx


def test_uniform_widths_tile_projected_width_and_cell_areas():
    p = W.config(0)
    g = rays.build(p.nx, p.ny, p.lx, p.ly, p.phi, p.h_moc, rays.UNIFORM)
    h = p.lx / p.nx
    for pr in g.pairs:
        W_ = p.lx * abs(pr.s) + p.ly * abs(pr.c)
        assert abs(pr.w.sum() - W_) < 1e-12
        assert np.all(pr.w <= p.h_moc * (1 + 1e-12))
        delta = pr.w[0]
        # traced area per cell: |delta sum l - h^2| <= delta^2 / (2 |s c|)
        # (midpoint rule on the piecewise-linear chord-length function)
        traced = np.zeros(p.nx * p.ny)
        for k in range(pr.K):
            np.add.at(traced, pr.cells[k], pr.lens[k] * pr.w[k])
        bound = delta ** 2 / (2 * abs(pr.s * pr.c))
        assert np.all(np.abs(traced - h * h) <= bound + 1e-13)
        # every chord fully cut
        for k in range(pr.K):
            assert abs(pr.lens[k].sum() - chord(p.lx, p.ly, pr.c, pr.s, pr.v[k])) < 1e-13


@pytest.mark.parametrize("n,h_moc", [(4, 0.5), (8, 0.2), (16, 0.05)])
def test_tube_construction_conserves_cell_area_exactly(n, h_moc):
    phi, _, _ = W.product_quadrature(8, 2)
    L = 6.0
    g = rays.build(n, n, L, L, phi, h_moc, rays.TUBES)
    h = L / n
    for pr in g.pairs:
        assert np.all(pr.w <= h_moc * (1 + 1e-12))
        traced = np.zeros(n * n)
        for k in range(pr.K):
            np.add.at(traced, pr.cells[k], pr.lens[k] * pr.w[k])
        assert np.allclose(traced, h * h, rtol=1e-12, atol=0)
        # no centreline passes a vertex: every grid-vertex projection is
        # at least a tiny distance from every centreline
        proj = np.array([-(i * h) * pr.s + (j * h) * pr.c for i in range(n + 1) for j in range(n + 1)])
        dmin = np.min(np.abs(proj[:, None] - pr.v[None, :]))
        assert dmin > 1e-9


def test_paper_claim_characteristics_per_cell():
    fc = json.load(open(os.path.join(GOLDEN, "fleck_cummings.json")))
    cl = fc["claim_min_characteristics_per_cell_per_direction"]
    h, hm = cl["h_mat_cm"], cl["h_moc_cm"]
    n = 8                                   # a 1.2 x 1.2 cm corner of the slab
    phi, _, _ = W.product_quadrature(8, 2)
    g = rays.build(n, n, n * h, n * h, phi[[0, 4]], hm, rays.TUBES)
    pr = g.pairs[0]
    count = np.zeros(n * n, dtype=int)
    for k in range(pr.K):
        count[np.unique(pr.cells[k])] += 1
    assert count.min() > cl["more_than"]


def test_paper_claim_halving_width_need_not_double():
    phi, _, _ = W.product_quadrature(16, 2)
    L, n = 6.0, 16
    ratios = []
    for a in range(8):
        k1 = len(rays.tube_offsets(n, n, L, L, math.cos(phi[a]), math.sin(phi[a]), L / n / 2)[0])
        k2 = len(rays.tube_offsets(n, n, L, L, math.cos(phi[a]), math.sin(phi[a]), L / n / 4)[0])
        assert k1 <= k2 <= 2 * k1
        ratios.append(k2 / k1)
    assert min(ratios) < 2.0


def test_global_segment_numbering():
    p = W.config(0)
    g = rays.build(p.nx, p.ny, p.lx, p.ly, p.phi, p.h_moc)
    ray_off, seg_off, cell, ln, w = g.flat()
    assert ray_off[-1] == g.n_rays and seg_off[-1] == g.n_seg == len(cell)
    j = 0
    for pr in g.pairs:
        assert pr.seg_base == j
        for k in range(pr.K):
            assert np.array_equal(cell[j:j + len(pr.cells[k])], pr.cells[k])
            j += len(pr.cells[k])


def test_subset_build_traces_exactly_the_crossing_characteristics():
    p = W.config(0)
    g = rays.build(p.nx, p.ny, p.lx, p.ly, p.phi, p.h_moc)
    cells = [0, 37, 200, 255]
    sub = rays.build(p.nx, p.ny, p.lx, p.ly, p.phi, p.h_moc, only_cells=cells)
    for full, part in zip(g.pairs, sub.pairs):
        want = [k for k in range(full.K) if set(cells) & set(full.cells[k].tolist())]
        assert np.array_equal(part.v, full.v[want])
        for q, k in enumerate(want):
            assert np.array_equal(part.cells[q], full.cells[k])
            assert np.array_equal(part.lens[q], full.lens[k])

