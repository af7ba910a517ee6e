"""Pins of the interior-face oracle (eq. (16) on interior faces): the widths
of the characteristics crossing a face add up to the face's projected width
exactly on the paper's vertex-avoiding grid; a point field equal to the
crossing coordinate reproduces the face position, which checks the face
assignment and the upwind point of both traversals; isotropic equilibrium
gives f = 1/3."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import faces as OF, rays as R, sweep as OS


def _grid(nx, ny, lx, ly, n_az, h_moc, mode):
    phi, mu, om = W.product_quadrature(n_az, 2)
    return R.build(nx, ny, lx, ly, phi, h_moc, mode), phi, mu, om


@pytest.mark.parametrize("nx,ny,lx,ly,n_az", [(5, 4, 1.0, 0.8, 8), (7, 7, 2.1, 2.1, 12), (3, 6, 0.6, 1.5, 16)])
def test_tube_widths_cover_each_face_exactly(nx, ny, lx, ly, n_az):
    g, phi, mu, om = _grid(nx, ny, lx, ly, n_az, 0.05, R.TUBES)
    hx, hy = lx / nx, ly / ny
    nf = OF.n_faces(nx, ny)
    nfx = (nx - 1) * ny
    for pr, (fs, ks, _, _) in zip(g.pairs, OF.crossings(g)):
        wsum = np.bincount(fs, weights=pr.w[ks], minlength=nf)
        want = np.concatenate([np.full(nfx, hy * abs(pr.c)), np.full(nf - nfx, hx * abs(pr.s))])
        assert np.allclose(wsum, want, rtol=1e-11, atol=1e-13), np.abs(wsum - want).max()


def test_uniform_widths_cover_each_face_within_one_width():
    nx, ny, lx, ly = 6, 5, 1.2, 1.0
    g, phi, mu, om = _grid(nx, ny, lx, ly, 8, 0.03, R.UNIFORM)
    nf = OF.n_faces(nx, ny)
    nfx = (nx - 1) * ny
    for pr, (fs, ks, _, _) in zip(g.pairs, OF.crossings(g)):
        wsum = np.bincount(fs, weights=pr.w[ks], minlength=nf)
        want = np.concatenate([np.full(nfx, ly / ny * abs(pr.c)), np.full(nf - nfx, lx / nx * abs(pr.s))])
        assert np.all(np.abs(wsum - want) <= pr.w.max() * (1 + 1e-12))


def _segment_points(g):
    """Forward start and end points of every segment, [n_seg][2] each."""
    starts, ends = [], []
    for pr in g.pairs:
        dvec = np.array([pr.c, pr.s])
        for k in range(pr.K):
            u = np.concatenate([[0.0], np.cumsum(pr.lens[k])])
            p = pr.entry_pt[k][None, :] + u[:, None] * dvec[None, :]
            starts.append(p[:-1]); ends.append(p[1:])
    return np.concatenate(starts), np.concatenate(ends)


@pytest.mark.parametrize("axis", [0, 1])
def test_point_field_equal_to_the_crossing_coordinate(axis):
    """points[j, d=0] = coordinate of the segment's forward start and
    points[j, d=1] = that of its forward end: both are the upwind point of
    the segment in that traversal.  On an x-face every crossing then carries
    the face's x, so E_f = 4 pi x_f / c and f_f = 1/3 (likewise y on
    y-faces)."""
    nx, ny, lx, ly = 5, 4, 1.0, 0.8
    g, phi, mu, om = _grid(nx, ny, lx, ly, 8, 0.04, R.TUBES)
    st, en = _segment_points(g)
    G = 2
    pts = np.zeros((g.n_seg, 2, len(mu), G))
    pts[:, 0] = st[:, axis][:, None, None]
    pts[:, 1] = en[:, axis][:, None, None]
    c = 3.0
    E, F, f = OF.face_moments(g, phi, mu, om, pts, c)
    nfx = (nx - 1) * ny
    if axis == 0:
        sel = np.arange(nfx)
        coord = (np.arange(nfx) % (nx - 1) + 1) * (lx / nx)
    else:
        sel = np.arange(nfx, OF.n_faces(nx, ny))
        coord = ((np.arange(len(sel)) // nx) + 1) * (ly / ny)
    assert np.allclose(E[:, sel], 4 * math.pi * coord[None, :] / c, rtol=1e-12)
    assert np.allclose(F[:, :, sel], 0.0, atol=1e-12)
    assert np.allclose(f[:, 0, sel], 1 / 3, atol=1e-12) and np.allclose(f[:, 2, sel], 1 / 3, atol=1e-12)
    assert np.allclose(f[:, 1, sel], 0.0, atol=1e-12)


def test_isotropic_equilibrium_on_interior_faces():
    nx, ny = 6, 5
    phi, mu, om = W.product_quadrature(8, 2)
    edges = W.group_edges(3, 0.01, 5.0)
    T = np.full(nx * ny, 0.5)
    kap = W.fc_opacity(W.group_midpoints(edges), T)
    B = W.group_planck(edges, T)
    g = R.build(nx, ny, 1.2, 1.0, phi, 0.05, R.UNIFORM)
    nb = 2 * (nx + ny)
    I_in = np.repeat(B[:, :1].T[None, :, :], nb, axis=0).repeat(len(phi) * len(mu), axis=1)
    state = OS.initial_state(g, len(mu), B)
    pts = np.zeros_like(state)
    OS.sweep(g, mu, kap, B, 3.0, state, I_in, points=pts)
    c = 2.0
    E, F, f = OF.face_moments(g, phi, mu, om, pts, c)
    assert np.allclose(E, 4 * math.pi * B[:, :1] / c, rtol=1e-12)
    assert np.allclose(F, 0.0, atol=1e-12 * B.max())
    assert np.allclose(f[:, [0, 2, 3]], 1 / 3, atol=1e-12) and np.allclose(f[:, 1], 0.0, atol=1e-12)
    # the face average of a constant field is that constant, whatever the face
    assert np.allclose(OF.face_direction_averages(g, len(mu), pts), B.T[0][None, None, :], rtol=1e-12)
