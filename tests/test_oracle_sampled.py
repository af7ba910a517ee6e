"""Pins of the sampled oracle (``solve.run_sampled`` over a grid built with
``rays.build(..., only_cells=..., only_faces=...)``), the checker of every
full-size GPU parity test.

* It equals the whole-grid oracle (``solve.run``) on the sampled cells and
  boundary faces, step after step, with material data that change every
  step: uniform and vertex-avoiding grids, ragged grids whose sampled cells
  sit on the corners, the domain edges and both sides of a 16-cell tile
  edge, and faces that a grazing direction leaves empty.  The segment states
  and exit intensities of the traced subset equal the whole grid's rows of
  the same characteristics.
* Planted mistakes in the subset selection and the sampled-row reductions
  fail that comparison.
* The empty-face stand-in (the characteristic whose exit point lies nearest
  the face centre) is worked by hand on a 3 x 2 grid, where the choice
  changes the factors (fixture tests/golden/grazing_boundary_face.json)."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import moments, rays, solve

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "grazing_boundary_face.json")


def _changing_problem(nx, ny, lx, ly, n_az, n_pol, G, h_moc, steps, seed):
    """Random incoming intensities on every face and a temperature field that
    changes every step (so a stale material step or a lost state shows)."""
    rng = np.random.default_rng(seed)
    Ts = [rng.uniform(0.01, 1.0, nx * ny) for _ in range(steps)]
    p = W.make_problem(nx, ny, lx, ly, n_az, n_pol, G, 0.001, 20.0, h_moc, 1.3, Ts, name="changing")
    p.I_in = rng.uniform(0.0, 0.4, p.I_in.shape)
    p.state0 = W.group_planck(p.edges, rng.uniform(0.005, 0.5, nx * ny))
    return p


def _empty_faces(grid):
    """Boundary faces that some outgoing direction leaves through no
    characteristic (on the whole grid)."""
    nb = 2 * (grid.nx + grid.ny)
    normals = moments.face_normals(grid.nx, grid.ny)
    out = set()
    for pr in grid.pairs:
        for d, fexit in ((0, pr.exit_face), (1, pr.entry_face)):
            dirn = (1.0 if d == 0 else -1.0) * np.array([pr.c, pr.s])
            for b in range(nb):
                if normals[b] @ dirn > 0.0 and not np.any(fexit == b):
                    out.add(b)
    return sorted(out)


def _sample(p, grid, rng):
    nx, ny = p.nx, p.ny
    corners = [0, nx - 1, (ny - 1) * nx, nx * ny - 1]
    edges = [rng.integers(1, nx - 1), (ny - 1) * nx + rng.integers(1, nx - 1),
             rng.integers(1, ny - 1) * nx, rng.integers(1, ny - 1) * nx + nx - 1]
    tile = []
    if nx > 16:                                   # both sides of the x = 16 h tile edge
        iy = int(rng.integers(0, ny))
        tile = [iy * nx + 15, iy * nx + 16]
    cells = np.array(sorted(set(int(c) for c in corners + edges + tile + list(rng.choice(nx * ny, 3)))))
    empty = _empty_faces(grid)
    faces = sorted(set([0, ny, 2 * ny, 2 * ny + nx, 2 * (nx + ny) - 1] + empty[:6]))
    return cells, faces, empty


def _row_map(sub, full):
    """Global segment rows and ray indices of the subset's characteristics in
    the whole grid (matched by offset, which both builds compute alike)."""
    rows, rays_ = [], []
    for ps, pf in zip(sub.pairs, full.pairs):
        ray_base = sum(q.K for q in full.pairs[:full.pairs.index(pf)])
        first = np.concatenate([[0], np.cumsum(pf.nseg)]) + pf.seg_base
        for k, v in enumerate(ps.v):
            kf = int(np.nonzero(pf.v == v)[0][0])
            assert np.array_equal(ps.cells[k], pf.cells[kf])
            rows.append(np.arange(first[kf], first[kf] + pf.nseg[kf]))
            rays_.append((ray_base + kf, kf))
    return np.concatenate(rows), rays_


CASES = [
    # nx, ny, lx, ly, n_az, n_pol, G, h_moc, mode
    (20, 12, 2.0, 1.2, 8, 2, 3, 0.045, rays.UNIFORM),
    (18, 5, 1.8, 0.5, 12, 3, 2, 0.04, rays.UNIFORM),
    (9, 7, 0.9, 0.7, 8, 2, 2, 0.05, rays.TUBES),
]


@pytest.mark.parametrize("case", CASES)
def test_sampled_run_equals_whole_run(case):
    nx, ny, lx, ly, n_az, n_pol, G, h, mode = case
    p = _changing_problem(nx, ny, lx, ly, n_az, n_pol, G, h, steps=3, seed=nx * 100 + ny)
    full_grid = rays.build(nx, ny, lx, ly, p.phi, h, mode)
    ref = solve.run(p, grid=full_grid)
    cells, faces, empty = _sample(p, full_grid, np.random.default_rng(7))
    assert len(empty) > 0 or mode == rays.TUBES          # grazing faces are sampled
    sub = rays.build(nx, ny, lx, ly, p.phi, h, mode, only_cells=cells, only_faces=faces)
    assert sub.n_rays < full_grid.n_rays
    got = solve.run_sampled(p, sub, cells, faces=faces)
    for t in range(3):
        r, g = ref["steps"][t], got["steps"][t]
        for k, sl in (("E", np.s_[:, cells]), ("F", np.s_[:, :, cells]), ("f", np.s_[:, :, cells])):
            assert np.allclose(g[k], r[k][sl], rtol=1e-14, atol=0), (t, k)
        assert np.allclose(g["bnd"], r["bnd"][:, faces], rtol=1e-14, atol=1e-300), t
    rows, rmap = _row_map(sub, full_grid)
    assert np.array_equal(got["state"], ref["state"][rows])
    for a, ps in enumerate(sub.pairs):
        pf = full_grid.pairs[a]
        ks = [int(np.nonzero(pf.v == v)[0][0]) for v in ps.v]
        assert np.array_equal(got["exits"][a], ref["exits"][a][:, ks])


def test_sampled_grid_selects_exactly_what_the_samples_need():
    """The subset holds every characteristic crossing a sampled cell or
    leaving through a sampled face, the nearest-exit stand-ins, and no other
    one crossing none of the cells (checked on the whole grid)."""
    p = _changing_problem(20, 12, 2.0, 1.2, 8, 2, 1, 0.045, steps=1, seed=3)
    full = rays.build(p.nx, p.ny, p.lx, p.ly, p.phi, p.h_moc)
    cells, faces, _ = _sample(p, full, np.random.default_rng(1))
    sub = rays.build(p.nx, p.ny, p.lx, p.ly, p.phi, p.h_moc, only_cells=cells, only_faces=faces)
    centres = rays.face_centres(p.nx, p.ny, p.lx, p.ly)
    for ps, pf in zip(sub.pairs, full.pairs):
        need = set()
        for k in range(pf.K):
            if set(pf.cells[k].tolist()) & set(cells.tolist()):
                need.add(k)
            if pf.entry_face[k] in faces or pf.exit_face[k] in faces:
                need.add(k)
        for b in faces:
            for pts in (pf.exit_pt, pf.entry_pt):
                dist = np.hypot(pts[:, 0] - centres[b, 0], pts[:, 1] - centres[b, 1])
                need |= set(np.nonzero(dist == dist.min())[0].tolist())
        have = {int(np.nonzero(pf.v == v)[0][0]) for v in ps.v}
        assert have == need


# ---------------------------------------------------------------------------
# planted mistakes: each must fail the comparison with the whole-grid run
# ---------------------------------------------------------------------------

def _narrow_crossing(v, nx, ny, lx, ly, c, s, cells):
    # mistake: a cell's projected extent taken as its centre's projection
    # +- half a cell width (misses the characteristics clipping its corners)
    hx, hy = lx / nx, ly / ny
    keep = np.zeros(len(v), dtype=bool)
    for cell in cells:
        ix, iy = int(cell) % nx, int(cell) // nx
        vc = -((ix + 0.5) * hx) * s + ((iy + 0.5) * hy) * c
        keep |= np.abs(v - vc) < 0.5 * hx
    return keep


def _no_stand_in(v, nx, ny, lx, ly, c, s, faces):
    # mistake: only characteristics entering or leaving through the faces
    keep = np.zeros(len(v), dtype=bool)
    for k, vv in enumerate(v):
        e = rays.endpoints(nx, ny, lx, ly, c, s, vv)
        if e is not None and (e[2] in faces or e[3] in faces):
            keep[k] = True
    return keep


_orig_cda = moments.cell_direction_averages


def _shifted_rows(grid, n_pol, state, cells=None):
    # mistake: sampled rows taken one cell off
    return _orig_cda(grid, n_pol, state, None if cells is None else np.minimum(np.asarray(cells) + 1,
                                                                                grid.nx * grid.ny - 1))


@pytest.mark.parametrize("target,bad", [(rays, ("_crossing", _narrow_crossing)),
                                        (rays, ("_leaving", _no_stand_in)),
                                        (moments, ("cell_direction_averages", _shifted_rows))])
def test_planted_mistakes_are_caught(monkeypatch, target, bad):
    monkeypatch.setattr(target, *bad)
    with pytest.raises((AssertionError, ValueError, IndexError)):
        test_sampled_run_equals_whole_run(CASES[0])


# ---------------------------------------------------------------------------
# the empty-face stand-in, worked by hand
# ---------------------------------------------------------------------------

def _grazing_problem(fx):
    gdef = fx["grid"]
    nx, ny, lx, ly = gdef["nx"], gdef["ny"], gdef["lx"], gdef["ly"]
    p0, p1 = fx["azimuths"]
    phi = np.array([p0, p1, p0 + math.pi, p1 + math.pi])
    mu = np.array([0.0])
    omega = np.full(4, math.pi)
    mat = fx["material"]
    cells = nx * ny
    kap = np.full((1, cells), mat["kappa"])
    pla = np.full((1, cells), mat["planck"])
    nb = 2 * (nx + ny)
    I_in = np.full((nb, 4, 1), fx["I_in_default"])
    for b, m, val in fx["I_in"]:
        I_in[b, m, 0] = val
    return W.Problem(nx, ny, lx, ly, phi, mu, omega, np.array([0.001, 10.0]), fx["h_moc"], mat["c_dt"],
                     [kap], [pla], I_in, np.full((1, cells), mat["state0"]), [np.ones(cells)], "grazing")


def _chord(expr):
    """A chord length written in the fixture as a closed form such as
    "3 / cos(0.15)"."""
    return float(eval(expr, {"__builtins__": {}, "cos": math.cos, "sin": math.sin}))


def test_empty_face_takes_the_nearest_exit_worked_by_hand():
    fx = json.load(open(GOLDEN))
    p = _grazing_problem(fx)
    out = solve.run(p)
    bnd = out["steps"][0]["bnd"][0]                          # [nb][8]
    kt = fx["material"]["kappa"]
    p0, p1 = fx["azimuths"]
    om_dir = {0: (math.cos(p0), math.sin(p0)), 1: (math.cos(p1), math.sin(p1)),
              2: (-math.cos(p0), -math.sin(p0)), 3: (-math.cos(p1), -math.sin(p1))}
    I_in = p.I_in[:, :, 0]
    for case in fx["cases"]:
        b = case["face"]
        n = np.array(case["normal"], float)
        near = case["nearest"]
        I = {}
        I[case["empty_direction"]] = I_in[near["enters_through"], case["empty_direction"]] * \
            math.exp(-kt * _chord(near["chord"]))
        oo = case["other_outgoing"]
        I[oo["direction"]] = np.mean([I_in[f, oo["direction"]] for f in oo["enter_through"]]) * \
            math.exp(-kt * _chord(oo["chord"].split(" each")[0]))
        for m in case["incoming"]:
            I[m] = I_in[b, m]
        w = math.pi
        dn = {m: om_dir[m][0] * n[0] + om_dir[m][1] * n[1] for m in range(4)}
        out_m = [case["empty_direction"], oo["direction"]]
        Pp = w * sum(I[m] for m in out_m)
        Jp = w * sum(dn[m] * I[m] for m in out_m)
        Pm = w * sum(I[m] for m in case["incoming"])
        Jm = w * sum(abs(dn[m]) * I[m] for m in case["incoming"])
        S = w * sum(I.values())
        fxx = w * sum(om_dir[m][0] ** 2 * I[m] for m in range(4)) / S
        fxy = w * sum(om_dir[m][0] * om_dir[m][1] * I[m] for m in range(4)) / S
        fyy = w * sum(om_dir[m][1] ** 2 * I[m] for m in range(4)) / S
        want = [Pp, Jp, Pm, Jm, Jp / Pp, fxx, fxy, fyy]
        assert np.allclose(bnd[b], want, rtol=1e-13, atol=1e-15), (b, bnd[b], want)
        # the pin discriminates: the other plausible choices give other factors
        for alt in case["alternatives"].values():
            I_alt = I_in[alt["enters_through"], case["empty_direction"]] * math.exp(-kt * _chord(alt["chord"]))
            Pp_alt = w * (I_alt + I[oo["direction"]])
            assert abs(Pp_alt - Pp) > 1e-3 * Pp
        # the nearest exit point is the one the fixture names
        pr = out["grid"].pairs[near["pair"]]
        pts = pr.exit_pt if case["empty_direction"] < 2 else pr.entry_pt
        c = rays.face_centres(p.nx, p.ny, p.lx, p.ly)[b]
        dist = np.hypot(pts[:, 0] - c[0], pts[:, 1] - c[1])
        assert int(np.argmin(dist)) == near["ray"]
        assert abs(dist.min() - near["distance"]) < 1e-6
        assert np.allclose(pts[near["ray"]], near["exit_point"], atol=1e-6)


def test_sampled_faces_include_the_stand_ins():
    """The grazing faces' factors from a subset that samples only them equal
    the whole-grid ones (the stand-in characteristic is in the subset)."""
    fx = json.load(open(GOLDEN))
    p = _grazing_problem(fx)
    ref = solve.run(p)["steps"][0]["bnd"]
    faces = [c["face"] for c in fx["cases"]]
    sub = rays.build(p.nx, p.ny, p.lx, p.ly, p.phi, p.h_moc, only_faces=faces)
    got = solve.run_sampled(p, sub, np.zeros(0, dtype=np.int64), faces=faces)["steps"][0]["bnd"]
    assert np.array_equal(got, ref[:, faces])


def test_worker_blocks_equal_the_whole_run():
    """The block-parallel form used at the largest sizes (tests/oracle_pool):
    blocks of samples in spawned workers, put side by side, equal the
    whole-grid oracle on those samples."""
    from tests import oracle_pool
    from tests.parity_util import sample_cells, sample_faces
    p = W.config(0, steps=2)
    ref = solve.run(p)["steps"]
    cells = sample_cells(p.nx, p.ny, 12, 0)
    faces, _ = sample_faces(p, 6, 0)
    jobs = [(("config", 0, 2), cb, fb) for cb, fb in zip(oracle_pool.blocks(cells, 3), oracle_pool.blocks(faces, 3))]
    res = oracle_pool.run_blocks(jobs)
    for t in range(2):
        for k, sl in (("E", np.s_[:, cells]), ("F", np.s_[:, :, cells]), ("f", np.s_[:, :, cells])):
            got = np.concatenate([r[t][k] for r in res], axis=-1)
            assert np.allclose(got, ref[t][k][sl], rtol=1e-14, atol=0)
        got_b = np.concatenate([r[t]["bnd"] for r in res], axis=1)
        assert np.allclose(got_b, ref[t]["bnd"][:, faces], rtol=1e-14, atol=1e-300)
