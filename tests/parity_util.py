"""Error metrics shared by the parity tests.

E: max over (g, i) of |E - E_ref| / E_ref where E_ref > floor * max_i E_ref[g]
   (the relative metric is meaningless where a group's intensity has
   underflowed); below the floor the absolute difference must be under the
   floor itself.
F: max |F - F_ref| / (c E_ref) over the same cells (|F| <= c E).
f: max |f_ab - f_ref_ab| over the same cells (f is dimensionless, trace 1).
"""
import numpy as np

FLOOR = 1e-30


def mask_of(E_ref, floor=FLOOR):
    return E_ref > floor * E_ref.max(axis=-1, keepdims=True)


def err_E(E, E_ref, floor=FLOOR):
    m = mask_of(E_ref, floor)
    rel = np.abs(E - E_ref)[m] / E_ref[m]
    below = np.abs(E - E_ref)[~m]
    lim = (floor * E_ref.max(axis=-1, keepdims=True) * np.ones_like(E_ref))[~m]
    assert np.all(below <= lim + 1e-300), "absolute error above the floor where E_ref is negligible"
    return float(rel.max()) if rel.size else 0.0


def err_F(F, F_ref, E_ref, c, floor=FLOOR):
    m = mask_of(E_ref, floor)
    d = np.abs(F - F_ref).max(axis=-2)          # over components
    return float((d[m] / (c * E_ref[m])).max()) if m.any() else 0.0


def err_f(f, f_ref, E_ref, floor=FLOOR):
    m = mask_of(E_ref, floor)
    d = np.abs(f - f_ref).max(axis=-2)
    return float(d[m].max()) if m.any() else 0.0


def err_rel(x, ref, floor=FLOOR):
    """Relative error of a non-negative field with a floor relative to its max."""
    scale = np.abs(ref).max()
    m = np.abs(ref) > floor * scale
    if not m.any():
        return float(np.abs(x - ref).max())
    return float((np.abs(x - ref)[m] / np.abs(ref)[m]).max())


# ---------------------------------------------------------------------------
# samples for the full-size comparisons
# ---------------------------------------------------------------------------

TILE = 16          # cells per side of the moment kernel's tiles


def sample_cells(nx, ny, n, seed):
    """At least n distinct cells: the four corners, cells on every domain
    edge, cells on both sides of tile edges (x = 16 j and y = 16 j cell
    lines), the rest at random.  Sorted."""
    rng = np.random.default_rng(seed)
    cells = {0, nx - 1, (ny - 1) * nx, nx * ny - 1}
    for _ in range(3):
        if nx > 2:
            ix = int(rng.integers(1, nx - 1))
            cells |= {ix, (ny - 1) * nx + ix}
        if ny > 2:
            iy = int(rng.integers(1, ny - 1))
            cells |= {iy * nx, iy * nx + nx - 1}
    for t in range(TILE, max(nx, ny), TILE):
        if t < nx:
            iy = int(rng.integers(0, ny))
            cells |= {iy * nx + t - 1, iy * nx + t}
        if t < ny:
            ix = int(rng.integers(0, nx))
            cells |= {(t - 1) * nx + ix, t * nx + ix}
        if len(cells) >= n // 2:
            break
    while len(cells) < min(n, nx * ny):
        cells.add(int(rng.integers(0, nx * ny)))
    return np.array(sorted(cells), dtype=np.int64)


def grazing_faces(prob, mode=0):
    """Boundary faces that some outgoing direction leaves through no
    characteristic, from the oracle's characteristic offsets and end points
    (no segment tracing)."""
    import math
    from oracle import rays as orays
    nx, ny, lx, ly = prob.nx, prob.ny, prob.lx, prob.ly
    nb = 2 * (nx + ny)
    normals = np.zeros((nb, 2))
    normals[:ny] = (-1, 0); normals[ny:2 * ny] = (1, 0)
    normals[2 * ny:2 * ny + nx] = (0, -1); normals[2 * ny + nx:] = (0, 1)
    empty = set()
    for a in range(prob.n_az // 2):
        c, s = math.cos(prob.phi[a]), math.sin(prob.phi[a])
        if mode == orays.UNIFORM:
            v, _ = orays.uniform_offsets(lx, ly, c, s, prob.h_moc)
        else:
            v, _ = orays.tube_offsets(nx, ny, lx, ly, c, s, prob.h_moc)
        ends = [orays.endpoints(nx, ny, lx, ly, c, s, vv) for vv in v]
        f_in = np.array([e[2] for e in ends if e is not None])
        f_out = np.array([e[3] for e in ends if e is not None])
        for d, fexit in ((0, f_out), (1, f_in)):
            dirn = (1.0 if d == 0 else -1.0) * np.array([c, s])
            hit = np.zeros(nb, dtype=bool)
            hit[fexit] = True
            empty |= set(np.nonzero((normals @ dirn > 0.0) & ~hit)[0].tolist())
    return sorted(empty)


def sample_faces(prob, n, seed, mode=0):
    """About n boundary faces: the faces next to the four corners, up to
    n / 2 faces that a grazing direction leaves empty, the rest at random."""
    rng = np.random.default_rng(seed)
    nx, ny = prob.nx, prob.ny
    nb = 2 * (nx + ny)
    faces = {0, ny - 1, ny, 2 * ny - 1, 2 * ny, 2 * ny + nx - 1, 2 * ny + nx, nb - 1}
    empty = grazing_faces(prob, mode)
    if empty:
        faces |= set(int(b) for b in rng.choice(empty, min(len(empty), n // 2), replace=False))
    while len(faces) < min(n, nb):
        faces.add(int(rng.integers(0, nb)))
    return np.array(sorted(faces), dtype=np.int64), empty


def bnd_errors(got, ref, floor=FLOOR):
    """Boundary factors [G][faces][8] (Phi+, J+, Phi-, J-, C, f_xx, f_xy,
    f_yy), in the metrics of E: per group, Phi+, J+, Phi- and J- relative
    where the reference exceeds `floor` times the group's largest over the
    faces (absolute error below that, bounded by the floor); C absolute where
    Phi+ exceeds the floor of Phi+; the face tensor absolute where Phi+ + Phi-
    exceeds the floor of Phi+ + Phi-.  floor = 0 compares every entry (C and
    the face tensor included).  Returns (worst relative, worst absolute)."""
    rel = 0.0
    for q in range(4):
        r = ref[..., q]
        m = r > floor * r.max(axis=-1, keepdims=True) if floor > 0 else np.abs(r) > 0
        d = np.abs(got[..., q] - r)
        if m.any():
            rel = max(rel, float((d[m] / np.abs(r[m])).max()))
        lim = (floor * np.abs(r).max(axis=-1, keepdims=True) * np.ones_like(r))[~m]
        assert np.all(d[~m] <= lim + 1e-300), "absolute boundary error above the floor where it is negligible"
    if floor > 0:
        pp = ref[..., 0]
        mc = pp > floor * pp.max(axis=-1, keepdims=True)
        s = ref[..., 0] + ref[..., 2]
        mf = s > floor * s.max(axis=-1, keepdims=True)
    else:
        mc = mf = np.ones(ref.shape[:-1], dtype=bool)
    ab = 0.0
    if mc.any():
        ab = max(ab, float(np.abs(got[..., 4] - ref[..., 4])[mc].max()))
    if mf.any():
        ab = max(ab, float(np.abs(got[..., 5:] - ref[..., 5:]).max(axis=-1)[mf].max()))
    return rel, ab


def bnd_worst(got, ref):
    """Where C differs most: (group, face, C, C_ref, Phi+_ref, the group's
    largest Phi+_ref) -- for the message of a failing comparison."""
    d = np.abs(got[..., 4] - ref[..., 4])
    g, b = np.unravel_index(int(np.argmax(d)), d.shape)
    return (int(g), int(b), float(got[g, b, 4]), float(ref[g, b, 4]), float(ref[g, b, 0]),
            float(ref[g, :, 0].max()))
