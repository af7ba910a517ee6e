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
