"""Consistency pin for the oracle (geometry + sweep + area-weighted cell
averages together): in a uniform medium with a uniform source S and a uniform
incoming intensity I_b, the exact intensity is
    I(r, Omega) = S + (I_b - S) exp(-kappa_t s(r) / sin zeta),
with s(r) the in-plane distance from r back to the boundary along -Omega
(eq. (10)-(12) integrated exactly).  As the characteristic spacing shrinks,
the per-direction cell averages of eq. (14)-(15) must converge, at second
order, to the cell average of that field, computed here independently (the
x-integral in closed form, the y-integral by Gauss-Legendre between kinks)."""
import math

import numpy as np

import workloads as W
from oracle import moments, rays, sweep

XG, WG = np.polynomial.legendre.leggauss(20)


def _exact_cell_average(x0, x1, y0, y1, c, s, kt, S, Ib):
    """(1/area) * integral over the cell of S + (Ib - S) exp(-kt * min(x/c, y/s))
    for a direction with c, s > 0 (entry through x = 0 or y = 0)."""
    def inner(y):                      # integral over x in [x0, x1] at fixed y
        xk = c * y / s                 # the back-trace leaves through x = 0 for x < xk
        a, b = x0, min(x1, xk)
        part = 0.0
        if b > a:
            part += (c / kt) * (math.exp(-kt * a / c) - math.exp(-kt * b / c))
        lo = max(x0, xk)
        if x1 > lo:
            part += (x1 - lo) * math.exp(-kt * y / s)
        return part
    cuts = sorted({y0, y1, *[min(max(s * x / c, y0), y1) for x in (x0, x1)]})
    tot = 0.0
    for ya, yb in zip(cuts[:-1], cuts[1:]):
        if yb <= ya:
            continue
        ys = 0.5 * (yb - ya) * XG + 0.5 * (ya + yb)
        tot += 0.5 * (yb - ya) * sum(w * inner(y) for w, y in zip(WG, ys))
    area = (x1 - x0) * (y1 - y0)
    return S + (Ib - S) * tot / area


def test_cell_averages_converge_to_the_exact_field():
    n, L = 4, 1.0
    h = L / n
    phi = np.array([0.4, 0.4 + math.pi])
    mu = np.array([0.0])
    kap = np.full((1, n * n), 2.5)
    B = np.full((1, n * n), 0.7)
    c_dt = 3.0
    kt = kap[0, 0] + 1.0 / c_dt
    Ib = 2.0
    c, s = math.cos(phi[0]), math.sin(phi[0])
    exact = np.array([_exact_cell_average((i % n) * h, (i % n + 1) * h, (i // n) * h, (i // n + 1) * h,
                                          c, s, kt, 0.7, Ib) for i in range(n * n)])
    # the opposite direction leaves through x = L or y = L: the mirrored field
    mirrored = exact.reshape(n, n)[::-1, ::-1].ravel()
    errs = []
    for refine in (8, 16, 32, 64):
        g = rays.build(n, n, L, L, phi, h / refine)
        st0 = sweep.initial_state(g, 1, B)            # previous intensity = B, so S = B
        I_in = np.full((4 * n, 2, 1), Ib)
        st, _ = sweep.sweep(g, mu, kap, B, c_dt, st0, I_in)
        avg = moments.cell_direction_averages(g, 1, st)[:, :, 0]   # directions 0.4 and 0.4 + pi
        errs.append(max(np.max(np.abs(avg[:, 0] - exact)), np.max(np.abs(avg[:, 1] - mirrored))))
    # second order: an error of 2.7e-3 at spacing h/8 falls to ~3e-5 at h/64
    assert errs[-1] < 5e-5, errs
    assert errs[0] / errs[-1] > 40.0, errs
    assert all(e0 / e1 > 2.5 for e0, e1 in zip(errs[:-1], errs[1:])), errs
