"""Cell-local grey closures of the effective grey problem (paper, eq. (8)-(9)),
formed from the multigroup cell moments of a sweep.  TEST INFRASTRUCTURE
ONLY, like the rest of this package.

Per material cell i, with E_g, F_g = (F_x,g, F_y,g) and the Eddington tensor
f_g = (f_xx, f_xy, f_yy, f_zz)_g of every group g, and the opacity kappa_g and
Planck source B_g of the cell:

    E            = sum_g E_g,            F = sum_g F_g
    <u>_E        = sum_g u_g E_g / sum_g E_g                          (8)
    <u>_B        = sum_g u_g B_g / sum_g B_g                          (5a)
    K_R          = diag(<kappa>_|F_x|, <kappa>_|F_y|)                 (8)
    <u>_|F_a|    = sum_g u_g |F_a,g| / sum_g |F_a,g|                  (9)
    eta_a        = sum_g (kappa_g - K_R,aa) F_a,g / sum_g E_g          (9)
    <f>_E        = sum_g f_g E_g / sum_g E_g  (the grey Eddington tensor)

Reading of <kappa>_B: eq. (5a) uses it without writing it out.  Summing the
multigroup balance (4a) over the groups gives c <kappa>_B a_R T^4 =
4 pi sum_g kappa_g B_g; with a_R T^4 taken as (4 pi / c) sum_g B_g (equal
when the groups span the whole spectrum) this is the Planck-weighted mean
over the group set above.

Sums run over g in increasing order.  Readings where the paper's ratios are
0/0 (no radiation, no emission or no flux in a cell):
    sum E = 0:      <kappa>_E = <kappa>_B if sum B > 0, else the mean of
                    kappa_g over the groups; eta = 0; <f>_E = 1/3 on the
                    diagonal, 0 off it;
    sum B = 0:      <kappa>_B = <kappa>_E;
    sum |F_a| = 0:  <kappa>_|F_a| = <kappa>_E.
In 2D x-y geometry F_z = 0, so the zz entry of K_R never acts and is not
formed.
"""
from __future__ import annotations

import numpy as np

# component order of the output, per cell
NAMES = ("E", "Fx", "Fy", "kappa_E", "kappa_B", "KR_xx", "KR_yy", "eta_x", "eta_y",
         "fE_xx", "fE_xy", "fE_yy", "fE_zz")
N_GREY = len(NAMES)


def _ordered_sum(terms):
    """Sum over the group axis (axis 0) in increasing g."""
    out = np.zeros(terms.shape[1:], dtype=np.float64)
    for g in range(terms.shape[0]):
        out = out + terms[g]
    return out


def grey_closures(E, F, f, kappa, planck):
    """E: [G][cells]; F: [G][2][cells]; f: [G][4][cells]; kappa, planck:
    [G][cells] (float64).  Returns [N_GREY][cells] in the order of NAMES."""
    E = np.asarray(E, np.float64)
    F = np.asarray(F, np.float64)
    f = np.asarray(f, np.float64)
    kap = np.asarray(kappa, np.float64)
    B = np.asarray(planck, np.float64)
    G, cells = E.shape
    out = np.zeros((N_GREY, cells))
    sE = _ordered_sum(E)
    sB = _ordered_sum(B)
    sF = [_ordered_sum(F[:, a]) for a in range(2)]
    out[0], out[1], out[2] = sE, sF[0], sF[1]
    mean_k = _ordered_sum(kap) / G
    with np.errstate(divide="ignore", invalid="ignore"):
        kB_raw = _ordered_sum(kap * B) / sB
        kE = np.where(sE > 0, _ordered_sum(kap * E) / sE, np.where(sB > 0, kB_raw, mean_k))
        kB = np.where(sB > 0, kB_raw, kE)
        out[3], out[4] = kE, kB
        for a in range(2):
            aF = np.abs(F[:, a])
            saF = _ordered_sum(aF)
            kF = np.where(saF > 0, _ordered_sum(kap * aF) / saF, kE)
            out[5 + a] = kF
            eta = _ordered_sum((kap - kF[None, :]) * F[:, a]) / sE
            out[7 + a] = np.where(sE > 0, eta, 0.0)
        iso = (1.0 / 3, 0.0, 1.0 / 3, 1.0 / 3)
        for c in range(4):
            fe = _ordered_sum(f[:, c] * E) / sE
            out[9 + c] = np.where(sE > 0, fe, iso[c])
    return out
