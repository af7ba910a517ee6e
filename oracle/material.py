"""The Fleck-Cummings test material of the paper's results section: the
spectral opacity 27/nu^3 (1 - e^(-nu/T)) and the group Planck functions
B_g(T), for the multilevel method's time steps.

TEST INFRASTRUCTURE ONLY (plain numpy + scipy quadrature).

B_g is the Planck intensity per steradian integrated over group g (the 4 pi
kappa B of eq. (4a)):
    B_g(T) = (a_R c T^4 / 4 pi) (15 / pi^4) int_{nu_{g-1}/T}^{nu_g/T} x^3 / (e^x - 1) dx,
so that the groups of a spectrum [0, inf) sum to a_R c T^4 / 4 pi.  The
integral is taken by adaptive quadrature over each group's own interval
(no differences of large integrals), an independent route from any series.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate


def fc_opacity(nu, T):
    """27/nu^3 (1 - e^(-nu/T)) for frequencies nu [G] (keV) and temperatures
    T [cells] (keV): [G][cells]."""
    nu = np.asarray(nu, dtype=np.float64)[:, None]
    T = np.asarray(T, dtype=np.float64)[None, :]
    return 27.0 / nu ** 3 * -np.expm1(-nu / T)


def _planck_integrand(x):
    if x <= 0.0:
        return 0.0
    if x < 1.0:
        return x ** 3 / math.expm1(x)
    return x ** 3 * math.exp(-x) / -math.expm1(-x)      # no overflow for large x


def planck_integral(x1, x2):
    """int_{x1}^{x2} x^3 / (e^x - 1) dx, 0 <= x1 <= x2 <= inf."""
    if x2 <= x1:
        return 0.0
    if x1 > 700.0:                     # the integrand is below 1e-300 there
        return 0.0
    val, _ = integrate.quad(_planck_integrand, x1, x2, epsabs=0.0, epsrel=2e-14, limit=400)
    return val


def group_planck(edges, T, a_R, c):
    """B_g(T) [G][cells] for group edges [G + 1] (keV; 0 and inf allowed)."""
    edges = np.asarray(edges, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    G = len(edges) - 1
    Tu, inv = np.unique(T, return_inverse=True)
    out = np.empty((G, len(Tu)))
    for j, t in enumerate(Tu):
        pref = a_R * c * t ** 4 / (4.0 * math.pi) * 15.0 / math.pi ** 4
        for g in range(G):
            out[g, j] = pref * planck_integral(edges[g] / t, edges[g + 1] / t)
    return out[:, inv]
