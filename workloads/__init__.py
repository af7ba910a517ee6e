"""Seeded synthetic problem inputs for the long-characteristics transport sweep.

This module is shared by the tests, the benchmark and the oracle's tests.  It
generates the *problem statement* only -- material grid, frequency groups,
angular quadrature, temperature fields, opacities, group Planck sources,
boundary and initial intensities -- and none of the sweep's arithmetic
(characteristic grid, attenuation, segment averages, moments).

Problem data follow the Fleck-Cummings test of the paper's results section:
a 6 x 6 cm slab, opacity kappa_nu = 27/nu^3 (1 - exp(-nu/T)) (nu, T in keV,
kappa in 1/cm), a 1 keV Planckian entering through the x = 0 face, vacuum on
the other faces, and an initial material temperature of 1 eV.  The paper's
own quadrature set (Abu-Shumays q461214) and 17-group bounds are not given in
its text; they are replaced by a product quadrature (uniform azimuths x
Gauss-Legendre polar cosines) and log-spaced group edges.

Units: cm, shake (1e-8 s), keV, GJ.  c = 299.792458 cm/sh and
a_R = 0.01372 GJ/(cm^3 keV^4).  B_g is the group Planck intensity per
steradian, so that sum_g 4*pi*B_g = a_R c T^4 (the 4*pi of the multigroup
energy equation of the paper's method section).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

C_LIGHT = 299.792458          # cm / shake
A_RAD = 0.01372               # GJ / (cm^3 keV^4)
SEED0 = 230511998             # base seed; configuration k uses SEED0 + k

__all__ = [
    "C_LIGHT", "A_RAD", "SEED0", "Problem", "product_quadrature",
    "group_edges", "group_midpoints", "fc_opacity", "planck_integral_0x",
    "group_planck", "boundary_faces", "inflow_left_planck",
    "t_field_iid", "t_field_gaussians", "t_field_front", "make_problem",
    "config", "batch_problems", "FcMlqd", "open_group_edges", "fc_mlqd",
]


# ---------------------------------------------------------------------------
# angular quadrature and groups
# ---------------------------------------------------------------------------

def product_quadrature(n_az: int, n_pol: int):
    """Product set: azimuths phi_a = (a + 1/2) 2 pi / n_az, polar cosines and
    weights from Gauss-Legendre on [-1, 1], omega_m = w_p 2 pi / n_az with
    direction index m = a * n_pol + p.  The weights sum to 4 pi.

    Returns (phi[n_az], mu[n_pol], omega[n_az * n_pol]) as float64 arrays.
    """
    if n_az < 2 or n_az % 2:
        raise ValueError("n_az must be even and >= 2")
    phi = np.array([(a + 0.5) * 2.0 * math.pi / n_az for a in range(n_az)])
    mu, wp = np.polynomial.legendre.leggauss(n_pol)
    # make the +-mu pairs exact mirror images
    mu = 0.5 * (mu - mu[::-1])
    wp = 0.5 * (wp + wp[::-1])
    omega = np.repeat(np.full(n_az, 2.0 * math.pi / n_az), n_pol) * np.tile(wp, n_az)
    return phi, mu, omega


def group_edges(G: int, nu_lo: float, nu_hi: float) -> np.ndarray:
    """G + 1 log-spaced group edges nu_j = nu_lo (nu_hi/nu_lo)^(j/G)."""
    j = np.arange(G + 1, dtype=np.float64)
    e = nu_lo * (nu_hi / nu_lo) ** (j / G)
    e[0], e[-1] = nu_lo, nu_hi
    return e


def group_midpoints(edges: np.ndarray) -> np.ndarray:
    """Arithmetic group midpoints."""
    return 0.5 * (edges[:-1] + edges[1:])


# ---------------------------------------------------------------------------
# material model
# ---------------------------------------------------------------------------

def fc_opacity(nu: np.ndarray, T: np.ndarray) -> np.ndarray:
    """Fleck-Cummings opacity 27/nu^3 (1 - exp(-nu/T)), evaluated at the
    group midpoints nu[G] for temperatures T[cells]; returns [G][cells]."""
    nu = np.asarray(nu, dtype=np.float64)[:, None]
    T = np.asarray(T, dtype=np.float64)[None, :]
    return 27.0 / nu ** 3 * (-np.expm1(-nu / T))


# Bernoulli numbers B_0..B_40 as exact fractions (B_1 = -1/2 convention).
def _bernoulli(n: int):
    from fractions import Fraction
    B = [Fraction(0)] * (n + 1)
    B[0] = Fraction(1)
    for m in range(1, n + 1):
        s = Fraction(0)
        for k in range(m):
            s += Fraction(math.comb(m + 1, k)) * B[k]
        B[m] = -s / (m + 1)
    return [float(b) for b in B]


_BERN = _bernoulli(40)
_PI4_15 = math.pi ** 4 / 15.0


def _planck_series(x: np.ndarray) -> np.ndarray:
    # int_0^x t^3/(e^t - 1) dt = sum_k B_k x^(k+3) / (k! (k+3)),  |x| < 2 pi
    out = np.zeros_like(x)
    xp = x ** 3
    fact = 1.0
    for k in range(0, 41):
        if k > 0:
            fact *= k
        if _BERN[k] != 0.0:
            out += _BERN[k] * xp / (fact * (k + 3))
        xp = xp * x
    return out


def _planck_tail(x: np.ndarray) -> np.ndarray:
    # int_x^inf t^3/(e^t - 1) dt = sum_n e^(-n x) (x^3/n + 3x^2/n^2 + 6x/n^3 + 6/n^4)
    out = np.zeros_like(x)
    fin = np.isfinite(x)
    xf = np.where(fin, x, 0.0)
    for n in range(1, 26):
        out += np.where(fin, np.exp(-n * xf) * (xf ** 3 / n + 3 * xf ** 2 / n ** 2 + 6 * xf / n ** 3 + 6 / n ** 4),
                        0.0)
    return out


def planck_integral_0x(x) -> np.ndarray:
    """P(x) = int_0^x t^3/(e^t - 1) dt for x >= 0 (P(inf) = pi^4/15)."""
    x = np.asarray(x, dtype=np.float64)
    lo = x < 2.0
    out = np.empty_like(x)
    out[lo] = _planck_series(x[lo])
    out[~lo] = _PI4_15 - _planck_tail(x[~lo])
    return out


def group_planck(edges: np.ndarray, T: np.ndarray) -> np.ndarray:
    """Group Planck intensity per steradian, [G][cells]:
    B_g(T) = (a_R c T^4 / 4 pi) (15/pi^4) int_{nu_{g-1}/T}^{nu_g/T} x^3/(e^x - 1) dx.
    The difference of the two integrals is formed from the series below x = 2
    and from the tails above, so no cancellation occurs in the far tail."""
    edges = np.asarray(edges, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    x1 = edges[:-1, None] / T[None, :]
    x2 = edges[1:, None] / T[None, :]
    both_hi = x1 >= 2.0
    both_lo = x2 < 2.0
    out = np.empty(x1.shape)
    # both in the tail region
    out[both_hi] = _planck_tail(x1[both_hi]) - _planck_tail(x2[both_hi])
    # both in the series region
    out[both_lo] = _planck_series(x2[both_lo]) - _planck_series(x1[both_lo])
    mid = ~(both_hi | both_lo)
    out[mid] = (_PI4_15 - _planck_tail(x2[mid])) - _planck_series(x1[mid])
    pref = A_RAD * C_LIGHT * T ** 4 / (4.0 * math.pi) * (15.0 / math.pi ** 4)
    return out * pref[None, :]


# ---------------------------------------------------------------------------
# boundary faces and intensities
# ---------------------------------------------------------------------------

def boundary_faces(nx: int, ny: int):
    """Boundary face numbering shared by every interface:
    [0, ny) x = 0 (row iy), [ny, 2ny) x = Lx, [2ny, 2ny + nx) y = 0 (column ix),
    [2ny + nx, 2ny + 2nx) y = Ly.  Returns the outward normals [nb][2]."""
    n = np.zeros((2 * (nx + ny), 2))
    n[:ny] = (-1.0, 0.0)
    n[ny:2 * ny] = (1.0, 0.0)
    n[2 * ny:2 * ny + nx] = (0.0, -1.0)
    n[2 * ny + nx:] = (0.0, 1.0)
    return n


def inflow_left_planck(nx, ny, phi, mu, edges, T_in=1.0) -> np.ndarray:
    """I_in[nb][M][G]: the group Planckian at T_in enters through the x = 0
    face (directions with Omega_x > 0); vacuum everywhere else."""
    n_az, n_pol = len(phi), len(mu)
    G = len(edges) - 1
    nb = 2 * (nx + ny)
    I_in = np.zeros((nb, n_az * n_pol, G))
    Bin = group_planck(edges, np.array([T_in]))[:, 0]
    for a in range(n_az):
        if math.cos(phi[a]) > 0.0:
            for p in range(n_pol):
                I_in[:ny, a * n_pol + p, :] = Bin[None, :]
    return I_in


# ---------------------------------------------------------------------------
# temperature fields (cell centred, keV)
# ---------------------------------------------------------------------------

def _centres(nx, ny, lx, ly):
    x = (np.arange(nx) + 0.5) * (lx / nx)
    y = (np.arange(ny) + 0.5) * (ly / ny)
    X, Y = np.meshgrid(x, y)           # [ny][nx] -> cell i = iy*nx + ix
    return X.ravel(), Y.ravel()


def t_field_iid(rng, nx, ny, t_lo=0.001, t_hi=1.0):
    return rng.uniform(t_lo, t_hi, size=nx * ny)


def t_field_gaussians(rng, nx, ny, lx, ly, n=8, t_lo=0.001, t_hi=1.0):
    """Sum of n random Gaussians, min-max normalised onto [t_lo, t_hi]."""
    X, Y = _centres(nx, ny, lx, ly)
    f = np.zeros_like(X)
    for _ in range(n):
        cx, cy = rng.uniform(0, lx), rng.uniform(0, ly)
        s = rng.uniform(0.3, 1.5)
        A = rng.uniform(0.2, 1.0)
        f += A * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * s * s))
    f = (f - f.min()) / (f.max() - f.min())
    return t_lo + (t_hi - t_lo) * f


def t_field_front(rng, nx, ny, lx, ly, offset=0.0, t_hot=1.0, t_cold=0.001):
    """Sharp front: hot where (r - p).n < offset, cold elsewhere."""
    X, Y = _centres(nx, ny, lx, ly)
    px, py = rng.uniform(1.0, lx - 1.0), rng.uniform(1.0, ly - 1.0)
    th = rng.uniform(0.0, 2.0 * math.pi)
    d = (X - px) * math.cos(th) + (Y - py) * math.sin(th)
    return np.where(d < offset, t_hot, t_cold)


# ---------------------------------------------------------------------------
# problems
# ---------------------------------------------------------------------------

@dataclass
class Problem:
    """One transport problem: everything the sweep's interface takes."""
    nx: int
    ny: int
    lx: float
    ly: float
    phi: np.ndarray            # [n_az]
    mu: np.ndarray             # [n_pol]
    omega: np.ndarray          # [n_az * n_pol]
    edges: np.ndarray          # [G + 1] keV
    h_moc: float               # maximum characteristic width, cm
    c_dt: float                # c * Delta t, cm
    kappa: list                # per step: [G][cells]
    planck: list               # per step: [G][cells]
    I_in: np.ndarray           # [nb][M][G]
    state0: np.ndarray         # [G][cells]: segment intensities start at this cell field
    T: list = field(default_factory=list)   # per step temperatures [cells]
    name: str = ""

    @property
    def G(self):
        return len(self.edges) - 1

    @property
    def n_az(self):
        return len(self.phi)

    @property
    def n_pol(self):
        return len(self.mu)

    @property
    def M(self):
        return len(self.omega)

    @property
    def cells(self):
        return self.nx * self.ny

    @property
    def steps(self):
        return len(self.kappa)


def make_problem(nx, ny, lx, ly, n_az, n_pol, G, nu_lo, nu_hi, h_moc, c_dt,
                 T_steps, T0=0.001, T_in=1.0, name=""):
    phi, mu, omega = product_quadrature(n_az, n_pol)
    edges = group_edges(G, nu_lo, nu_hi)
    numid = group_midpoints(edges)
    kap, B = [], []
    for T in T_steps:
        # evaluate on the distinct temperatures only (fronts have two)
        Tu, inv = np.unique(np.asarray(T, dtype=np.float64), return_inverse=True)
        kap.append(fc_opacity(numid, Tu)[:, inv])
        B.append(group_planck(edges, Tu)[:, inv])
    I_in = inflow_left_planck(nx, ny, phi, mu, edges, T_in)
    s0 = np.repeat(group_planck(edges, np.array([T0])), nx * ny, axis=1)
    return Problem(nx, ny, lx, ly, phi, mu, omega, edges, h_moc, c_dt,
                   kap, B, I_in, s0, list(T_steps), name)


def group_subset(prob: Problem, g0: int, g1: int, h_moc: float | None = None, name: str = "") -> Problem:
    """Groups [g0, g1) of a problem as a problem of their own, optionally
    with another characteristic spacing (every input sliced, nothing else)."""
    return Problem(prob.nx, prob.ny, prob.lx, prob.ly, prob.phi, prob.mu, prob.omega, prob.edges[g0:g1 + 1].copy(),
                   prob.h_moc if h_moc is None else h_moc, prob.c_dt,
                   [np.ascontiguousarray(k[g0:g1]) for k in prob.kappa],
                   [np.ascontiguousarray(b[g0:g1]) for b in prob.planck],
                   np.ascontiguousarray(prob.I_in[:, :, g0:g1]), np.ascontiguousarray(prob.state0[g0:g1]),
                   list(prob.T), name or f"{prob.name}[{g0}:{g1}]")


def config(k: int, steps: int | None = None) -> Problem:
    """The five workloads, built from seed SEED0 + k:

    0  16x16 cells on 6x6 cm, G = 4 (0.001-10 keV), 16 x 2 directions,
       spacing 0.05 cm, iid T in [0.001, 1] keV, 1 step.
    1  128x128, G = 17 (0.001-30 keV), 32 x 2, spacing h/4, smooth T from 8
       Gaussians, 5 steps with T held fixed.
    2  256x256, G = 51 (0.001-30 keV), 32 x 4, spacing h/2, sharp front, 1 step.
    3  see batch_problems().
    4  512x512, G = 51, 48 x 6, spacing h/2, front moving 0.25 cm per step,
       10 steps.
    c dt = 3 cm throughout; the first step starts from B_g(1 eV).
    """
    rng = np.random.default_rng(SEED0 + k)
    L = 6.0
    if k == 0:
        n = 16
        T = t_field_iid(rng, n, n)
        ns = 1 if steps is None else steps
        return make_problem(n, n, L, L, 16, 2, 4, 0.001, 10.0, 0.05, 3.0,
                            [T] * ns, name="c0")
    if k == 1:
        n = 128
        T = t_field_gaussians(rng, n, n, L, L)
        ns = 5 if steps is None else steps
        return make_problem(n, n, L, L, 32, 2, 17, 0.001, 30.0, L / n / 4, 3.0,
                            [T] * ns, name="c1")
    if k == 2:
        n = 256
        T = t_field_front(rng, n, n, L, L)
        ns = 1 if steps is None else steps
        return make_problem(n, n, L, L, 32, 4, 51, 0.001, 30.0, L / n / 2, 3.0,
                            [T] * ns, name="c2")
    if k == 4:
        n = 512
        ns = 10 if steps is None else steps
        st = rng.bit_generator.state
        Ts = []
        for s in range(ns):
            rng.bit_generator.state = st       # same line, moving offset
            Ts.append(t_field_front(rng, n, n, L, L, offset=0.25 * s))
        return make_problem(n, n, L, L, 48, 6, 51, 0.001, 30.0, L / n / 2, 3.0,
                            Ts, name="c4")
    raise ValueError(f"no single-problem configuration {k}")


def batch_spec(n_problems=64, seed=SEED0 + 3):
    """Sizes of the batched workload: problem j draws mesh N from
    {32, 64, 128, 256}, G from {8, 17, 51} and M from {16, 64, 128}
    independently with seed + 1000 j."""
    specs = []
    for j in range(n_problems):
        r = np.random.default_rng(seed + 1000 * j)
        N = int(r.choice([32, 64, 128, 256]))
        G = int(r.choice([8, 17, 51]))
        M = int(r.choice([16, 64, 128]))
        specs.append((N, G, M, int(r.integers(0, 2 ** 31))))
    return specs


_M_SPLIT = {16: (8, 2), 64: (32, 2), 128: (32, 4), 288: (48, 6)}


def batch_problems(n_problems=64, steps=5, seed=SEED0 + 3, only=None):
    """The batched workload: n_problems independent problems of uneven mesh,
    group and direction counts, spacing h/2, smooth T fields."""
    out = []
    for j, (N, G, M, s) in enumerate(batch_spec(n_problems, seed)):
        if only is not None and j not in only:
            continue
        rng = np.random.default_rng(s)
        L = 6.0
        T = t_field_gaussians(rng, N, N, L, L)
        n_az, n_pol = _M_SPLIT[M]
        out.append(make_problem(N, N, L, L, n_az, n_pol, G, 0.001, 30.0,
                                L / N / 2, 3.0, [T] * steps, name=f"b{j}"))
    return out


# ---------------------------------------------------------------------------
# the Fleck-Cummings problem of the multilevel method's time steps
# ---------------------------------------------------------------------------

def open_group_edges(G: int, nu_lo: float, nu_hi: float) -> np.ndarray:
    """G + 1 edges covering the whole spectrum: 0, then G - 1 log-spaced
    edges from nu_lo to nu_hi, then infinity (so that the group Planck
    functions sum to a_R c T^4 / 4 pi exactly)."""
    e = np.empty(G + 1)
    e[0] = 0.0
    e[1:G] = group_edges(G - 2, nu_lo, nu_hi) if G > 2 else [nu_lo]
    e[G] = math.inf
    return e


@dataclass
class FcMlqd:
    """The Fleck-Cummings problem as the multilevel method's time steps take
    it: a 6 x 6 cm slab of cells h_mat wide, opacity 27/nu^3 (1 - e^(-nu/T))
    at the representative frequencies nu, eps = c_v T with
    c_v = 0.5917 a_R keV^-3, T^0 = 1 eV, the Planckian of T_in = 1 keV
    entering at x = 0, vacuum elsewhere."""
    nx: int
    ny: int
    lx: float
    ly: float
    phi: np.ndarray
    mu: np.ndarray
    omega: np.ndarray
    edges: np.ndarray          # [G + 1] keV, 0 and inf at the ends
    nu: np.ndarray             # [G] representative frequencies of the opacity
    h_moc: float
    c_dt: float
    c_v: float
    T0: float
    T_in: float
    I_in: np.ndarray           # [nb][M][G]
    state0: np.ndarray         # [G][cells]: B_g(T^0)
    name: str = ""

    @property
    def G(self):
        return len(self.nu)

    @property
    def cells(self):
        return self.nx * self.ny

    @property
    def n_pol(self):
        return len(self.mu)

    @property
    def kappa0(self):
        return fc_opacity(self.nu, np.full(self.cells, self.T0))

    @property
    def planck0(self):
        return self.state0


def fc_mlqd(h_mat: float, h_moc: float, n_az: int = 36, n_pol: int = 4, G: int = 17, nu_lo: float = 0.01,
            nu_hi: float = 20.0, dt_ns: float = 0.02, L: float = 6.0, name: str = "") -> FcMlqd:
    """Representative frequencies: arithmetic midpoints of the finite groups,
    half the upper edge for [0, nu_lo], the lower edge for [nu_hi, inf).
    Default 36 x 4 = 144 directions and 17 groups, the paper's counts, and
    Delta t = 0.02 ns."""
    n = int(round(L / h_mat))
    if n < 1 or abs(n * h_mat - L) > 1e-9 * L:
        raise ValueError("h_mat must divide the 6 cm slab")
    phi, mu, omega = product_quadrature(n_az, n_pol)
    edges = open_group_edges(G, nu_lo, nu_hi)
    nu = np.empty(G)
    nu[0] = 0.5 * edges[1]
    nu[1:G - 1] = 0.5 * (edges[1:G - 1] + edges[2:G])
    nu[G - 1] = edges[G - 1]
    T0, T_in = 0.001, 1.0
    c_dt = C_LIGHT * dt_ns * 0.1          # 1 shake = 10 ns
    I_in = inflow_left_planck(n, n, phi, mu, edges, T_in)
    s0 = np.repeat(group_planck(edges, np.array([T0])), n * n, axis=1)
    return FcMlqd(n, n, L, L, phi, mu, omega, edges, nu, h_moc, c_dt, 0.5917 * A_RAD, T0, T_in, I_in, s0,
                  name or f"fc_{n}x{n}")
