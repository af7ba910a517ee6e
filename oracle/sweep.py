"""Transport sweep along the characteristics (paper, eq. (10)-(13)).

Along a characteristic the backward-Euler BTE reads
    dI^n/du + kappa_t I^n = Q,
    kappa_t = kappa + 1/(c dt),   Q = kappa B + I^{n-1}/(c dt)          (10)-(11)
With kappa, B constant in a material cell, each segment is integrated exactly:
    tau   = kappa_t l / sin(zeta)                                         (13)
    I_out = I_in e^{-tau} + (Q/kappa_t)(1 - e^{-tau})                     (12)
    alpha = 1/tau - e^{-tau}/(1 - e^{-tau})                               (13)
    I_bar = alpha I_in + (1 - alpha) I_out                                (12)

Readings where the text is silent:
* I^{n-1} in Q is the previous step's segment-average intensity of the same
  segment and direction, so Q is constant on the segment and (12) stays exact;
* the intensity entering a characteristic is the boundary intensity of the
  face it enters through (eq. (2));
* 1 - e^{-tau} is evaluated as -expm1(-tau), and alpha by its Bernoulli
  series 1/2 - tau/12 + tau^3/720 - tau^5/30240 + tau^7/1209600 below
  tau = 0.1, where the closed form loses digits to cancellation (the series
  truncation error there is below 1e-16 relative).

State layout (canonical, also the library's export layout):
state[j][d][p][g] with j the global segment index, d = 0 forward / 1 reverse,
p the polar index and g the group.  Exit intensities: per pair an array
[2][K][P][G].
"""
from __future__ import annotations

import numpy as np

ALPHA_SERIES_BELOW = 0.1


def alpha_of_tau(tau):
    """Weight of the entering intensity in the segment average, eq. (13)."""
    tau = np.asarray(tau, dtype=np.float64)
    out = np.empty_like(tau)
    big = tau >= ALPHA_SERIES_BELOW
    t = tau[big]
    out[big] = 1.0 / t - np.exp(-t) / (-np.expm1(-t))
    t = tau[~big]
    t2 = t * t
    out[~big] = 0.5 - t / 12.0 + t * t2 / 720.0 - t * t2 * t2 / 30240.0 \
        + t * t2 * t2 * t2 / 1209600.0
    return out


def segment_step(I, kappa_t, Q, length, sin_zeta):
    """One segment of eq. (12)-(13): returns (I_out, I_bar)."""
    tau = kappa_t * length / sin_zeta
    e = np.exp(-tau)
    one_minus_e = -np.expm1(-tau)
    src = Q / kappa_t
    I_out = I * e + src * one_minus_e
    a = alpha_of_tau(tau)
    I_bar = a * I + (1.0 - a) * I_out
    return I_out, I_bar


def direction_index(a, d, p, n_az, n_pol):
    """m = azimuth * n_pol + p; d = 1 selects the opposite azimuth."""
    return (a + d * (n_az // 2)) * n_pol + p


def sweep_pair(grid, a, mu, kappa, planck, c_dt, state_prev, I_in, rays=None,
               local_state=False, points=None):
    """Sweep both directions of azimuth pair a, all polar angles and groups.

    kappa, planck: [G][cells]; state_prev: canonical [n_seg][2][P][G] (only
    the rows of this pair's segments are read); I_in: [nb][M][G].  ``rays``
    optionally limits the sweep to a subset of characteristics (for sampled
    checks); with ``local_state`` the state rows are indexed like the
    returned rows (only the chosen rays' segments, in their order) instead of
    by global segment index.  ``points`` ([n_seg][2][P][G], optional)
    receives the intensity entering each segment in each traversal (the
    value at its upwind face, I_{k,s} of eq. (12) and (16)).  Returns
    (j [n], rows [n][2][P][G],
    I_exit [2][K'][P][G], ray ids) where j are the global indices of the
    swept segments.
    """
    pr = grid.pairs[a]
    n_pol = len(mu)
    G = kappa.shape[0]
    sin_zeta = np.sqrt(1.0 - np.asarray(mu) ** 2)          # [P]
    ks = np.arange(pr.K) if rays is None else np.asarray(rays)
    nseg = pr.nseg[ks]
    first = np.concatenate([[0], np.cumsum(pr.nseg)])[ks] + pr.seg_base
    Smax = int(nseg.max())
    cellpad = np.zeros((len(ks), Smax), dtype=np.int64)
    lenpad = np.zeros((len(ks), Smax))
    for q, k in enumerate(ks):
        cellpad[q, :nseg[q]] = pr.cells[k]
        lenpad[q, :nseg[q]] = pr.lens[k]
    local = np.concatenate([[0], np.cumsum(nseg)])
    jglob = np.concatenate([np.arange(f, f + n) for f, n in zip(first, nseg)])
    rows = np.zeros((int(local[-1]), 2, n_pol, G))
    kap_t = kappa + 1.0 / c_dt                              # eq. (11)
    emis = kappa * planck                                   # kappa B
    I_exit = np.zeros((2, len(ks), n_pol, G))
    for d in (0, 1):
        I = np.zeros((len(ks), n_pol, G))
        face_in = (pr.entry_face if d == 0 else pr.exit_face)[ks]
        for p in range(n_pol):
            m = direction_index(a, d, p, grid.n_az, n_pol)
            I[:, p, :] = I_in[face_in, m, :]
        for t in range(Smax):
            kk = np.nonzero(t < nseg)[0]                    # rays still inside
            s = np.full(len(kk), t) if d == 0 else nseg[kk] - 1 - t
            cell = cellpad[kk, s]
            ln = lenpad[kk, s]
            kt = kap_t[:, cell].T[:, None, :]               # [k][1][G]
            row_prev = (local[kk] + s) if local_state else (first[kk] + s)
            Q = emis[:, cell].T[:, None, :] + state_prev[row_prev, d] / c_dt
            if points is not None:
                points[first[kk] + s, d] = I[kk]
            I_out, I_bar = segment_step(I[kk], kt, Q, ln[:, None, None],
                                        sin_zeta[None, :, None])
            rows[local[kk] + s, d] = I_bar
            I[kk] = I_out
        I_exit[d] = I
    return jglob, rows, I_exit, ks


def sweep(grid, mu, kappa, planck, c_dt, state_prev, I_in, points=None):
    """Full sweep: every pair, both directions, all polar angles and groups.
    Returns (state_new [n_seg][2][P][G], I_exit list per pair [2][K][P][G]);
    ``points`` as for sweep_pair."""
    state_new = np.zeros_like(state_prev)
    exits = []
    for a in range(len(grid.pairs)):
        j, rows, I_exit, _ = sweep_pair(grid, a, mu, kappa, planck, c_dt,
                                        state_prev, I_in, points=points)
        state_new[j] = rows
        exits.append(I_exit)
    return state_new, exits


def initial_state(grid, n_pol, field):
    """Segment intensities set to a cell field X[G][cells] in every direction:
    state[j][d][p][g] = X[g][cell(j)]."""
    _, _, cell, _, _ = grid.flat()
    G = field.shape[0]
    st = np.empty((len(cell), 2, n_pol, G))
    st[:] = field[:, cell].T[:, None, None, :]
    return st
