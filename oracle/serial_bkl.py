"""Independent serial n-fold-way (BKL) simulation (test infrastructure only).

Rejection-free continuous-time kMC of the whole periodic lattice with no
domains: every site i carries the rate w_i (Metropolis or Barker), the next
event is site i with probability w_i / R, and time advances by an
exponential variate of mean 1/R, R = sum_i w_i (Sec. 2.1: tau_S = 1/R).
Written with numpy over many independent runs at once; it shares nothing
with kmco.c and is used to pin the oracle's relaxation curves.
"""
import numpy as np


def site_rates(s, J, h, T, model):
    n = (np.roll(s, 1, 1) + np.roll(s, -1, 1) + np.roll(s, 1, 2) +
         np.roll(s, -1, 2))
    dE = 2.0 * s * (J * n + h)
    if model == 0:
        return np.where(dE <= 0, 1.0, np.exp(-np.maximum(dE, 0) / T))
    return 1.0 / (1.0 + np.exp(dE / T))


def relaxation(start, nruns, t_grid, J=1.0, h=0.0, T=2.0, model=0, seed=0):
    """Energy per site -(J B + h M)/N and magnetisation per site of each run
    at the times t_grid (state after the last event at or before t)."""
    rng = np.random.default_rng(seed)
    L = start.shape[0]
    N = L * L
    s = np.repeat(start[None].astype(np.float64), nruns, axis=0)
    t = np.zeros(nruns)
    t_grid = np.asarray(t_grid, float)
    e_out = np.zeros((nruns, t_grid.size))
    m_out = np.zeros((nruns, t_grid.size))
    k = np.zeros(nruns, dtype=np.int64)  # next grid point to fill per run
    active = np.ones(nruns, bool)
    rows = np.arange(nruns)
    while active.any():
        w = site_rates(s, J, h, T, model).reshape(nruns, N)
        R = w.sum(axis=1)
        dt = rng.exponential(1.0, nruns) / R
        t_next = t + dt
        # record the current state at every grid time passed before the event
        bonds = (s * np.roll(s, -1, 1) + s * np.roll(s, -1, 2)).sum(axis=(1, 2))
        M = s.sum(axis=(1, 2))
        e = -(J * bonds + h * M) / N
        for _ in range(t_grid.size):
            fill = active & (k < t_grid.size)
            fill &= t_grid[np.minimum(k, t_grid.size - 1)] < t_next
            if not fill.any():
                break
            e_out[rows[fill], k[fill]] = e[fill]
            m_out[rows[fill], k[fill]] = M[fill] / N
            k[fill] += 1
        active = k < t_grid.size
        # choose the event site proportionally to its rate and flip it
        u = rng.random(nruns) * R
        idx = np.minimum((np.cumsum(w, axis=1) < u[:, None]).sum(axis=1), N - 1)
        flat = s.reshape(nruns, N)
        flat[rows[active], idx[active]] *= -1
        t = t_next
    return e_out, m_out
