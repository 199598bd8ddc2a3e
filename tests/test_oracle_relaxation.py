"""Pins of the oracle's relaxation curves against independent serial BKL.

With one domain (N_D = 1) the oracle's tick chain with its n-fold-way clock
is serial continuous-time kMC in law, so the ensemble energy at fixed times
must equal that of oracle/serial_bkl.py (a separate rejection-free code)
within statistical error.  With N_D > 1 the paper expects the response to be
preserved approximately when N_I is small against the relaxation time
(Sec. 3.3, Sec. 4); that is checked with a loose tolerance.
"""
import numpy as np
import pytest

from oracle import serial_bkl

T_GRID = np.array([0.25, 0.5, 1.0, 2.0, 4.0])


def oracle_curve(kmco, L, B, NI, T, start, nruns, seed, record_every=1):
    e = np.zeros((nruns, T_GRID.size))
    for rep in range(nruns):
        r = kmco.Replica(L, B, T=T, steps_per_visit=NI, init=kmco.INIT_GIVEN,
                         spins=start, seed=seed, replica=rep)
        n_sweeps = int(np.ceil(T_GRID[-1] * 1.5 * L * L / (NI * (L // B) ** 2))) + 8
        recs = [r.run(n_sweeps, record_every)]
        while recs[-1]["t"][-1] <= T_GRID[-1]:  # the clock is random: extend
            recs.append(r.run(n_sweeps, record_every))
        rec = np.concatenate(recs)
        t = np.concatenate([[0.0], rec["t"]])
        s0 = start.astype(np.int64)
        b0 = (s0 * np.roll(s0, -1, 0) + s0 * np.roll(s0, -1, 1)).sum()
        ee = np.concatenate([[-b0], -rec["B"]]) / L**2
        assert t[-1] > T_GRID[-1]
        pos = np.searchsorted(t, T_GRID, side="right") - 1
        e[rep] = ee[pos]
    return e


def start_config(L):
    rng = np.random.default_rng(42)
    return np.where(rng.random((L, L)) < 0.5, 1, -1).astype(np.int8)


def test_single_domain_is_serial_bkl(oracle_lib):
    L, T = 8, 2.0
    start = start_config(L)
    e_or = oracle_curve(oracle_lib, L, L, 1, T, start, 1500, seed=3)
    e_bkl, _ = serial_bkl.relaxation(start, 3000, T_GRID, T=T, seed=4)
    for k in range(T_GRID.size):
        a, b = e_or[:, k], e_bkl[:, k]
        z = (a.mean() - b.mean()) / np.sqrt(a.var() / a.size + b.var() / b.size)
        assert abs(z) < 4.5, (T_GRID[k], a.mean(), b.mean(), z)


@pytest.mark.parametrize("B,NI", [(4, 4), (2, 1)])
def test_decomposed_relaxation_close_to_serial(oracle_lib, B, NI):
    L, T = 8, 2.0
    start = start_config(L)
    e_par = oracle_curve(oracle_lib, L, B, NI, T, start, 1500, seed=9)
    e_bkl, _ = serial_bkl.relaxation(start, 3000, T_GRID, T=T, seed=10)
    diff = np.abs(e_par.mean(axis=0) - e_bkl.mean(axis=0))
    assert (diff[1:] < 0.06).all(), diff
