"""Pins of the oracle's ring (the paper's 1D system, Sec. 3.1).

* The transfer-matrix energy of the periodic ring equals brute-force
  enumeration (with and without a field), and gives the exact equilibrium
  energy of the paper's 1 x 8 ring at 1/(beta J) = 2.
* The ring's rate table: a flip and its reverse have rates in the ratio
  e^{-dE/T}, with dE from a direct count of the two neighbour bonds.
* The oracle's state histogram after a few sweeps, over many independent
  replicas started from one of the paper's initial conditions (two adjacent
  up spins), matches exact propagation of the probability vector with the
  ring's T_PAR over 2^N states (oracle/exact.py, written separately), for
  N_D in {1, 2, 4, 8} and N_I in {1, 2, 5} (Eq. (1D partitions), Table 1),
  Barker and Metropolis rates, random orders and the palindrome.
* Replicas started from exact Boltzmann samples stay Boltzmann-distributed,
  and long runs reproduce the transfer-matrix energy.
A wrong neighbour (a vertical one left over from the square lattice), a
wrong rate sign, halo or colour fails one of these.
"""
import itertools

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import exact
from tests.test_oracle_dynamics import chi2_pvalue


def ring_state_index(spins):
    bits = (np.asarray(spins) > 0).astype(np.int64)
    return int((bits << np.arange(bits.size)).sum())


def two_up(N, i):
    s = -np.ones(N, np.int8)
    s[i % N] = 1
    s[(i + 1) % N] = 1
    return s


@pytest.mark.parametrize("N,J,h,T", [(5, 1.0, 0.0, 2.0), (8, 1.0, 0.0, 2.0),
                                     (8, 0.7, 0.3, 1.5), (9, 1.0, -0.2, 3.0),
                                     (10, -0.5, 0.1, 1.0)])
def test_ring_transfer_matrix_equals_enumeration(N, J, h, T):
    pi, M, B, E = exact.ring_boltzmann(N, J, h, T)
    assert abs((pi * E).sum() - cf.ring_energy(N, T, J, h)) < 1e-7 * N
    sd = np.sqrt((pi * E ** 2).sum() - (pi * E).sum() ** 2)
    assert abs(sd - cf.ring_energy_std(N, T, J, h)) < 1e-4 * N


def test_paper_ring_equilibrium_energy():
    """The 1 x 8 ring at 1/(beta J) = 2: <H>/N_S = -0.465649 J exactly (the
    paper's Table 1 prints -0.237; no unit convention reproduces it, so the
    exact value is the pin)."""
    e = cf.ring_energy(8, 2.0) / 8
    assert abs(e - (-0.4656492509)) < 1e-8
    pi, M, B, E = exact.ring_boltzmann(8, 1.0, 0.0, 2.0)
    assert abs((pi * E).sum() / 8 - e) < 1e-9


@pytest.mark.parametrize("model", [0, 1])
def test_ring_rate_table(oracle_lib, model):
    J, h, T = 1.0, 0.3, 1.7
    r, w, gJ, gh = oracle_lib.rates(J, h, T, model, z=2)
    for up, k in itertools.product((0, 1), range(3)):
        s = 1 if up else -1
        dE = 2 * s * (J * (2 * k - 2) + h)  # the two bonds and the field
        c, cbar = 5 * up + k, 5 * (1 - up) + k
        assert np.isclose(w[c] / w[cbar], np.exp(-dE / T), rtol=1e-12)
    # d ln w / dJ by central differences
    d = 1e-6
    wp = oracle_lib.rates(J + d, h, T, model, z=2)[1]
    wm = oracle_lib.rates(J - d, h, T, model, z=2)[1]
    for c in (0, 1, 2, 5, 6, 7):
        assert np.isclose(gJ[c], (np.log(wp[c]) - np.log(wm[c])) / (2 * d), atol=1e-6)


RING_CASES = [  # N, B, N_I, model, palindrome, sweeps
    (8, 8, 1, 1, False, 3),
    (8, 4, 2, 1, False, 2),
    (8, 2, 5, 1, False, 2),
    (8, 1, 1, 1, False, 3),
    (8, 2, 1, 0, True, 2),
    (6, 2, 2, 1, False, 2),   # three domains: three colours
]


def sample_ring(kmco, N, B, NI, model, pal, sweeps, start, nrep, seed=23, T=2.0, h=0.0):
    counts = np.zeros(1 << N)
    for rep in range(nrep):
        r = kmco.Replica(N, B, T=T, h=h, steps_per_visit=NI, rate_model=model,
                         schedule=1 if pal else 0, init=kmco.INIT_GIVEN, spins=start,
                         seed=seed, replica=rep, dims=1)
        r.run(sweeps)
        counts[ring_state_index(r.spins())] += 1
    return counts


@pytest.mark.parametrize("N,B,NI,model,pal,sweeps", RING_CASES)
def test_ring_finite_time_distribution(oracle_lib, N, B, NI, model, pal, sweeps):
    start = two_up(N, 3)
    p = np.zeros(1 << N)
    p[ring_state_index(start)] = 1.0
    op = exact.RingSweepOperator(N, B, 1.0, 0.0, 2.0, model, NI, quantise=True,
                                 palindrome=pal)
    for _ in range(sweeps):
        p = op.par(p)
    counts = sample_ring(oracle_lib, N, B, NI, model, pal, sweeps, start, 20000)
    assert chi2_pvalue(counts, p) > 1e-4


def test_ring_boltzmann_is_stationary(oracle_lib):
    N, T, h = 8, 2.0, 0.2
    pi, *_ = exact.ring_boltzmann(N, 1.0, h, T)
    rng = np.random.default_rng(4)
    states = rng.choice(1 << N, size=20000, p=pi)
    counts = np.zeros(1 << N)
    for rep, st in enumerate(states):
        start = np.where((st >> np.arange(N)) & 1, 1, -1).astype(np.int8)
        r = oracle_lib.Replica(N, 2, T=T, h=h, steps_per_visit=3, rate_model=1,
                               init=oracle_lib.INIT_GIVEN, spins=start, seed=31,
                               replica=rep, dims=1)
        r.run(2)
        counts[ring_state_index(r.spins())] += 1
    assert chi2_pvalue(counts, pi) > 1e-4


def test_ring_long_run_energy(oracle_lib):
    """Time average of H over a long run of a 64-site ring (4 domains,
    N_I = 16) against the transfer matrix, with batch-means error bars."""
    N, T = 64, 2.0
    r = oracle_lib.Replica(N, 16, T=T, steps_per_visit=16, rate_model=1, seed=5, dims=1)
    r.run(500, 500)
    rec = r.run(40000, 4)
    e = -rec["B"].astype(float) / N
    b = e.reshape(20, -1).mean(axis=1)
    err = b.std(ddof=1) / np.sqrt(len(b))
    assert abs(b.mean() - cf.ring_energy(N, T) / N) < 4.5 * err + 1e-3


def test_ring_records_are_consistent(oracle_lib):
    r = oracle_lib.Replica(12, 3, T=1.5, h=0.1, steps_per_visit=4, seed=2, dims=1)
    rec = r.run(30, 1, check=True)
    assert r.check_failures() == 0
    s = r.spins().astype(int)
    assert s.shape == (12,)
    assert rec["M"][-1] == s.sum()
    assert rec["B"][-1] == (s * np.roll(s, -1)).sum()
    assert (rec["steps"] == np.arange(1, 31) * 4 * 4).all()
    col, ncol = r.partition()
    assert list(col) == [0, 1, 0, 1] and ncol == 2
