"""Pins of the oracle's rejection-free variant with fixed time slices (the
synchronous time-horizon methods the paper contrasts itself with, Sec. 1).

* Its logarithm (the atanh series) is within 2 ulp of libm's over (0, 1],
  exact at 1, and monotone, so the stop decision t + dt > tau is the one the
  exact waiting time takes except within rounding.
* A domain process is the domain's continuous-time chain observed at time
  tau, exp(Q_d tau): the oracle's state histogram after a few sweeps over
  many replicas matches exact propagation with sparse matrix exponentials
  (oracle/exact.py) on the 3 x 3 torus (stripes, single sites, one domain),
  the 4 x 4 torus in 2 x 2 domains and the 1 x 8 ring; Boltzmann samples
  stay Boltzmann-distributed.
* With one domain, slices compose: k slices of tau equal one slice of
  k tau in law (the semigroup exp(Q tau)^k = exp(Q k tau)), i.e. serial
  continuous-time BKL.
* With all rates 1 the events of a visit are Poisson(n_d tau).
* Records: the clock advances by exactly tau per visit, the step count stays
  0, and the class bookkeeping recounts clean.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import exact
from tests.test_oracle_dynamics import chi2_pvalue, state_index


def ulp(x):
    return math.ulp(abs(x)) if x != 0 else 0.0


def test_slice_log_against_libm(oracle_lib):
    rng = np.random.default_rng(3)
    us = np.concatenate([rng.random(20000), 2.0 ** -rng.uniform(0, 53, 5000),
                         1 - 2.0 ** -rng.uniform(1, 52, 5000),
                         [2.0 ** -53, 0.5, 0.25, 1 - 2.0 ** -53, math.sqrt(0.5)]])
    us = us[(us > 0) & (us <= 1)]
    for u in us:
        a, b = oracle_lib.slice_log(u), math.log(u)
        assert abs(a - b) <= 2 * ulp(b), (u, a, b)
    assert oracle_lib.slice_log(1.0) == 0.0
    v = np.sort(rng.random(4000))
    lv = [oracle_lib.slice_log(x) for x in v]
    assert all(a <= b for a, b in zip(lv, lv[1:]))


SLICE_CASES = [  # L, Bx, By, tau, model, palindrome, ring, sweeps
    (3, 1, 3, 0.7, 0, False, False, 2),   # three vertical stripes
    (3, 1, 1, 0.4, 1, False, False, 1),   # nine one-site domains (palindrome only for >4 colours)
    (3, 3, 3, 1.3, 0, False, False, 2),   # one periodic domain: serial BKL
    (4, 2, 2, 0.5, 0, False, False, 2),   # 2 x 2 checkerboard
    (4, 2, 2, 0.9, 1, True, False, 1),    # palindrome
    (8, 2, 0, 0.6, 1, False, True, 3),    # the ring, four domains
]


def sample(kmco, L, Bx, By, tau, model, pal, ring, sweeps, start, nrep, seed=5, T=2.3, h=0.1):
    counts = np.zeros(1 << (L if ring else L * L))
    for rep in range(nrep):
        r = kmco.Replica(L, Bx, T=T, h=h, rate_model=model, tile_rows=By,
                         schedule=1 if pal else 0, init=kmco.INIT_GIVEN, spins=start,
                         seed=seed, replica=rep, dims=1 if ring else 2, time_slice=tau)
        r.run(sweeps)
        counts[state_index(r.spins())] += 1
    return counts


@pytest.mark.parametrize("L,Bx,By,tau,model,pal,ring,sweeps", SLICE_CASES)
def test_slice_finite_time_distribution(oracle_lib, L, Bx, By, tau, model, pal, ring, sweeps):
    if L == 3 and Bx == 1 and By == 1:
        pal = True  # nine colours: only the palindrome is mixed exactly
    rng = np.random.default_rng(L + Bx)
    start = np.where(rng.random(L if ring else (L, L)) < 0.5, 1, -1).astype(np.int8)
    op = exact.SliceSweepOperator(L, Bx, 1.0, 0.1, 2.3, model, tau, palindrome=pal,
                                  By=By or None, ring=ring)
    p = np.zeros(1 << (L if ring else L * L))
    p[state_index(start)] = 1.0
    for _ in range(sweeps):
        p = op.par(p)
    counts = sample(oracle_lib, L, Bx, By, tau, model, pal, ring, sweeps, start, 20000)
    assert chi2_pvalue(counts, np.maximum(p, 0.0)) > 1e-4


def test_slice_boltzmann_is_stationary(oracle_lib):
    L, T, h = 3, 2.0, 0.2
    pi, *_ = exact.boltzmann(L, 1.0, h, T)
    rng = np.random.default_rng(8)
    states = rng.choice(1 << 9, size=20000, p=pi)
    counts = np.zeros(1 << 9)
    for rep, st in enumerate(states):
        start = np.where((st >> np.arange(9)) & 1, 1, -1).astype(np.int8).reshape(3, 3)
        r = oracle_lib.Replica(L, 1, T=T, h=h, tile_rows=3, init=oracle_lib.INIT_GIVEN,
                               spins=start, seed=13, replica=rep, time_slice=0.8)
        r.run(2)
        counts[state_index(r.spins())] += 1
    assert chi2_pvalue(counts, pi) > 1e-4


def test_slices_compose_with_one_domain(oracle_lib):
    """One periodic domain: 4 slices of 0.25 against 1 slice of 1.0 and the
    exact exp(Q) (serial continuous-time kinetics)."""
    L = 3
    start = np.array([[1, -1, 1], [-1, -1, 1], [1, 1, -1]], np.int8)
    op = exact.SliceSweepOperator(L, 3, 1.0, 0.1, 2.3, 0, 1.0, By=3)
    p = np.zeros(512)
    p[state_index(start)] = 1.0
    p = op.par(p)
    for tau, sweeps in ((0.25, 4), (1.0, 1)):
        counts = sample(oracle_lib, L, 3, 3, tau, 0, False, False, sweeps, start, 20000,
                        seed=int(100 * tau))
        assert chi2_pvalue(counts, np.maximum(p, 0.0)) > 1e-4


def test_slice_event_count_is_poisson(oracle_lib):
    """J = h = 0, Metropolis: every rate is 1, so a visit of a domain of n_d
    sites has Poisson(n_d tau) events."""
    nd, tau = 16, 0.75
    ev = []
    for rep in range(3000):
        r = oracle_lib.Replica(8, 4, J=0.0, h=0.0, T=1.0, seed=2, replica=rep, time_slice=tau)
        r.run(1)
        ev.extend(r.domain_events())
    ev = np.array(ev)
    lam = nd * tau
    assert abs(ev.mean() - lam) < 4.5 * math.sqrt(lam / ev.size)
    counts = np.bincount(ev, minlength=30)[:30]
    probs = stats.poisson.pmf(np.arange(30), lam)
    assert chi2_pvalue(counts, probs / probs.sum()) > 1e-4


def test_slice_records(oracle_lib):
    r = oracle_lib.Replica(16, 4, T=2.2, h=0.05, seed=4, time_slice=0.3,
                           schedule=oracle_lib.SCHED_PALINDROME)
    rec = r.run(12, 3, check=True)
    assert r.check_failures() == 0
    assert (rec["steps"] == 0).all()
    np.testing.assert_allclose(rec["t"], np.array([3, 6, 9, 12]) * 2 * 0.3, rtol=1e-14)
    s, c = r.domain_clocks()
    np.testing.assert_allclose(s + c, 12 * 2 * 0.3, rtol=1e-14)
    spins = r.spins().astype(int)
    assert rec["M"][-1] == spins.sum()
    with pytest.raises(ValueError):
        r.run(2, 1, score=True)  # no score for the time-slice variant
