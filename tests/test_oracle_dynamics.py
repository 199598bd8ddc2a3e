"""Pins of the oracle's dynamics against exact probability propagation.

The paper evolves the probability vector with the parallel transition
matrix to obtain its reference values (Sec. 3.1, Eq. (CK_parallel in s)).
oracle/exact.py does the same on 2^N states, independently of kmco.c:
  * the oracle's state histogram after w sweeps over many independent
    replicas must match T_PAR^w applied to the start state (chi-square);
  * replicas started from exact Boltzmann samples must stay Boltzmann-
    distributed (Eq. (equilibrium distribution)), which Eq. (general
    reversibility condition) guarantees for every domain size, N_I and
    schedule, and random starts must converge to it.
A wrong halo, neighbour index, class prefix, member order, rate sign or
schedule changes these distributions and fails the chi-square tests.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import exact

PMIN = 1e-5


def state_index(spins):
    bits = (np.asarray(spins).reshape(-1) > 0).astype(np.int64)
    return int((bits << np.arange(bits.size)).sum())


def chi2_pvalue(counts, probs):
    n = counts.sum()
    exp_ = probs * n
    big = exp_ >= 5
    obs = np.append(counts[big], counts[~big].sum())
    ex = np.append(exp_[big], exp_[~big].sum())
    if ex[-1] < 5:  # fold a tiny remainder into the last big bin
        obs[-2] += obs[-1]
        ex[-2] += ex[-1]
        obs, ex = obs[:-1], ex[:-1]
    return stats.chisquare(obs, ex * obs.sum() / ex.sum()).pvalue


def sample_states(kmco, L, B, nrep, sweeps, start=None, seed=17, **kw):
    counts = np.zeros(1 << (L * L))
    for rep in range(nrep):
        if start is not None:
            r = kmco.Replica(L, B, init=kmco.INIT_GIVEN, spins=start, seed=seed,
                             replica=rep, **kw)
        else:
            r = kmco.Replica(L, B, seed=seed, replica=rep, **kw)
        r.run(sweeps)
        counts[state_index(r.spins())] += 1
    return counts


def start_state(L, seed=3):
    rng = np.random.default_rng(seed)
    return np.where(rng.random((L, L)) < 0.5, 1, -1).astype(np.int8)


FINITE_TIME = [
    # L, B, N_I, T, J, h, model, palindrome, sweeps
    (4, 2, 4, 2.5, 1.0, 0.1, 0, False, 1),
    (4, 2, 3, 2.0, 1.0, -0.2, 1, False, 2),
    (4, 1, 1, 2.5, 1.0, 0.1, 0, False, 2),
    (4, 2, 2, 2.5, 0.8, 0.3, 0, True, 1),
    (2, 1, 2, 1.5, 1.0, 0.2, 1, False, 3),
    (3, 3, 9, 2.0, 1.0, 0.1, 0, False, 1),   # N_D = 1, domain wraps on itself
]


@pytest.mark.parametrize("L,B,NI,T,J,h,model,pal,sweeps", FINITE_TIME)
def test_finite_time_distribution(oracle_lib, L, B, NI, T, J, h, model, pal,
                                  sweeps):
    start = start_state(L)
    op = exact.SweepOperator(L, B, J, h, T, model, NI, palindrome=pal)
    p = np.zeros(1 << (L * L))
    p[state_index(start)] = 1.0
    for _ in range(sweeps):
        p = op.par(p)
    assert abs(p.sum() - 1) < 1e-12
    counts = sample_states(oracle_lib, L, B, 12000, sweeps, start, J=J, h=h,
                           T=T, steps_per_visit=NI, rate_model=model,
                           schedule=1 if pal else 0)
    assert chi2_pvalue(counts, p) > PMIN


STATIONARY = [
    # L, B, N_I, T, J, h, model, palindrome, sweeps
    (4, 2, 4, 2.5, 1.0, 0.1, 0, False, 3),
    (4, 1, 2, 3.0, 1.0, 0.0, 1, False, 3),
    (4, 2, 1, 2.5, 1.0, -0.1, 0, True, 4),
    (3, 3, 9, 2.5, 1.0, 0.0, 0, False, 3),
    (4, 4, 16, 2.2, 1.0, 0.1, 0, False, 2),
    (4, 2, 5, 1.8, 1.0, 0.25, 1, False, 3),
]


@pytest.mark.parametrize("L,B,NI,T,J,h,model,pal,sweeps", STATIONARY)
def test_boltzmann_is_stationary(oracle_lib, L, B, NI, T, J, h, model, pal,
                                 sweeps):
    """Replicas started from exact Boltzmann samples stay Boltzmann-
    distributed at every sweep endpoint (Eq. (general reversibility
    condition) implies pi T_PAR = pi)."""
    pi, *_ = exact.boltzmann(L, J, h, T)
    rng = np.random.default_rng(2024)
    starts = rng.choice(pi.size, size=12000, p=pi)
    counts = np.zeros(pi.size)
    for rep, i in enumerate(starts):
        spins = np.where((i >> np.arange(L * L)) & 1, 1, -1).astype(np.int8)
        r = oracle_lib.Replica(L, B, J=J, h=h, T=T, steps_per_visit=NI,
                               rate_model=model, schedule=1 if pal else 0,
                               init=oracle_lib.INIT_GIVEN, spins=spins, seed=8,
                               replica=rep)
        r.run(sweeps)
        counts[state_index(r.spins())] += 1
    assert chi2_pvalue(counts, pi) > PMIN


@pytest.mark.parametrize("L,B,NI,T,J,h,model,sweeps", [
    (4, 1, 2, 3.0, 1.0, 0.0, 1, 30)])
def test_converges_to_boltzmann(oracle_lib, L, B, NI, T, J, h, model, sweeps):
    """From random starts the endpoint distribution converges to pi; the
    exact operator certifies that the burn-in is long enough."""
    pi, *_ = exact.boltzmann(L, J, h, T)
    op = exact.SweepOperator(L, B, J, h, T, model, NI)
    p = np.full(pi.size, 1.0 / pi.size)
    for _ in range(sweeps):
        p = op.par(p)
    assert 0.5 * np.abs(p - pi).sum() < 1e-3
    counts = sample_states(oracle_lib, L, B, 12000, sweeps, None, J=J, h=h, T=T,
                           steps_per_visit=NI, rate_model=model)
    assert chi2_pvalue(counts, pi) > PMIN


@pytest.mark.parametrize("L,B,NI,pal", [(4, 2, 4, False), (4, 1, 2, False),
                                        (4, 2, 3, True)])
def test_exact_parallel_kernel_is_reversible(L, B, NI, pal):
    """Eq. (general reversibility condition) and the mixture of Eq. (sum of
    sequential tms): pi is stationary for T_PAR, T_PAR D_pi is symmetric, and
    T_SEQ(Lambda) D_pi = (T_SEQ(reverse Lambda) D_pi)^T for each schedule."""
    J, h, T = 1.0, 0.15, 2.3
    pi, *_ = exact.boltzmann(L, J, h, T)
    op = exact.SweepOperator(L, B, J, h, T, 0, NI, palindrome=pal)
    assert np.abs(op.par(pi) - pi).max() < 1e-13
    rng = np.random.default_rng(0)
    a, b = rng.random(pi.size), rng.random(pi.size)
    lhs = a @ op.par(pi * b)
    rhs = b @ op.par(pi * a)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    for order in op.orders()[:5]:
        rev = tuple(reversed(order))
        lhs = a @ op.seq(pi * b, order)
        rhs = b @ op.seq(pi * a, rev)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_single_order_is_not_reversible():
    """A fixed non-palindromic order is not reversible by itself; the
    mixture over reversed pairs is what restores Eq. (general reversibility
    condition).  Guards the test above against being vacuous."""
    L, B, NI = 4, 2, 4
    pi, *_ = exact.boltzmann(L, 1.0, 0.15, 2.3)
    op = exact.SweepOperator(L, B, 1.0, 0.15, 2.3, 0, NI)
    rng = np.random.default_rng(1)
    a, b = rng.random(pi.size), rng.random(pi.size)
    order = (0, 1, 2, 3)
    lhs = a @ op.seq(pi * b, order)
    rhs = b @ op.seq(pi * a, order)
    assert abs(lhs - rhs) > 1e-6 * abs(lhs)


def test_bookkeeping_check_mode(oracle_lib):
    for L, B in [(8, 4), (12, 6), (8, 2), (6, 6)]:
        r = oracle_lib.Replica(L, B, T=2.2, h=0.05, seed=4)
        r.run(20, check=True)
        assert r.check_failures() == 0


def test_records_match_lattice(oracle_lib):
    r = oracle_lib.Replica(16, 8, T=2.5, steps_per_visit=64, seed=1)
    rec = r.run(5)
    s = r.spins().astype(np.int64)
    M = s.sum()
    Bs = (s * np.roll(s, -1, 1)).sum() + (s * np.roll(s, -1, 0)).sum()
    assert rec[-1]["M"] == M and rec[-1]["B"] == Bs
    assert rec[-1]["steps"] == 5 * 64 * 4 and rec[-1]["sweep"] == 5
    assert r.domain_events().sum() == rec[-1]["events"]


def test_determinism(oracle_lib):
    a = oracle_lib.Replica(16, 8, T=2.0, seed=99, replica=3)
    b = oracle_lib.Replica(16, 8, T=2.0, seed=99, replica=3)
    ra, rb = a.run(30), b.run(30)
    assert (ra == rb).all()
    assert (a.spins() == b.spins()).all()


def test_resume_equals_uninterrupted(oracle_lib):
    a = oracle_lib.Replica(16, 4, T=2.3, seed=5)
    b = oracle_lib.Replica(16, 4, T=2.3, seed=5)
    ra = a.run(40, record_every=2)
    rb = np.concatenate([b.run(10, record_every=2), b.run(30, record_every=2)])
    assert (ra == rb).all() and (a.spins() == b.spins()).all()
