"""Pins of the oracle's event clock and likelihood-ratio score.

Clock: with all rates equal to 1 every tick is an event and a domain visit
of N_I ticks lasts an Erlang(N_I, tau_S = 1/n_d) time, the density of
Eq. (Poisson Distribution).  In general the n-fold-way clock advances by
N_I/n_d per visit in expectation (each tick fires with probability R_w/n_d
and then adds 1/R_w on average).

Score: the derivative of an endpoint expectation computed by finite
differences of the exact propagated distribution (oracle/exact.py) must
equal E[O * score] from the oracle's trajectories.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import exact


def test_clock_is_erlang_when_all_rates_are_one(oracle_lib):
    L, B, NI = 16, 4, 8
    nd = B * B
    samples = []
    for rep in range(600):
        r = oracle_lib.Replica(L, B, J=0.0, h=0.0, T=1.0, steps_per_visit=NI,
                               seed=21, replica=rep)
        rec = r.run(1)
        assert rec[0]["events"] == rec[0]["steps"] == NI * (L // B) ** 2
        s, c = r.domain_clocks()
        samples.append(s + c)
    samples = np.concatenate(samples)
    res = stats.kstest(samples, stats.gamma(a=NI, scale=1.0 / nd).cdf)
    assert res.pvalue > 1e-4
    assert abs(samples.mean() - NI / nd) < 4 * samples.std() / np.sqrt(samples.size)


@pytest.mark.parametrize("T,h,B,NI", [(2.5, 0.05, 8, 64), (1.7, 0.2, 4, 10),
                                      (3.2, -0.3, 8, 20)])
def test_clock_mean_advance_per_visit(oracle_lib, T, h, B, NI):
    L, sweeps = 16, 4
    nd = B * B
    vals = []
    for rep in range(300):
        r = oracle_lib.Replica(L, B, T=T, h=h, steps_per_visit=NI, seed=5,
                               replica=rep)
        r.run(sweeps)
        s, c = r.domain_clocks()
        vals.append(s + c)
    vals = np.concatenate(vals)
    expect = sweeps * NI / nd
    z = (vals.mean() - expect) / (vals.std() / np.sqrt(vals.size))
    assert abs(z) < 4.5


def exact_expectations(L, B, NI, T, J, h, model, start, sweeps):
    op = exact.SweepOperator(L, B, J, h, T, model, NI)
    p = np.zeros(1 << (L * L))
    p[int(((start.reshape(-1) > 0).astype(np.int64) << np.arange(L * L)).sum())] = 1
    for _ in range(sweeps):
        p = op.par(p)
    M, Bs = exact.magnetisation_and_bonds(L)
    return p @ M, p @ Bs


@pytest.mark.parametrize("model,T,J,h", [(0, 2.5, 1.0, 0.1), (1, 2.0, 0.8, -0.15)])
def test_score_matches_exact_derivative(oracle_lib, model, T, J, h):
    L, B, NI, sweeps = 4, 2, 4, 2
    rng = np.random.default_rng(7)
    start = np.where(rng.random((L, L)) < 0.5, 1, -1).astype(np.int8)
    eps = 1e-5
    dM_dh = (exact_expectations(L, B, NI, T, J, h + eps, model, start, sweeps)[0] -
             exact_expectations(L, B, NI, T, J, h - eps, model, start, sweeps)[0]) / (2 * eps)
    dB_dJ = (exact_expectations(L, B, NI, T, J + eps, h, model, start, sweeps)[1] -
             exact_expectations(L, B, NI, T, J - eps, h, model, start, sweeps)[1]) / (2 * eps)
    n = 30000
    M = np.zeros(n)
    Bs = np.zeros(n)
    S = np.zeros((n, 2))
    for rep in range(n):
        r = oracle_lib.Replica(L, B, J=J, h=h, T=T, steps_per_visit=NI,
                               rate_model=model, init=oracle_lib.INIT_GIVEN,
                               spins=start, seed=31, replica=rep)
        rec, sc = r.run(sweeps, record_every=1, score=True)
        M[rep], Bs[rep] = rec[-1]["M"], rec[-1]["B"]
        S[rep] = sc.sum(axis=0)
    for obs, sc, exact_d in [(M, S[:, 1], dM_dh), (Bs, S[:, 0], dB_dJ)]:
        est = (obs - obs.mean()) * sc
        z = (est.mean() - exact_d) / (est.std() / np.sqrt(n))
        assert abs(z) < 4.5, (est.mean(), exact_d, z)
        # the score has mean zero
        zs = sc.mean() / (sc.std() / np.sqrt(n))
        assert abs(zs) < 4.5
    assert abs(dM_dh) > 0.5 and abs(dB_dJ) > 0.5  # non-trivial derivatives


def test_score_bins_partition_the_run(oracle_lib):
    """Bins per record interval add up to the one-bin score of the same run."""
    kw = dict(L=8, tile=4, T=2.4, h=0.1, seed=3)
    a = oracle_lib.Replica(**kw)
    b = oracle_lib.Replica(**kw)
    _, sa = a.run(12, record_every=3, score=True)
    _, sb = b.run(12, record_every=12, score=True)
    assert sa.shape == (4, 2) and sb.shape == (1, 2)
    np.testing.assert_allclose(sa.sum(axis=0), sb[0], rtol=1e-12, atol=1e-12)
