"""The ring study's analysis (Sec. 3.1, App. B) on oracle trajectories (no
GPU): the fitted decay time of A = H m of the serial reference against the
same fit applied to the exact equilibrium autocorrelation of the 1 x 8 ring
(oracle/exact.py), and the bookkeeping of the study (settings, starts,
sampling in steps)."""
import numpy as np

from oracle import exact
from paper_1403_4674_amd import analysis, experiments


def exact_tau_ref(N=8, T=2.0, lags=400):
    """tau of A = H m for serial Barker dynamics (one tick per step), from
    C(k) = sum_s pi(s) A(s) E[A(sigma_k) | sigma_0 = s] - <A>^2."""
    pi, M, B, E = exact.ring_boltzmann(N, 1.0, 0.0, T)
    A = (E / N) * (M / N)
    kern = exact.RingTickKernel(N, range(N), 1.0, 0.0, T, 1, quantise=True)
    v, C = A.copy(), []
    mean = (pi * A).sum()
    for _ in range(lags):
        C.append((pi * A * v).sum() - mean ** 2)
        v = kern.apply_transpose(v, 1)
    return analysis.fit_tau(np.array(C), 1.0)


def oracle_study(kmco, settings, N=8, n_traj=1500, steps=800, seed=7):
    starts = experiments.ring_starts(N, n_traj)
    out = []
    for k, (label, B, NI) in enumerate(settings):
        nd = N // B
        sweeps = steps // (nd * NI)
        recs = []
        for rho in range(n_traj):
            o = kmco.Replica(N, B, T=2.0, steps_per_visit=NI, rate_model=1,
                             init=kmco.INIT_GIVEN, spins=starts[rho], seed=seed + k,
                             replica=rho, dims=1)
            recs.append(o.run(sweeps, 1))
        rec = np.concatenate([analysis.start_records(starts, kmco.RECORD_DTYPE),
                              np.array(recs)], axis=1)
        out.append(dict(label=label, tile=B, NI=NI, ND=nd, rec=rec, sec=1.0, ticks=0))
    return out


def test_ring_settings_and_starts():
    s = experiments.settings_ring(8)
    assert s[0] == ("reference", 8, 1)
    assert ("N_D=8 N_I=10", 1, 10) in s and len(s) == 1 + 3 * 4
    st = experiments.ring_starts(8, 10)
    for k, x in enumerate(st):
        assert x.sum() == -4 and x[k % 8] == 1 and x[(k + 1) % 8] == 1


def test_ring_reference_tau_matches_exact(oracle_lib):
    tau_exact = exact_tau_ref()
    assert 25 < tau_exact < 35  # Table 1 prints tau_REF = 31.80 for this ring
    res = oracle_study(oracle_lib, [("reference", 8, 1), ("N_D=2 N_I=1", 4, 1)])
    rows = experiments.analyse_ring(res, 8, n_boot=20)
    ref = rows[0]
    assert ref["eta"] == 1.0 and ref["chi2"] == 0.0
    assert abs(ref["tau_steps"] - tau_exact) < 4.5 * ref["tau_se"] + 0.5, (ref, tau_exact)
    # the equilibrium energy of the second half against the exact ring value
    pi, M, B, E = exact.ring_boltzmann(8, 1.0, 0.0, 2.0)
    assert abs(ref["e_eq"] - (pi * E).sum() / 8) < 0.02
    assert np.isfinite(rows[1]["eta"]) and rows[1]["chi2"] >= 0.0
