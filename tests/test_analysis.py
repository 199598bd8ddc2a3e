"""Pins of the analysis of parallel runs (Sec. 2.3, Eq. (efficiency), Eq.
(error metric)) on processes whose answers are known in closed form."""
import numpy as np
import pytest

from paper_1403_4674_amd import analysis


def ar1(n_traj, n, phi, x0, rng, sigma=1.0):
    """x_{k+1} = phi x_k + sigma e_k: mean x0 phi^k, stationary
    autocorrelation phi^lag, i.e. tau = -1 / ln(phi) samples."""
    x = np.empty((n_traj, n))
    x[:, 0] = x0
    e = rng.standard_normal((n_traj, n)) * sigma
    for k in range(1, n):
        x[:, k] = phi * x[:, k - 1] + e[:, k]
    return x


def test_fit_tau_recovers_an_exact_exponential():
    for tau, dt in [(7.0, 1.0), (1130.0, 144.0), (3.3, 0.5)]:
        C = 2.5 * np.exp(-np.arange(60) * dt / tau)
        assert analysis.fit_tau(C, dt) == pytest.approx(tau, rel=1e-12)


def test_autocorrelation_of_ar1_gives_its_decay_constant():
    rng = np.random.default_rng(0)
    phi = 0.9
    x = ar1(400, 2000, phi, 0.0, rng)
    C = analysis.autocorrelation(x[:, 200:], 60)
    tau = analysis.fit_tau(C, 3.0)  # samples 3 steps apart
    assert tau == pytest.approx(-3.0 / np.log(phi), rel=0.03)
    assert C[0] == pytest.approx(1.0 / (1 - phi * phi), rel=0.03)


def test_efficiency_is_the_ratio_of_decay_constants():
    assert analysis.efficiency(1130.0, 1130.0) == 1.0
    assert analysis.efficiency(1000.0, 500.0) == 2.0


def test_response_error_of_identical_means_is_zero():
    rng = np.random.default_rng(1)
    x = ar1(50, 300, 0.95, 5.0, rng)
    s = np.arange(300) * 10.0
    assert analysis.response_error(s, x, s, x, 195.0, 195.0) == pytest.approx(0.0, abs=1e-20)


def test_response_error_of_two_ensembles_of_one_process_is_about_two():
    """Equal dynamics, equal ensemble sizes: each squared difference of the
    means has expectation twice the squared standard error of one mean."""
    rng = np.random.default_rng(2)
    vals = []
    for _ in range(8):
        a = ar1(200, 400, 0.97, 8.0, rng)
        b = ar1(200, 400, 0.97, 8.0, rng)
        s = np.arange(400) * 1.0
        vals.append(analysis.response_error(s, a, s, b, 33.0, 33.0, S=399.0))
    assert np.mean(vals) == pytest.approx(2.0, rel=0.25)


def test_time_rescaling_maps_a_stretched_response_onto_the_reference():
    """A parallel run whose dynamics is the reference slowed by kappa has
    tau_PAR = kappa tau_REF; after s -> s tau_REF / tau_PAR the mean curves
    coincide, so chi^2 only measures interpolation error."""
    tau_ref, kappa = 40.0, 2.5
    s_ref = np.arange(0, 400, 2.0)
    s_par = np.arange(0, 400 * kappa, 5.0)
    ref = np.exp(-s_ref / tau_ref)[None, :] + np.array([[1e-3], [-1e-3]])
    par = np.exp(-s_par / (kappa * tau_ref))[None, :].repeat(2, 0)
    chi2 = analysis.response_error(s_ref, ref, s_par, par, tau_ref, kappa * tau_ref)
    assert chi2 < 1e-6
    wrong = analysis.response_error(s_ref, ref, s_par, par, tau_ref, tau_ref)
    assert wrong > 1e3


def test_circle_start_is_the_half_area_disc():
    for L in (12, 40, 100):
        ic = analysis.circle_initial_condition(L)
        assert abs((ic == 1).mean() - 0.5) < 0.03
        assert np.array_equal(ic, ic[::-1, :]) and np.array_equal(ic, ic[:, ::-1])
    # 76 of 144 sites inside the disc for 12 x 12: m = 8/144
    assert analysis.circle_initial_condition(12).sum() == 8


def test_observables_from_records():
    rec = np.zeros((1, 2), [("M", "<i8"), ("B", "<i8")])
    rec["M"] = [[144, -10]]
    rec["B"] = [[288, 40]]
    H = analysis.observable(rec, 12, J=1.0, h=0.0, kind="H")
    assert np.allclose(H, [[-2.0, -40 / 144]])
    Hm = analysis.observable(rec, 12, kind="Hm")
    assert np.allclose(Hm, [[-2.0, -40 / 144 * (-10 / 144)]])
    r = analysis.start_record(analysis.circle_initial_condition(12), 3,
                              [("M", "<i8"), ("B", "<i8")])
    assert r.shape == (3, 1) and int(r["M"][0, 0]) == 8


def test_study_save_and_load_round_trip(tmp_path):
    from paper_1403_4674_amd import experiments
    rng = np.random.default_rng(3)
    res = []
    for label, B, By, NI in [("reference", 12, 12, 144), ("stripes N_D=4 N_I=2", 3, 12, 2)]:
        rec = np.zeros((5, 7), [("steps", "<i8"), ("M", "<i8"), ("B", "<i8"), ("t", "<f8")])
        rec["steps"] = np.arange(7)[None, :] * 144
        rec["M"] = rng.integers(-144, 145, (5, 7))
        rec["B"] = rng.integers(-288, 289, (5, 7))
        res.append(dict(label=label, tile=B, tile_rows=By, NI=NI, ND=(12 // B) * (12 // By),
                        rec=rec, sec=1.0, ticks=1))
    p = tmp_path / "study.npz"
    experiments.save_study(str(p), res, 12)
    back, L = experiments.load_study(str(p))
    assert L == 12 and [r["label"] for r in back] == [r["label"] for r in res]
    for a, b in zip(res, back):
        assert (a["tile"], a["tile_rows"], a["NI"], a["ND"]) == \
            (b["tile"], b["tile_rows"], b["NI"], b["ND"])
        for f in ("steps", "M", "B"):
            assert np.array_equal(a["rec"][f], b["rec"][f])


def test_study_settings_cover_the_papers_partitions():
    from paper_1403_4674_amd import experiments
    st = experiments.settings_2d(12)
    labels = [x[0] for x in st]
    assert labels[0] == "reference" and st[0][1:] == (12, 12, 144)
    for n in (2, 4):
        for NI in (1, 2, 5, 10):
            assert (f"stripes N_D={n} N_I={NI}", 12 // n, 12, NI) in st
    for n in (4, 16):
        for NI in (1, 2, 5, 10):
            side = 12 // int(n ** 0.5)
            assert (f"checkerboard N_D={n} N_I={NI}", side, side, NI) in st
    big = experiments.settings_2d(100)   # resident form: the full reference
    assert big[0] == ("reference", 100, 100, 10000)
    assert {x[0].split(" N_I")[0] for x in big[1:]} == {
        "stripes N_D=2", "stripes N_D=4", "checkerboard N_D=4", "checkerboard N_D=16"}
    huge = experiments.settings_2d(256)  # beyond the resident form: domains <= 64
    assert all(By <= 64 and Bx <= 64 for _, Bx, By, _ in huge)


def test_autocorrelation_and_tau_against_exact_propagation(oracle_lib):
    """The analysis on sampled trajectories against the exact equilibrium
    autocorrelation of A = H m for the unpartitioned 3 x 3 lattice (Barker,
    1/(beta J) = 2.4, h = 0.15, one sweep = 9 steps): C(k) = A . T^k (pi A) - <A>^2
    with T the exact sweep operator (oracle/exact.py).  Trajectories come
    from the oracle, started from exact Boltzmann samples."""
    from oracle import exact
    L, T, NI, h = 3, 2.4, 9, 0.15  # a field: <A> != 0, so the connected part matters
    pi, M, B, _ = exact.boltzmann(L, 1.0, h, T)
    A = ((-B - h * M) / 9.0) * (M / 9.0)
    op = exact.SweepOperator(L, L, 1.0, h, T, model=1, NI=NI, quantise=True)
    v = pi * A
    mean = float(pi @ A)
    C_exact = []
    for _ in range(13):
        C_exact.append(float(A @ v) - mean * mean)
        v = op.par(v)
    C_exact = np.array(C_exact)
    rng = np.random.default_rng(5)
    n_traj, n_sw = 240, 2500
    starts = rng.choice(pi.size, size=n_traj, p=pi)
    traj = []
    for rep, i in enumerate(starts):
        spins = np.where((i >> np.arange(L * L)) & 1, 1, -1).astype(np.int8)
        r = oracle_lib.Replica(L, L, T=T, h=h, rate_model=1, steps_per_visit=NI,
                               init=oracle_lib.INIT_GIVEN, spins=spins, seed=77, replica=rep)
        traj.append(r.run(n_sw, 1))
    rec = np.array(traj)
    Am = analysis.observable(rec, L, h=h, kind="Hm")
    C = analysis.autocorrelation(Am, 12)
    np.testing.assert_allclose(C / C[0], C_exact / C_exact[0], atol=0.03)
    t_hat, t_exact = analysis.fit_tau(C, NI), analysis.fit_tau(C_exact, NI)
    assert t_hat == pytest.approx(t_exact, rel=0.08)
