"""The paper's analysis of parallel runs: time rescaling, ideal efficiency and
response error (Sec. 2.3; App. B, Eq. (efficiency) and Eq. (error metric)).

Host-side post-processing of the observables the GPU records at sweep
endpoints (many replicas = many trajectories).  Time is the integer step
count s of Eq. (CK_parallel in s): a sweep advances it by N_I * N_D, which is
the `steps` field of every record.

Readings (where the printed formulas leave a choice):
* The decay constant is fitted to the connected autocorrelation
  <dA(s) dA(s + ds)> of the equilibrium part of each trajectory (dA = A minus
  the trajectory's mean), averaged over trajectories: for A = H, whose mean is
  far from zero, the raw product <A(s) A(s + ds)> would not decay.  The fit is
  C(ds) = C(0) exp(-ds / tau) by least squares on log(C/C(0)) over the lags
  where C/C(0) is above exp(-2).
* tau_PAR is counted in the paper's sampling interval of N_I steps, so
  eta = tau_REF / (tau_PAR N_I) = tau_REF / tau_PAR when both are in steps
  (eta = 1 for an unpartitioned run, whatever N_I).
* Response error: the parallel ensemble mean, as a function of the rescaled
  time t = s tau_REF / tau_PAR, is interpolated with a cubic spline at the
  reference's sample times s in [0, S], S = 5 tau_REF; each squared
  difference is divided by the squared standard error of the reference mean
  at s (ensemble variance / number of reference trajectories); samples where
  that variance is zero (the common start) are left out.  With equal
  dynamics and equal ensemble sizes its expectation is 2, the value the paper
  reports for well-behaved settings.
"""
import numpy as np


def ensemble_mean(A):
    """<A(s)> over trajectories (rows), Eq. (time dependent averages)."""
    return np.asarray(A, float).mean(axis=0)


def ensemble_sem2(A):
    """Squared standard error of the ensemble mean at every sample."""
    A = np.asarray(A, float)
    return A.var(axis=0, ddof=1) / A.shape[0]


def autocorrelation(A, max_lag, center="trajectory"):
    """Connected autocorrelation C(k) = <dA(i) dA(i + k)> for k = 0..max_lag
    samples, per trajectory (rows of A), averaged over trajectories.  dA is A
    minus each trajectory's own mean (center="trajectory"), or minus the mean
    over every trajectory and sample (center="ensemble"): the paper's
    C_A = <A(s) A(s + ds)> - <A>^2.  The trajectory mean of a window W
    samples long lowers C by about 2 tau / W of C(0), which shortens the
    fitted tau when W is only ten or twenty tau; the ensemble mean does not."""
    A = np.asarray(A, float)
    if center == "ensemble":
        dA = A - A.mean()
    else:
        dA = A - A.mean(axis=1, keepdims=True)
    n = A.shape[1]
    max_lag = min(max_lag, n - 1)
    C = np.empty(max_lag + 1)
    for k in range(max_lag + 1):
        C[k] = np.mean(dA[:, : n - k] * dA[:, k:])
    return C


def fit_tau(C, dt):
    """Decay constant tau of C(k dt) = C(0) exp(-k dt / tau): least squares on
    log(C/C(0)) through the origin, over the leading lags with
    C/C(0) > exp(-2)."""
    C = np.asarray(C, float)
    r = C / C[0]
    k = 1
    while k < len(r) and r[k] > np.exp(-2.0):
        k += 1
    lags = np.arange(1, k) * float(dt)
    if lags.size == 0:
        return float(dt) / max(-np.log(max(r[1], 1e-300)), 1e-300)
    y = np.log(r[1:k])
    return float(-np.sum(lags * lags) / np.sum(lags * y))


def efficiency(tau_ref, tau_par):
    """Ideal efficiency eta = tau_REF / (tau_PAR N_I) with tau_PAR in units of
    N_I steps, i.e. tau_REF / tau_PAR with both in steps (Eq. (efficiency))."""
    return float(tau_ref) / float(tau_par)


def response_error(s_ref, A_ref, s_par, A_par, tau_ref, tau_par, S=None):
    """Response error chi^2 of Eq. (error metric).  A_ref, A_par: trajectories
    (rows) sampled at steps s_ref, s_par.  The parallel mean is rescaled to
    t = s tau_REF / tau_PAR and spline-interpolated at the reference samples
    with s <= S (default 5 tau_REF)."""
    from scipy.interpolate import CubicSpline
    s_ref = np.asarray(s_ref, float)
    s_par = np.asarray(s_par, float)
    S = 5.0 * tau_ref if S is None else S
    m_ref = ensemble_mean(A_ref)
    e2_ref = ensemble_sem2(A_ref)
    m_par = ensemble_mean(A_par)
    t_par = s_par * (tau_ref / tau_par)
    # samples where every reference trajectory agrees (the common start) carry
    # no statistical error and are left out
    keep = (s_ref <= S) & (s_ref >= t_par[0]) & (s_ref <= t_par[-1]) & (e2_ref > 0)
    spline = CubicSpline(t_par, m_par)
    d = m_ref[keep] - spline(s_ref[keep])
    return float(np.mean(d * d / e2_ref[keep]))


def circle_initial_condition(L):
    """The paper's filled-circle start (Sec. 3.2): +1 inside the disc of
    diameter sqrt(2/pi) L centred at ((L-1)/2, (L-1)/2), -1 outside.  The
    printed length 0.7975 sqrt(N_S) is taken as the diameter (as a radius the
    disc would cover the whole lattice); the disc then holds half the area."""
    y, x = np.mgrid[0:L, 0:L]
    c = (L - 1) / 2.0
    r = 0.5 * np.sqrt(2.0 / np.pi) * L
    return np.where((y - c) ** 2 + (x - c) ** 2 <= r * r, 1, -1).astype(np.int8)


def observable(records, L, J=1.0, h=0.0, kind="H", n_sites=None):
    """A(s) of every trajectory from records [replica, record]: the energy
    per site H/N_S (kind "H", the paper's 2D choice) or H m (kind "Hm", its
    1D choice).  N_S = L^2 unless n_sites is given (L on the ring)."""
    N = float(n_sites or L * L)
    H = (-J * records["B"] - h * records["M"]) / N
    if kind == "H":
        return H
    return H * (records["M"] / N)


def run_setting(kmc, L, tile, steps_per_visit, T, n_traj, n_sweeps, record_every, seed,
                J=1.0, h=0.0, rate_model=1, init_spins=None, flags=None, tile_rows=0):
    """n_traj trajectories of one parallelisation setting on the GPU (one
    batched persistent launch; domains `tile` wide and `tile_rows` high).
    Returns records [n_traj, n_records]; with a given start configuration a
    first column holds the start state (s = 0)."""
    d = dict(L=L, tile=tile, T=T, J=J, h=h, steps_per_visit=steps_per_visit,
             rate_model=rate_model, tile_rows=tile_rows)
    given = None
    if init_spins is not None:
        d["init"] = kmc.INIT_GIVEN
        given = [init_spins] * n_traj
    lat = kmc.Lattice([d] * n_traj, seed, given_spins=given)
    lat.run(n_sweeps, record_every, kmc.F_PERSISTENT if flags is None else flags)
    rec = lat.records()
    lat.close()
    if init_spins is not None:
        rec = np.concatenate([start_record(init_spins, n_traj, kmc.RECORD_DTYPE), rec], axis=1)
    return rec


def start_record(spins, n_traj, dtype):
    """Record of a start configuration: M and the right/down bond sum B (the
    right bonds only on a ring, a 1D array of spins)."""
    s = np.asarray(spins).astype(np.int64)
    rec = np.zeros((n_traj, 1), dtype)
    rec["M"] = int(s.sum())
    if s.ndim == 1:
        rec["B"] = int((s * np.roll(s, -1)).sum())
    else:
        rec["B"] = int((s * np.roll(s, -1, 1)).sum() + (s * np.roll(s, -1, 0)).sum())
    return rec


def start_records(starts, dtype):
    """Start records of trajectories with different start configurations."""
    return np.concatenate([start_record(s, 1, dtype) for s in starts], axis=0)
