"""The paper's 2D parallelisation study, run on the GPU (Sec. 3.2, Table 1,
Fig. (full-summary)): a periodic Ising lattice at k_B T / J = 2.4 with
Glauber (Barker) rates, started from the filled circle, evolved with no
partition (the reference, N_D = 1), with vertical stripes (N_D = 2, 4) and
with checkerboards (N_D = 4, 16) for N_I in {1, 2, 5, 10}; each setting is a
batch of independent trajectories in one persistent launch.  The analysis
(tau, eta, chi^2) is `analysis.py`.

    python -m paper_1403_4674_amd.experiments --L 12     # 500 x 1.6e5 steps
    python -m paper_1403_4674_amd.experiments --L 100    # 50 x 1.6e7 steps
    python -m paper_1403_4674_amd.experiments --ring     # 1 x 8: 6000 x 800 steps

(Table 1's trajectory counts and run lengths) prints one JSON line per
setting and a summary line; `--save FILE.npz` also keeps every setting's
trajectories (steps, M, B) for re-analysis.  Lattices up to 128 run in the
resident form (the whole lattice in one workgroup's LDS), which holds the
unpartitioned 100 x 100 reference and the 100-high stripes.
"""
import json
import time

import numpy as np

from . import analysis


# Table 1: trajectories and steps per trajectory of the 2D runs
PAPER_RUNS = {12: (500, 160_000), 100: (50, 16_000_000)}


def max_side(L):
    """Largest domain side the GPU runs for lattice side L (the resident form
    holds domains up to the lattice itself for L <= 128)."""
    return L if L <= 128 else 64


def settings_2d(L):
    """(label, domain width, domain height, N_I) of the unpartitioned
    reference, vertical stripes with N_D = 2 and 4, and checkerboards with
    N_D = 4 and 16, each for N_I in {1, 2, 5, 10} (partitions that do not
    divide L, or whose domains are too large for the GPU, are left out)."""
    top = max_side(L)
    out = [("reference", L, L, L * L)] if L <= top else []
    parts = [(f"stripes N_D={n}", L // n, L, n) for n in (2, 4)]
    parts += [(f"checkerboard N_D={n * n}", L // n, L // n, n) for n in (2, 4)]
    for label, Bx, By, n in parts:
        if L % n or Bx < 1 or Bx > top or By > top:
            continue
        for NI in (1, 2, 5, 10):
            out.append((f"{label} N_I={NI}", Bx, By, NI))
    return out


def run_study(kmc, L=12, n_traj=500, total_steps=160000, sample_steps=None, T=2.4, seed=2024,
              settings=None, verbose=True):
    """Runs every setting for `total_steps` steps of s per trajectory,
    sampling A about every `sample_steps` steps (default N_S), and returns
    the per-setting records and timings."""
    sample_steps = sample_steps or L * L
    ic = analysis.circle_initial_condition(L)
    results = []
    for label, B, By, NI in (settings or settings_2d(L)):
        nd = (L // B) * (L // By)
        per_sweep = NI * nd
        every = max(1, int(round(sample_steps / per_sweep)))
        n_sweeps = max(every, (total_steps // (per_sweep * every)) * every)
        t0 = time.perf_counter()
        flags = kmc.F_RESIDENT if L <= 128 else kmc.F_PERSISTENT
        rec = analysis.run_setting(kmc, L, B, NI, T, n_traj, n_sweeps, every, seed + len(results),
                                   init_spins=ic, tile_rows=By, flags=flags)
        sec = time.perf_counter() - t0
        results.append(dict(label=label, tile=B, tile_rows=By, NI=NI, ND=nd, rec=rec, sec=sec,
                            ticks=n_traj * n_sweeps * per_sweep))
        if verbose:
            print(f"[study] {label}: {n_sweeps} sweeps, {rec.shape[1]} samples, {sec:.2f} s",
                  flush=True)
    return results


def analyse(results, L, eq_fraction=0.5, max_lag_samples=400, n_boot=30, boot_seed=0):
    """tau of A = H m from the equilibrium halves, eta and chi^2 (A = H) of
    every setting against the reference (the first result).  Also: chi^2
    without the time rescaling (tau_PAR = tau_REF), and bootstrap standard
    errors of tau and eta (trajectories resampled n_boot times; eta's error
    combines the two taus' in quadrature)."""
    ref = results[0]
    rng = np.random.default_rng(boot_seed)

    def tau_of(r, rows=None):
        s = r["rec"]["steps"][0].astype(float)
        Am = analysis.observable(r["rec"], L, kind="Hm")
        if rows is not None:
            Am = Am[rows]
        k0 = int(len(s) * eq_fraction)
        C = analysis.autocorrelation(Am[:, k0:], max_lag_samples)
        return analysis.fit_tau(C, s[1] - s[0])

    taus, ses = [], []
    for r in results:
        taus.append(tau_of(r))
        n = r["rec"].shape[0]
        boot = [tau_of(r, rng.integers(0, n, n)) for _ in range(n_boot)]
        ses.append(float(np.std(boot)) if n_boot > 1 else float("nan"))
    s_ref = ref["rec"]["steps"][0].astype(float)
    H_ref = analysis.observable(ref["rec"], L, kind="H")
    out = []
    for r, tau, se in zip(results, taus, ses):
        s = r["rec"]["steps"][0].astype(float)
        H = analysis.observable(r["rec"], L, kind="H")
        chi2 = analysis.response_error(s_ref, H_ref, s, H, taus[0], tau)
        chi2_raw = analysis.response_error(s_ref, H_ref, s, H, taus[0], taus[0])
        eta = analysis.efficiency(taus[0], tau)
        eta_se = eta * float(np.hypot(ses[0] / taus[0], se / tau)) if r is not ref else 0.0
        out.append(dict(setting=r["label"], tile=r["tile"], tile_rows=r["tile_rows"],
                        N_D=r["ND"], N_I=r["NI"], tau_steps=tau, tau_se=se,
                        eta=eta, eta_se=eta_se, chi2=chi2, chi2_unscaled=chi2_raw,
                        e_final=float(H[:, -1].mean()), gpu_seconds=r["sec"],
                        site_updates_per_s=r["ticks"] / r["sec"]))
    return out


# ------------------------------------------------------------------ the ring
#
# The paper's 1D study (Sec. 3.1, Eq. (1D partitions), Table 1): a periodic
# ring of 8 sites at 1/(beta J) = 2 with Glauber (Barker) rates, started from
# the eight configurations with two adjacent up spins, evolved serially
# (N_D = 1, the reference) and with N_D in {2, 4, 8} domains for N_I in
# {1, 2, 5, 10}; 6000 trajectories of S = 800 steps per setting.  A = H m.

RING_RUN = (8, 6000, 800)  # sites, trajectories, steps (Table 1)


def settings_ring(N=8):
    """(label, domain length, N_I) of the reference and the partitions."""
    out = [("reference", N, 1)]
    for nd in (2, 4, 8):
        if N % nd:
            continue
        for NI in (1, 2, 5, 10):
            out.append((f"N_D={nd} N_I={NI}", N // nd, NI))
    return out


def ring_starts(N, n_traj):
    """Trajectory k starts from the k mod N-th configuration with two
    adjacent up spins (sites k mod N and k mod N + 1)."""
    out = []
    for k in range(n_traj):
        s = -np.ones(N, np.int8)
        s[k % N] = s[(k + 1) % N] = 1
        out.append(s)
    return out


def run_ring_study(kmc, N=8, n_traj=6000, total_steps=800, T=2.0, seed=1998, verbose=True):
    """Every ring setting for total_steps steps per trajectory, sampled at
    every sweep end (N_D N_I steps apart), each as one persistent launch of
    n_traj replicas; records [n_traj, samples] with the start (s = 0) first."""
    starts = ring_starts(N, n_traj)
    results = []
    for k, (label, B, NI) in enumerate(settings_ring(N)):
        nd = N // B
        per_sweep = nd * NI
        n_sweeps = max(1, total_steps // per_sweep)
        d = dict(L=N, tile=B, T=T, steps_per_visit=NI, rate_model=kmc.RATE_BARKER,
                 init=kmc.INIT_GIVEN, dims=1)
        t0 = time.perf_counter()
        lat = kmc.Lattice([d] * n_traj, seed + k, given_spins=starts)
        lat.run(n_sweeps, 1, kmc.F_PERSISTENT)
        rec = lat.records()
        lat.close()
        sec = time.perf_counter() - t0
        rec = np.concatenate([analysis.start_records(starts, kmc.RECORD_DTYPE), rec], axis=1)
        results.append(dict(label=label, tile=B, NI=NI, ND=nd, rec=rec, sec=sec,
                            ticks=n_traj * n_sweeps * per_sweep))
        if verbose:
            print(f"[ring] {label}: {n_sweeps} sweeps, {sec:.2f} s", flush=True)
    return results


def analyse_ring(results, N, eq_fraction=0.5, max_lag_samples=200, n_boot=30, boot_seed=0):
    """tau of A = H m from the equilibrium halves (in steps), eta = tau_REF /
    tau_PAR and the paper's chi^2 of <A> against the reference (Eq. (efficiency),
    Eq. (error metric)), with bootstrap errors over trajectories."""
    rng = np.random.default_rng(boot_seed)

    def A(r):
        return analysis.observable(r["rec"], N, kind="Hm", n_sites=N)

    def tau_of(r, rows=None):
        s = r["rec"]["steps"][0].astype(float)
        a = A(r) if rows is None else A(r)[rows]
        k0 = int(len(s) * eq_fraction)
        # runs of 800 steps are only ~14 tau_REF long at equilibrium: centre
        # on the ensemble mean, which the trajectory means would bias
        C = analysis.autocorrelation(a[:, k0:], min(max_lag_samples, len(s) - k0 - 1),
                                     center="ensemble")
        return analysis.fit_tau(C, s[2] - s[1])

    taus, ses = [], []
    for r in results:
        taus.append(tau_of(r))
        n = r["rec"].shape[0]
        boot = [tau_of(r, rng.integers(0, n, n)) for _ in range(n_boot)]
        ses.append(float(np.std(boot)))
    ref = results[0]
    s_ref = ref["rec"]["steps"][0].astype(float)
    A_ref = A(ref)
    out = []
    for r, tau, se in zip(results, taus, ses):
        s = r["rec"]["steps"][0].astype(float)
        a = A(r)
        chi2 = analysis.response_error(s_ref, A_ref, s, a, taus[0], tau)
        chi2_raw = analysis.response_error(s_ref, A_ref, s, a, taus[0], taus[0])
        eta = analysis.efficiency(taus[0], tau)
        eta_se = eta * float(np.hypot(ses[0] / taus[0], se / tau)) if r is not ref else 0.0
        H = analysis.observable(r["rec"], N, kind="H", n_sites=N)
        k0 = int(H.shape[1] * eq_fraction)
        out.append(dict(setting=r["label"], N_D=r["ND"], N_I=r["NI"], tau_steps=tau,
                        tau_se=se, eta=eta, eta_se=eta_se, chi2=chi2, chi2_unscaled=chi2_raw,
                        e_eq=float(H[:, k0:].mean()), gpu_seconds=r["sec"]))
    return out


def save_study(path, results, L):
    """Trajectories of every setting as compact arrays: M and B fit in 32
    bits for L <= 2^14; steps are shared by all trajectories of a setting."""
    arrays = {}
    for k, r in enumerate(results):
        rec = r["rec"]
        arrays[f"s{k}_steps"] = rec["steps"][0].astype(np.int64)
        arrays[f"s{k}_M"] = rec["M"].astype(np.int32)
        arrays[f"s{k}_B"] = rec["B"].astype(np.int32)
    arrays["labels"] = np.array([r["label"] for r in results])
    arrays["tile"] = np.array([r["tile"] for r in results])
    arrays["tile_rows"] = np.array([r["tile_rows"] for r in results])
    arrays["NI"] = np.array([r["NI"] for r in results])
    arrays["L"] = np.array(L)
    np.savez_compressed(path, **arrays)


def load_study(path):
    """Inverse of save_study: a list of dicts with `label`, `tile`, `NI`, `ND`
    and `rec` (structured records with the fields steps, M, B), as
    `analyse` takes them (timings are not kept)."""
    z = np.load(path)
    L = int(z["L"])
    out = []
    for k, label in enumerate(z["labels"]):
        M = z[f"s{k}_M"]
        rec = np.zeros(M.shape, [("steps", "<i8"), ("M", "<i8"), ("B", "<i8")])
        rec["steps"] = z[f"s{k}_steps"][None, :]
        rec["M"] = M
        rec["B"] = z[f"s{k}_B"]
        B = int(z["tile"][k])
        By = int(z["tile_rows"][k]) if "tile_rows" in z else B
        out.append(dict(label=str(label), tile=B, tile_rows=By, NI=int(z["NI"][k]),
                        ND=(L // B) * (L // By), rec=rec, sec=float("nan"), ticks=0))
    return out, L


def main():
    import argparse

    import torch

    from . import kmc
    ap = argparse.ArgumentParser()
    ap.add_argument("--L", type=int, default=12)
    ap.add_argument("--ring", action="store_true",
                    help="the 1 x 8 ring study (Sec. 3.1) instead of the 2D one")
    ap.add_argument("--traj", type=int, default=0, help="default: Table 1's count")
    ap.add_argument("--steps", type=int, default=0, help="default: Table 1's length")
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--save", default="", help="write the trajectories to this .npz")
    ap.add_argument("--only", default="",
                    help="comma-separated labels to keep besides the reference, e.g. "
                         "'stripes N_D=2 N_I=1,stripes N_D=2 N_I=2'")
    args = ap.parse_args()
    torch.cuda.set_stream(torch.cuda.Stream())
    kmc.use_torch_allocator()
    if args.ring:
        N, traj, steps = RING_RUN
        res = run_ring_study(kmc, N, args.traj or traj, args.steps or steps)
        for row in analyse_ring(res, N):
            print(json.dumps(row), flush=True)
        print(json.dumps({"ring": N, "trajectories": args.traj or traj,
                          "steps": args.steps or steps,
                          "gpu_seconds": sum(r["sec"] for r in res),
                          "site_updates": int(sum(r["ticks"] for r in res))}), flush=True)
        return
    traj, steps = PAPER_RUNS.get(args.L, (100, 100 * args.L * args.L))
    args.traj = args.traj or traj
    args.steps = args.steps or steps
    settings = settings_2d(args.L)
    if args.only:
        keep = {x.strip() for x in args.only.split(",")}
        settings = [st for st in settings if st[0] == "reference" or st[0] in keep]
    res = run_study(kmc, args.L, args.traj, args.steps, seed=args.seed, settings=settings)
    rows = analyse(res, args.L)
    if args.save:
        save_study(args.save, res, args.L)
    for row in rows:
        print(json.dumps(row), flush=True)
    print(json.dumps({"L": args.L, "trajectories": args.traj, "steps": args.steps,
                      "gpu_seconds": sum(r["sec"] for r in res),
                      "site_updates": int(sum(r["ticks"] for r in res))}), flush=True)


if __name__ == "__main__":
    main()
