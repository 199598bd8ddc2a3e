"""The paper's 2D parallelisation study, run on the GPU (Sec. 3.2, Table 1,
Fig. (full-summary)): a periodic Ising lattice at k_B T / J = 2.4 with
Glauber (Barker) rates, started from the filled circle, evolved with no
partition (the reference, N_D = 1), with vertical stripes (N_D = 2, 4) and
with checkerboards (N_D = 4, 16) for N_I in {1, 2, 5, 10}; each setting is a
batch of independent trajectories in one persistent launch.  The analysis
(tau, eta, chi^2) is `analysis.py`.

    python -m paper_1403_4674_amd.experiments --L 12 --traj 500

prints one JSON line per setting and a summary line; `--save FILE.npz`
also keeps every setting's trajectories (steps, M, B) for re-analysis.
"""
import json
import time

import numpy as np

from . import analysis


def settings_2d(L):
    """(label, domain width, domain height, N_I) of the unpartitioned
    reference, vertical stripes with N_D = 2 and 4, and checkerboards with
    N_D = 4 and 16, each for N_I in {1, 2, 5, 10} (partitions that do not
    divide L, or whose domains exceed 64 sites a side, are left out)."""
    out = [("reference", L, L, L * L)] if L <= 64 else []
    parts = [(f"stripes N_D={n}", L // n, L, n) for n in (2, 4)]
    parts += [(f"checkerboard N_D={n * n}", L // n, L // n, n) for n in (2, 4)]
    for label, Bx, By, n in parts:
        if L % n or Bx < 1 or Bx > 64 or By > 64:
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
        rec = analysis.run_setting(kmc, L, B, NI, T, n_traj, n_sweeps, every, seed + len(results),
                                   init_spins=ic, tile_rows=By)
        sec = time.perf_counter() - t0
        results.append(dict(label=label, tile=B, tile_rows=By, NI=NI, ND=nd, rec=rec, sec=sec,
                            ticks=n_traj * n_sweeps * per_sweep))
        if verbose:
            print(f"[study] {label}: {n_sweeps} sweeps, {rec.shape[1]} samples, {sec:.2f} s",
                  flush=True)
    return results


def analyse(results, L, eq_fraction=0.5, max_lag_samples=400):
    """tau of A = H m from the equilibrium halves, eta and chi^2 (A = H) of
    every setting against the reference (the first result)."""
    ref = results[0]
    out = []
    taus = []
    for r in results:
        s = r["rec"]["steps"][0].astype(float)
        Am = analysis.observable(r["rec"], L, kind="Hm")
        k0 = int(len(s) * eq_fraction)
        C = analysis.autocorrelation(Am[:, k0:], max_lag_samples)
        taus.append(analysis.fit_tau(C, s[1] - s[0]))
    s_ref = ref["rec"]["steps"][0].astype(float)
    H_ref = analysis.observable(ref["rec"], L, kind="H")
    for r, tau in zip(results, taus):
        s = r["rec"]["steps"][0].astype(float)
        H = analysis.observable(r["rec"], L, kind="H")
        chi2 = analysis.response_error(s_ref, H_ref, s, H, taus[0], tau)
        out.append(dict(setting=r["label"], tile=r["tile"], tile_rows=r["tile_rows"],
                        N_D=r["ND"], N_I=r["NI"],
                        tau_steps=tau, eta=analysis.efficiency(taus[0], tau), chi2=chi2,
                        e_final=float(H[:, -1].mean()), gpu_seconds=r["sec"],
                        site_updates_per_s=r["ticks"] / r["sec"]))
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
    ap.add_argument("--traj", type=int, default=500)
    ap.add_argument("--steps", type=int, default=160000)
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--save", default="", help="write the trajectories to this .npz")
    args = ap.parse_args()
    torch.cuda.set_stream(torch.cuda.Stream())
    kmc.use_torch_allocator()
    res = run_study(kmc, args.L, args.traj, args.steps, seed=args.seed)
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
