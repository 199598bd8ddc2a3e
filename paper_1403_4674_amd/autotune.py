"""Tile autotuner for batched runs.

The domain side B of every lattice side L in a batch is chosen by timing
the real batch: coordinate descent over L, trying each valid B (B % 4 == 0,
L/B even, B <= max_tile) with the other sides fixed, keeping the fastest in
site-updates/s of the persistent kernel.  The choice changes the dynamics
(the paper's T_PAR depends on the partition) but not the equilibrium, which
Eq. (general reversibility condition) guarantees for any partition; the
chosen tile is written into the descriptors, so every run and its oracle
replay use the same partition.  Choices persist as JSON keyed by workload.
"""
import json
import os
import time

from . import kmc

DEFAULT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_tiles.json")


def valid_tiles(L, max_tile=32, min_tile=8):
    return [B for B in range(min_tile, min(max_tile, L // 2) + 1, 4)
            if L % B == 0 and (L // B) % 2 == 0]


def _rate(descs, seed, sweeps, warmup=4, repeats=2):
    """Site-updates/s of the persistent kernel on the batch: `warmup` sweeps
    first (the random start relaxes fastest and has the most events), then
    the best of `repeats` timed runs of `sweeps` sweeps."""
    import torch
    stream = torch.cuda.current_stream()
    lat = kmc.Lattice(descs, seed)
    lat.run(warmup, warmup, kmc.F_PERSISTENT)
    best = 0.0
    for _ in range(repeats):
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        lat.run(sweeps, sweeps, kmc.F_PERSISTENT)
        b.record(stream)
        torch.cuda.synchronize()
        best = max(best, sweeps * sum(d["L"] ** 2 for d in descs) / (a.elapsed_time(b) / 1e3))
    lat.close()
    return best


def tune_batch(name, descs, seed, sweeps=30, max_tile=32, passes=1, path=DEFAULT_PATH,
               verbose=False, starts=None):
    """Chooses a tile per lattice side for the batch `descs` (dicts with L,
    tile, ...), records the choice under `name` and returns {L: tile}.

    Coordinate descent from the best of several starting points: the
    descriptors' tiles, the largest valid tiles up to 16 (the range of the
    four-domains-per-wavefront kernel, which only pays once most replicas
    use it, so single-coordinate moves from large tiles never reach it), and
    any `starts` given."""
    Ls = sorted({int(d["L"]) for d in descs})
    with_tiles = lambda tl: [dict(d, tile=tl[int(d["L"])]) for d in descs]
    cands = [{L: int(next(d["tile"] for d in descs if d["L"] == L)) for L in Ls}]
    small = {L: max(valid_tiles(L, 16, 4)) for L in Ls}
    if small not in cands:
        cands.append(small)
    cands += [dict(s) for s in (starts or []) if s not in cands]
    trials = []
    best, tiles = -1.0, None
    for c in cands:
        r = _rate(with_tiles(c), seed, sweeps)
        trials.append({"tiles": dict(c), "site_updates_per_s": r})
        if verbose:
            print(f"[autotune] {name} start {c}: {r:.3e} site-updates/s", flush=True)
        if r > best:
            best, tiles = r, dict(c)
    for _ in range(passes):
        for L in Ls:
            for B in valid_tiles(L, max_tile):
                if B == tiles[L]:
                    continue
                cand = dict(tiles)
                cand[L] = B
                r = _rate(with_tiles(cand), seed, sweeps)
                trials.append({"tiles": dict(cand), "site_updates_per_s": r})
                if verbose:
                    print(f"[autotune] {name} L={L} B={B}: {r:.3e} site-updates/s", flush=True)
                if r > best:
                    best, tiles = r, cand
    table = load(path)
    table[name] = {"tiles": {str(k): v for k, v in tiles.items()},
                   "site_updates_per_s": best, "sweeps": sweeps,
                   "trials": [{"tiles": {str(k): v for k, v in t["tiles"].items()},
                               "site_updates_per_s": t["site_updates_per_s"]}
                              for t in trials],
                   "when": time.strftime("%Y-%m-%dT%H:%M:%S")}
    save(table, path)
    return tiles


def load(path=DEFAULT_PATH):
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save(table, path=DEFAULT_PATH):
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tiles_for(name, path=DEFAULT_PATH):
    """The tuned {L: tile} of workload `name`, or None."""
    entry = load(path).get(name)
    if not entry:
        return None
    return {int(k): int(v) for k, v in entry["tiles"].items()}


def main():
    """Tunes the two batched benchmark workloads on the current GPU and
    writes the table to --out (default: next to this file)."""
    import argparse

    import torch

    from . import workloads
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_PATH)
    ap.add_argument("--sweeps", type=int, default=30)
    args = ap.parse_args()
    torch.cuda.set_stream(torch.cuda.Stream())
    kmc.use_torch_allocator()
    DEF = workloads.DEFAULT_TILE
    seed, descs, _ = workloads.batched_4096(tiles=DEF)
    print("batched_4096", tune_batch("batched_4096", descs, seed, sweeps=args.sweeps,
                                     path=args.out, verbose=True), flush=True)
    seed, descs, _ = workloads.differentiable_1024(tile=32)
    print("differentiable_1024", tune_batch("differentiable_1024", descs, seed,
                                            sweeps=args.sweeps, path=args.out,
                                            verbose=True), flush=True)


if __name__ == "__main__":
    main()
