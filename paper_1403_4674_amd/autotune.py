"""Tile autotuner for batched runs.

For every lattice side L of a workload the tuner times short persistent runs
of a probe batch with each valid domain side B (B % 4 == 0, L/B even,
B <= max_tile) and keeps the fastest in site-updates/s.  The choice changes
the dynamics (the paper's T_PAR depends on the partition) but not the
equilibrium, which Eq. (general reversibility condition) guarantees for any
partition; the chosen tile is written into the descriptors, so every run
(and its oracle replay) uses the same partition.  Choices persist as JSON.
"""
import json
import os
import time

from . import kmc

DEFAULT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_tiles.json")


def valid_tiles(L, max_tile=32, min_tile=8):
    return [B for B in range(min_tile, min(max_tile, L // 2) + 1, 4)
            if L % B == 0 and (L // B) % 2 == 0]


def tune(Ls, T=2.5, h=0.0, probe_replicas=512, sweeps=20, max_tile=32, seed=1234,
         path=DEFAULT_PATH, steps_per_visit=0):
    """Returns {L: best tile} and writes it to `path` (merged with what is
    there).  Timing uses the persistent batched kernel on the GPU."""
    import torch
    table = load(path)
    stream = torch.cuda.current_stream()
    for L in sorted(set(int(x) for x in Ls)):
        best, best_rate = None, -1.0
        timings = {}
        for B in valid_tiles(L, max_tile):
            descs = [dict(L=L, tile=B, T=T, h=h, steps_per_visit=steps_per_visit)] * \
                probe_replicas
            lat = kmc.Lattice(descs, seed)
            lat.run(2, 2, kmc.F_PERSISTENT)
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            lat.run(sweeps, sweeps, kmc.F_PERSISTENT)
            b.record(stream)
            torch.cuda.synchronize()
            sec = a.elapsed_time(b) / 1e3
            lat.close()
            rate = probe_replicas * sweeps * L * L / sec
            timings[B] = rate
            if rate > best_rate:
                best, best_rate = B, rate
        table[str(L)] = {"tile": best, "site_updates_per_s": timings,
                         "probe": dict(T=T, h=h, replicas=probe_replicas, sweeps=sweeps),
                         "when": time.strftime("%Y-%m-%dT%H:%M:%S")}
    save(table, path)
    return {int(k): v["tile"] for k, v in table.items()}


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


def tiles_for(Ls, path=DEFAULT_PATH, fallback=None):
    """Tuned tile per L, falling back to `fallback` (or the largest valid
    tile <= 32) for sides that were never tuned."""
    table = load(path)
    out = {}
    for L in set(int(x) for x in Ls):
        if str(L) in table:
            out[L] = int(table[str(L)]["tile"])
        elif fallback and L in fallback:
            out[L] = fallback[L]
        else:
            out[L] = max(valid_tiles(L, 32, 4))
    return out
