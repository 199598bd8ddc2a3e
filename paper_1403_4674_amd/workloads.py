"""Seeded synthetic workloads shaped like the paper's 2D Ising runs.

Only parameter draws live here (lattice sizes, temperatures, fields, seeds);
none of the method's arithmetic.  Both the HIP path and the oracle-based
tests take their inputs from these functions.

The paper studies periodic square Ising lattices at 1/(beta J) = 2.4 with
checkerboard or stripe domains (Sec. 3.2, Table 1); the five workloads below
extend that shape to GPU sizes.
"""
import json
import os

import numpy as np

METROPOLIS = 0

# tile side per lattice side for batched runs: the largest valid tile <= 32
# (L/tile even), unless the autotuner chose otherwise
DEFAULT_TILE = {16: 8, 24: 12, 32: 16, 48: 24, 64: 32, 128: 32}


def single_16(seed_list=range(1, 9)):
    """16x16, J=1, h=0, T=2.5, 2x2 domains of 8x8, N_I=64, 1000 sweeps,
    record every sweep; one replica per seed."""
    desc = dict(L=16, tile=8, J=1.0, h=0.0, T=2.5, steps_per_visit=64,
                rate_model=METROPOLIS)
    return [(s, [desc]) for s in seed_list], dict(sweeps=1000, record_every=1)


def single_1024(T):
    """1024x1024, 32x32 domains (1024 domains, 256 per colour), N_I=1024,
    random start, seed 2, 10^4 sweeps, record every 10."""
    desc = dict(L=1024, tile=32, J=1.0, h=0.0, T=float(T), steps_per_visit=1024,
                rate_model=METROPOLIS)
    return 2, [desc], dict(sweeps=10_000, record_every=10)


def quench_4096():
    """4096x4096 quench from a random start to T=1.5, 64x64 domains,
    N_I=4096, seed 3, 2000 sweeps, record every 10."""
    desc = dict(L=4096, tile=64, J=1.0, h=0.0, T=1.5, steps_per_visit=4096,
                rate_model=METROPOLIS)
    return 3, [desc], dict(sweeps=2000, record_every=10)


TUNED_TILES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_tiles.json")


def _tuned(name):
    """(Bx, By, N_I) per lattice side chosen for workload `name` by the
    autotuner (a JSON table next to this file), or None.  Entries written
    before the tuner searched rectangles and visit lengths hold a square side
    only (N_I = B^2)."""
    if not os.path.exists(TUNED_TILES):
        return None
    with open(TUNED_TILES) as f:
        entry = json.load(f).get(name)
    if not entry:
        return None
    if "shapes" in entry:
        return {int(k): tuple(int(x) for x in v) for k, v in entry["shapes"].items()}
    return {int(k): (int(v), int(v), int(v) ** 2) for k, v in entry["tiles"].items()}


def _desc(L, shape, **kw):
    bx, by, ni = shape
    return dict(L=int(L), tile=int(bx), tile_rows=int(by) if by != bx else 0,
                steps_per_visit=int(ni), rate_model=METROPOLIS, **kw)


def batched_4096(n=4096, tiles=None, seed=4, shapes=None):
    """n replicas, L uniform in {16,24,32,48,64,128}, T ~ U[1.5, 3.5],
    h ~ U[-0.5, 0.5] from numpy default_rng(4); domain shape and N_I per L
    from `shapes` {L: (Bx, By, N_I)}, else square `tiles` {L: B} with
    N_I = B^2, else the autotuner's table, else DEFAULT_TILE; 5000 sweeps."""
    rng = np.random.default_rng(seed)
    Ls = rng.choice([16, 24, 32, 48, 64, 128], size=n)
    Ts = rng.uniform(1.5, 3.5, size=n)
    hs = rng.uniform(-0.5, 0.5, size=n)
    if shapes is None and tiles is not None:
        shapes = {L: (B, B, B * B) for L, B in tiles.items()}
    shapes = shapes or _tuned("batched_4096") or {L: (B, B, B * B)
                                                  for L, B in DEFAULT_TILE.items()}
    descs = [_desc(L, shapes[int(L)], J=1.0, h=float(h), T=float(T))
             for L, T, h in zip(Ls, Ts, hs)]
    return 4, descs, dict(sweeps=5000, record_every=100)


def differentiable_1024(n=1024, tile=None, seed=5, shape=None):
    """n replicas of 64x64, T=2.5, J=1, h ~ U[-0.2, 0.2] from default_rng(5),
    domain shape and N_I from `shape` (Bx, By, N_I), else a square `tile`
    with N_I = tile^2, else the autotuner's table, else 32 x 32 with
    N_I = 1024; 20000 sweeps, score on."""
    if shape is None and tile is not None:
        shape = (tile, tile, tile * tile)
    if shape is None:
        shape = (_tuned("differentiable_1024") or {64: (32, 32, 1024)})[64]
    rng = np.random.default_rng(seed)
    hs = rng.uniform(-0.2, 0.2, size=n)
    descs = [_desc(64, shape, J=1.0, h=float(h), T=2.5) for h in hs]
    return 5, descs, dict(sweeps=20_000, record_every=10)
