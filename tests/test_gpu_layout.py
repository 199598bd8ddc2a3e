"""The device lattice is held domain by domain, with a table of every
domain's edge columns (needs an MI355X).

* Start lattices (random, all up, given) read back row-major equal to the
  oracle's, for square, rectangular, striped, single-domain, odd-sided,
  resident-sized and ring shapes: the layout kernels and the random start
  map every site to its place.
* One context run through every execution form in turn ends bit-exact with
  the oracle: the edge table is rebuilt from the spins before each run of
  the staged visits, whatever form wrote the spins last (the multi-slot and
  resident kernels do not keep it).
"""
import numpy as np
import pytest

from paper_1403_4674_amd import kmc
from tests.gpu_helpers import assert_replica_equal, oracle_for, say

pytestmark = pytest.mark.gpu

SHAPES = [
    dict(L=32, tile=8),                 # square domains
    dict(L=24, tile=12, tile_rows=6),   # rectangles, 4 x 2 domains of 12 x 6
    dict(L=20, tile=5),                 # odd sides (byte staging)
    dict(L=18, tile=3, tile_rows=9),    # 3 x 9 domains, odd widths
    dict(L=16, tile=4, tile_rows=16),   # vertical stripes
    dict(L=16, tile=16, tile_rows=4),   # horizontal stripes
    dict(L=12, tile=12),                # one domain
    dict(L=128, tile=64),               # domains over 32 sites a side
    dict(L=96, tile=96),                # one resident-only domain
    dict(L=30, tile=5, dims=1),         # ring of 30 sites, domains of 5
]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU test on a host without a GPU"
    return torch


@pytest.mark.parametrize("init", ["random", "all_up", "given"])
def test_start_lattices_read_back(torch_cuda, oracle_lib, init):
    descs = [dict(d, T=2.3) for d in SHAPES]
    given = None
    if init == "all_up":
        descs = [dict(d, init=kmc.INIT_ALL_UP) for d in descs]
    elif init == "given":
        rng = np.random.default_rng(41)
        descs = [dict(d, init=kmc.INIT_GIVEN) for d in descs]
        given = [rng.choice(np.array([-1, 1], np.int8),
                            size=(d["L"],) if d.get("dims", 0) == 1 else (d["L"], d["L"]))
                 for d in descs]
    say(f"start lattices, {init}, {len(descs)} shapes")
    lat = kmc.Lattice(descs, 9, given_spins=given)
    for rho, d in enumerate(descs):
        o = oracle_for(oracle_lib, d, 9, rho, None if given is None else given[rho])
        g = lat.spins(rho)
        assert np.array_equal(g, o.spins()), (init, d)
        if given is not None:
            assert np.array_equal(g, given[rho]), (init, d)
    lat.close()


FORMS = [
    ("phase", 0, 2),
    ("resident", kmc.F_RESIDENT, 3),
    ("dataflow", kmc.F_FLOW, 2),
    ("persistent multi-slot", kmc.F_PERSISTENT | kmc.F_MULTI, 3),
    ("persistent wavefront", kmc.F_PERSISTENT | kmc.F_NO_MULTI, 2),
    ("dataflow", kmc.F_FLOW, 1),
    ("resident", kmc.F_RESIDENT, 1),
    ("phase", 0, 1),
]


def test_forms_in_turn_on_one_context(torch_cuda, oracle_lib):
    # shapes every form runs: square lattices up to 128 with at most 16
    # domains along x, the multi-slot ones with sides <= 16
    descs = [dict(L=32, tile=8, T=2.6, h=0.1),
             dict(L=24, tile=6, T=2.0, h=-0.2),
             dict(L=40, tile=10, tile_rows=8, T=2.269),
             dict(L=64, tile=16, T=3.2, h=0.05, schedule=kmc.SCHED_PALINDROME),
             dict(L=16, tile=4, tile_rows=16, T=1.8)]
    seed = 17
    lat = kmc.Lattice(descs, seed)
    total = 0
    for name, flags, n in FORMS:
        say(f"forms in turn: {name}, {n} sweeps")
        lat.run(n, 1, flags)
        total += n
    rec = lat.records()
    for rho, d in enumerate(descs):
        o = oracle_for(oracle_lib, d, seed, rho)
        orec = o.run(total, 1)
        assert_replica_equal(lat, rho, o, rec[rho], orec, f"forms in turn, replica {rho}")
    lat.close()
