"""Degenerate and boundary cases of the method on the GPU (needs an MI355X).

Each case runs through the C-ABI in the phase-by-phase form and in the
persistent forms (multi-slot where the domains allow it, and forced
one-domain-per-wavefront), and must match the oracle bit for bit:

* rates that round to 0 (T -> 0: uphill flips never happen) and rates at or
  next to 2^32 (T -> infinity: hardly any null ticks), Barker's w = 1/2;
* J = 0 (independent spins in a field), J < 0 (antiferromagnet), a field
  that dominates the coupling;
* N_I = 1 (one tick per visit) and N_I far above the domain size and not a
  multiple of the 64-tick batch;
* the smallest checkerboard (2 x 2 domains of 4 x 4), 32 x 32 and 64 x 64
  domains (rows that fill a 32-bit or a 64-bit mask, so the last column is
  a neighbour of the next to last), and a 12 x 12 domain (the slot draw
  rejects 2^32 mod 144);
* calls with no sweeps and calls with no record point.
"""
import numpy as np
import pytest

from paper_1403_4674_amd import kmc
from tests.gpu_helpers import assert_records_equal, assert_replica_equal, oracle_for, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU test on a host without a GPU"
    return torch


CASES = {
    "frozen": dict(L=32, tile=8, T=0.05, h=0.0),
    "hot": dict(L=32, tile=8, T=1.0e6, h=0.0),
    "barker_hot": dict(L=24, tile=12, T=1.0e6, rate_model=kmc.RATE_BARKER),
    "free_spins": dict(L=16, tile=8, J=0.0, h=0.3, T=1.0),
    "antiferro": dict(L=32, tile=16, J=-1.0, h=0.0, T=1.5),
    "strong_field": dict(L=32, tile=8, J=1.0, h=5.0, T=2.0),
    "one_tick": dict(L=32, tile=8, T=2.3, steps_per_visit=1),
    "long_visit": dict(L=16, tile=8, T=2.3, steps_per_visit=1000),
    "smallest": dict(L=8, tile=4, T=2.0),
    "tile64": dict(L=128, tile=64, T=2.6, h=-0.05),
    "tile32": dict(L=64, tile=32, T=2.4, h=0.05),
    "odd_domain": dict(L=48, tile=12, T=2.2, h=0.1),
}
FORMS = {"phased": 0,
         "persistent_multi": kmc.F_PERSISTENT | kmc.F_MULTI,
         "persistent_wave": kmc.F_PERSISTENT | kmc.F_NO_MULTI}


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("case", list(CASES))
def test_degenerate_case_matches_oracle(torch_cuda, oracle_lib, case, form):
    d = CASES[case]
    sweeps, every = 12, 4
    say(f"edge case {case}, {form}")
    lat = kmc.Lattice([d], 21)
    lat.run(sweeps, every, FORMS[form])
    rec = lat.records()
    o = oracle_for(oracle_lib, d, 21, 0)
    orec = o.run(sweeps, every)
    assert_replica_equal(lat, 0, o, rec[0], orec, f"{case} {form}")
    if case == "frozen":
        # from a random start at T -> 0 only downhill and level flips occur
        e = -rec[0]["B"]
        assert (np.diff(e) <= 0).all()
    if case == "hot":
        assert rec[0]["events"][-1] > 0.99 * rec[0]["steps"][-1]
    lat.close()


def test_calls_without_sweeps_or_record_points(torch_cuda, oracle_lib):
    d = dict(L=16, tile=8, T=2.4, h=0.2)
    say("zero sweeps / no record point")
    lat = kmc.Lattice([d], 5)
    o = oracle_for(oracle_lib, d, 5, 0)
    lat.run(0, 1)
    assert lat.records().shape == (1, 0)
    lat.run(3, 5)  # no record inside this call
    assert len(o.run(3, 5)) == 0
    assert lat.records().shape == (1, 0)
    lat.run(10, 4, kmc.F_PERSISTENT)  # records after sweeps 7 and 11
    orec = o.run(10, 4)
    rec = lat.records()
    assert list(rec[0]["sweep"]) == [7, 11]
    assert_records_equal(rec[0], orec, "sparse records")
    assert np.array_equal(lat.spins(0), o.spins())


SHAPES = {
    "tile1": dict(L=8, tile=1, T=2.2),                      # one site per domain
    "tile2": dict(L=8, tile=2, T=2.4, h=0.1),
    "tile3": dict(L=12, tile=3, T=2.0),
    "tile5": dict(L=20, tile=5, T=2.6, rate_model=kmc.RATE_BARKER),
    "tile6": dict(L=12, tile=6, T=2.4, rate_model=kmc.RATE_BARKER),   # the paper's 12^2, N_D = 4
    "tile25": dict(L=100, tile=25, T=2.4, rate_model=kmc.RATE_BARKER, steps_per_visit=300),
    "tile50": dict(L=100, tile=50, T=2.4, rate_model=kmc.RATE_BARKER, steps_per_visit=900),
    "tile36_palin": dict(L=72, tile=36, T=2.3, schedule=kmc.SCHED_PALINDROME, steps_per_visit=500),
    "single3": dict(L=3, tile=3, T=2.0),                    # N_D = 1: periodic in itself
    "single12": dict(L=12, tile=12, T=2.4, rate_model=kmc.RATE_BARKER),
    "single16_palin": dict(L=16, tile=16, T=2.1, h=0.2, schedule=kmc.SCHED_PALINDROME),
    "single40": dict(L=40, tile=40, T=2.5, steps_per_visit=700),   # 64-bit rows
    # general partitions: vertical stripes (wrap in y), odd domain counts
    # (3 colours per axis), rectangles, horizontal stripes (wrap in x)
    "stripes2": dict(L=12, tile=6, tile_rows=12, T=2.4, rate_model=kmc.RATE_BARKER),
    "stripes4": dict(L=12, tile=3, tile_rows=12, T=2.4, rate_model=kmc.RATE_BARKER,
                     steps_per_visit=10),
    "stripes5_palin": dict(L=20, tile=4, tile_rows=20, T=2.2, h=0.1,
                           schedule=kmc.SCHED_PALINDROME),
    "odd3x3": dict(L=12, tile=4, T=2.3),                 # 9 colours
    "odd3x3_palin": dict(L=15, tile=5, T=2.0, schedule=kmc.SCHED_PALINDROME),
    "rect8x4": dict(L=16, tile=8, tile_rows=4, T=2.5, h=-0.1),
    "rect3x5": dict(L=15, tile=3, tile_rows=5, T=2.6, steps_per_visit=40),
    "hstripes": dict(L=12, tile=12, tile_rows=6, T=2.4),
    "tall48": dict(L=48, tile=16, tile_rows=48, T=2.3, steps_per_visit=500),  # 48 rows
    "wide64x8": dict(L=64, tile=64, tile_rows=8, T=2.7, steps_per_visit=600),
}


@pytest.mark.parametrize("form", ["phased", "flow", "persistent"])
@pytest.mark.parametrize("case", list(SHAPES))
def test_domain_shapes_match_oracle(torch_cuda, oracle_lib, case, form):
    """Domain sides that are not multiples of 4 (byte-wise staging), the
    unpartitioned lattice as one periodic domain, stripes, odd domain counts
    and rectangular domains, in every execution form."""
    d = SHAPES[case]
    flags = {"phased": 0, "flow": kmc.F_FLOW, "persistent": kmc.F_PERSISTENT | kmc.F_MULTI}[form]
    say(f"shape {case}, {form}")
    lat = kmc.Lattice([d], 13)
    lat.run(10, 5, flags)
    o = oracle_for(oracle_lib, d, 13, 0)
    orec = o.run(10, 5)
    assert_replica_equal(lat, 0, o, lat.records()[0], orec, f"{case} {form}")
    lat.close()


def test_mixed_shapes_in_one_batch(torch_cuda, oracle_lib):
    descs = list(SHAPES.values())
    say("all shapes in one persistent batch")
    lat = kmc.Lattice(descs, 29)
    lat.run(6, 3, kmc.F_PERSISTENT)
    rec = lat.records()
    for rho, d in enumerate(descs):
        o = oracle_for(oracle_lib, d, 29, rho)
        assert_replica_equal(lat, rho, o, rec[rho], o.run(6, 3), f"batch {rho}")
