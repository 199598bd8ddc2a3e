"""The resident form (KMC_F_RESIDENT: one workgroup keeps a whole replica in
LDS) on the GPU (needs an MI355X).

* Bit-exact against the oracle on every partition shape, including domains
  over 64 sites a side that only this form holds: the unpartitioned 100^2
  and 128^2 lattices, 100-high stripes, 128 x 64 halves.
* Bit-exact against the phase-by-phase form where both apply, on a mixed
  batch (one launch, a workgroup per replica sized for the largest).
* Score: fused bins equal the replayed ones bit for bit and the oracle's
  within the score tolerance.
* Flag and shape errors: KMC_EINVAL with other forms or L > 128,
  KMC_EUNSUPPORTED for big domains outside the resident form.
"""
import numpy as np
import pytest

from paper_1403_4674_amd import kmc
from tests.gpu_helpers import (assert_records_equal, assert_replica_equal, assert_score_close,
                               oracle_for, oracle_score, say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


SHAPES = {
    "checker16": dict(L=16, tile=8, T=2.4, h=0.1),
    "stripes12x3": dict(L=12, tile=3, tile_rows=12, T=2.4, rate_model=kmc.RATE_BARKER,
                        steps_per_visit=7),
    "odd15": dict(L=15, tile=5, T=2.2, schedule=kmc.SCHED_PALINDROME),
    "single12": dict(L=12, tile=12, T=2.4, rate_model=kmc.RATE_BARKER),
    "tile1": dict(L=8, tile=1, T=2.0, steps_per_visit=2),
    "rect": dict(L=24, tile=8, tile_rows=3, T=2.6, h=-0.2),
    "single100": dict(L=100, tile=100, T=2.4, rate_model=kmc.RATE_BARKER,
                      steps_per_visit=4000),
    "stripes100x50": dict(L=100, tile=50, tile_rows=100, T=2.4, rate_model=kmc.RATE_BARKER,
                          steps_per_visit=700),
    "stripes100x25": dict(L=100, tile=25, tile_rows=100, T=2.3, steps_per_visit=300),
    "single128": dict(L=128, tile=128, T=3.0, steps_per_visit=6000, h=0.05),
    "halves128": dict(L=128, tile=128, tile_rows=64, T=2.2, steps_per_visit=3000),
    "stripes99x33": dict(L=99, tile=33, tile_rows=99, T=2.5, steps_per_visit=900),  # 3 colours
}


@pytest.mark.parametrize("case", list(SHAPES))
def test_resident_matches_oracle(torch_cuda, oracle_lib, case):
    d = SHAPES[case]
    say(f"resident {case}")
    lat = kmc.Lattice([d], 31)
    lat.run(6, 2, kmc.F_RESIDENT)
    lat.run(3, 3, kmc.F_RESIDENT)  # a second call starts from the stored lattice
    o = oracle_for(oracle_lib, d, 31, 0)
    orec = np.concatenate([o.run(6, 2), o.run(3, 3)])
    assert_replica_equal(lat, 0, o, lat.records()[0], orec, f"resident {case}")
    lat.close()


def test_resident_equals_phase_form_on_a_mixed_batch(torch_cuda, oracle_lib):
    small = [d for k, d in SHAPES.items() if d["L"] <= 64 and d.get("tile", 0) <= 64]
    descs = small + [dict(L=32, tile=16, T=2.0 + 0.1 * i, h=0.02 * i) for i in range(6)]
    say("resident vs phased, mixed batch")
    a = kmc.Lattice(descs, 44)
    b = kmc.Lattice(descs, 44)
    a.run(5, 1, kmc.F_RESIDENT)
    b.run(5, 1, 0)
    ra, rb = a.records(), b.records()
    for rho in range(len(descs)):
        assert_records_equal(ra[rho], rb[rho], f"replica {rho}")
        assert np.array_equal(a.spins(rho), b.spins(rho))
    o = oracle_for(oracle_lib, descs[-1], 44, len(descs) - 1)
    assert_records_equal(ra[-1], o.run(5, 1), "oracle")


def test_resident_score_fused_equals_replay_and_oracle(torch_cuda, oracle_lib):
    descs = [SHAPES["stripes12x3"], SHAPES["checker16"],
             dict(L=100, tile=50, tile_rows=100, T=2.4, steps_per_visit=500)]
    sweeps, every = 8, 4
    say("resident score")
    f = kmc.Lattice(descs, 13)
    f.run(sweeps, every, kmc.F_RESIDENT | kmc.F_SCORE)
    fused = f.score(sweeps // every)
    r = kmc.Lattice(descs, 13)
    r.run(sweeps, every, kmc.F_RESIDENT | kmc.F_CHECKPOINT)
    replay = r.score(sweeps // every)
    assert np.array_equal(fused, replay)
    for rho, d in enumerate(descs):
        _, _, sc, mag = oracle_score(oracle_lib, d, 13, rho, sweeps, every)
        assert_score_close(fused[rho], sc, mag, f"replica {rho}")


def test_resident_flag_and_shape_errors(torch_cuda):
    lat = kmc.Lattice([SHAPES["checker16"]], 1)
    for bad in (kmc.F_PERSISTENT, kmc.F_FLOW, kmc.F_GRAPH):
        with pytest.raises(kmc.KmcError) as e:
            lat.run(1, 1, kmc.F_RESIDENT | bad)
        assert e.value.status == kmc.KMC_EINVAL
    lat.close()
    big = kmc.Lattice([SHAPES["stripes100x50"]], 1)
    for form in (0, kmc.F_FLOW, kmc.F_PERSISTENT):
        with pytest.raises(kmc.KmcError) as e:
            big.run(1, 1, form)
        assert e.value.status == kmc.KMC_EUNSUPPORTED
    assert big.records().shape == (1, 0)  # nothing ran
    big.close()
    wide = kmc.Lattice([dict(L=256, tile=16, T=2.0)], 1)  # 16 domains along x but L > 128
    with pytest.raises(kmc.KmcError) as e:
        wide.run(1, 1, kmc.F_RESIDENT)
    assert e.value.status == kmc.KMC_EINVAL
    wide.close()
