"""The rejection-free variant with fixed time slices on the GPU (needs an
MI355X), through the C-ABI.

* Bit-exact against the oracle (lattices, per-domain event counts, every
  record; the clocks, exactly tau per visit) on checkerboards, stripes, one
  periodic domain, the ring, the palindrome, Barker rates and a field, in
  the phase, dataflow and persistent forms, and on the 1024^2 workload shape.
  Every stop decision compares FP64 times, so parity holds only because both
  sides evaluate the same logarithm in the same IEEE operations.
* The histogram of 100000 GPU replicas of the 4 x 4 torus after two sweeps
  matches exact propagation with exp(Q_d tau) per domain visit.
* Refusals: contexts mixing time slices and ticks, the score, checkpoints,
  the resident form, and exact propagation of a time-slice descriptor.
"""
import numpy as np
import pytest

from oracle import exact
from paper_1403_4674_amd import kmc, workloads
from tests.gpu_helpers import assert_replica_equal, oracle_for, say
from tests.test_oracle_dynamics import chi2_pvalue, state_index

pytestmark = pytest.mark.gpu

FORMS = {"phase": 0, "flow": kmc.F_FLOW, "persistent": kmc.F_PERSISTENT}

SLICES = [dict(L=32, tile=8, T=2.3, h=0.1, time_slice=1.0),
          dict(L=16, tile=8, T=1.6, time_slice=0.5, rate_model=kmc.RATE_BARKER),
          dict(L=24, tile=12, T=3.0, h=-0.2, time_slice=2.0, schedule=kmc.SCHED_PALINDROME),
          dict(L=20, tile=4, tile_rows=20, T=2.0, time_slice=0.7),      # stripes
          dict(L=12, tile=12, T=2.4, time_slice=3.0),                    # one periodic domain
          dict(L=128, tile=64, T=2.269, time_slice=0.25),               # 64-bit row masks
          dict(L=64, tile=32, T=1.2, h=0.3, time_slice=1.5),
          dict(L=15, tile=5, T=2.6, time_slice=0.9)]                     # odd: 9 colours


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def compare(kmco, descs, seed, sweeps, every, flags, what):
    lat = kmc.Lattice(descs, seed)
    lat.run(sweeps, every, flags)
    g = lat.records()
    for rho, d in enumerate(descs):
        o = oracle_for(kmco, d, seed, rho)
        orec = o.run(sweeps, every)
        assert (orec["steps"] == 0).all()
        assert_replica_equal(lat, rho, o, g[rho], orec, f"{what} replica {rho}")
    lat.close()


@pytest.mark.parametrize("form", list(FORMS))
def test_slices_bit_exact(torch_cuda, oracle_lib, form):
    say(f"time slices, {len(SLICES)} replicas, {form}")
    compare(oracle_lib, SLICES, 29, 24, 4, FORMS[form], form)


@pytest.mark.parametrize("form", list(FORMS))
def test_ring_slices_bit_exact(torch_cuda, oracle_lib, form):
    descs = [dict(L=64, tile=8, T=2.0, time_slice=1.0, dims=1, rate_model=kmc.RATE_BARKER),
             dict(L=8, tile=8, T=2.0, time_slice=2.5, dims=1),
             dict(L=30, tile=10, T=1.5, h=0.2, time_slice=0.6, dims=1)]
    say(f"ring time slices, {form}")
    compare(oracle_lib, descs, 3, 40, 5, FORMS[form], f"ring {form}")


def test_slices_on_the_1024_shape(torch_cuda, oracle_lib):
    seed, descs, _ = workloads.single_1024(2.269)
    d = dict(descs[0], time_slice=1.0, steps_per_visit=0)
    say("1024^2 time slices, 3 sweeps, dataflow form")
    compare(oracle_lib, [d], seed, 3, 1, kmc.F_FLOW, "1024 slices")


def test_slice_histogram_matches_exact(torch_cuda):
    L, B, tau, n_rep = 4, 2, 0.5, 100000
    rng = np.random.default_rng(6)
    start = np.where(rng.random((L, L)) < 0.5, 1, -1).astype(np.int8)
    d = dict(L=L, tile=B, T=2.3, h=0.1, time_slice=tau, init=kmc.INIT_GIVEN)
    say(f"time-slice histogram, {n_rep} replicas of 4x4")
    lat = kmc.Lattice([d] * n_rep, 8, given_spins=[start] * n_rep)
    lat.run(2, 2, kmc.F_PERSISTENT)
    counts = np.zeros(1 << 16)
    for rho in range(n_rep):
        counts[state_index(lat.spins(rho))] += 1
    lat.close()
    op = exact.SliceSweepOperator(L, B, 1.0, 0.1, 2.3, 0, tau)
    p = np.zeros(1 << 16)
    p[state_index(start)] = 1.0
    for _ in range(2):
        p = op.par(p)
    assert chi2_pvalue(counts, np.maximum(p, 0.0)) > 1e-4


def test_slice_refusals(torch_cuda):
    with pytest.raises(kmc.KmcError) as e:
        kmc.Lattice([SLICES[0], dict(L=16, tile=8, T=2.0)], 1)
    assert e.value.status == kmc.KMC_EINVAL
    lat = kmc.Lattice([SLICES[1]], 1)
    for flags in (kmc.F_SCORE, kmc.F_CHECKPOINT, kmc.F_RESIDENT):
        with pytest.raises(kmc.KmcError) as e:
            lat.run(1, 1, flags)
        assert e.value.status == kmc.KMC_EUNSUPPORTED
    with pytest.raises(kmc.KmcError) as e:
        lat.score(1)
    assert e.value.status == kmc.KMC_ESTATE
    lat.close()
    import torch
    p = torch.zeros(1 << 16, dtype=torch.float64, device="cuda")
    w = torch.zeros(3 << 16, dtype=torch.float64, device="cuda")
    with pytest.raises(kmc.KmcError) as e:
        kmc.kmc_exact_sweeps(dict(L=4, tile=2, T=2.0, time_slice=0.5), p, w, 1)
    assert e.value.status == kmc.KMC_EUNSUPPORTED
