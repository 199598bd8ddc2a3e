"""The paper's 1D system on the GPU: the periodic ring (Sec. 3.1,
Eq. (1D partitions), Table 1), through the C-ABI (needs an MI355X).

* The 1 x 8 ring at 1/(beta J) = 2 with Barker rates, started from the
  paper's eight initial conditions (two adjacent up spins), for
  N_D in {1, 2, 4, 8} and N_I in {1, 2, 5, 10}: lattices, per-domain event
  counts and clocks, and every record bit-exact against the oracle, in the
  phase, dataflow and persistent forms.
* Longer rings (random starts, Metropolis, a field, the palindrome, odd
  domain counts, 64-site domains) in all three forms.
* Exact propagation of the ring's distribution on the GPU
  (kmc_exact_sweeps) equals the numpy tool; the histogram of many GPU
  replicas after two sweeps matches it.
"""
import numpy as np
import pytest

from oracle import exact
from paper_1403_4674_amd import kmc
from tests.gpu_helpers import assert_replica_equal, oracle_for, say
from tests.test_oracle_dynamics import chi2_pvalue

pytestmark = pytest.mark.gpu

FORMS = {"phase": 0, "flow": kmc.F_FLOW, "persistent": kmc.F_PERSISTENT}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def paper_ics(N=8):
    out = []
    for i in range(N):
        s = -np.ones(N, np.int8)
        s[i] = s[(i + 1) % N] = 1
        out.append(s)
    return out


def compare(kmco, descs, seed, sweeps, every, flags, given=None, what=""):
    lat = kmc.Lattice(descs, seed, given_spins=given)
    lat.run(sweeps, every, flags)
    g = lat.records()
    for rho, d in enumerate(descs):
        o = oracle_for(kmco, d, seed, rho, None if given is None else given[rho])
        orec = o.run(sweeps, every)
        assert_replica_equal(lat, rho, o, g[rho], orec, f"{what} replica {rho}")
    lat.close()


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("ND", [1, 2, 4, 8])
def test_paper_ring_bit_exact(torch_cuda, oracle_lib, ND, form):
    ics = paper_ics()
    for NI in (1, 2, 5, 10):
        descs = [dict(L=8, tile=8 // ND, T=2.0, rate_model=kmc.RATE_BARKER, steps_per_visit=NI,
                      init=kmc.INIT_GIVEN, dims=1) for _ in ics]
        sweeps = max(1, 800 // (ND * NI))
        say(f"ring 1x8 N_D={ND} N_I={NI}: {sweeps} sweeps, {form}")
        compare(oracle_lib, descs, 17, sweeps, 1, FORMS[form], ics, f"N_D={ND} N_I={NI}")


RINGS = [dict(L=256, tile=32, T=1.5, h=0.1, dims=1),
         dict(L=96, tile=32, T=2.5, dims=1, rate_model=kmc.RATE_BARKER),  # 3 domains, 3 colours
         dict(L=128, tile=64, T=1.2, h=-0.3, dims=1, schedule=kmc.SCHED_PALINDROME),
         dict(L=60, tile=60, T=2.0, dims=1, steps_per_visit=100),          # one periodic domain
         dict(L=30, tile=5, T=1.8, dims=1, steps_per_visit=7),             # 6 domains, bytes
         dict(L=9, tile=3, T=2.2, h=0.4, dims=1, rate_model=kmc.RATE_BARKER)]


@pytest.mark.parametrize("form", list(FORMS))
def test_rings_bit_exact(torch_cuda, oracle_lib, form):
    say(f"rings, {form}")
    compare(oracle_lib, RINGS, 5, 40, 4, FORMS[form], what=form)


def test_ring_rejects_the_resident_form(torch_cuda):
    lat = kmc.Lattice([RINGS[0]], 1)
    with pytest.raises(kmc.KmcError) as e:
        lat.run(1, 1, kmc.F_RESIDENT)
    assert e.value.status == kmc.KMC_EUNSUPPORTED
    lat.close()


@pytest.mark.parametrize("B,NI,pal", [(8, 3, False), (4, 2, False), (2, 5, True), (1, 1, False)])
def test_ring_exact_propagation(torch_cuda, B, NI, pal):
    import torch
    N = 8
    d = dict(L=N, tile=B, T=2.0, h=0.15, rate_model=kmc.RATE_BARKER, steps_per_visit=NI,
             dims=1, schedule=kmc.SCHED_PALINDROME if pal else kmc.SCHED_RANDOM_PERM)
    start = np.zeros(1 << N)
    start[0b00011000] = 1.0
    op = exact.RingSweepOperator(N, B, 1.0, 0.15, 2.0, 1, NI, quantise=True, palindrome=pal)
    ref = start.copy()
    for _ in range(3):
        ref = op.par(ref)
    p = torch.tensor(start, dtype=torch.float64, device="cuda")
    work = torch.empty(3 << N, dtype=torch.float64, device="cuda")
    say(f"ring exact propagation B={B} N_I={NI}")
    kmc.kmc_exact_sweeps(d, p, work, 3, quantised=True)
    torch.cuda.synchronize()
    np.testing.assert_allclose(p.cpu().numpy(), ref, rtol=0, atol=1e-14)


def test_ring_histogram_matches_exact(torch_cuda):
    N, B, NI = 8, 2, 3
    n_rep = 100000
    d = dict(L=N, tile=B, T=2.0, rate_model=kmc.RATE_BARKER, steps_per_visit=NI, dims=1,
             init=kmc.INIT_GIVEN)
    start = paper_ics()[2]
    say(f"ring histogram, {n_rep} replicas")
    lat = kmc.Lattice([d] * n_rep, 3, given_spins=[start] * n_rep)
    lat.run(2, 2, kmc.F_PERSISTENT)
    counts = np.zeros(1 << N)
    for rho in range(0, n_rep):
        s = lat.spins(rho)
        counts[int(((s > 0).astype(np.int64) << np.arange(N)).sum())] += 1
    lat.close()
    p = np.zeros(1 << N)
    p[int(((start > 0).astype(np.int64) << np.arange(N)).sum())] = 1.0
    op = exact.RingSweepOperator(N, B, 1.0, 0.0, 2.0, 1, NI, quantise=True)
    for _ in range(2):
        p = op.par(p)
    assert chi2_pvalue(counts, p) > 1e-4
