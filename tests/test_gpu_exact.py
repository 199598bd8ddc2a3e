"""Exact propagation of state distributions on the GPU (kmc_exact_sweeps;
needs an MI355X).

* Equal to the oracle's exact tool (oracle/exact.py, numpy over 2^N states)
  after a few sweeps on every partition shape, schedule and rate model, with
  and without the Q32 rate quantisation.
* At 5 x 5 (2^25 states, beyond what the numpy tool reaches in seconds):
  probability is conserved and the Boltzmann distribution is stationary
  (Eq. (general reversibility condition)) for the unpartitioned lattice, for
  the 25 one-site domains (9 colours, palindrome) and for five horizontal
  stripes (3 colours mixed over their 6 orders).
* The kMC path at scale against it: the joint (M, B) histogram of 200 000
  replicas of a 4 x 4 lattice run by the batched persistent kernel after two
  sweeps from the all-up start matches the exact (quantised) distribution
  (chi-square).
* Large systems, where a tick runs as two passes over tiles in LDS (one over
  runs of 2^(28 - N) consecutive states, one over 2^14 consecutive states):
  rings of 20 and 22 sites (one domain; two domains and two colour orders),
  of 13 and 14 (one tile, one pass) and of 15 (three domains, six orders,
  two tiles of the strided pass) equal to the numpy tool over the whole
  vector; one tick of the 5 x 5 lattice (2^25 states) and of the 24-
  and 26-site rings (2^26, the largest system) equal to the oracle's value
  at 4096 sampled states and their flip partners.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import exact
from paper_1403_4674_amd import kmc
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def gpu_exact(torch, desc, p0, sweeps, quantised):
    n = p0.size
    p = torch.tensor(p0, dtype=torch.float64, device="cuda")
    work = torch.empty(3 * n, dtype=torch.float64, device="cuda")
    kmc.kmc_exact_sweeps(desc, p, work, sweeps, quantised=quantised)
    torch.cuda.synchronize()
    return p.cpu().numpy()


SYSTEMS = [
    # desc, sweeps
    (dict(L=4, tile=2, T=2.5, h=0.1, steps_per_visit=4), 2),
    (dict(L=4, tile=2, tile_rows=4, T=2.0, h=-0.2, steps_per_visit=3,
          rate_model=kmc.RATE_BARKER), 2),
    (dict(L=4, tile=2, T=2.3, steps_per_visit=2, schedule=kmc.SCHED_PALINDROME), 2),
    (dict(L=3, tile=3, T=2.0, h=0.1, steps_per_visit=9), 3),
    (dict(L=3, tile=1, tile_rows=3, T=2.4, steps_per_visit=2,
          rate_model=kmc.RATE_BARKER), 2),
    (dict(L=4, tile=1, T=3.0, h=0.2, steps_per_visit=1), 2),
    (dict(L=4, tile=4, tile_rows=2, T=2.2, steps_per_visit=5), 1),
    (dict(L=3, tile=1, T=2.5, steps_per_visit=1, schedule=kmc.SCHED_PALINDROME), 1),
]


@pytest.mark.parametrize("quantised", [True, False])
@pytest.mark.parametrize("k", range(len(SYSTEMS)))
def test_exact_equals_the_oracle_tool(torch_cuda, k, quantised):
    d, sweeps = SYSTEMS[k]
    say(f"exact propagation {d} quantised={quantised}")
    L = d["L"]
    rng = np.random.default_rng(k)
    p0 = rng.random(1 << (L * L))
    p0 /= p0.sum()
    op = exact.SweepOperator(L, d["tile"], d.get("J", 1.0), d.get("h", 0.0), d["T"],
                             d.get("rate_model", 0), d["steps_per_visit"], quantise=quantised,
                             palindrome=d.get("schedule", 0) == 1, By=d.get("tile_rows"))
    ref = p0
    for _ in range(sweeps):
        ref = op.par(ref)
    got = gpu_exact(torch_cuda, d, p0, sweeps, quantised)
    assert np.abs(got - ref).max() < 1e-14
    assert abs(got.sum() - 1.0) < 1e-13


def boltzmann_gpu(torch, L, J, h, T):
    """pi over the 2^(L L) states, computed with torch on the device."""
    N = L * L
    s = torch.arange(1 << N, device="cuda", dtype=torch.int64)
    spin = lambda i: ((s >> i) & 1).to(torch.float64) * 2 - 1
    M = torch.zeros(1 << N, dtype=torch.float64, device="cuda")
    B = torch.zeros_like(M)
    for y in range(L):
        for x in range(L):
            a = spin(y * L + x)
            M += a
            B += a * spin(y * L + (x + 1) % L) + a * spin(((y + 1) % L) * L + x)
    lw = (J * B + h * M) / T
    w = torch.exp(lw - lw.max())
    return w / w.sum()


@pytest.mark.parametrize("d", [
    dict(L=5, tile=5, T=2.3, h=0.1, steps_per_visit=25),
    dict(L=5, tile=1, T=2.6, h=-0.05, steps_per_visit=1, schedule=kmc.SCHED_PALINDROME,
         rate_model=kmc.RATE_BARKER),
    # five horizontal stripes, three colours mixed over their six orders;
    # the stripes below site 14 tick in one pass, the others in two
    dict(L=5, tile=5, tile_rows=1, T=2.4, h=0.05, steps_per_visit=3),
])
def test_boltzmann_is_stationary_at_5x5(torch_cuda, d):
    torch = torch_cuda
    say(f"exact 5x5 stationarity {d}")
    pi = boltzmann_gpu(torch, 5, d.get("J", 1.0), d["h"], d["T"])
    p = pi.clone()
    work = torch.empty(3 * p.numel(), dtype=torch.float64, device="cuda")
    kmc.kmc_exact_sweeps(d, p, work, 1, quantised=False)
    torch.cuda.synchronize()
    assert abs(float(p.sum()) - 1.0) < 1e-12
    assert float((p - pi).abs().max()) < 1e-12 * float(pi.max())
    # a start far from equilibrium moves towards it
    q = torch.zeros_like(pi)
    q[-1] = 1.0  # all up
    kmc.kmc_exact_sweeps(d, q, work, 3, quantised=False)
    torch.cuda.synchronize()
    assert abs(float(q.sum()) - 1.0) < 1e-12 and float(q.min()) >= 0.0


def test_kmc_histogram_matches_exact_distribution(torch_cuda):
    torch = torch_cuda
    d = dict(L=4, tile=2, T=2.5, h=0.1, steps_per_visit=4, init=kmc.INIT_ALL_UP)
    n_rep, sweeps = 200_000, 2
    say("200000 replicas of 4x4 against the exact distribution")
    lat = kmc.Lattice([d] * n_rep, 2024)
    lat.run(sweeps, sweeps, kmc.F_PERSISTENT)
    rec = lat.records()[:, -1]
    lat.close()
    p0 = np.zeros(1 << 16)
    p0[-1] = 1.0
    p = gpu_exact(torch, d, p0, sweeps, quantised=True)
    M, B = exact.magnetisation_and_bonds(4)
    keys = (M + 16) * 100 + (B + 32)
    uniq, inv = np.unique(keys, return_inverse=True)
    prob = np.bincount(inv, weights=p, minlength=uniq.size)
    obs_keys = (rec["M"] + 16) * 100 + (rec["B"] + 32)
    pos = np.searchsorted(uniq, obs_keys)
    assert np.array_equal(uniq[pos], obs_keys)  # every observed (M, B) is possible
    counts = np.bincount(pos, minlength=uniq.size).astype(float)
    exp_ = prob * n_rep
    big = exp_ >= 5
    obs = np.append(counts[big], counts[~big].sum())
    ex = np.append(exp_[big], exp_[~big].sum())
    assert stats.chisquare(obs, ex * obs.sum() / ex.sum()).pvalue > 1e-5


@pytest.mark.parametrize("N,B,NI", [(13, 13, 2), (14, 7, 1), (15, 5, 1), (20, 20, 2),
                                      (22, 11, 2)])
def test_two_pass_ticks_equal_the_ring_tool(torch_cuda, N, B, NI):
    d = dict(L=N, tile=B, T=2.0, h=0.15, rate_model=kmc.RATE_BARKER, steps_per_visit=NI,
             dims=1)
    rng = np.random.default_rng(N)
    p0 = rng.random(1 << N)
    p0 /= p0.sum()
    op = exact.RingSweepOperator(N, B, 1.0, 0.15, 2.0, 1, NI, quantise=True)
    ref = op.par(p0)
    say(f"exact propagation, ring of {N}, domains of {B}, N_I={NI}")
    got = gpu_exact(torch_cuda, d, p0, 1, quantised=True)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=0)


@pytest.mark.parametrize("system", ["square 5x5", "ring 24", "ring 26"])
def test_one_tick_of_the_largest_systems_at_sampled_states(torch_cuda, system):
    if system == "square 5x5":
        N, d = 25, dict(L=5, tile=5, T=2.3, h=0.1, steps_per_visit=1)
        nb = exact.square_neighbours(5)
        J, h, T, model = 1.0, 0.1, 2.3, 0
    else:
        N = int(system.split()[1])
        d = dict(L=N, tile=N, T=2.0, h=-0.1, steps_per_visit=1, dims=1,
                 rate_model=kmc.RATE_BARKER)
        nb = exact.ring_neighbours(N)
        J, h, T, model = 1.0, -0.1, 2.0, 1
    rng = np.random.default_rng(N)
    p0 = rng.random(1 << N)
    p0 /= p0.sum()
    say(f"one exact tick of the {system} lattice, 2^{N} states")
    got = gpu_exact(torch_cuda, d, p0, 1, quantised=False)
    s = rng.integers(0, 1 << N, 4096)
    s = np.concatenate([s, s ^ (1 << rng.integers(0, N, s.size)), [0, (1 << N) - 1]])
    ref = exact.tick_at(p0, s, list(range(N)), nb, J, h, T, model)
    np.testing.assert_allclose(got[s], ref, rtol=1e-12, atol=0)
    assert abs(got.sum() - 1.0) < 1e-12
