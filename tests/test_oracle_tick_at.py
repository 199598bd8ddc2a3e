"""The oracle's one-tick value at sampled states (oracle/exact.py tick_at),
which checks the GPU's exact propagation on systems too large for the
whole-vector tools.

* Equal to TickKernel.apply (square lattices, any domain, both rate models,
  quantised or not) and RingTickKernel.apply at every state, including the
  side-2 lattices whose two neighbours along an axis are one site.
* Conserves probability (Eq. (Glauber_TM) is stochastic) and keeps the
  Boltzmann distribution stationary at every state (each flip obeys
  detailed balance, Eq. (equilibrium distribution)), pins that do not go
  through the whole-vector tools.
"""
import numpy as np
import pytest

from oracle import exact

SQUARE = [(2, [0, 3], 0, False), (3, list(range(9)), 1, True), (4, [2, 3, 6, 7], 0, True),
          (4, list(range(16)), 1, False), (4, [5], 0, False)]


@pytest.mark.parametrize("L,sites,model,quantise", SQUARE)
def test_tick_at_equals_the_whole_vector_tick(L, sites, model, quantise):
    J, h, T = 1.0, 0.15, 2.3
    rng = np.random.default_rng(L * 31 + len(sites))
    p = rng.random(1 << (L * L))
    p /= p.sum()
    ref = exact.TickKernel(L, sites, J, h, T, model, quantise).apply(p)
    got = exact.tick_at(p, np.arange(p.size), sites, exact.square_neighbours(L), J, h, T,
                        model, quantise)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=0)


@pytest.mark.parametrize("N,sites", [(2, [0]), (8, list(range(8))), (10, [4, 5, 6, 7, 8])])
def test_tick_at_equals_the_whole_vector_ring_tick(N, sites):
    J, h, T = 1.0, -0.2, 2.0
    rng = np.random.default_rng(N)
    p = rng.random(1 << N)
    p /= p.sum()
    ref = exact.RingTickKernel(N, sites, J, h, T, 1, True).apply(p)
    got = exact.tick_at(p, np.arange(p.size), sites, exact.ring_neighbours(N), J, h, T, 1, True)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=0)


@pytest.mark.parametrize("model", [0, 1])
def test_tick_at_conserves_probability_and_keeps_boltzmann(model):
    L, J, h, T = 4, 1.0, 0.1, 2.5
    sites = [0, 1, 4, 5, 10]
    rng = np.random.default_rng(5)
    p = rng.random(1 << 16)
    p /= p.sum()
    allst = np.arange(p.size)
    nb = exact.square_neighbours(L)
    assert abs(exact.tick_at(p, allst, sites, nb, J, h, T, model).sum() - 1.0) < 1e-13
    pi = exact.boltzmann(L, J, h, T)[0]
    np.testing.assert_allclose(exact.tick_at(pi, allst, sites, nb, J, h, T, model), pi,
                               rtol=1e-12, atol=0)
    # a wrong neighbour breaks both detailed balance and stationarity
    bad = lambda i: nb(i)[:3] + [i ^ 1]
    assert np.abs(exact.tick_at(pi, allst, sites, bad, J, h, T, model) - pi).max() > 1e-6
