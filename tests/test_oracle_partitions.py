"""Pins of the oracle's general domain partitions (Sec. 2.2, Fig. 1:
checkerboards with even or odd domain counts, vertical stripes, a single
domain) and of the schedule over their colours (Eq. (schedule), Eq. (sum of
sequential tms)).

* The colouring must be proper: two domains that share an edge (some site of
  one is a 4-neighbour, periodically, of a site of the other) never share a
  colour.  Checked against the site adjacency itself, not the formula.
* The schedule index is uniform on [0, n!) and equals the Lemire definition
  recomputed from the Python Philox; ranks map to lexicographic orders.
* The oracle's state distribution after a few sweeps on every partition shape
  matches exact propagation over 2^N states, and Boltzmann starts stay
  Boltzmann-distributed (Eq. (general reversibility condition)).
"""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

from oracle import exact
from tests.test_oracle_dynamics import PMIN, chi2_pvalue, sample_states, start_state, state_index
from tests.test_oracle_rng import MASK, philox_py

SHAPES = [
    # L, Bx, By
    (8, 4, 4), (12, 4, 4), (12, 6, 12), (12, 3, 12), (12, 4, 12), (9, 3, 3),
    (10, 2, 5), (12, 12, 4), (6, 2, 3), (15, 5, 3), (8, 8, 8), (7, 7, 1),
]


def touching(L, doms):
    """Pairs of distinct domains with a 4-neighbour site pair (periodic)."""
    owner = np.empty(L * L, int)
    for q, d in enumerate(doms):
        owner[d] = q
    pairs = set()
    for i in range(L * L):
        y, x = divmod(i, L)
        for j in (((y + 1) % L) * L + x, y * L + (x + 1) % L):
            a, b = owner[i], owner[j]
            if a != b:
                pairs.add((min(a, b), max(a, b)))
    return pairs


@pytest.mark.parametrize("L,Bx,By", SHAPES)
def test_colouring_is_proper(oracle_lib, L, Bx, By):
    r = oracle_lib.Replica(L, Bx, tile_rows=By, T=2.0)
    col, n = r.partition()
    doms, ecols, en = exact.partition(L, Bx, By)
    assert n == en and list(col) == list(ecols)
    assert sorted(set(col)) == list(range(n))
    for a, b in touching(L, doms):
        assert col[a] != col[b], (a, b)
    nx, ny = L // Bx, L // By

    def axis_colours(m):
        return 1 if m == 1 else (3 if m % 2 else 2)

    assert n == axis_colours(nx) * axis_colours(ny)
    if nx % 2 == 0 and ny % 2 == 0:  # the 4-colour checkerboard
        assert list(col) == [2 * (q // nx % 2) + q % nx % 2 for q in range(nx * ny)]


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_perm_from_index_n_is_lexicographic(oracle_lib, n):
    for i, p in enumerate(itertools.permutations(range(n))):
        assert tuple(oracle_lib.perm_from_index_n(i, n)) == p


@pytest.mark.parametrize("n_perm", [1, 2, 6, 24, 120, 720])
def test_schedule_index_n_matches_definition(oracle_lib, n_perm):
    seed, rep = 0x0F1E_2D3C_4B5A_6978, 5
    thr = (1 << 32) % n_perm
    for w in range(150):
        expect = None
        for call in itertools.count():
            for word in philox_py([call, 2 << 24, w, rep], [seed & MASK, seed >> 32]):
                m = word * n_perm
                if (m & MASK) >= thr:
                    expect = m >> 32
                    break
            if expect is not None:
                break
        assert oracle_lib.schedule_index_n(seed, rep, w, n_perm) == expect
    if n_perm == 24:
        assert all(oracle_lib.schedule_index_n(seed, rep, w, 24) ==
                   oracle_lib.schedule_index(seed, rep, w) for w in range(50))


@pytest.mark.parametrize("n_perm", [2, 6, 120])
def test_schedule_index_n_uniform(oracle_lib, n_perm):
    counts = np.zeros(n_perm)
    for w in range(300 * n_perm):
        counts[oracle_lib.schedule_index_n(11, 2, w, n_perm)] += 1
    assert stats.chisquare(counts).pvalue > 1e-4


FINITE_TIME = [
    # L, Bx, By, N_I, T, J, h, model, palindrome, sweeps
    (4, 2, 4, 4, 2.5, 1.0, 0.1, 0, False, 1),   # two vertical stripes (wrap in y)
    (4, 2, 4, 3, 2.0, 1.0, 0.1, 0, True, 2),    # stripes, palindrome
    (3, 1, 3, 2, 2.0, 1.0, 0.1, 1, False, 2),   # three stripes: 3 colours, 3! orders
    (4, 4, 2, 3, 2.5, 1.0, -0.1, 0, False, 1),  # horizontal stripes (wrap in x)
    (4, 2, 1, 2, 2.2, 1.0, 0.2, 0, False, 1),   # 1 x 2 domains on a 2 x 4 grid
    (3, 1, 1, 1, 2.5, 1.0, 0.1, 0, True, 1),    # 3 x 3 grid of sites: 9 colours
]


@pytest.mark.parametrize("L,Bx,By,NI,T,J,h,model,pal,sweeps", FINITE_TIME)
def test_finite_time_distribution_general(oracle_lib, L, Bx, By, NI, T, J, h, model, pal,
                                          sweeps):
    start = start_state(L, seed=5)
    op = exact.SweepOperator(L, Bx, J, h, T, model, NI, palindrome=pal, By=By)
    p = np.zeros(1 << (L * L))
    p[state_index(start)] = 1.0
    for _ in range(sweeps):
        p = op.par(p)
    assert abs(p.sum() - 1) < 1e-12
    counts = sample_states(oracle_lib, L, Bx, 12000, sweeps, start, J=J, h=h, T=T,
                           steps_per_visit=NI, rate_model=model,
                           schedule=1 if pal else 0, tile_rows=By)
    assert chi2_pvalue(counts, p) > PMIN


@pytest.mark.parametrize("L,Bx,By,NI,model,pal", [
    (4, 2, 4, 4, 0, False), (3, 1, 3, 3, 1, False), (3, 1, 1, 1, 0, True),
    (4, 4, 2, 5, 0, False)])
def test_boltzmann_is_stationary_general(oracle_lib, L, Bx, By, NI, model, pal):
    J, h, T = 1.0, 0.1, 2.4
    pi, *_ = exact.boltzmann(L, J, h, T)
    rng = np.random.default_rng(77)
    starts = rng.choice(pi.size, size=12000, p=pi)
    counts = np.zeros(pi.size)
    for rep, i in enumerate(starts):
        spins = np.where((i >> np.arange(L * L)) & 1, 1, -1).astype(np.int8)
        r = oracle_lib.Replica(L, Bx, tile_rows=By, J=J, h=h, T=T, steps_per_visit=NI,
                               rate_model=model, schedule=1 if pal else 0,
                               init=oracle_lib.INIT_GIVEN, spins=spins, seed=12, replica=rep)
        r.run(2)
        counts[state_index(r.spins())] += 1
    assert chi2_pvalue(counts, pi) > PMIN


@pytest.mark.parametrize("L,Bx,By,pal", [(4, 2, 4, False), (3, 1, 3, False),
                                         (3, 1, 1, True), (4, 2, 1, False)])
def test_exact_parallel_kernel_is_reversible_general(L, Bx, By, pal):
    """pi T_PAR = pi and T_PAR D_pi symmetric for every partition shape;
    T_SEQ(Lambda) D_pi = (T_SEQ(reverse Lambda) D_pi)^T order by order."""
    J, h, T = 1.0, 0.15, 2.3
    pi, *_ = exact.boltzmann(L, J, h, T)
    op = exact.SweepOperator(L, Bx, J, h, T, 0, 2, palindrome=pal, By=By)
    assert len(op.orders()) == (1 if pal else math.factorial(op.ncol))
    assert np.abs(op.par(pi) - pi).max() < 1e-13
    rng = np.random.default_rng(3)
    a, b = rng.random(pi.size), rng.random(pi.size)
    assert abs(a @ op.par(pi * b) - b @ op.par(pi * a)) < 1e-12 * abs(a @ op.par(pi * b))
    for order in op.orders()[:4]:
        lhs = a @ op.seq(pi * b, order)
        rhs = b @ op.seq(pi * a, tuple(reversed(order)))
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_stripe_records_are_consistent(oracle_lib):
    """Records of a stripe partition: steps = N_I N_D per sweep, M and B
    recomputed from the lattice, the bookkeeping check mode clean."""
    r = oracle_lib.Replica(12, 3, tile_rows=12, T=2.4, h=0.1, seed=6, steps_per_visit=20)
    rec = r.run(6, 1, check=True)
    assert r.check_failures() == 0
    assert list(rec["steps"]) == [20 * 4 * (k + 1) for k in range(6)]
    s = r.spins().astype(np.int64)
    assert rec["M"][-1] == s.sum()
    assert rec["B"][-1] == (s * np.roll(s, -1, 1)).sum() + (s * np.roll(s, -1, 0)).sum()
