"""Pins of the oracle's counter-based generator, schedule draw and slot draw.

Philox4x32-10 follows Salmon et al., SC'11.  The oracle's C generator is
checked against the published known-answer vectors and against a second
implementation written here in plain Python.
"""
import itertools
import os

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))
MASK = 0xFFFFFFFF


def philox_py(ctr, key, rounds=10):
    """Philox4x32: S-box of two 32x32->64 products per round (Salmon et al.)."""
    c = list(ctr)
    k0, k1 = key
    for r in range(rounds):
        if r:
            k0 = (k0 + 0x9E3779B9) & MASK
            k1 = (k1 + 0xBB67AE85) & MASK
        p0 = 0xD2511F53 * c[0]
        p1 = 0xCD9E8D57 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & MASK, p1 & MASK,
             ((p0 >> 32) ^ c[3] ^ k1) & MASK, p0 & MASK]
    return c


def load_kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(oracle_lib):
    for ctr, key, out in load_kat():
        assert list(oracle_lib.philox(ctr, key)) == out
        assert philox_py(ctr, key) == out


def test_philox_matches_second_implementation(oracle_lib):
    rng = np.random.default_rng(11)
    for _ in range(500):
        ctr = [int(x) for x in rng.integers(0, 2**32, 4)]
        key = [int(x) for x in rng.integers(0, 2**32, 2)]
        assert list(oracle_lib.philox(ctr, key)) == philox_py(ctr, key)


def test_perm_from_index_is_lexicographic(oracle_lib):
    perms = list(itertools.permutations(range(4)))
    for i, p in enumerate(perms):
        assert tuple(oracle_lib.perm_from_index(i)) == p


def test_schedule_index_uniform(oracle_lib):
    counts = np.zeros(24)
    for w in range(24000):
        counts[oracle_lib.schedule_index(5, 0, w)] += 1
    assert stats.chisquare(counts).pvalue > 1e-4


def test_schedule_index_matches_definition(oracle_lib):
    # first accepted word of the schedule stream, Lemire rejection of low < 16
    seed, rep = 0x1234_5678_9ABC_DEF0, 3
    for w in range(200):
        expect = None
        for call in itertools.count():
            o = philox_py([call, 2 << 24, w, rep],
                          [seed & MASK, seed >> 32])
            for word in o:
                m = word * 24
                if (m & MASK) >= 16:
                    expect = m >> 32
                    break
            if expect is not None:
                break
        assert oracle_lib.schedule_index(seed, rep, w) == expect


@pytest.mark.parametrize("n", [64, 144, 576, 1024, 4096])
def test_tick_slot_uniform(oracle_lib, n):
    counts = np.zeros(n)
    draws = 40 * n
    for t in range(draws):
        s, _ = oracle_lib.tick_slot(9, 1, 7, t % 17, 0, t, n)
        counts[s] += 1
    assert stats.chisquare(counts).pvalue > 1e-4


def test_tick_slot_power_of_two_is_top_bits(oracle_lib):
    for t in range(300):
        o = philox_py([t, 5, 11, 2], [42, 0])
        s, r = oracle_lib.tick_slot(42, 2, 11, 5, 0, t, 1024)
        assert r == 0 and s == o[1] >> 22


def test_tick_slot_rejection_and_retry_streams(oracle_lib):
    # n = 2^31 + 1 rejects about half the first draws, exercising the retry
    # streams 3, 4, ...; the accepted slot must be uniform on [0, n).
    n = 2**31 + 1
    thr = (2**32) % n
    retries, low = [], 0
    for t in range(4000):
        s, r = oracle_lib.tick_slot(3, 0, 1, 2, 1, t, n)
        retries.append(r)
        low += s < n // 2
        # recompute the rule independently
        c1 = 2 | (1 << 20)
        word = philox_py([t, c1, 1, 0], [3, 0])[1]
        k = 0
        while (word * n) & MASK < thr and k < 12:
            k += 1
            word = philox_py([t, c1 | ((3 + k - 1) << 24), 1, 0], [3, 0])[1]
        assert (r, s) == (k, (word * n) >> 32)
    retries = np.array(retries)
    assert 0.45 < (retries > 0).mean() < 0.55
    assert abs(low / 4000 - 0.5) < 0.03


def init_lattice_py(seed, replica, L):
    """The random start recomputed from the generator: site i (row-major) is
    +1 when bit i % 32 of word (i / 32) % 4 of INIT-stream call i / 128
    (counter (call, 1 << 24, 0, replica)) is set."""
    out = np.empty(L * L, np.int8)
    key = [seed & MASK, seed >> 32]
    for call in range(-(-(L * L) // 128)):
        words = philox_py([call, 1 << 24, 0, replica], key)
        for i in range(call * 128, min(L * L, call * 128 + 128)):
            out[i] = 1 if (words[(i >> 5) & 3] >> (i & 31)) & 1 else -1
    return out.reshape(L, L)


@pytest.mark.parametrize("L,seed,replica", [(20, 7, 0), (24, 0x1234_5678_9ABC_DEF0, 5),
                                            (33, 2, 3)])
def test_random_start_recomputed(oracle_lib, L, seed, replica):
    r = oracle_lib.Replica(L, L if L % 2 else L // 2, T=2.0, seed=seed, replica=replica)
    assert np.array_equal(r.spins(), init_lattice_py(seed, replica, L))


def test_random_start_is_uniform_and_uncorrelated(oracle_lib):
    """The random start is i.i.d. +-1 with probability 1/2: the fraction of
    up spins, the nearest-neighbour bond averages along both axes and the
    correlation between replicas are all zero within 4.5 standard errors, and
    the 16 patterns of 2 x 2 blocks are uniform (chi-square)."""
    L = 256
    a = oracle_lib.Replica(L, 32, T=2.0, seed=9, replica=0).spins().astype(np.int64)
    b = oracle_lib.Replica(L, 32, T=2.0, seed=9, replica=1).spins().astype(np.int64)
    n = L * L
    se = 1.0 / np.sqrt(n)
    assert set(np.unique(a)) == {-1, 1}
    assert abs(a.mean()) < 4.5 * se
    assert abs((a * np.roll(a, 1, 0)).mean()) < 4.5 * se
    assert abs((a * np.roll(a, 1, 1)).mean()) < 4.5 * se
    assert abs((a * b).mean()) < 4.5 * se
    blocks = ((a[0::2, 0::2] > 0) + 2 * (a[0::2, 1::2] > 0) + 4 * (a[1::2, 0::2] > 0)
              + 8 * (a[1::2, 1::2] > 0))
    counts = np.bincount(blocks.ravel(), minlength=16)
    assert stats.chisquare(counts).pvalue > 1e-4
