"""Host-side checks of the identities the GPU event chain relies on.

The kernels keep, per domain row, the spin mask and three bit planes of the
up-neighbour count k, and per rate class a count n_c.  After a flip they do
not recount: they step the planes of the four neighbours by one and update
the counts from packed 3-bit per-class tallies (the flipped site's old and
new class, every neighbour's class moving by one).  The member index is
formed in floating point.  These tests emulate those steps bit for bit in
Python and compare them with direct recounts, so that a wrong carry, field
or shift fails here on the CPU.  They share nothing with the oracle.
"""
import numpy as np
import pytest


def planes_full(S, top, bot, hl, hr, B):
    VM = (1 << B) - 1
    s0, s1, s2 = [0] * B, [0] * B, [0] * B
    for y in range(B):
        U = (S[y - 1] if y > 0 else top) & VM
        D = (S[y + 1] if y < B - 1 else bot) & VM
        Lf = ((S[y] << 1) | hl[y]) & VM
        Rt = ((S[y] >> 1) | (hr[y] << (B - 1))) & VM
        p1, q1, p2, q2 = U ^ D, U & D, Lf ^ Rt, Lf & Rt
        c0 = p1 & p2
        s0[y], s1[y], s2[y] = p1 ^ p2, q1 ^ q2 ^ c0, (q1 & q2) | (c0 & (q1 ^ q2))
    return [s0, s1, s2]


def site_class(S, P, y, x):
    s = (S[y] >> x) & 1
    k = ((P[0][y] >> x) & 1) + 2 * ((P[1][y] >> x) & 1) + 4 * ((P[2][y] >> x) & 1)
    return 5 * s + k


def direct_counts(S, P, B):
    n = [0] * 10
    for y in range(B):
        for x in range(B):
            n[site_class(S, P, y, x)] += 1
    return n


def neighbour_count_by_definition(S, top, bot, hl, hr, B, y, x):
    up = lambda v, b: (v >> b) & 1
    k = up(S[y - 1], x) if y > 0 else up(top, x)
    k += up(S[y + 1], x) if y < B - 1 else up(bot, x)
    k += up(S[y], x - 1) if x > 0 else hl[y]
    k += up(S[y], x + 1) if x < B - 1 else hr[y]
    return k


def flip_step(S, P, n, ys, xs, B, width=32):
    """The kernel's update for a flip at (ys, xs): returns the new counts and
    steps S and P in place (tallies in 32-bit words, as on the GPU)."""
    M32 = 0xFFFFFFFF
    c = site_class(S, P, ys, xs)
    up = c >= 5
    c_new = c - 5 if up else c + 5
    nb = [0] * 64
    for lane in range(64):
        on_row = lane == ys
        adj = (lane in (ys - 1, ys + 1)) and lane < B
        ca = xs - 1 if on_row else xs
        va = xs > 0 if on_row else adj
        vb = on_row and xs < B - 1
        pa = 3 * site_class(S, P, lane, ca & (width - 1)) if lane < B else 0
        pb = 3 * site_class(S, P, lane, (xs + 1) & (width - 1)) if lane < B else 0
        nb[lane] = ((int(va) << pa) + (int(vb) << pb)) & M32
    nb_s = (nb[ys] + (nb[ys - 1] if ys > 0 else 0) + (nb[ys + 1] if ys < 63 else 0)) & M32
    sub_s = (nb_s + (1 << (3 * c))) & M32
    add_s = ((((nb_s << 3) & ((1 << 64) - 1)) >> (6 if up else 0)) + (1 << (3 * c_new))) & M32
    n2 = [n[c2] + ((add_s >> (3 * c2)) & 7) - ((sub_s >> (3 * c2)) & 7) for c2 in range(10)]
    bx = 1 << xs
    mrow = ((bx << 1) | (bx >> 1)) & ((1 << B) - 1)
    S[ys] ^= bx
    inv = 0 if not up else M32
    for lane in range(B):
        m = mrow if lane == ys else (bx if lane in (ys - 1, ys + 1) else 0)
        c1 = (P[0][lane] ^ inv) & m
        c2 = (P[1][lane] ^ inv) & c1
        P[0][lane] ^= m
        P[1][lane] ^= c1
        P[2][lane] ^= c2
    return n2


@pytest.mark.parametrize("B", [4, 8, 12, 16, 32])
def test_planes_hold_the_neighbour_count(B):
    rng = np.random.default_rng(B)
    S = [int(v) for v in rng.integers(0, 1 << B, B)]
    top, bot = int(rng.integers(0, 1 << B)), int(rng.integers(0, 1 << B))
    hl = [int(v) for v in rng.integers(0, 2, B)]
    hr = [int(v) for v in rng.integers(0, 2, B)]
    P = planes_full(S, top, bot, hl, hr, B)
    for y in range(B):
        for x in range(B):
            k = site_class(S, P, y, x) % 5 if (S[y] >> x) & 1 == 0 else site_class(S, P, y, x) - 5
            assert k == neighbour_count_by_definition(S, top, bot, hl, hr, B, y, x)


@pytest.mark.parametrize("B", [4, 8, 12, 16, 32])
def test_incremental_tallies_and_planes_match_recounts(B):
    rng = np.random.default_rng(100 + B)
    for trial in range(12):
        S = [int(v) for v in rng.integers(0, 1 << B, B)]
        if trial % 3 == 0:  # ordered tiles reach classes 0 and 9 (all four
            S = [(1 << B) - 1] * B  # neighbours in the top or bottom class)
        top = int(rng.integers(0, 1 << B)) if trial % 3 else (1 << B) - 1
        bot = int(rng.integers(0, 1 << B)) if trial % 3 else (1 << B) - 1
        hl = [int(v) for v in rng.integers(0, 2, B)] if trial % 3 else [1] * B
        hr = [int(v) for v in rng.integers(0, 2, B)] if trial % 3 else [1] * B
        P = planes_full(S, top, bot, hl, hr, B)
        n = direct_counts(S, P, B)
        for _ in range(60):
            ys, xs = int(rng.integers(0, B)), int(rng.integers(0, B))
            n = flip_step(S, P, n, ys, xs, B)
            assert P == planes_full(S, top, bot, hl, hr, B)
            assert n == direct_counts(S, P, B)


def test_top_class_tally_does_not_overflow():
    """A class-9 site (up, four up neighbours) flipping down moves four class-9
    neighbours to class 8: the tally field of class 9 holds 4 (bit 29), and
    the shift that moves it must not lose it."""
    B = 8
    S = [(1 << B) - 1] * B
    P = planes_full(S, (1 << B) - 1, (1 << B) - 1, [1] * B, [1] * B, B)
    n = direct_counts(S, P, B)
    assert n[9] == B * B
    n = flip_step(S, P, n, 3, 4, B)
    assert n == direct_counts(S, P, B)
    assert n[8] == 4 and n[4] == 1 and n[9] == B * B - 5


def member_index_fp64(a, r):
    """The kernels' member index: trunc((a + 1/2) fl(1/r)) in IEEE doubles."""
    inv = np.float64(1.0) / np.float64(r)
    return int(np.trunc((np.float64(a) + np.float64(0.5)) * inv))


def test_member_index_in_fp64_is_exact_floor():
    """j = floor(a / r) for 0 <= a < n r, n <= 4096, 1 <= r <= 2^32: the
    quotient lies at least 1/(2r) from an integer and the double product is
    within 2^-39 of it.  Exhaustive at the edges (a = j r, j r - 1, j r + r - 1)
    and random in between."""
    rng = np.random.default_rng(7)
    rs = [1, 2, 3, 7, 2 ** 31 - 1, 2 ** 31, 2 ** 32 - 1, 2 ** 32, 12345677, 99991]
    rs += [int(v) for v in rng.integers(1, 2 ** 32 + 1, 400, dtype=np.uint64)]
    for r in rs:
        for j in [0, 1, 2, 1023, 4094, 4095] + [int(v) for v in rng.integers(0, 4096, 20)]:
            for m in {0, 1, r - 1, r // 2, int(rng.integers(0, r))}:
                if m >= r:
                    continue
                a = j * r + m
                assert member_index_fp64(a, r) == j, (a, r, j)


def test_rate_sums_are_exact_in_fp64():
    """n_c r_c < 2^44 and ten of them sum below 2^48: doubles hold every
    prefix exactly, so comparisons with x < n_d 2^32 are exact."""
    rng = np.random.default_rng(3)
    for _ in range(200):
        n = rng.integers(0, 4097, 10)
        r = rng.integers(0, 2 ** 32 + 1, 10, dtype=np.uint64)
        exact = np.cumsum([int(a) * int(b) for a, b in zip(n, r)])
        fp = np.cumsum(n.astype(np.float64) * r.astype(np.float64))
        assert all(int(v) == e for v, e in zip(fp, exact))
