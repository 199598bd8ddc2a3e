"""Exact reference tools on tiny lattices (test infrastructure only).

These do not simulate trajectories; they work on the full probability vector
over all 2^N configurations, which is how the paper itself obtained its
reference equilibrium values (Sec. 3.1: the distribution is evolved to
equilibrium with Eq. (CK_parallel in s)).  They share no code with the
serial oracle in kmco.c or with the HIP library, so they can pin both.

State encoding: configuration index i in [0, 2^N), bit (y*L + x) of i is 1
when spin (y, x) is +1.
"""
import itertools
import math

import numpy as np


def spins_of_states(L):
    N = L * L
    idx = np.arange(1 << N, dtype=np.int64)
    bits = (idx[:, None] >> np.arange(N)[None, :]) & 1
    return (2 * bits - 1).astype(np.int8)  # [2^N, N]


def magnetisation_and_bonds(L, S=None):
    """M = sum of spins, B = sum over right and down periodic bonds of s s'
    (Eq. (Hamiltonian Definition) with each bond counted once)."""
    if S is None:
        S = spins_of_states(L)
    s = S.reshape(-1, L, L).astype(np.int64)
    M = s.sum(axis=(1, 2))
    B = (s * np.roll(s, -1, axis=2)).sum(axis=(1, 2)) + \
        (s * np.roll(s, -1, axis=1)).sum(axis=(1, 2))
    return M, B


def boltzmann(L, J, h, T):
    """pi_i = exp(-H_i/T), H = -J B - h M (Eq. (equilibrium distribution))."""
    M, B = magnetisation_and_bonds(L)
    E = -J * B - h * M
    a = -E / T
    p = np.exp(a - a.max())
    return p / p.sum(), M, B, E


def rate(dE, T, model):
    """Acceptance w for energy change dE: Metropolis min(1, e^{-dE/T}) or the
    Barker/Glauber form 1/(1 + e^{dE/T}) of Eq. (Glauber_TM)."""
    if model == 0:
        return np.where(dE <= 0, 1.0, np.exp(-np.maximum(dE, 0.0) / T))
    return 1.0 / (1.0 + np.exp(dE / T))


class TickKernel:
    """The single-site kernel of one domain, applied to probability vectors.

    In one tick, a site i of the domain (n_d sites) is selected with
    probability 1/n_d and flipped with probability w_i(sigma); otherwise the
    configuration is unchanged (Eq. (Glauber_TM), selection probability
    N_D/N_S = 1/n_d).  The operator acts on the column vector p in the
    left-stochastic convention of Eq. (CK_canonical in s).
    """

    def __init__(self, L, sites, J, h, T, model=0, quantise=False):
        S = spins_of_states(L).astype(np.float64)
        self.N = L * L
        self.sites = list(sites)
        nd = len(self.sites)
        self.flip_prob = []
        for i in self.sites:
            y, x = divmod(i, L)
            nb = [((y - 1) % L) * L + x, ((y + 1) % L) * L + x,
                  y * L + (x - 1) % L, y * L + (x + 1) % L]
            n = S[:, nb].sum(axis=1)
            dE = 2.0 * S[:, i] * (J * n + h)
            w = rate(dE, T, model)
            if quantise:
                w = np.minimum(np.floor(w * 2.0 ** 32 + 0.5), 2.0 ** 32) / 2.0 ** 32
            self.flip_prob.append(w / nd)

    def apply(self, p, times=1):
        idx = np.arange(1 << self.N)
        for _ in range(times):
            out = p.copy()
            for i, q in zip(self.sites, self.flip_prob):
                moved = q * p
                out -= moved
                out[idx ^ (1 << i)] += moved
            p = out
        return p

    def apply_transpose(self, v, times=1):
        """v^T T (row-vector action); used for reversibility checks."""
        idx = np.arange(1 << self.N)
        for _ in range(times):
            out = v.copy()
            for i, q in zip(self.sites, self.flip_prob):
                out += q * (v[idx ^ (1 << i)] - v)
            v = out
        return v


def partition(L, Bx, By=None):
    """Domains Bx wide and By high in row-major order over the domain grid,
    their colours and the number of colours.  Each axis of n domains is
    coloured with one colour (n = 1), t mod 2 (n even), or t mod 2 with the
    last domain given a third colour (n odd); the colour is ax + cx ay."""
    By = By or Bx
    NTx, NTy = L // Bx, L // By

    def axis(t, n):
        return 0 if n == 1 else (2 if n % 2 and t == n - 1 else t % 2)

    def ncol(n):
        return 1 if n == 1 else (3 if n % 2 else 2)

    doms, cols = [], []
    for ty in range(NTy):
        for tx in range(NTx):
            doms.append([(ty * By + ly) * L + tx * Bx + lx
                         for ly in range(By) for lx in range(Bx)])
            cols.append(axis(tx, NTx) + ncol(NTx) * axis(ty, NTy))
    return doms, cols, ncol(NTx) * ncol(NTy)


def checkerboard(L, B):
    """Square domains of side B (4 colours when L/B is even)."""
    doms, cols, _ = partition(L, B, B)
    return doms, cols


class SweepOperator:
    """T_SEQ(Lambda) for one colour order and T_PAR, the uniform mixture over
    all n! orders of the n colours (Eq. (replica detailed balance of
    sequential tm) and Eq. (sum of sequential tms)), or the fixed palindrome
    0 1 .. n-1 n-1 .. 1 0.  Domains are B wide and By (default B) high."""

    def __init__(self, L, B, J, h, T, model=0, NI=None, quantise=False,
                 palindrome=False, By=None):
        self.doms, self.cols, self.ncol = partition(L, B, By)
        self.kern = [TickKernel(L, d, J, h, T, model, quantise) for d in self.doms]
        self.NI = NI if NI else B * (By or B)
        self.palindrome = palindrome

    def orders(self):
        n = self.ncol
        if self.palindrome:
            return [tuple(range(n)) + tuple(reversed(range(n)))]
        return list(itertools.permutations(range(n)))

    def seq(self, p, order):
        for c in order:
            for k, col in zip(self.kern, self.cols):
                if col == c:
                    p = k.apply(p, self.NI)
        return p

    def seq_transpose(self, v, order):
        for c in reversed(order):
            for k, col in zip(self.kern, self.cols):
                if col == c:
                    v = k.apply_transpose(v, self.NI)
        return v

    def par(self, p):
        outs = [self.seq(p, o) for o in self.orders()]
        return sum(outs) / len(outs)


def perm_rank(perm):
    """Lexicographic rank of a permutation of range(n)."""
    rank, avail = 0, list(range(len(perm)))
    for i, v in enumerate(perm):
        a = avail.index(v)
        rank += a * math.factorial(len(perm) - 1 - i)
        avail.pop(a)
    return rank


# ------------------------------------------------------------------ the ring
#
# The paper's 1D system (Sec. 3.1): a periodic ring of N sites, site i with
# the two neighbours i - 1 and i + 1, cut into N_D domains of B consecutive
# sites (Eq. (1D partitions)).  State index bit i set when spin i is +1.

def ring_spins(N):
    idx = np.arange(1 << N, dtype=np.int64)
    return (2 * ((idx[:, None] >> np.arange(N)[None, :]) & 1) - 1).astype(np.int8)


def ring_boltzmann(N, J, h, T):
    """pi over the 2^N ring states, with M and the bond sum B = sum s_i s_{i+1}."""
    s = ring_spins(N).astype(np.int64)
    M = s.sum(axis=1)
    B = (s * np.roll(s, -1, axis=1)).sum(axis=1)
    E = -J * B - h * M
    a = -E / T
    p = np.exp(a - a.max())
    return p / p.sum(), M, B, E


class RingTickKernel:
    """One tick of a ring domain: site i of the domain's n_d sites is chosen
    with probability 1/n_d and flipped with probability w (two neighbours)."""

    def __init__(self, N, sites, J, h, T, model=0, quantise=False):
        S = ring_spins(N).astype(np.float64)
        self.N, self.sites = N, list(sites)
        nd = len(self.sites)
        self.flip_prob = []
        for i in self.sites:
            n = S[:, (i - 1) % N] + S[:, (i + 1) % N]
            dE = 2.0 * S[:, i] * (J * n + h)
            w = rate(dE, T, model)
            if quantise:
                w = np.minimum(np.floor(w * 2.0 ** 32 + 0.5), 2.0 ** 32) / 2.0 ** 32
            self.flip_prob.append(w / nd)

    def apply(self, p, times=1):
        idx = np.arange(1 << self.N)
        for _ in range(times):
            out = p.copy()
            for i, q in zip(self.sites, self.flip_prob):
                moved = q * p
                out -= moved
                out[idx ^ (1 << i)] += moved
            p = out
        return p

    def apply_transpose(self, v, times=1):
        idx = np.arange(1 << self.N)
        for _ in range(times):
            out = v.copy()
            for i, q in zip(self.sites, self.flip_prob):
                out += q * (v[idx ^ (1 << i)] - v)
            v = out
        return v


def tick_at(p, states, sites, neighbours, J, h, T, model=0, quantise=False):
    """p' at the given states after one tick of the domain `sites` applied to
    the full vector p (Eq. (Glauber_TM): site i of the n_d sites is chosen with
    probability 1/n_d and flipped with probability w_i), for systems whose
    2^N x N tables TickKernel cannot hold:

        p'(s) = p(s) - sum_i q_i(s) p(s) + sum_i q_i(s ^ 2^i) p(s ^ 2^i),

    q_i(s) = w(dE_i(s)) / n_d, dE_i = 2 s_i (J sum of the neighbours' spins + h).
    neighbours(i) lists the sites bonded to i, a site met twice counted twice
    (the two neighbours along an axis of length 2)."""
    states = np.asarray(states, dtype=np.int64)
    nd = len(sites)

    def q(s, i):
        spin = lambda j: 2.0 * ((s >> j) & 1) - 1.0
        n = sum(spin(j) for j in neighbours(i))
        w = rate(2.0 * spin(i) * (J * n + h), T, model)
        if quantise:
            w = np.minimum(np.floor(w * 2.0 ** 32 + 0.5), 2.0 ** 32) / 2.0 ** 32
        return w / nd

    out = p[states].copy()
    for i in sites:
        partner = states ^ (1 << i)
        out -= q(states, i) * p[states]
        out += q(partner, i) * p[partner]
    return out


def square_neighbours(L):
    """The four bonded sites of site i = y L + x on the periodic L x L lattice."""
    def nb(i):
        y, x = divmod(i, L)
        return [((y - 1) % L) * L + x, ((y + 1) % L) * L + x,
                y * L + (x - 1) % L, y * L + (x + 1) % L]
    return nb


def ring_neighbours(N):
    """The two bonded sites of site i on the periodic ring of N sites."""
    return lambda i: [(i - 1) % N, (i + 1) % N]


def ring_partition(N, B):
    """Domains of B consecutive sites, their colours along the ring (one
    colour for one domain, t mod 2 for an even count, t mod 2 with the last
    domain given a third colour for an odd count) and the colour count."""
    n = N // B
    doms = [list(range(t * B, (t + 1) * B)) for t in range(n)]
    cols = [0 if n == 1 else (2 if n % 2 and t == n - 1 else t % 2) for t in range(n)]
    return doms, cols, 1 if n == 1 else (3 if n % 2 else 2)


class RingSweepOperator(SweepOperator):
    """T_PAR of the ring: the mixture over all orders of its colours (or the
    palindrome), N_I ticks per domain visit (Eq. (1D partitions))."""

    def __init__(self, N, B, J, h, T, model=0, NI=None, quantise=False, palindrome=False):
        self.doms, self.cols, self.ncol = ring_partition(N, B)
        self.kern = [RingTickKernel(N, d, J, h, T, model, quantise) for d in self.doms]
        self.NI = NI if NI else B
        self.palindrome = palindrome


# ------------------------------------------------ time-slice domain processes
#
# The rejection-free variant with fixed time slices: a domain process runs
# its continuous-time kinetics (each site of the domain flips at rate w,
# nothing outside moves) for a time tau, so it acts on p as exp(Q_d tau),
# Q_d the domain's generator.  The sweep applies these in colour order.

class SliceKernel:
    """exp(Q_d tau) of one domain, applied to probability vectors with a
    sparse matrix exponential (scipy's expm_multiply)."""

    def __init__(self, n_sites, sites, neighbours, J, h, T, model, tau, quantise=True):
        import scipy.sparse as sp
        S = ((np.arange(1 << n_sites)[:, None] >> np.arange(n_sites)[None, :]) & 1) * 2 - 1
        S = S.astype(np.float64)
        idx = np.arange(1 << n_sites)
        rows, cols, vals = [], [], []
        diag = np.zeros(1 << n_sites)
        for i in sites:
            n = S[:, neighbours[i]].sum(axis=1)
            dE = 2.0 * S[:, i] * (J * n + h)
            w = rate(dE, T, model)
            if quantise:
                w = np.minimum(np.floor(w * 2.0 ** 32 + 0.5), 2.0 ** 32) / 2.0 ** 32
            rows.append(idx ^ (1 << i))
            cols.append(idx)
            vals.append(w)
            diag -= w
        rows.append(idx)
        cols.append(idx)
        vals.append(diag)
        self.Q = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                               shape=(1 << n_sites, 1 << n_sites))
        self.tau = tau

    def apply(self, p, times=1):
        from scipy.sparse.linalg import expm_multiply
        for _ in range(times):
            p = expm_multiply(self.Q * self.tau, p)
        return p


class SliceSweepOperator(SweepOperator):
    """T_PAR of the time-slice variant on the L x L torus (domains Bx x By) or
    on the ring of L sites (ring=True, domains of Bx sites): each domain
    visit is exp(Q_d tau); colour orders as for the tick chain."""

    def __init__(self, L, B, J, h, T, model, tau, palindrome=False, By=None, ring=False,
                 quantise=True):
        if ring:
            n_sites = L
            self.doms, self.cols, self.ncol = ring_partition(L, B)
            nb = {i: [(i - 1) % L, (i + 1) % L] for i in range(L)}
        else:
            n_sites = L * L
            self.doms, self.cols, self.ncol = partition(L, B, By)
            nb = {}
            for i in range(n_sites):
                y, x = divmod(i, L)
                nb[i] = [((y - 1) % L) * L + x, ((y + 1) % L) * L + x,
                         y * L + (x - 1) % L, y * L + (x + 1) % L]
        self.kern = [SliceKernel(n_sites, d, nb, J, h, T, model, tau, quantise)
                     for d in self.doms]
        self.NI = 1
        self.palindrome = palindrome
