"""Closed forms for the periodic Ising model (test infrastructure only).

* The periodic ring (the paper's 1D system): transfer-matrix free energy.

* Onsager (1944) energy per site and Yang (1952) spontaneous magnetisation
  of the infinite square lattice, J = 1, k_B = 1.
* Kaufman (1949) partition function of the finite m x n torus; the paper
  compares its 12x12 and 100x100 runs with the finite-lattice result of
  Ferdinand and Fisher (Sec. 3.2 and Table 1), which follows from it.
These pin the oracle's equilibrium statistics at sizes too large to
enumerate.
"""
import math

import numpy as np
from scipy.special import ellipk

T_CRITICAL = 2.0 / math.log(1.0 + math.sqrt(2.0))


def onsager_energy(T, J=1.0):
    """Energy per site u(T) = -J coth(2K) [1 + (2/pi)(2 tanh^2(2K) - 1) K1(k)],
    K = J/T, k = 2 sinh(2K)/cosh^2(2K), K1 the complete elliptic integral of
    the first kind (scipy's parameter m = k^2)."""
    K = J / T
    k = 2.0 * math.sinh(2 * K) / math.cosh(2 * K) ** 2
    a = 2.0 * math.tanh(2 * K) ** 2 - 1.0
    if abs(a) < 1e-15:  # T = T_c: a -> 0 while K1 -> infinity, product -> 0
        return -J / math.tanh(2 * K)
    K1 = ellipk(k * k)
    return -J / math.tanh(2 * K) * (1.0 + 2.0 / math.pi * a * K1)


def onsager_magnetisation(T, J=1.0):
    """Spontaneous magnetisation per site (1 - sinh(2K)^-4)^(1/8) below T_c."""
    K = J / T
    s = math.sinh(2 * K)
    if s <= 1.0:
        return 0.0
    return (1.0 - s ** -4) ** 0.125


def _log2cosh(y):
    y = abs(y)
    return y + math.log1p(math.exp(-2.0 * y))


def _log_abs_2sinh(y):
    """log|2 sinh y| and its sign (y != 0)."""
    a = abs(y)
    return a + math.log1p(-math.exp(-2.0 * a)), math.copysign(1.0, y)


def _log_abs_sum(terms):
    """log|sum| of signed terms given as (sign, log|term|)."""
    mx = max(l for _, l in terms)
    tot = sum(s * math.exp(l - mx) for s, l in terms)
    return mx + math.log(abs(tot)), math.copysign(1.0, tot)


def kaufman_log_z(K, m, n):
    """ln Z of the m x n periodic Ising model at coupling K = J/T, h = 0.

    Z = 1/2 (2 sinh 2K)^{mn/2} (Z1 + Z2 + Z3 + Z4) with
      Z1 = prod_r 2 cosh(m g_{2r+1}/2),  Z2 = prod_r 2 sinh(m g_{2r+1}/2),
      Z3 = prod_r 2 cosh(m g_{2r}/2),    Z4 = prod_r 2 sinh(m g_{2r}/2),
    r = 0..n-1, cosh g_l = cosh 2K coth 2K - cos(l pi/n), and g_0 taken
    with its sign, g_0 = 2K + ln tanh K.
    """
    c = math.cosh(2 * K) / math.tanh(2 * K)

    def gamma(l):
        if l == 0:
            return 2 * K + math.log(math.tanh(K))
        return math.acosh(c - math.cos(l * math.pi / n))

    terms = []
    for parity in (1, 0):
        g = [gamma(2 * r + parity) for r in range(n)]
        # cosh product (always positive)
        lc = sum(_log2cosh(m * x / 2) for x in g)
        terms.append((1.0, lc))
        if all(x != 0.0 for x in g):
            sign, ls = 1.0, 0.0
            for x in g:
                l, sg = _log_abs_2sinh(m * x / 2)
                sign *= sg
                ls += l
            terms.append((sign, ls))
    lsum, sgn = _log_abs_sum(terms)
    assert sgn > 0
    return -math.log(2.0) + 0.5 * m * n * math.log(2 * math.sinh(2 * K)) + lsum


def kaufman_energy(T, L, J=1.0, dK=1e-5):
    """Mean energy per site <H>/N of the L x L torus, -(1/N) d ln Z/dK * J,
    by a fourth-order central difference of kaufman_log_z."""
    K = J / T
    f = lambda k: kaufman_log_z(k, L, L)
    d = (-f(K + 2 * dK) + 8 * f(K + dK) - 8 * f(K - dK) + f(K - 2 * dK)) / (12 * dK)
    return -J * d / (L * L)


def kaufman_energy_std(T, L, J=1.0, dK=1e-4):
    """Standard deviation of H/N per sample: sqrt(d^2 ln Z/dK^2) J / N."""
    K = J / T
    f = lambda k: kaufman_log_z(k, L, L)
    d2 = (-f(K + 2 * dK) + 16 * f(K + dK) - 30 * f(K) + 16 * f(K - dK)
          - f(K - 2 * dK)) / (12 * dK * dK)
    return J * math.sqrt(d2) / (L * L)


def ring_energy(N, T, J=1.0, h=0.0):
    """Mean energy <H> of the periodic Ising ring of N sites (the paper's 1D
    system, Sec. 3.1), H = -J sum s_i s_{i+1} - h sum s_i, from the 2 x 2
    transfer matrix V_{s s'} = exp(K s s' + (h/2T)(s + s')), K = J/T
    (Kramers-Wannier): Z = lam_+^N + lam_-^N with lam the eigenvalues of V,
    and <H> = T^2 d ln Z/dT, here by a central difference in 1/T."""
    def log_z(beta):
        a = beta * J
        b = beta * h
        disc = math.sqrt(math.exp(2 * a) * math.sinh(b) ** 2 + math.exp(-2 * a))
        lp = math.exp(a) * math.cosh(b) + disc
        lm = math.exp(a) * math.cosh(b) - disc
        # lam_-^N may be negative for odd N when lam_- < 0
        return N * math.log(lp) + math.log1p((lm / lp) ** N)

    beta, d = 1.0 / T, 1e-6
    return -(log_z(beta + d) - log_z(beta - d)) / (2 * d)


def ring_energy_std(N, T, J=1.0, h=0.0, d=1e-4):
    """Standard deviation of H on the ring: Var(H) = d^2 ln Z/d beta^2."""
    beta = 1.0 / T
    e = lambda b: ring_energy(N, 1.0 / b, J, h)
    var = -(e(beta + d) - e(beta - d)) / (2 * d)
    return math.sqrt(max(var, 0.0))
