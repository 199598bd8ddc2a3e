"""Pins of the oracle's per-class rate table (Appendix A, Eq. (Glauber_TM)).

Classes: c = 5*[s = +1] + k, k = number of up neighbours, n = 2k - 4,
dE = 2 s (J n + h).  The pins use properties fixed by the physics rather
than the formula itself: the detailed-balance ratio of a move and its
reverse, the Barker sum rule, the Q32 quantisation and finite-difference
derivatives.
"""
import math

import numpy as np
import pytest

CASES = [(1.0, 0.0, 2.5), (1.0, 0.3, 1.5), (0.7, -0.45, 3.3), (-1.0, 0.2, 2.0),
         (1.0, 0.0, 2.269)]


def energy_change(c, J, h):
    """Flip energy from a direct count of the bonds around one site."""
    up, k = divmod(c, 5)
    s = 1 if up else -1
    nb = [1] * k + [-1] * (4 - k)
    before = -J * sum(s * x for x in nb) - h * s
    after = -J * sum(-s * x for x in nb) + h * s
    return after - before


@pytest.mark.parametrize("J,h,T", CASES)
@pytest.mark.parametrize("model", [0, 1])
def test_detailed_balance_ratio(oracle_lib, J, h, T, model):
    r, w, gJ, gh = oracle_lib.rates(J, h, T, model)
    for c in range(10):
        up, k = divmod(c, 5)
        rev = 5 * (1 - up) + k  # same neighbours, flipped centre spin
        dE = energy_change(c, J, h)
        # w(c)/w(rev) = exp(-dE/T): stationarity of exp(-H/T)
        assert w[c] / w[rev] == pytest.approx(math.exp(-dE / T), rel=1e-13)
        if model == 1:
            assert w[c] + w[rev] == pytest.approx(1.0, abs=1e-15)
        else:
            assert max(w[c], w[rev]) == 1.0


@pytest.mark.parametrize("J,h,T", CASES)
@pytest.mark.parametrize("model", [0, 1])
def test_q32_quantisation(oracle_lib, J, h, T, model):
    r, w, _, _ = oracle_lib.rates(J, h, T, model)
    for c in range(10):
        q = w[c] * 2.0 ** 32
        assert abs(int(r[c]) - q) <= 0.5
        assert int(r[c]) <= 2 ** 32
        if w[c] == 1.0:
            assert int(r[c]) == 2 ** 32


@pytest.mark.parametrize("J,h,T", CASES[1:4])
@pytest.mark.parametrize("model", [0, 1])
def test_log_derivatives(oracle_lib, J, h, T, model):
    eps = 1e-6
    _, _, gJ, gh = oracle_lib.rates(J, h, T, model)
    lw = lambda JJ, hh: np.log(oracle_lib.rates(JJ, hh, T, model)[1])
    dJ = (lw(J + eps, h) - lw(J - eps, h)) / (2 * eps)
    dh = (lw(J, h + eps) - lw(J, h - eps)) / (2 * eps)
    np.testing.assert_allclose(gJ, dJ, atol=1e-6)
    np.testing.assert_allclose(gh, dh, atol=1e-6)


def test_rejects_bad_parameters(oracle_lib):
    for bad in [(1.0, 0.0, 0.0), (1.0, 0.0, -1.0), (float("nan"), 0.0, 1.0),
                (1.0, float("inf"), 1.0)]:
        with pytest.raises(ValueError):
            oracle_lib.rates(*bad)
