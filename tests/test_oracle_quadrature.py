"""Pins of the oracle's Gauss rules against closed forms and a library routine.

Half-range rule: Q nodes on a semi-axis recover the half-space moments up to order
2Q-1 (paper Sec. I / Sec. III); the moments of exp(-p^2/2)/sqrt(2 pi) on [0, inf) are
mu_k = 2^((k-1)/2) Gamma((k+1)/2) / sqrt(2 pi).  Full-range rule: numpy's hermegauss.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import quadrature as quad


def mu_half(k):
    return 2.0 ** ((k - 1) / 2.0) * math.gamma((k + 1) / 2.0) / math.sqrt(2 * math.pi)


@pytest.mark.parametrize("Q", [1, 2, 3, 4, 7, 11, 16, 30, 50])
def test_half_range_moment_exactness(Q):
    x, w = quad.half_range_rule(Q)
    assert np.all(np.diff(x) > 0) and np.all(x > 0) and np.all(w > 0)
    for k in range(2 * Q):
        got = math.fsum(w * x ** k)
        assert abs(got / mu_half(k) - 1) < 1e-13, (Q, k)
    # degree 2Q is not integrated exactly: the error of a Gauss rule on p^2Q is the squared
    # norm of the monic P_Q, i.e. the Hankel-determinant ratio det H_{Q+1} / det H_Q
    if Q <= 7:
        with mp.workdps(80):
            mom = quad.half_range_moments(2 * Q + 1, 80)
            H = lambda n: mp.det(mp.matrix([[mom[i + j] for j in range(n)] for i in range(n)]))
            gamma_Q = H(Q + 1) / H(Q)
        err = mu_half(2 * Q) - math.fsum(w * x ** (2 * Q))
        assert err == pytest.approx(float(gamma_Q), rel=1e-8)


def test_half_range_one_node_closed_form():
    x, w = quad.half_range_rule(1)
    assert x[0] == pytest.approx(math.sqrt(2 / math.pi), rel=1e-15)
    assert w[0] == pytest.approx(0.5, rel=1e-15)


def test_half_range_two_nodes_closed_form():
    # the two nodes are the zeros of the monic x^2 + b x + c orthogonal to 1 and x:
    #   m2 + b m1 + c m0 = 0,  m3 + b m2 + c m1 = 0   (Cramer's rule below)
    m0, m1, m2, m3 = (mu_half(k) for k in range(4))
    det = m1 * m1 - m0 * m2
    b = (m0 * m3 - m1 * m2) / det
    c = (m2 * m2 - m1 * m3) / det
    r = np.sort(np.roots([1.0, b, c]))
    x, w = quad.half_range_rule(2)
    assert np.allclose(x, r, rtol=1e-12)


def test_half_range_precision_is_stable():
    # the mp construction at two working precisions agrees to far below float64 rounding
    Q = 40
    x1, w1, a, b, dps = quad.half_range_rule_mp(Q)
    mom = quad.half_range_moments(2 * Q + 2, dps + 40)
    a2, b2 = quad.chebyshev_recurrence(mom, Q + 1, dps + 40)
    x2, w2 = quad.gauss_rule(a2, b2, Q, dps + 40)
    with mp.workdps(dps):
        assert max(abs(u / v - 1) for u, v in zip(x1, x2)) < mp.mpf(10) ** -25
        assert max(abs(u / v - 1) for u, v in zip(w1, w2)) < mp.mpf(10) ** -25


@pytest.mark.parametrize("Q", [1, 2, 3, 4, 5, 6, 7, 8])
def test_full_range_matches_hermegauss(Q):
    x, w = quad.full_range_rule(Q)
    xr, wr = np.polynomial.hermite_e.hermegauss(Q)
    wr = wr / math.sqrt(2 * math.pi)
    assert np.allclose(x, xr, rtol=0, atol=1e-14)
    assert np.allclose(w, wr, rtol=1e-13, atol=0)
    assert math.fsum(w) == pytest.approx(1.0, abs=1e-15)


@pytest.mark.parametrize("Q", [2, 3, 4, 5, 6, 7])
def test_full_range_symmetry_bitwise(Q):
    x, w = quad.full_range_rule(Q)
    assert np.array_equal(x, -x[::-1])
    assert np.array_equal(w, w[::-1])
    if Q % 2:
        assert x[Q // 2] == 0.0


@pytest.mark.parametrize("Q", [4, 16])
def test_x_axis_layout(Q):
    x, w = quad.x_axis(Q)
    assert len(x) == 2 * Q
    assert np.array_equal(x, -x[::-1]) and np.array_equal(w, w[::-1])
    assert np.all(np.diff(x) > 0)
    assert math.fsum(w) == pytest.approx(1.0, abs=1e-15)
