"""Pins of the oracle's discrete equilibrium (paper Sec. III: direct-product expansion,
g_x in half-range Hermite polynomials up to N_x on each semi-axis, g_y (and g_z) in
full-range Hermite polynomials up to N = Q - 1; Shakhov factor of Eq. sdef)."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import equilibrium as eq
from oracle import solver as sv

RNG = np.random.default_rng(1702)


def gauss_pdf(p, u, T):
    return mp.exp(-(p - u) ** 2 / (2 * T)) / mp.sqrt(2 * mp.pi * T)


@pytest.mark.parametrize("u,T", [(0.0, 1.0), (0.37, 1.3), (-0.8, 0.6), (1.4, 2.2)])
def test_half_gaussian_moments_vs_numerical_integration(u, T):
    I = eq.half_gaussian_moments(8, u, T)
    for k in range(9):
        ref = mp.quad(lambda p: p ** k * gauss_pdf(p, u, T), [0, mp.inf])
        assert I[k] == pytest.approx(float(ref), rel=1e-13, abs=1e-15)
    E = eq.gaussian_moments(8, u, T)
    for k in range(9):
        ref = mp.quad(lambda p: p ** k * gauss_pdf(p, u, T), [-mp.inf, mp.inf])
        assert E[k] == pytest.approx(float(ref), rel=1e-13, abs=1e-15)


@pytest.mark.parametrize("Q,N", [(4, 3), (7, 6), (16, 6), (50, 6)])
def test_half_range_factor_recovers_moments(Q, N):
    ax = eq.AxisProjection('half', Q, N)
    x = ax.nodes
    for _ in range(4):
        u, T = RNG.uniform(-0.6, 0.6), RNG.uniform(0.6, 1.6)
        g = ax.factor(u, T)
        Ip, Im, E = eq.half_gaussian_moments(N, u, T), eq.half_gaussian_moments(N, -u, T), eq.gaussian_moments(N, u, T)
        for k in range(N + 1):
            pos = math.fsum(g[x > 0] * x[x > 0] ** k)
            neg = math.fsum(g[x < 0] * x[x < 0] ** k)
            assert pos == pytest.approx(Ip[k], rel=1e-12, abs=1e-14)
            assert neg == pytest.approx((-1) ** k * Im[k], rel=1e-12, abs=1e-14)
            assert pos + neg == pytest.approx(E[k], rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("Q", [2, 4, 5, 6, 7])
def test_full_range_factor_recovers_moments(Q):
    ax = eq.AxisProjection('full', Q, Q - 1)
    x = ax.nodes
    for _ in range(4):
        u, T = RNG.uniform(-0.6, 0.6), RNG.uniform(0.6, 1.6)
        g = ax.factor(u, T)
        E = eq.gaussian_moments(Q - 1, u, T)
        for k in range(Q):
            assert math.fsum(g * x ** k) == pytest.approx(E[k], rel=1e-12, abs=1e-14)


def test_full_range_factor_projection_coefficients():
    # the expansion coefficients of Eq. Fmn_def are int G He_l; He_l are the probabilists'
    # Hermite polynomials (orthogonality of Eq. H_ortho); numerical integration in mpmath
    Q = 6
    ax = eq.AxisProjection('full', Q, Q - 1)
    u, T = 0.31, 1.17
    He = [lambda p: 1, lambda p: p, lambda p: p ** 2 - 1, lambda p: p ** 3 - 3 * p,
          lambda p: p ** 4 - 6 * p ** 2 + 3, lambda p: p ** 5 - 10 * p ** 3 + 15 * p]
    coef = [mp.quad(lambda p: gauss_pdf(p, u, T) * He[l](p), [-mp.inf, mp.inf]) for l in range(Q)]
    x, w = ax.nodes, ax.weights
    ref = [w[j] * sum(float(coef[l]) * float(He[l](x[j])) / math.factorial(l) for l in range(Q)) for j in range(Q)]
    assert np.allclose(ax.factor(u, T), ref, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("kind,Q,N", [('half', 4, 3), ('half', 16, 6), ('half', 50, 6), ('full', 5, 4)])
def test_rest_state_is_the_weights(kind, Q, N):
    """At u = 0, T = 1 the 1D Maxwellian equals the weight function, so J_0 = gamma_0 and
    J_l = 0 (l >= 1) and g_i = w_i.  In float64 the J_l carry rounding of size
    eps * sum_k |C_lk| I_k, amplified at node i by sum_l |w_i P_l(x_i) / gamma_l|; the test
    bounds the deviation by that product (it reaches ~1e-9 relative at the outermost
    node of Q = 50, where w ~ 1e-52)."""
    ax = eq.AxisProjection(kind, Q, N)
    g = ax.factor(0.0, 1.0)
    if kind == 'half':
        mom = eq.half_gaussian_moments(N, 0.0, 1.0)
        amp = np.abs(ax.Phi).sum(1)
        amp = np.concatenate([amp[::-1], amp])
    else:
        mom = np.abs(eq.gaussian_moments(N, 0.0, 1.0))
        amp = np.abs(ax.Phi).sum(1)
    jerr = 8 * np.finfo(float).eps * (np.abs(ax.C) @ mom).max()
    assert np.all(np.abs(g - ax.weights) <= jerr * amp + 4 * np.finfo(float).eps * ax.weights)


def test_shakhov_target_moments():
    """For N >= 6 on every axis the discrete F^eq(1+S) has density n, velocity u,
    pressure tensor n T delta_ab and heat flux (1 - Pr) q  [derived from Eq. sdef and the
    Gaussian moments <xi_a^2> = T, <xi^2 xi_a^2> = 5 T^2, <xi^4 xi_a^2> = 35 T^3]."""
    p = sv.Params(Qx=8, Qy=7, Qz=7, S=3, dt=1e-3, pr=2.0 / 3.0)
    m = sv.Model(p)
    n = np.array([0.9, 1.1, 1.0])
    u = (np.array([0.05, -0.1, 0.0]), np.array([0.3, -0.2, 0.1]), np.array([0.02, 0.0, -0.05]))
    T = np.array([1.1, 0.95, 1.2])
    q = (np.array([0.02, -0.01, 0.05]), np.array([-0.03, 0.04, 0.01]), np.array([0.0, 0.01, -0.02]))
    mom = sv.Moments(n, u, None, T, q)
    FS = sv.shakhov_target(mom, m)
    got = sv.moments(FS, m)
    assert np.allclose(got.n, n, rtol=1e-13)
    for a in range(3):
        assert np.allclose(got.u[a], u[a], rtol=0, atol=1e-13)
        assert np.allclose(got.q[a], (1 - p.pr) * q[a], rtol=0, atol=1e-13)
    assert np.allclose(got.T, T, rtol=1e-13)
    for key in ('xx', 'yy', 'zz'):
        assert np.allclose(got.P[key], n * T, rtol=1e-13)
    for key in ('xy', 'xz', 'yz'):
        assert np.allclose(got.P[key], 0.0, atol=1e-13)


def test_bgk_target_is_plain_maxwellian():
    p = sv.Params(Qx=4, Qy=4, Qz=4, S=2, dt=1e-3, pr=1.0)
    m = sv.Model(p)
    mom = sv.Moments(np.array([1.0, 1.2]), (np.zeros(2), np.array([0.1, 0.2]), np.zeros(2)), None,
                     np.array([1.0, 1.1]), (np.array([0.1, 0.0]), np.zeros(2), np.zeros(2)))
    FS = sv.shakhov_target(mom, m)
    assert np.array_equal(FS, m.vs.maxwellian(mom.n, *mom.u, mom.T))


def test_compensated_dot_meets_its_published_error_bound():
    """Dot2 (Ogita, Rump and Oishi 2005, their error bound for the twice-precision dot
    product): |res - s| <= eps |s| + gamma_n^2 sum |c_k m_k|, gamma_n = n eps / (1 - n eps),
    with s the exact sum of the double inputs (rational arithmetic), on the projection inputs
    at rest and at random states, where the terms cancel to 1e-17 of their size."""
    from fractions import Fraction
    from oracle import equilibrium as eq
    eps = 2.0 ** -53
    rng = np.random.default_rng(5)
    ax = eq.AxisProjection('half', 50, 6)
    states = [(0.0, 1.0)] + [(rng.uniform(-0.3, 0.3), rng.uniform(0.8, 1.2)) for _ in range(6)]
    for u, T in states:
        M = eq.half_gaussian_moments(6, u, T)
        J = eq.compensated_dot(ax.C, M)
        for l in range(7):
            exact = sum(Fraction(float(ax.C[l, k])) * Fraction(float(M[k])) for k in range(7))
            n = l + 1
            gam = n * eps / (1 - n * eps)
            bound = eps * abs(float(exact)) + gam ** 2 * float(np.abs(ax.C[l] * M).sum())
            assert abs(Fraction(float(J[l])) - exact) <= Fraction(bound), (u, T, l)


@pytest.mark.parametrize("Q", [4, 7, 16, 50])
def test_projected_factor_matches_exact_evaluation(Q):
    """The float64 half-range factor against its mpmath evaluation from the rule's unrounded
    nodes, weights and polynomials: the difference is the rounding of the tabulated
    coefficients C_lk and of the moments I_k, amplified by the outer nodes, and stays within
    2 eps sum_l |Phi_il| sum_k |C_lk I_k| + 2 eps |g_i| (first-order bound; measured at most
    0.56 of it with a factor 1), at rest and at moving states; at rest and Q = 4 it is a few
    ulp, at Q = 50 6.6e-8 relative at the outermost node."""
    from oracle import equilibrium as eq
    eps = 2.0 ** -53
    ax = eq.AxisProjection('half', Q, min(6, Q - 1))
    for u, T in ((0.0, 1.0), (0.05, 0.97), (-0.2, 1.1), (0.4, 1.3)):
        f, e = ax.factor(u, T), ax.factor_exact(u, T)
        for Mv, half in ((eq.half_gaussian_moments(ax.N, u, T), slice(Q, 2 * Q)),
                         (eq.half_gaussian_moments(ax.N, -u, T), slice(Q - 1, None, -1))):
            amp = np.abs(ax.Phi) @ (np.abs(ax.C) @ np.abs(Mv))
            bound = 2 * eps * amp + 2 * eps * np.abs(e[half])
            assert np.all(np.abs(f[half] - e[half]) <= bound), (u, T)
        if Q == 4 and u == 0.0:
            assert np.abs(f / e - 1).max() < 1e-14
