"""Oracle quadrature rules (test infrastructure only; see ``oracle/__init__``).

Half-range Gauss-Hermite rule (paper Sec. I and Sec. III: Q nodes per semi-axis recover
the half-space moments up to order N = Q - 1; the construction itself is in the
authors' earlier work and is restated here from the definition of a Gauss rule):

* weight function on [0, inf): omega(p) = exp(-p^2/2) / sqrt(2 pi)   (Eq. H_omega)
* its moments are known in closed form:
      mu_k = int_0^inf p^k omega(p) dp = 2^((k-1)/2) Gamma((k+1)/2) / sqrt(2 pi)
* the monic orthogonal polynomials P_k obey P_{k+1} = (p - a_k) P_k - b_k P_{k-1};
  (a_k, b_k) follow from the moments by Chebyshev's algorithm, run in mpmath at a
  working precision high enough to absorb its ill-conditioning;
* nodes are the zeros of P_Q (Newton-polished in mpmath), weights are the Christoffel
  numbers w_i = 1 / sum_{k<Q} P_k(x_i)^2 / (b_0 b_1 ... b_k).

Full-range rule on y and z: the same construction for omega on the whole real line
(probabilists' Hermite polynomials He_k, Eq. H_ortho), whose moments are
mu_{2m} = (2m-1)!!, mu_{odd} = 0, so the weights sum to one.

Pins (tests/test_oracle_quadrature.py): half-range rule integrates p^k exactly against
the closed-form mu_k for k <= 2Q-1; full-range rule equals numpy's hermegauss / sqrt(2 pi);
node symmetry; Q=1 closed form.
"""
from functools import lru_cache

import mpmath as mp
import numpy as np


def _work_dps(Q):
    # Chebyshev's algorithm loses roughly a fixed number of digits per degree on this
    # weight; 40 guard digits plus 2 per node keeps > 30 correct digits for Q <= 128
    # (checked in the tests by comparing two precisions).
    return 40 + 2 * Q


def half_range_moments(n, dps):
    """mu_k = int_0^inf p^k exp(-p^2/2)/sqrt(2 pi) dp for k = 0..n-1 (closed form)."""
    with mp.workdps(dps):
        c = 1 / mp.sqrt(2 * mp.pi)
        return [c * mp.power(2, mp.mpf(k - 1) / 2) * mp.gamma(mp.mpf(k + 1) / 2) for k in range(n)]


def full_range_moments(n, dps):
    """mu_k = int_R p^k exp(-p^2/2)/sqrt(2 pi) dp: (k-1)!! for even k, 0 for odd k."""
    with mp.workdps(dps):
        out = []
        for k in range(n):
            if k % 2:
                out.append(mp.mpf(0))
            else:
                out.append(mp.fac2(k - 1) if k > 0 else mp.mpf(1))
        return out


def chebyshev_recurrence(mom, n, dps):
    """Recurrence coefficients (a_k, b_k), k < n, of the monic orthogonal polynomials of a
    measure from its first 2n moments (Chebyshev's algorithm; b_0 = mu_0)."""
    with mp.workdps(dps):
        a = [mp.mpf(0)] * n
        b = [mp.mpf(0)] * n
        sig_prev = [mp.mpf(0)] * (2 * n)          # sigma_{-1, l}
        sig = [mp.mpf(m) for m in mom[:2 * n]]     # sigma_{0, l} = mu_l
        a[0] = sig[1] / sig[0]
        b[0] = sig[0]
        for k in range(1, n):
            new = [mp.mpf(0)] * (2 * n)
            for l in range(k, 2 * n - k):
                new[l] = sig[l + 1] - a[k - 1] * sig[l] - b[k - 1] * sig_prev[l]
            a[k] = new[k + 1] / new[k] - sig[k] / sig[k - 1]
            b[k] = new[k] / sig[k - 1]
            sig_prev, sig = sig, new
        return a, b


def _monic_values(x, a, b, upto):
    """P_0(x) .. P_upto(x) of the monic family with recurrence (a, b)."""
    vals = [mp.mpf(1), x - a[0]]
    for k in range(1, upto):
        vals.append((x - a[k]) * vals[k] - b[k] * vals[k - 1])
    return vals[:upto + 1]


def gauss_rule(a, b, Q, dps):
    """Nodes (zeros of P_Q) and Christoffel weights of the Q-point Gauss rule."""
    # initial guesses: eigenvalues of the Jacobi matrix in float64
    J = np.diag([float(v) for v in a[:Q]])
    off = [float(mp.sqrt(v)) for v in b[1:Q]]
    J += np.diag(off, 1) + np.diag(off, -1)
    guesses = np.sort(np.linalg.eigvalsh(J)) if Q > 1 else np.array([float(a[0])])
    nodes, weights = [], []
    with mp.workdps(dps):
        norms = [b[0]]
        for k in range(1, Q):
            norms.append(norms[-1] * b[k])
        for g in guesses:
            x = mp.mpf(g)
            for _ in range(100):
                # Newton on P_Q using P_Q' from the differentiated recurrence
                p0, p1 = mp.mpf(1), x - a[0]
                d0, d1 = mp.mpf(0), mp.mpf(1)
                for k in range(1, Q):
                    p0, p1 = p1, (x - a[k]) * p1 - b[k] * p0
                    d0, d1 = d1, p0 + (x - a[k]) * d1 - b[k] * d0
                step = p1 / d1
                x -= step
                if abs(step) <= abs(x) * mp.mpf(10) ** (-dps + 8) + mp.mpf(10) ** (-dps + 8):
                    break
            vals = _monic_values(x, a, b, Q - 1)
            w = 1 / mp.fsum(vals[k] ** 2 / norms[k] for k in range(Q))
            nodes.append(x)
            weights.append(w)
    return nodes, weights


@lru_cache(maxsize=None)
def half_range_rule_mp(Q):
    """Half-range rule in mpmath precision: (nodes, weights, a, b, dps), ascending nodes > 0,
    weights summing to mu_0 = 1/2."""
    dps = _work_dps(Q)
    mom = half_range_moments(2 * Q + 2, dps)
    a, b = chebyshev_recurrence(mom, Q + 1, dps)
    x, w = gauss_rule(a, b, Q, dps)
    return x, w, a, b, dps


@lru_cache(maxsize=None)
def full_range_rule_mp(Q):
    """Full-range (probabilists') Gauss-Hermite rule in mpmath precision."""
    dps = _work_dps(Q)
    mom = full_range_moments(2 * Q + 2, dps)
    a, b = chebyshev_recurrence(mom, Q + 1, dps)
    x, w = gauss_rule(a, b, Q, dps)
    return x, w, a, b, dps


def half_range_rule(Q):
    """float64 nodes and weights on the positive semi-axis (ascending), sum(w) = 1/2."""
    x, w, _, _, _ = half_range_rule_mp(Q)
    return np.array([float(v) for v in x]), np.array([float(v) for v in w])


def full_range_rule(Q):
    """float64 full-range nodes (ascending, exactly antisymmetric) and weights (sum 1)."""
    x, w, _, _, _ = full_range_rule_mp(Q)
    xs = np.array([float(v) for v in x])
    ws = np.array([float(v) for v in w])
    # the mp nodes are symmetric to working precision; enforce it bitwise in float64
    xs = 0.5 * (xs - xs[::-1])
    ws = 0.5 * (ws + ws[::-1])
    return xs, ws


def x_axis(Qx):
    """The 2Qx nodes on the whole x axis, ascending: (-p_Q..-p_1, p_1..p_Q), and weights."""
    p, w = half_range_rule(Qx)
    return np.concatenate([-p[::-1], p]), np.concatenate([w[::-1], w])
