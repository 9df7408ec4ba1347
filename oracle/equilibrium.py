"""Oracle discrete equilibrium (test infrastructure only; see ``oracle/__init__``).

The paper builds the discrete equilibrium as a direct product of one-dimensional factors
(Sec. III, text after Eq. H_ortho): the Maxwellian factor along x is expanded in
half-range Hermite polynomials up to order N_x, each semi-axis separately, and the
factors along y (and here z) in full-range Hermite polynomials up to order N = Q - 1
(Eqs. fyz, Fmn_def, H_ortho).  Written out for one axis with weight omega, monic
orthogonal family P_l (norms gamma_l = int omega P_l^2) and Gauss rule (x_i, w_i):

    g^N(p)   = omega(p) * sum_{l<=N} (J_l / gamma_l) P_l(p),   J_l = int G(p) P_l(p) dp
    g_i      = w_i * g^N(x_i) / omega(x_i) = w_i * sum_{l<=N} P_l(x_i) J_l / gamma_l

with G(p; u, T) = exp(-(p-u)^2 / 2T) / sqrt(2 pi T) the 1D Maxwellian factor of Eq. phieq
(m = 1).  On a half axis the integral runs over that half only, so J_l is a combination
of the half-range Gaussian moments I_k = int_0^inf p^k G dp; on the full axis it is a
combination of the raw Gaussian moments E[X^k].  The discrete population is
F^eq_ijk = n g_{x,i} g_{y,j} g_{z,k}, and the Shakhov-corrected target is
F^eq (1 + S(xi)) with S from Eq. sdef evaluated at the discrete velocity.

Pins (tests/test_oracle_equilibrium.py): the closed-form I_k against mpmath numerical
integration; exact recovery sum_i g_i x_i^k = E[X^k] (and half sums = I_k) for k <= N;
g = w at u = 0, T = 1; Shakhov moments (density, momentum, energy unchanged; heat flux
scaled by Pr) for N >= 6.
"""
import math

import mpmath as mp
import numpy as np
from scipy.special import erfc

from . import quadrature as quad


def half_gaussian_moments(kmax, u, T):
    """I_k(u, T) = int_0^inf p^k exp(-(p-u)^2/2T)/sqrt(2 pi T) dp for k = 0..kmax.

    Closed form: I_0 = erfc(-u / sqrt(2T)) / 2, and integrating p G = u G - T G' by parts,
    I_1 = u I_0 + T G(0), I_k = u I_{k-1} + (k-1) T I_{k-2} for k >= 2.
    ``u`` and ``T`` may be arrays of equal shape; the result has a trailing axis k.
    """
    u = np.asarray(u, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    G0 = np.exp(-u * u / (2 * T)) / np.sqrt(2 * np.pi * T)
    out = np.empty(u.shape + (kmax + 1,))
    out[..., 0] = 0.5 * erfc(-u / np.sqrt(2 * T))
    if kmax >= 1:
        out[..., 1] = u * out[..., 0] + T * G0
    for k in range(2, kmax + 1):
        out[..., k] = u * out[..., k - 1] + (k - 1) * T * out[..., k - 2]
    return out


def gaussian_moments(kmax, u, T):
    """E[X^k] for X ~ N(u, T), k = 0..kmax (E[X^k] = u E[X^{k-1}] + (k-1) T E[X^{k-2}])."""
    u = np.asarray(u, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    out = np.empty(u.shape + (kmax + 1,))
    out[..., 0] = 1.0
    if kmax >= 1:
        out[..., 1] = u
    for k in range(2, kmax + 1):
        out[..., k] = u * out[..., k - 1] + (k - 1) * T * out[..., k - 2]
    return out


def _two_sum(a, b):
    """s + e = a + b exactly (Knuth's TwoSum)."""
    s = a + b
    bb = s - a
    return s, (a - (s - bb)) + (b - bb)


def _two_prod(a, b):
    """p + e = a b exactly (Dekker's TwoProduct with Veltkamp's splitting into 26-bit halves)."""
    p = a * b

    def split(x):
        c = 134217729.0 * x
        hi = c - (c - x)
        return hi, x - hi
    ah, al = split(a)
    bh, bl = split(b)
    return p, ((ah * bh - p) + ah * bl + al * bh) + al * bl


def compensated_dot(C, m):
    """J[..., l] = sum_k C[l, k] m[..., k] for every row l of C, each by Dot2 (Ogita, Rump and
    Oishi, SIAM J. Sci. Comput. 26 (2005)): exact products and exact two-term sums over
    k = 0, 1, ..., the rounding errors accumulated on the side, so the result is as accurate
    as a dot product carried out in twice the working precision.  The projection
    coefficients need it: J_l = sum_k C_lk I_k cancels (at rest it vanishes for l >= 1 while
    its terms reach 1e3), and the outer half-range nodes multiply what is left by up to 1e7
    (Qx = 50), so a plain sum's rounding would be the largest error of the equilibrium there.
    (C is lower triangular; its zero entries add exact zeros.)"""
    h, r = _two_prod(C, m[..., None, :])          # (..., l, k)
    p, s = h[..., 0], r[..., 0]
    for k in range(1, C.shape[1]):
        p, q = _two_sum(p, h[..., k])
        s = s + (q + r[..., k])
    return p + s


def monic_coefficients(a, b, N, dps):
    """Monomial coefficients C[l, k] of the monic orthogonal P_l (l <= N) and their norms
    gamma_l = b_0 b_1 ... b_l, from the recurrence P_{l+1} = (p - a_l) P_l - b_l P_{l-1}."""
    with mp.workdps(dps):
        C = [[mp.mpf(0)] * (N + 1) for _ in range(N + 1)]
        C[0][0] = mp.mpf(1)
        if N >= 1:
            C[1][0] = -a[0]
            C[1][1] = mp.mpf(1)
        for l in range(1, N):
            for k in range(N + 1):
                v = -a[l] * C[l][k] - b[l] * C[l - 1][k]
                if k > 0:
                    v += C[l][k - 1]
                C[l + 1][k] = v
        gam = [b[0]]
        for l in range(1, N + 1):
            gam.append(gam[-1] * b[l])
        return C, gam


class AxisProjection:
    """Projection of a 1D Maxwellian onto one Gauss-Hermite axis.

    ``kind`` is 'half' (x axis: nodes -p_Q..-p_1, p_1..p_Q, each semi-axis projected on
    its own half-range family) or 'full' (y, z axes).
    """

    def __init__(self, kind, Q, N):
        self.kind, self.Q, self.N = kind, Q, N
        if kind == 'half':
            x, w, a, b, dps = quad.half_range_rule_mp(Q)
        else:
            x, w, a, b, dps = quad.full_range_rule_mp(Q)
        if N > Q - 1 or N < 0:
            raise ValueError("expansion order must satisfy 0 <= N <= Q-1")
        C, gam = monic_coefficients(a, b, N, dps)
        with mp.workdps(dps):
            # Phi[i, l] = w_i P_l(x_i) / gamma_l on the rule's own nodes
            Phi = [[w[i] * mp.fsum(C[l][k] * x[i] ** k for k in range(l + 1)) / gam[l]
                    for l in range(N + 1)] for i in range(Q)]
        self._mp = (x, w, C, gam, dps)
        self.C = np.array([[float(v) for v in row] for row in C])  # (N+1, N+1)
        self.Phi = np.array([[float(v) for v in row] for row in Phi])  # (Q, N+1)
        if kind == 'half':
            self.nodes, self.weights = quad.x_axis(Q)
        else:
            self.nodes, self.weights = quad.full_range_rule(Q)

    def factor(self, u, T):
        """Discrete factor g_i(u, T); u, T arrays of shape (...), result (..., nodes)."""
        u = np.asarray(u, dtype=np.float64)
        T = np.asarray(T, dtype=np.float64)
        if self.kind == 'full':
            J = gaussian_moments(self.N, u, T) @ self.C.T           # J_l = sum_k C_lk E[X^k]
            return J @ self.Phi.T
        # positive semi-axis: J+_l = int_0^inf G(p) P_l(p) dp = sum_k C_lk I_k(u, T)
        # negative semi-axis, node -x_i: J-_l = int_0^inf G(-p) P_l(p) dp = sum_k C_lk I_k(-u, T)
        # (compensated sums over k <= l: see compensated_dot)
        Ip = half_gaussian_moments(self.N, u, T)
        Im = half_gaussian_moments(self.N, -u, T)
        Jp = compensated_dot(self.C, Ip)
        Jm = compensated_dot(self.C, Im)
        gp = Jp @ self.Phi.T            # nodes x_1 .. x_Q (ascending)
        gm = (Jm @ self.Phi.T)[..., ::-1]  # nodes -x_Q .. -x_1 (ascending)
        return np.concatenate([gm, gp], axis=-1)


    def factor_exact(self, u, T):
        """The same discrete factor g_i(u, T) for scalar u, T, evaluated in mpmath at the rule's
        working precision from the rule's own (unrounded) nodes, weights and polynomials, and
        rounded once to float64: the reference the float64 evaluations are measured against
        (their error is the rounding of J_l = sum_k C_lk M_k amplified by P_l at the outer
        nodes, which reaches 1e-9 relative at Qx = 50)."""
        x, w, C, gam, dps = self._mp
        N = self.N
        with mp.workdps(dps):
            u, T = mp.mpf(u), mp.mpf(T)

            def moments(uu):
                # I_k (half) or E[X^k] (full) for X ~ N(uu, T), k <= N, by the recursions of
                # half_gaussian_moments / gaussian_moments, in mpmath
                m = [mp.mpf(0)] * (N + 1)
                if self.kind == 'half':
                    m[0] = mp.erfc(-uu / mp.sqrt(2 * T)) / 2
                    if N >= 1:
                        m[1] = uu * m[0] + T * mp.exp(-uu * uu / (2 * T)) / mp.sqrt(2 * mp.pi * T)
                else:
                    m[0] = mp.mpf(1)
                    if N >= 1:
                        m[1] = uu
                for k in range(2, N + 1):
                    m[k] = uu * m[k - 1] + (k - 1) * T * m[k - 2]
                return m

            def g(nodes, J):
                return [w[i] * mp.fsum(mp.fsum(C[l][k] * nodes[i] ** k for k in range(l + 1)) * J[l] / gam[l]
                                       for l in range(N + 1)) for i in range(len(nodes))]

            def coeffs(uu):
                M = moments(uu)
                return [mp.fsum(C[l][k] * M[k] for k in range(l + 1)) for l in range(N + 1)]

            if self.kind == 'full':
                return np.array([float(v) for v in g(x, coeffs(u))])
            gp = g(x, coeffs(u))
            gm = g(x, coeffs(-u))[::-1]
            return np.array([float(v) for v in gm + gp])


class VelocitySet:
    """Product velocity set p_ijk = (p_x,i, p_y,j, p_z,k), i < 2Qx, j < Qy, k < Qz, with
    flat index v = (i Qy + j) Qz + k, and the Hermite-projected equilibrium on it."""

    def __init__(self, Qx, Qy, Qz, Nx=None, Ny=None, Nz=None):
        Nx = min(6, Qx - 1) if Nx is None else Nx
        Ny = Qy - 1 if Ny is None else Ny
        Nz = Qz - 1 if Nz is None else Nz
        self.Qx, self.Qy, self.Qz = Qx, Qy, Qz
        self.Nx, self.Ny, self.Nz = Nx, Ny, Nz
        self.X = AxisProjection('half', Qx, Nx)
        self.Y = AxisProjection('full', Qy, Ny)
        self.Z = AxisProjection('full', Qz, Nz)
        self.V = 2 * Qx * Qy * Qz
        px, py, pz = np.meshgrid(self.X.nodes, self.Y.nodes, self.Z.nodes, indexing='ij')
        self.px, self.py, self.pz = px.ravel(), py.ravel(), pz.ravel()

    def maxwellian(self, n, ux, uy, uz, T):
        """F^eq[..., v] = n g_x,i(u_x, T) g_y,j(u_y, T) g_z,k(u_z, T)."""
        gx = self.X.factor(ux, T)
        gy = self.Y.factor(uy, T)
        gz = self.Z.factor(uz, T)
        n = np.asarray(n, dtype=np.float64)
        prod = n[..., None, None, None] * gx[..., :, None, None] * gy[..., None, :, None] * gz[..., None, None, :]
        return prod.reshape(prod.shape[:-3] + (self.V,))

    def shakhov_factor(self, n, u, T, q, pr):
        """S(xi_v) of Eq. sdef (m = k_B = 1): (1-Pr)/(n T^2) (xi^2/(5T) - 1) q.xi, per velocity.
        ``u`` and ``q`` are tuples of three arrays of the cell shape."""
        xi = [self.px - u[0][..., None], self.py - u[1][..., None], self.pz - u[2][..., None]]
        xi2 = xi[0] ** 2 + xi[1] ** 2 + xi[2] ** 2
        qxi = q[0][..., None] * xi[0] + q[1][..., None] * xi[1] + q[2][..., None] * xi[2]
        n = np.asarray(n)[..., None]
        T = np.asarray(T)[..., None]
        return (1.0 - pr) / (n * T ** 2) * (xi2 / (5.0 * T) - 1.0) * qxi
