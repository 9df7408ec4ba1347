"""Oracle observables of the Couette solution (test infrastructure only).

Sec. IV: slip velocity by quadratic extrapolation to the wall (Eqs. uslip, uslip_extra),
centre-line derivative by the three-point even/odd formula (Eq. ud0_extra), half-channel
mass flow by the rectangle rule in eta (Eq. mflow) and its hydrodynamic value
(Eq. mflow_hydro), channel-averaged shear stress (Eq. Txy) and its ballistic value
(Eq. Txy_bal).  Sec. VI: velocity gradient nu (Eq. vgrad), reduced shear stress Pi
(Eq. stress) and centre temperature T_0 (Eq. T0).

``x`` are the node positions x_1..x_S of the grid; profiles are arrays over those nodes.
Pins: tests/test_oracle_diagnostics.py (exact on the polynomial profiles each formula is
built to reproduce).
"""
import math

import numpy as np


def wall_value(x, f, L=1.0):
    """f(L/2) from nodes S, S-1, S-2 by quadratic (Lagrange) extrapolation, Eq. uslip_extra."""
    xw = L / 2
    x1, x2, x3 = x[-1], x[-2], x[-3]
    return ((xw - x2) * (xw - x3) / ((x1 - x2) * (x1 - x3)) * f[-1]
            + (xw - x1) * (xw - x3) / ((x2 - x1) * (x2 - x3)) * f[-2]
            + (xw - x1) * (xw - x2) / ((x3 - x1) * (x3 - x2)) * f[-3])


def u_slip(x, uy, u_w, L=1.0):
    """Eq. uslip: u_w - u_y(L/2)."""
    return u_w - wall_value(x, uy, L)


def centre_derivative(x, f):
    """f'(0) for an odd profile from nodes 1, 2, 3 (Eq. ud0_extra)."""
    x1, x2, x3 = x[0], x[1], x[2]
    return (x2 ** 2 * x3 ** 2 * f[0] / (x1 * (x1 ** 2 - x2 ** 2) * (x1 ** 2 - x3 ** 2))
            + x1 ** 2 * x3 ** 2 * f[1] / (x2 * (x2 ** 2 - x1 ** 2) * (x2 ** 2 - x3 ** 2))
            + x1 ** 2 * x2 ** 2 * f[2] / (x3 * (x3 ** 2 - x1 ** 2) * (x3 ** 2 - x2 ** 2)))


def centre_value(x, f):
    """f(0) for an even profile from nodes 1, 2, 3 (Eq. T0)."""
    x1, x2, x3 = x[0], x[1], x[2]
    return (x2 ** 2 * x3 ** 2 * f[0] / ((x1 ** 2 - x2 ** 2) * (x1 ** 2 - x3 ** 2))
            + x3 ** 2 * x1 ** 2 * f[1] / ((x2 ** 2 - x1 ** 2) * (x2 ** 2 - x3 ** 2))
            + x1 ** 2 * x2 ** 2 * f[2] / ((x3 ** 2 - x1 ** 2) * (x3 ** 2 - x2 ** 2)))


def _eta_weights(S, A):
    """Rectangle-rule weights of Eq. mflow in eta, per unit length: artanh(A) / (A S cosh^2 eta_s);
    the equidistant grid (A -> 0) gives 1/S."""
    if A == 0.0:
        return np.full(S, 1.0 / S)
    eta = (np.arange(1, S + 1) - 0.5) * math.atanh(A) / S
    return math.atanh(A) / (A * S) / np.cosh(eta) ** 2


def mass_flow(n, uy, A, L=1.0):
    """Half-channel mass flow, Eq. mflow (m = 1, rho = n)."""
    return L / 2 * np.sum(_eta_weights(len(n), A) * n * uy)


def mass_flow_hydro(rho, u_w, L=1.0):
    """Eq. mflow_hydro: rho u_w L / 4."""
    return rho * u_w * L / 4


def mean_shear_stress(Txy, A):
    """Channel-averaged T_xy, Eq. Txy."""
    return np.sum(_eta_weights(len(Txy), A) * Txy)


def ballistic_shear_stress(rho, u_w, T_w=1.0):
    """Eq. Txy_bal with m = 1."""
    return -rho * u_w * math.sqrt(2 * T_w / math.pi)


def velocity_gradient(x, uy, u_w, L=1.0):
    """nu = (L / 2u_w) du_y/dx at x = 0, Eq. vgrad."""
    return L / (2 * u_w) * centre_derivative(x, uy)


def reduced_shear_stress(Txy_mean, u_w):
    """Pi = -T_xy / (u_w sqrt 2), Eq. stress."""
    return -Txy_mean / (u_w * math.sqrt(2))
