"""Pins of the Sec. IV / VI observables on profiles they reproduce exactly."""
import math

import numpy as np
import pytest

from oracle import diagnostics as dg
from oracle import solver as sv


@pytest.mark.parametrize("A", [0.0, 0.98])
def test_wall_extrapolation_exact_on_quadratics(A):
    x = sv.Grid(16, A).x(np.arange(1, 17))
    f = 0.3 + 1.1 * x - 2.0 * x * x
    assert dg.wall_value(x, f) == pytest.approx(0.3 + 0.55 - 0.5, rel=1e-13)
    assert dg.u_slip(x, f, 1.0) == pytest.approx(1 - 0.35, rel=1e-12)


@pytest.mark.parametrize("A", [0.0, 0.98])
def test_centre_formulas_exact_on_odd_and_even_polynomials(A):
    x = sv.Grid(16, A).x(np.arange(1, 17))
    odd = 0.7 * x - 1.3 * x ** 3 + 2.1 * x ** 5     # sixth order for odd profiles
    even = 1.2 + 0.4 * x ** 2 - 0.9 * x ** 4
    assert dg.centre_derivative(x, odd) == pytest.approx(0.7, rel=1e-11)
    assert dg.centre_value(x, even) == pytest.approx(1.2, rel=1e-12)
    assert dg.velocity_gradient(x, odd, 0.35) == pytest.approx(0.7 / 0.7, rel=1e-11)


def test_mass_flow_and_mean_stress():
    S, A = 400, 0.98
    x = sv.Grid(S, A).x(np.arange(1, S + 1))
    # hydrodynamic profile u = 2 u_w x / L -> m_dot = rho u_w L / 4 (Eq. mflow_hydro)
    u_w = 0.3
    assert dg.mass_flow(np.ones(S), 2 * u_w * x, A) == pytest.approx(dg.mass_flow_hydro(1.0, u_w), rel=1e-4)
    # constant stress averages to itself; uniform grid limit
    assert dg.mean_shear_stress(np.full(S, -0.2), A) == pytest.approx(-0.2, rel=1e-4)
    assert dg.mean_shear_stress(np.full(8, -0.2), 0.0) == pytest.approx(-0.2, rel=1e-15)
    # ballistic stress and Pi = 1/sqrt(pi) in the free-molecular limit
    Tb = dg.ballistic_shear_stress(1.0, u_w)
    assert dg.reduced_shear_stress(Tb, u_w) == pytest.approx(1 / math.sqrt(math.pi), rel=1e-15)
