"""Pins of the oracle's space-time discretisation (paper App. A): WENO-5 (Eqs. weno5_flux,
weno5_omega, weno_sigma, Table II), second-order upwind, TVD RK3 (Eq. rk3, Table rk3),
tanh grid (Eqs. stretch, etas) and the quadratic ghost extrapolation (App. A.4)."""
import math

import numpy as np
import pytest

from oracle import solver as sv

RNG = np.random.default_rng(20170204)


def weno(a, b, c, d, e, scheme='weno5', px=1.0):
    return sv.interface_flux(*(np.asarray(t, dtype=float) for t in (a, b, c, d, e)), px, scheme)


def test_ideal_weights_give_textbook_five_point_flux():
    # 0.1 f1 + 0.6 f2 + 0.3 f3 is the fifth-order upwind-biased interpolation
    # (2 F_{s-2} - 13 F_{s-1} + 47 F_s + 27 F_{s+1} - 3 F_{s+2}) / 60
    v = RNG.normal(size=(5, 100))
    ref = (2 * v[0] - 13 * v[1] + 47 * v[2] + 27 * v[3] - 3 * v[4]) / 60
    assert np.allclose(weno(*v, scheme='linear5'), ref, rtol=1e-14, atol=1e-15)


def test_table_II_rows_are_limits_of_the_weight_formula():
    """Each row of Table II is the limit of Eq. weno5_omega as the listed indicators go to
    zero together (checked with the quotient formula at sigma = 1e-150 instead of 0)."""
    tiny = 1e-150
    for key, vals in sv.WENO_LIMITS.items():
        sig = [tiny if q in key else RNG.uniform(0.5, 2.0) for q in range(3)]
        d = sv.WENO_DELTA
        wt = [d[q] / sig[q] ** 2 if sig[q] > tiny else d[q] / tiny / tiny for q in range(3)]
        # exact limit with equal tiny sigmas: the non-vanishing ones drop out
        tot = sum(wt)
        lim = [t / tot for t in wt]
        assert np.allclose(lim, vals, atol=1e-12), key
        got = sv.weno5_weights(*(np.array([0.0 if q in key else sig[q]]) for q in range(3)))
        assert np.allclose([g[0] for g in got], vals, rtol=0, atol=1e-15), key


def test_flat_stencils_select_table_rows():
    # sigma_q = 0 exactly iff candidate stencil q is constant
    w = sv.weno5_weights(*(np.array([x]) for x in (0.0, 1.0, 2.0)))
    assert [x[0] for x in w] == [1.0, 0.0, 0.0]
    # b = c = d = e, a different: sigma_2 = sigma_3 = 0 -> (0, 2/3, 1/3)
    a, b = 3.0, 1.0
    f = weno([a], [b], [b], [b], [b])
    assert f[0] == pytest.approx(b, rel=1e-15)


def test_weno_matches_quotient_definition_on_random_data():
    v = RNG.normal(size=(5, 1000))
    a, b, c, d, e = v
    s1 = 13 / 12 * (a - 2 * b + c) ** 2 + 0.25 * (a - 4 * b + 3 * c) ** 2
    s2 = 13 / 12 * (b - 2 * c + d) ** 2 + 0.25 * (b - d) ** 2
    s3 = 13 / 12 * (c - 2 * d + e) ** 2 + 0.25 * (3 * c - 4 * d + e) ** 2
    wt = [0.1 / s1 ** 2, 0.6 / s2 ** 2, 0.3 / s3 ** 2]
    tot = wt[0] + wt[1] + wt[2]
    f1 = a / 3 - 7 * b / 6 + 11 * c / 6
    f2 = -b / 6 + 5 * c / 6 + d / 3
    f3 = c / 3 + 5 * d / 6 - e / 6
    ref = (wt[0] * f1 + wt[1] * f2 + wt[2] * f3) / tot
    assert np.allclose(weno(*v), ref, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("scale_exp", [-450, -300, -170, -60, 0, 60, 300])
def test_weno_scale_homogeneity_bitwise(scale_exp):
    """Without the customary epsilon the scheme is homogeneous of degree one; power-of-two
    scaling is exact in floating point, so the flux must scale bitwise (App. A.3) as long
    as the indicators stay normal numbers (|F| above ~1e-150; the smallest population of
    the 50-node-per-half set is ~1e-52)."""
    v = np.abs(RNG.normal(size=(5, 400))) + 0.1
    base = weno(*v)
    sc = 2.0 ** scale_exp
    assert np.array_equal(weno(*(v * sc)), base * sc)


def test_weno_mirror_symmetry():
    # the p_x < 0 flux on a field equals minus the p_x > 0 flux on the mirrored field
    S = 20
    G = np.abs(RNG.normal(size=(S + 6, 1))) + 0.5
    fp = sv.stencil_fluxes(G, np.array([1.3]), 'weno5', 2, S - 2)
    Gm = G[::-1].copy()
    fm = sv.stencil_fluxes(Gm, np.array([-1.3]), 'weno5', 2, S - 2)
    # interface s+1/2 of G is interface (S+1-s)-1/2 ... in mirrored indices: t = S - s
    assert np.allclose(fp[::-1, 0], -fm[:, 0], rtol=1e-14)


@pytest.mark.parametrize("scheme,order", [('weno5', 5), ('linear5', 5), ('upwind2', 2)])
def test_convergence_order_on_smooth_monotone_data(scheme, order):
    """Flux-form derivative of a smooth profile without critical points: error ratio on
    grid halving approaches 2^order (weights tend to the ideal ones)."""
    errs = []
    for S in (10, 20, 40):
        h = 1.0 / S
        xc = (np.arange(-2, S + 4) - 0.5) * h          # node t at (t - 1/2) h, t = -2..S+3
        f = lambda x: np.exp(0.8 * x) + 0.3 * x
        Fint = lambda x: np.exp(0.8 * x) / 0.8 + 0.15 * x * x
        # cell averages -> WENO reconstructs point values at interfaces
        Gc = ((Fint(xc + h / 2) - Fint(xc - h / 2)) / h)[:, None]
        phi = sv.stencil_fluxes(Gc, np.array([1.0]), scheme, 0, S)[:, 0]
        xi = np.arange(0, S + 1) * h
        errs.append(np.abs(phi - f(xi)).max())
    for k in range(2):
        assert errs[k] / errs[k + 1] == pytest.approx(2 ** order, rel=0.1), errs


def test_rk3_stability_polynomial():
    # dF/dt = lam F: one step multiplies F by 1 + z + z^2/2 + z^3/6, z = lam dt (Table rk3)
    for z in (0.3, -1.2, 1.5 + 0.7j, -0.4 + 2.0j):
        lam, dt = z / 0.01, 0.01
        got = sv.rk3(np.array([1.0 + 0j]), lambda F: lam * F, dt)[0]
        assert got == pytest.approx(1 + z + z * z / 2 + z ** 3 / 6, rel=1e-14)


def test_rk3_is_third_order():
    # nonlinear ODE dF/dt = -F^2, F(0) = 1, exact 1/(1+t)
    errs = []
    for nsteps in (20, 40, 80):
        dt = 1.0 / nsteps
        F = np.array([1.0])
        for _ in range(nsteps):
            F = sv.rk3(F, lambda G: -G * G, dt)
        errs.append(abs(F[0] - 0.5))
    assert errs[0] / errs[1] == pytest.approx(8, rel=0.1)
    assert errs[1] / errs[2] == pytest.approx(8, rel=0.1)


@pytest.mark.parametrize("A", [0.0, 0.5, 0.98])
def test_grid(A):
    S = 16
    g = sv.Grid(S, A)
    s = np.arange(1, S + 1)
    # interfaces of node 1 and node S are the centre line and the wall
    assert g.x(0.5) == 0.0
    assert g.x(S + 0.5) == pytest.approx(0.5, rel=1e-15)
    assert math.fsum(g.widths()) == pytest.approx(0.5, rel=1e-14)
    assert np.all(np.diff(g.x(s)) > 0)
    if A > 0:
        assert np.allclose(g.x(s), np.tanh((s - 0.5) * np.arctanh(A) / S) / (2 * A), rtol=1e-15)
        # stretching refines towards the wall
        assert g.widths()[-1] < g.widths()[0]


def test_small_A_tends_to_uniform_grid():
    S = 10
    s = np.arange(1, S + 1)
    assert np.allclose(sv.Grid(S, 1e-6).x(s), sv.Grid(S, 0.0).x(s), rtol=1e-10)


@pytest.mark.parametrize("A", [0.0, 0.98])
def test_extrapolation_exact_on_quadratics(A):
    p = sv.Params(Qx=2, Qy=2, Qz=2, S=12, dt=1e-3, A=A)
    m = sv.Model(p)
    quadf = lambda x: 1.7 - 2.3 * x + 4.1 * x * x
    for s in (p.S + 1, p.S + 2):
        c1, c2, c3 = m.extrap[s]
        got = c1 * quadf(m.grid.x(s - 1)) + c2 * quadf(m.grid.x(s - 2)) + c3 * quadf(m.grid.x(s - 3))
        assert got == pytest.approx(quadf(m.grid.x(s)), rel=1e-12)
