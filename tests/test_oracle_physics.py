"""Integration pins of the oracle time step against what the paper and the mathematics fix:
a gas at rest stays at rest, mass is conserved (bounce-back centre line, diffuse wall with
zero net mass flux, App. A.4), and the collisionless Couette problem has the closed-form
free-molecular solution (paper Eq. Txy_bal and its companions, derived in the test)."""
import math

import numpy as np
import pytest

from oracle import solver as sv

SPLIT = np.random.default_rng(11)


def seeded(m, eps=0.05, seed=3):
    r = np.random.default_rng(seed).uniform(-1, 1, size=(m.p.S, m.V))
    return sv.seeded_state(m, r, eps)


@pytest.mark.parametrize("scheme,pr,law,A", [('upwind2', 1.0, 'power', 0.0), ('weno5', 2 / 3, 'power', 0.98),
                                             ('weno5', 2 / 3, 'sutherland', 0.0)])
def test_gas_at_rest_stays_at_rest(scheme, pr, law, A):
    p = sv.Params(Qx=4, Qy=4, Qz=4, S=12, dt=2e-3 if A == 0 else 2e-4, kn=0.3, u_w=0.0, pr=pr, law=law,
                  omega=0.5, suth_S=0.5239, A=A, scheme=scheme)
    m = sv.Model(p)
    F0 = sv.equilibrium_state(m)
    F = sv.run(F0, m, 300)
    assert np.abs(F - F0).max() / F0.max() < 1e-13
    mom = sv.moments(F, m)
    assert np.abs(mom.u[1]).max() < 1e-14 and np.abs(mom.u[0]).max() < 1e-14


@pytest.mark.parametrize("scheme,A,pr", [('upwind2', 0.0, 1.0), ('weno5', 0.98, 2 / 3), ('upwind2', 0.5, 2 / 3)])
def test_mass_conservation(scheme, A, pr):
    # (the ideal-weight 'linear5' switch is excluded: without the Table II limit its incoming
    # wall flux is not p_x n_w F^eq_w, so the wall density formula of App. A.4 does not make
    # the net wall flux vanish)
    p = sv.Params(Qx=5, Qy=4, Qz=4, S=14, dt=2e-4, kn=0.2, u_w=0.5, pr=pr, A=A, scheme=scheme)
    m = sv.Model(p)
    F = seeded(m)
    mass0 = math.fsum((m.dx[:, None] * F).ravel())
    for _ in range(4):
        F = sv.run(F, m, 25)
        assert math.fsum((m.dx[:, None] * F).ravel()) == pytest.approx(mass0, rel=1e-13)


def test_boundary_fluxes_carry_no_mass():
    p = sv.Params(Qx=6, Qy=5, Qz=3, S=10, dt=1e-4, kn=0.1, u_w=0.4, pr=2 / 3, A=0.9, scheme='weno5')
    m = sv.Model(p)
    F = seeded(m)
    G, n_w = sv.build_ghosts(F, m)
    phi = sv.stencil_fluxes(G, m.vs.px, 'weno5', 0, p.S)
    # centre line: the bounce-back pairs carry opposite fluxes
    assert np.array_equal(phi[0], -phi[0][m.mirror])
    # wall: zero net mass flux, incoming flux is exactly p_x n_w F^eq_w (Table II limit)
    assert abs(math.fsum(phi[-1])) < 1e-15 * np.abs(phi[-1]).sum()
    assert np.allclose(phi[-1][m.neg], m.vs.px[m.neg] * n_w * m.g_wall[m.neg], rtol=1e-15, atol=0)


def free_molecular_state(m):
    """x-uniform collisionless steady state: populations leaving the wall (p_x < 0) are the
    wall Maxwellian; those with p_x > 0 are their bounce-back images."""
    f = np.where(m.neg, m.g_wall, m.g_wall[m.mirror])
    return np.tile(f, (m.p.S, 1))


def closed_form(u_w):
    # derived: n = 1, u = 0, T = 1 + u_w^2/3, P_xx = P_zz = 1, P_yy = 1 + u_w^2,
    # P_xy = -u_w sqrt(2/pi) (= T_xy^bal of Eq. Txy_bal with rho = T_w = 1), q = 0
    return {'n': 1.0, 'T': 1 + u_w ** 2 / 3, 'xx': 1.0, 'yy': 1 + u_w ** 2, 'zz': 1.0,
            'xy': -u_w * math.sqrt(2 / math.pi)}


@pytest.mark.parametrize("scheme,A", [('weno5', 0.98), ('upwind2', 0.0)])
def test_free_molecular_fixed_point(scheme, A):
    u_w = 0.4
    p = sv.Params(Qx=6, Qy=5, Qz=5, S=10, dt=1e-4, u_w=u_w, A=A, scheme=scheme, collisionless=True)
    m = sv.Model(p)
    F0 = free_molecular_state(m)
    F = sv.run(F0, m, 50)
    assert np.abs(F - F0).max() / F0.max() < 1e-13
    mom = sv.moments(F, m)
    cf = closed_form(u_w)
    assert np.allclose(mom.n, cf['n'], rtol=1e-13)
    assert np.allclose(mom.T, cf['T'], rtol=1e-13)
    for k in ('xx', 'yy', 'zz', 'xy'):
        assert np.allclose(mom.P[k], cf[k], rtol=1e-13), k
    for a in range(3):
        assert np.abs(mom.q[a]).max() < 1e-13 and np.abs(mom.u[a]).max() < 1e-13


def test_collisionless_run_converges_to_free_molecular_solution():
    u_w = 0.2
    p = sv.Params(Qx=4, Qy=4, Qz=4, S=8, dt=1e-2, u_w=u_w, A=0.0, scheme='upwind2', collisionless=True)
    m = sv.Model(p)
    F, steps, R = sv.run_to_steady(sv.equilibrium_state(m), m, tol=1e-11, max_steps=20000)
    assert R < 1e-11
    mom = sv.moments(F, m)
    cf = closed_form(u_w)
    assert np.allclose(mom.n, cf['n'], rtol=1e-9)
    assert np.allclose(mom.T, cf['T'], rtol=1e-9)
    assert np.allclose(mom.P['xy'], cf['xy'], rtol=1e-9)
    # Pi = -T_xy / (u_w sqrt 2) (Eq. stress) -> 1/sqrt(pi)
    assert np.allclose(-mom.P['xy'] / (u_w * math.sqrt(2)), 1 / math.sqrt(math.pi), rtol=1e-9)


def test_lowmach_law_is_constant_and_gives_linear_response():
    """Sec. IV: at wall speeds ~1e-5 the flow is the linear response of the gas at rest, with
    tau = k / sqrt(2) (Eq. knLuo) independent of n and T, on HHLB(N_x; Q_x) x HLB(1; 2)."""
    base = dict(Qx=4, Qy=2, Qz=1, S=8, dt=2e-3, kn=0.5, pr=1.0, law='lowmach', scheme='upwind2')
    p = sv.Params(u_w=1e-5, **base)
    tau = sv.relaxation_time(np.array([0.5, 1.0, 2.0]), np.array([0.7, 1.0, 1.9]), p)
    assert np.all(tau == 0.5 / np.sqrt(2.0))
    prof = []
    for u in (1e-5, 2e-5):
        m = sv.Model(sv.Params(u_w=u, **base))
        F = sv.run(sv.equilibrium_state(m), m, 400)
        prof.append(sv.moments(F, m).u[1] / u)
    assert np.abs(prof[0]).max() > 0.05
    assert np.abs(prof[0] - prof[1]).max() <= 1e-4 * np.abs(prof[0]).max()
