"""Pins of the warm-start reconstruction oracle: the seed reproduces the profiles it was
built from when the equilibrium is exact to order 6 (Gaussian moment identities), reduces
to the discrete equilibrium without stress and heat flux, and its heat-flux term scaled by
(1 - Pr) is the Shakhov factor of Eq. sdef."""
import numpy as np
import pytest

from oracle import solver as sv
from oracle import warmstart as ws
from oracle.equilibrium import VelocitySet


def random_table(rng, S):
    n = rng.uniform(0.8, 1.2, S)
    uy = rng.uniform(-0.3, 0.3, S)
    T = rng.uniform(0.9, 1.1, S)
    Pxx = n * T * (1 + rng.uniform(-0.05, 0.05, S))
    Pyy = n * T * (1 + rng.uniform(-0.05, 0.05, S))
    Pxy = rng.uniform(-0.05, 0.05, S)
    qx = rng.uniform(-0.05, 0.05, S)
    qy = rng.uniform(-0.05, 0.05, S)
    return ws.table_from_profiles(np.stack([n, uy, T, Pxx, Pxy, Pyy, qx, qy], axis=-1))


def test_seed_reproduces_profiles_with_order6_equilibrium():
    p = sv.Params(Qx=7, Qy=7, Qz=7, S=9, dt=1e-3, Nx=6, Ny=6, Nz=6)
    m = sv.Model(p)
    tab = random_table(np.random.default_rng(1), p.S)
    f = ws.seed(tab, m.vs)
    got = sv.moments(f, m).table()
    assert np.abs(got - tab).max() <= 1e-12 * np.abs(tab).max()


def test_seed_reproduces_general_table():
    """Off-Couette entries (u_x, u_z, P_xz, P_yz, q_z) are carried as well."""
    p = sv.Params(Qx=8, Qy=7, Qz=7, S=5, dt=1e-3, Nx=6, Ny=6, Nz=6)
    m = sv.Model(p)
    rng = np.random.default_rng(2)
    tab = random_table(rng, p.S)
    tab[:, 1] = rng.uniform(-0.1, 0.1, p.S)
    tab[:, 3] = rng.uniform(-0.1, 0.1, p.S)
    tab[:, 9] = rng.uniform(-0.03, 0.03, p.S)
    tab[:, 10] = rng.uniform(-0.03, 0.03, p.S)
    tab[:, 13] = rng.uniform(-0.03, 0.03, p.S)
    tab[:, 7] = 3 * tab[:, 0] * tab[:, 4] - tab[:, 5] - tab[:, 6]
    got = sv.moments(ws.seed(tab, m.vs), m).table()
    assert np.abs(got - tab).max() <= 1e-12 * np.abs(tab).max()


def test_seed_without_stress_and_heat_flux_is_the_equilibrium():
    vs = VelocitySet(4, 5, 5)
    rng = np.random.default_rng(3)
    S = 6
    n, uy, T = rng.uniform(0.8, 1.2, S), rng.uniform(-0.3, 0.3, S), rng.uniform(0.8, 1.2, S)
    tab = ws.table_from_profiles(np.stack([n, uy, T, n * T, 0 * n, n * T, 0 * n, 0 * n], axis=-1))
    f = ws.seed(tab, vs)
    assert np.abs(f - vs.maxwellian(n, 0 * n, uy, 0 * n, T)).max() <= 1e-15 * np.abs(f).max()


def test_heat_term_is_shakhov_factor():
    vs = VelocitySet(5, 4, 4)
    rng = np.random.default_rng(4)
    S, pr = 4, 2.0 / 3.0
    n, uy, T = rng.uniform(0.8, 1.2, S), rng.uniform(-0.3, 0.3, S), rng.uniform(0.8, 1.2, S)
    qx, qy = rng.uniform(-0.05, 0.05, S), rng.uniform(-0.05, 0.05, S)
    z = 0 * n
    tab = ws.table_from_profiles(np.stack([n, uy, T, n * T, z, n * T, (1 - pr) * qx, (1 - pr) * qy], axis=-1))
    f = ws.seed(tab, vs)
    feq = vs.maxwellian(n, z, uy, z, T)
    ref = feq * (1 + vs.shakhov_factor(n, (z, uy, z), T, (qx, qy, z), pr))
    assert np.abs(f - ref).max() <= 1e-14 * np.abs(ref).max()


def test_profile_table_round_trip():
    tab = random_table(np.random.default_rng(5), 7)
    assert np.array_equal(ws.table_from_profiles(ws.profiles_from_table(tab)), tab)
    T = tab[:, 4]
    assert np.allclose(tab[:, 5] + tab[:, 6] + tab[:, 7], 3 * tab[:, 0] * T, rtol=1e-15)


def test_mass_preserving_scale():
    p = sv.Params(Qx=5, Qy=4, Qz=4, S=11, dt=1e-3, A=0.9, n0=1.3)
    m = sv.Model(p)
    rng = np.random.default_rng(6)
    tab = ws.table_from_profiles(np.stack([rng.uniform(0.8, 1.2, p.S), rng.uniform(-0.2, 0.2, p.S),
                                           rng.uniform(0.9, 1.1, p.S), np.ones(p.S), 0.01 * np.ones(p.S),
                                           np.ones(p.S), 0.01 * np.ones(p.S), -0.01 * np.ones(p.S)], axis=-1))
    scaled = ws.mass_preserving(tab, m.dx, p.n0)
    f = ws.seed(scaled, m.vs)
    mass = np.sum(f.sum(axis=1) * m.dx)
    assert abs(mass - p.n0 * np.sum(m.dx)) <= 1e-14 * mass
    # the equilibrium start has that mass too
    assert abs(np.sum(sv.equilibrium_state(m).sum(axis=1) * m.dx) - mass) <= 1e-14 * mass
    # u and T are intensive: unchanged
    m0, m1 = sv.moments(ws.seed(tab, m.vs), m), sv.moments(f, m)
    assert np.allclose(m0.u[1], m1.u[1], rtol=1e-13, atol=1e-15) and np.allclose(m0.T, m1.T, rtol=1e-13)
    assert np.allclose(ws.seed(scaled, m.vs), ws.seed(tab, m.vs) * scaled[0, 0] / tab[0, 0], rtol=1e-13)
