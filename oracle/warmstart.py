"""Oracle of the warm-start reconstruction (test infrastructure only; see ``oracle/__init__``).

A warm start seeds the populations of every node from predicted macroscopic profiles
instead of the equilibrium at rest.  The seed is the discrete equilibrium of the node
(the Hermite-projected F^eq of Sec. III at the node's n, u, T) times a polynomial
correction in the peculiar velocity xi = p - u:

    f = F^eq (1 + Pi_ab xi_a xi_b / (2 n T^2) + (xi^2 / (5T) - 1) xi.q / (n T^2)),
    Pi_ab = P_ab - n T delta_ab.

The heat-flux term is the polynomial of the Shakhov factor (Eq. sdef) with the factor
(1 - Pr) replaced by 1, so that the seed carries the heat flux q itself; the stress term is
the second-order Hermite term that carries the traceless pressure deviator.  Over a
continuous Maxwellian the corrected f has density n, velocity u, pressure tensor P and
heat flux q (Gaussian moment identities E[xi_a xi_b xi_c xi_d] = T^2 (d_ab d_cd + d_ac d_bd
+ d_ad d_bc), E[xi^2 xi_a xi_b] = 5 T^2 d_ab, E[xi^4 xi_a xi_b] = 35 T^3 d_ab).  On the
discrete set the same holds exactly when the equilibrium reproduces the Gaussian
moments up to order 6 on every axis (N_x, N_y, N_z >= 6).

The network predicts eight profiles of the Couette problem, in this order:
n, u_y, T, P_xx, P_xy, P_yy, q_x, q_y.  The remaining entries follow from the symmetry of
plane Couette flow (u_x = u_z = 0, P_xz = P_yz = 0, q_z = 0) and from T = tr P / (3n),
which fixes P_zz = 3 n T - P_xx - P_yy.

Pins (tests/test_oracle_warmstart.py): with N >= 6 on every axis the moments of the seed
equal the profiles it was built from (n, u, T, P, q) to rounding; with Pi = 0 and q = 0 the
seed is the discrete equilibrium; the heat-flux term with q scaled by (1 - Pr) equals the
Shakhov target of the solver oracle; the mass-preserving scaling gives the seed the mass
of the equilibrium start and leaves u and T unchanged.
"""
import numpy as np

CHANNELS = ('n', 'uy', 'T', 'Pxx', 'Pxy', 'Pyy', 'qx', 'qy')


def profiles_from_table(table):
    """The eight predicted channels from a moment table (..., 14) in the column order
    n, ux, uy, uz, T, Pxx, Pyy, Pzz, Pxy, Pxz, Pyz, qx, qy, qz."""
    t = np.asarray(table)
    return np.stack([t[..., 0], t[..., 2], t[..., 4], t[..., 5], t[..., 8], t[..., 6], t[..., 11], t[..., 12]], axis=-1)


def table_from_profiles(prof):
    """Inverse of profiles_from_table under the Couette symmetries."""
    p = np.asarray(prof, dtype=np.float64)
    n, uy, T, Pxx, Pxy, Pyy, qx, qy = (p[..., k] for k in range(8))
    z = np.zeros_like(n)
    Pzz = 3.0 * n * T - Pxx - Pyy
    return np.stack([n, z, uy, z, T, Pxx, Pyy, Pzz, Pxy, z, z, qx, qy, z], axis=-1)


def seed(table, vs):
    """Seed populations f[..., v] from a moment table (..., 14) on the velocity set vs
    (an oracle.equilibrium.VelocitySet)."""
    t = np.asarray(table, dtype=np.float64)
    n, ux, uy, uz, T = t[..., 0], t[..., 1], t[..., 2], t[..., 3], t[..., 4]
    P = {'xx': t[..., 5], 'yy': t[..., 6], 'zz': t[..., 7], 'xy': t[..., 8], 'xz': t[..., 9], 'yz': t[..., 10]}
    q = (t[..., 11], t[..., 12], t[..., 13])
    feq = vs.maxwellian(n, ux, uy, uz, T)
    xi = {'x': vs.px - ux[..., None], 'y': vs.py - uy[..., None], 'z': vs.pz - uz[..., None]}
    nT = (n * T)[..., None]
    denom = (n * T * T)[..., None]
    stress = np.zeros_like(feq)
    for a, b in (('x', 'x'), ('y', 'y'), ('z', 'z')):
        stress = stress + (P[a + b][..., None] - nT) * xi[a] * xi[b]
    for a, b in (('x', 'y'), ('x', 'z'), ('y', 'z')):
        stress = stress + 2.0 * P[a + b][..., None] * xi[a] * xi[b]
    xi2 = xi['x'] ** 2 + xi['y'] ** 2 + xi['z'] ** 2
    qxi = q[0][..., None] * xi['x'] + q[1][..., None] * xi['y'] + q[2][..., None] * xi['z']
    heat = (xi2 / (5.0 * T[..., None]) - 1.0) * qxi
    return feq * (1.0 + stress / (2.0 * denom) + heat / denom)


def mass_preserving(table, dx, n0):
    """The table scaled by the one factor c = n0 sum_s dx_s / sum_s n_s dx_s that gives the
    seed the mass of the equilibrium start (extensive columns n, P, q times c; u and T
    unchanged), for table (S, 14) and node widths dx (S,).  The scheme conserves mass
    (bounce-back centre line, zero net mass flux through the diffuse wall, App. A.4), so
    the steady state reached from a seed depends on its mass."""
    t = np.array(table, dtype=np.float64)
    c = n0 * np.sum(dx) / np.sum(t[:, 0] * dx)
    for k in (0, 5, 6, 7, 8, 9, 10, 11, 12, 13):
        t[:, k] *= c
    return t


def features(kn, u_w, omega, pr, x_half):
    """Network inputs of one node: log10 kn, u_w, omega, Pr and the node position as a
    fraction of the half channel, x / (L/2)."""
    return np.array([np.log10(kn), u_w, omega, pr, x_half], dtype=np.float64)
