"""Oracle time step of the mixed-quadrature LB solver for 3D Couette flow
(test infrastructure only; see ``oracle/__init__``).

State: F[s, v], s = 1..S fluid nodes on the half channel 0 <= x <= L/2 (L = 1), stored
0-based as F[s-1]; v = (i Qy + j) Qz + k over the product velocity set.  One evaluation of
the right-hand side L[F] (Eq. L_def) takes these steps, in the paper's order:

1. moments n, u, pressure tensor, T, q of F (Eq. qdef; P = n T);
2. relaxation time tau (Eq. mw_tau; power law mu ~ T^omega of Sec. VI; Eq. sutherland_tau;
   the constant tau of the linearised regime, Eq. knLuo);
3. Shakhov target F^eq (1 + S) (Eqs. phieq, sdef; discrete construction of Sec. III);
4. ghost nodes: bounce-back at x = 0 (Eq. widetildei), quadratic extrapolation of the
   outgoing populations and diffuse-reflection wall Maxwellian with the wall density fixed
   by zero net mass flux at x = L/2 (App. A.4);
5. interface fluxes by WENO-5 (Eqs. weno5_flux, weno5_omega, weno_sigma, Table II) or
   second-order upwind, and the flux-form derivative on the (stretched) grid (Eqs. flux,
   stretch, etas);
6. L[F] = -D - (F - F^eq(1+S)) / tau.
The time step is the three-stage TVD Runge-Kutta scheme of Eq. rk3 (Butcher tableau in
Table rk3).  Ghosts and the wall density are rebuilt from each stage's input.

Where the paper leaves a point open, the reading taken is stated at the function that
takes it.
"""
from dataclasses import dataclass

import numpy as np

from .equilibrium import VelocitySet

# ideal WENO-5 weights delta_q (text after Eq. weno5_omega)
WENO_DELTA = (0.1, 0.6, 0.3)

# Table II: limiting weights when some smoothness indicators vanish, keyed by the set of
# vanishing indicators (0-based q).
WENO_LIMITS = {
    (0, 1, 2): (0.1, 0.6, 0.3),
    (1, 2): (0.0, 2.0 / 3.0, 1.0 / 3.0),
    (0, 2): (0.25, 0.0, 0.75),
    (0, 1): (1.0 / 7.0, 6.0 / 7.0, 0.0),
    (0,): (1.0, 0.0, 0.0),
    (1,): (0.0, 1.0, 0.0),
    (2,): (0.0, 0.0, 1.0),
}


@dataclass
class Params:
    """Physical and numerical parameters of one Couette instance (non-dimensional, Sec. II.B).

    kn          rarefaction: viscosity mu(T) = kn * T^omega (power law) or Sutherland's
                law scaled to mu(1) = kn (kn = 1/(delta sqrt 2) of Sec. VI).
    law         'power', 'sutherland' or 'lowmach' (constant tau = kn / sqrt 2, kn = k of
                Sec. IV).
    collisionless  drop the collision term (1/tau = 0).
    A           tanh stretching parameter of Eq. stretch; A = 0 is the equidistant grid.
    scheme      'weno5', 'upwind2' or 'linear5' (WENO-5 stencils with the ideal weights; a
                test switch only: its incoming wall flux is not the wall Maxwellian's, so
                the wall-density rule of App. A.4 does not conserve mass with it).
    """
    Qx: int
    Qy: int
    Qz: int
    S: int
    dt: float
    kn: float = 0.1
    u_w: float = 0.0
    T_w: float = 1.0
    n0: float = 1.0
    pr: float = 1.0
    law: str = 'power'
    omega: float = 1.0
    suth_S: float = 0.0
    A: float = 0.0
    scheme: str = 'weno5'
    collisionless: bool = False
    Nx: int = None
    Ny: int = None
    Nz: int = None


class Grid:
    """Cell centres and interfaces of App. A.2 (Eqs. stretch, etas), 1-based node index s.

    x(eta) = L tanh(eta) / (2A), eta_s = (s - 1/2) artanh(A) / S; interfaces at
    eta_s +- d_eta/2.  A = 0 is the equidistant limit x_s = (s - 1/2) L / (2S).  The same
    formulas continue to ghost nodes s > S (used by the extrapolation of App. A.4).
    """

    def __init__(self, S, A, L=1.0):
        self.S, self.A, self.L = S, A, L
        if A == 0.0:
            self.eta_max = None
        else:
            self.eta_max = np.arctanh(A)

    def x(self, s):
        """Position of (possibly fractional) node index s, 1-based."""
        s = np.asarray(s, dtype=np.float64)
        if self.A == 0.0:
            return (s - 0.5) * self.L / (2 * self.S)
        eta = (s - 0.5) * self.eta_max / self.S
        return self.L * np.tanh(eta) / (2 * self.A)

    def eta(self, s):
        s = np.asarray(s, dtype=np.float64)
        return (s - 0.5) * self.eta_max / self.S

    def widths(self):
        """x_{s+1/2} - x_{s-1/2} for s = 1..S."""
        s = np.arange(1, self.S + 1, dtype=np.float64)
        return self.x(s + 0.5) - self.x(s - 0.5)


class Model:
    """Tables of one instance: velocity set, grid, wall Maxwellian, bounce-back map."""

    def __init__(self, p: Params):
        self.p = p
        self.vs = VelocitySet(p.Qx, p.Qy, p.Qz, p.Nx, p.Ny, p.Nz)
        self.V = self.vs.V
        self.grid = Grid(p.S, p.A)
        self.dx = self.grid.widths()
        Qx, Qy, Qz = p.Qx, p.Qy, p.Qz
        idx = np.arange(self.V).reshape(2 * Qx, Qy, Qz)
        # bounce-back partner of v: (2Qx-1-i, Qy-1-j, k) -- p_x and p_y reversed, p_z kept
        self.mirror = idx[::-1, ::-1, :].ravel()
        self.pos = self.vs.px > 0
        self.neg = self.vs.px < 0
        # wall Maxwellian per unit density, wall at x = L/2 moving with +u_w along y
        self.g_wall = self.vs.maxwellian(1.0, 0.0, p.u_w, 0.0, p.T_w)
        self.wall_den = np.sum(self.vs.px[self.neg] * self.g_wall[self.neg])
        # Lagrange weights extrapolating node s from s-1, s-2, s-3 (App. A.4), s = S+1, S+2
        self.extrap = {}
        for s in (p.S + 1, p.S + 2):
            xs = self.grid.x(s)
            x1, x2, x3 = self.grid.x(s - 1), self.grid.x(s - 2), self.grid.x(s - 3)
            self.extrap[s] = (
                (xs - x2) * (xs - x3) / ((x1 - x2) * (x1 - x3)),
                (xs - x1) * (xs - x3) / ((x2 - x1) * (x2 - x3)),
                (xs - x1) * (xs - x2) / ((x3 - x1) * (x3 - x2)),
            )


@dataclass
class Moments:
    n: np.ndarray
    u: tuple
    P: dict          # pressure tensor T_ab of Eq. qdef, keys 'xx','yy','zz','xy','xz','yz'
    T: np.ndarray
    q: tuple

    def table(self):
        """(S, 14): n, ux, uy, uz, T, Pxx, Pyy, Pzz, Pxy, Pxz, Pyz, qx, qy, qz."""
        cols = [self.n, *self.u, self.T] + [self.P[k] for k in ('xx', 'yy', 'zz', 'xy', 'xz', 'yz')] + list(self.q)
        return np.stack(cols, axis=-1)


def moments(F, m: Model) -> Moments:
    """Eq. qdef with m = 1: n = sum F, u = sum F p / n, T_ab = sum F xi_a xi_b,
    T = (T_xx + T_yy + T_zz) / (3n) (P = nT), q = sum F xi^2 xi / 2, with xi = p - u.
    Central moments are taken in a second pass over F."""
    vs = m.vs
    n = F.sum(axis=-1)
    ux = (F * vs.px).sum(axis=-1) / n
    uy = (F * vs.py).sum(axis=-1) / n
    uz = (F * vs.pz).sum(axis=-1) / n
    xx = vs.px - ux[..., None]
    xy = vs.py - uy[..., None]
    xz = vs.pz - uz[..., None]
    P = {
        'xx': (F * xx * xx).sum(-1), 'yy': (F * xy * xy).sum(-1), 'zz': (F * xz * xz).sum(-1),
        'xy': (F * xx * xy).sum(-1), 'xz': (F * xx * xz).sum(-1), 'yz': (F * xy * xz).sum(-1),
    }
    T = (P['xx'] + P['yy'] + P['zz']) / (3.0 * n)
    xi2 = xx * xx + xy * xy + xz * xz
    q = (0.5 * (F * xi2 * xx).sum(-1), 0.5 * (F * xi2 * xy).sum(-1), 0.5 * (F * xi2 * xz).sum(-1))
    return Moments(n, (ux, uy, uz), P, T, q)


def relaxation_time(n, T, p: Params):
    """tau with mu = tau n T (Chapman-Enskog, Sec. II.A):
    power law mu = kn T^omega -> tau = kn T^(omega-1) / n (omega = 1: Eq. mw_tau);
    Sutherland (Eq. sutherland_tau with 1/(delta sqrt 2) = kn):
        tau = kn (1 + S) / (n sqrt(T) (1 + S/T));
    linearised low-Mach regime of Sec. IV (Eq. knLuo, kn = k): tau = k / sqrt(2), constant."""
    if p.law == 'power':
        return p.kn * T ** (p.omega - 1.0) / n
    if p.law == 'sutherland':
        return p.kn * (1.0 + p.suth_S) / (n * np.sqrt(T) * (1.0 + p.suth_S / T))
    if p.law == 'lowmach':
        return np.full_like(np.asarray(n, dtype=np.float64), p.kn / np.sqrt(2.0))
    raise ValueError(p.law)


def shakhov_target(mom: Moments, m: Model):
    """F^eq (1 + S) per cell and velocity (Eqs. phieq, sdef; S evaluated pointwise at the
    discrete velocity on the Hermite-projected F^eq)."""
    feq = m.vs.maxwellian(mom.n, mom.u[0], mom.u[1], mom.u[2], mom.T)
    if m.p.pr == 1.0:
        return feq
    return feq * (1.0 + m.vs.shakhov_factor(mom.n, mom.u, mom.T, mom.q, m.p.pr))


def weno5_weights(s1, s2, s3):
    """Normalised nonlinear weights of Eq. weno5_omega, w_q = (d_q / s_q^2) / sum_r (d_r / s_r^2),
    evaluated as w_q = 1 / (1 + sum_{r != q} (d_r / d_q) (s_q / s_r)^2) (the same quotient with
    numerator and denominator divided by d_q / s_q^2; this form neither overflows nor
    underflows for the tiny populations of high-order half-range sets).  Where one or more
    indicators vanish the weights are read from Table II, as the paper prescribes."""
    sig = (s1, s2, s3)
    d = WENO_DELTA
    w = []
    with np.errstate(divide='ignore', invalid='ignore', over='ignore'):
        for q in range(3):
            acc = np.ones_like(s1)
            for r in range(3):
                if r != q:
                    acc = acc + (d[r] / d[q]) * (sig[q] / sig[r]) ** 2
            w.append(1.0 / acc)
    z = [s == 0.0 for s in sig]
    for key, vals in WENO_LIMITS.items():
        mask = np.ones_like(s1, dtype=bool)
        for q in range(3):
            mask &= z[q] if q in key else ~z[q]
        if mask.any():
            for q in range(3):
                w[q] = np.where(mask, vals[q], w[q])
    return w


def interface_flux(a, b, c, d, e, px, scheme):
    """Flux through the interface s+1/2 from the upwind-ordered stencil (a..e) =
    (F_{s-2}, F_{s-1}, F_s, F_{s+1}, F_{s+2}) for p_x > 0, and the mirrored stencil
    (F_{s+3}, F_{s+2}, F_{s+1}, F_s, F_{s-1}) for p_x < 0 (reading: the paper writes only the
    p_x > 0 case, Eqs. weno5_flux and its candidates)."""
    if scheme == 'upwind2':
        return px * (3.0 * c - b) / 2.0
    f1 = a / 3.0 - 7.0 * b / 6.0 + 11.0 * c / 6.0
    f2 = -b / 6.0 + 5.0 * c / 6.0 + d / 3.0
    f3 = c / 3.0 + 5.0 * d / 6.0 - e / 6.0
    if scheme == 'linear5':
        w1, w2, w3 = WENO_DELTA
    else:
        s1 = 13.0 / 12.0 * (a - 2 * b + c) ** 2 + 0.25 * (a - 4 * b + 3 * c) ** 2
        s2 = 13.0 / 12.0 * (b - 2 * c + d) ** 2 + 0.25 * (b - d) ** 2
        s3 = 13.0 / 12.0 * (c - 2 * d + e) ** 2 + 0.25 * (3 * c - 4 * d + e) ** 2
        w1, w2, w3 = weno5_weights(s1, s2, s3)
    return px * (w1 * f1 + w2 * f2 + w3 * f3)


def stencil_fluxes(G, px, scheme, lo, hi):
    """Fluxes at interfaces s+1/2 for s = lo..hi (1-based; s = 0 is the centre line) from
    the ghost-extended array G, where G[t + 2] holds node t (t = -2 .. S+3)."""
    s = np.arange(lo, hi + 1)
    pos = px > 0
    at = lambda off: G[s + 2 + off]
    # upwind-ordered stencils, chosen per velocity by the sign of p_x
    a = np.where(pos, at(-2), at(3))
    b = np.where(pos, at(-1), at(2))
    c = np.where(pos, at(0), at(1))
    d = np.where(pos, at(1), at(0))
    e = np.where(pos, at(2), at(-1))
    return interface_flux(a, b, c, d, e, px, scheme)


def build_ghosts(F, m: Model):
    """Ghost-extended array G (S+6 rows; G[t+2] = node t, t = -2..S+3) and the wall density.

    * x = 0: bounce-back F_{1-m; ijk} = F_{m; i~ j~ k} for m = 1, 2, 3 (Eq. widetildei;
      reading: p_z is kept, i.e. the map is the rotation by pi about z that carries the
      Couette flow onto itself).
    * x = L/2, p_x > 0: F_{S+1}, F_{S+2} by quadratic extrapolation from the three nodes
      below (App. A.4).  F_{S+3} is never read for p_x > 0 and is set to NaN.
    * x = L/2, p_x < 0: F_{S+1} = F_{S+2} = F_{S+3} = n_w F^eq_w / n_w with
      n_w = -sum_{p_x>0} Phi_{S+1/2} / sum_{p_x<0} p_x F^eq_w / n_w.
    Rebuilt from every Runge-Kutta stage input (reading of "at every time step").
    """
    S = m.p.S
    V = m.V
    G = np.full((S + 6, V), np.nan)
    G[3:S + 3] = F
    for k in (1, 2, 3):
        G[3 - k] = F[k - 1][m.mirror]
    pos, neg = m.pos, m.neg
    for s in (S + 1, S + 2):
        c1, c2, c3 = m.extrap[s]
        G[s + 2, pos] = c1 * G[s + 1, pos] + c2 * G[s, pos] + c3 * G[s - 1, pos]
    phi_wall = stencil_fluxes(G[:, pos], m.vs.px[pos], m.p.scheme, S, S)[0]
    n_w = -np.sum(phi_wall) / m.wall_den
    for s in (S + 1, S + 2, S + 3):
        G[s + 2, neg] = n_w * m.g_wall[neg]
    return G, n_w


def rhs(F, m: Model):
    """L[F] of Eq. L_def for one instance; returns (L, n_w)."""
    p = m.p
    G, n_w = build_ghosts(F, m)
    phi = stencil_fluxes(G, m.vs.px, p.scheme, 0, p.S)          # interfaces 1/2 .. S+1/2
    D = (phi[1:] - phi[:-1]) / m.dx[:, None]
    if p.collisionless:
        return -D, n_w
    mom = moments(F, m)
    tau = relaxation_time(mom.n, mom.T, p)
    return -D - (F - shakhov_target(mom, m)) / tau[:, None], n_w


def rk3(F, L, dt):
    """Shu-Osher TVD RK3 of Eq. rk3 for dF/dt = L(F):
    F1 = F + dt L(F); F2 = 3/4 F + 1/4 F1 + 1/4 dt L(F1); F_next = 1/3 F + 2/3 F2 + 2/3 dt L(F2)."""
    F1 = F + dt * L(F)
    F2 = 0.75 * F + 0.25 * F1 + 0.25 * dt * L(F1)
    return F / 3.0 + 2.0 / 3.0 * F2 + 2.0 / 3.0 * dt * L(F2)


def rk3_step(F, m: Model):
    """One time step of the solver: Eq. rk3 applied to L[F] of Eq. L_def."""
    return rk3(F, lambda G: rhs(G, m)[0], m.p.dt)


def residual(F_new, F_old, dt):
    """R = ||F_{l+1} - F_l||_2 / (dt ||F_l||_2) over the fluid nodes (reading: the paper runs
    to a steady state without defining the stopping rule; this is a relative rate per
    unit time, independent of dt)."""
    return np.sqrt(np.sum((F_new - F_old) ** 2)) / (dt * np.sqrt(np.sum(F_old ** 2)))


def equilibrium_state(m: Model):
    """Initial state: the discrete equilibrium at rest, n = n0, u = 0, T = T_w, in every node
    (reading: the paper does not state its initial condition)."""
    p = m.p
    f = m.vs.maxwellian(p.n0, 0.0, 0.0, 0.0, p.T_w)
    return np.tile(f, (p.S, 1))


def seeded_state(m: Model, r, eps):
    """Equilibrium state times (1 + eps r) for a caller-supplied r[s, v] in [-1, 1)."""
    return equilibrium_state(m) * (1.0 + eps * r)


def run(F, m: Model, steps):
    for _ in range(steps):
        F = rk3_step(F, m)
    return F


def run_to_steady(F, m: Model, tol, max_steps, check_every=100):
    """Advance until the residual of one step falls below ``tol``; returns (F, steps, R)."""
    steps = 0
    R = np.inf
    while steps < max_steps:
        for _ in range(check_every - 1):
            F = rk3_step(F, m)
        Fn = rk3_step(F, m)
        steps += check_every
        R = residual(Fn, F, m.p.dt)
        F = Fn
        if R < tol:
            break
    return F, steps, R


class TwoWallModel:
    """Test-only mode: the whole channel -L/2 <= x <= L/2 in 2S equidistant nodes, a diffuse
    wall on each side (x = -L/2 moving with -u_w, x = +L/2 with +u_w, both at T_w), and no
    centre line.  The paper solves only the half channel, with bounce-back at x = 0 standing
    in for the other half by the symmetry of the flow (App. A.4); this mode exists to check
    that symmetry.  Each wall is treated as App. A.4 treats the wall at L/2: outgoing
    populations extrapolated quadratically into the ghost nodes, incoming ones the wall
    Maxwellian with the density that makes the net mass flux through the wall vanish.
    ``p.S`` is the node count of a half channel; ``p.A`` must be 0."""

    def __init__(self, p: Params):
        if p.A != 0.0:
            raise ValueError("the two-wall mode uses the equidistant grid")
        self.p = p
        self.vs = VelocitySet(p.Qx, p.Qy, p.Qz, p.Nx, p.Ny, p.Nz)
        self.V = self.vs.V
        self.N = 2 * p.S
        self.dx = np.full(self.N, 1.0 / self.N)
        self.pos = self.vs.px > 0
        self.neg = self.vs.px < 0
        self.g_right = self.vs.maxwellian(1.0, 0.0, p.u_w, 0.0, p.T_w)
        self.g_left = self.vs.maxwellian(1.0, 0.0, -p.u_w, 0.0, p.T_w)
        self.den_right = np.sum(self.vs.px[self.neg] * self.g_right[self.neg])
        self.den_left = np.sum(self.vs.px[self.pos] * self.g_left[self.pos])
        x = lambda s: -0.5 + (s - 0.5) / self.N   # node s (1-based), ghosts continue the map

        def lagrange(xs, x1, x2, x3):
            return ((xs - x2) * (xs - x3) / ((x1 - x2) * (x1 - x3)),
                    (xs - x1) * (xs - x3) / ((x2 - x1) * (x2 - x3)),
                    (xs - x1) * (xs - x2) / ((x3 - x1) * (x3 - x2)))
        N = self.N
        # ghost t from the three nodes on its inner side, nearest first
        self.ex_right = {t: lagrange(x(t), x(t - 1), x(t - 2), x(t - 3)) for t in (N + 1, N + 2)}
        self.ex_left = {t: lagrange(x(t), x(t + 1), x(t + 2), x(t + 3)) for t in (0, -1)}


def rhs_two_walls(F, m: TwoWallModel):
    """L[F] of Eq. L_def on the whole channel (F has 2S rows); returns (L, n_w left, n_w right)."""
    p, N, V = m.p, m.N, m.V
    G = np.full((N + 6, V), np.nan)      # G[t + 2] = node t, t = -2 .. N+3
    G[3:N + 3] = F
    pos, neg = m.pos, m.neg
    for t in (N + 1, N + 2):             # outgoing at the right wall: p_x > 0
        c1, c2, c3 = m.ex_right[t]
        G[t + 2, pos] = c1 * G[t + 1, pos] + c2 * G[t, pos] + c3 * G[t - 1, pos]
    for t in (0, -1):                    # outgoing at the left wall: p_x < 0
        c1, c2, c3 = m.ex_left[t]
        G[t + 2, neg] = c1 * G[t + 3, neg] + c2 * G[t + 4, neg] + c3 * G[t + 5, neg]
    phi_r = stencil_fluxes(G[:, pos], m.vs.px[pos], p.scheme, N, N)[0]
    n_r = -np.sum(phi_r) / m.den_right
    phi_l = stencil_fluxes(G[:, neg], m.vs.px[neg], p.scheme, 0, 0)[0]
    n_l = -np.sum(phi_l) / m.den_left
    for t in (N + 1, N + 2, N + 3):
        G[t + 2, neg] = n_r * m.g_right[neg]
    for t in (0, -1, -2):
        G[t + 2, pos] = n_l * m.g_left[pos]
    phi = stencil_fluxes(G, m.vs.px, p.scheme, 0, N)
    D = (phi[1:] - phi[:-1]) / m.dx[:, None]
    if p.collisionless:
        return -D, n_l, n_r
    mom = moments(F, m)
    tau = relaxation_time(mom.n, mom.T, p)
    return -D - (F - shakhov_target(mom, m)) / tau[:, None], n_l, n_r


def rk3_step_two_walls(F, m: TwoWallModel):
    return rk3(F, lambda G: rhs_two_walls(G, m)[0], m.p.dt)
