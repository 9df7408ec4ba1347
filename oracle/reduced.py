"""Oracle of the paper's own z-elimination: the reduced distributions phi = int f dp_z and
chi = int f p_z^2 dp_z (Eq. reduced_def), evolved by Eq. boltz_red with
phi^eq = n g_x g_y (Eq. phieq), chi^eq = T phi^eq and the reduced Shakhov factors of
Eq. sred_def (test infrastructure only).

The solver under test keeps p_z explicit on a full-range Gauss-Hermite axis instead.  For
states even in p_z, with a scheme linear in F (second-order upwind) and N_z >= 4, the
z-sums of the explicit populations follow exactly these reduced equations, which is what
tests/test_oracle_reduced.py checks; it ties the explicit-z model to the paper's
literal equations.

Reduced moments (u_z = 0, q_z = 0 by symmetry):
    n = sum phi, n u_a = sum p_a phi (a = x, y), P_ab = sum xi_a xi_b phi, P_zz = sum chi,
    3 n T = sum (xi_x^2 + xi_y^2) phi + sum chi,
    q_a = 1/2 [sum (xi_x^2 + xi_y^2) xi_a phi + sum xi_a chi].
Boundary conditions as in App. A.4, with chi_w = T_w phi_w and n_w from the phi fluxes.
"""
import numpy as np

from . import solver as sv
from .equilibrium import AxisProjection


class ReducedModel:
    def __init__(self, p: sv.Params):
        self.p = p
        Nx = min(6, p.Qx - 1) if p.Nx is None else p.Nx
        Ny = p.Qy - 1 if p.Ny is None else p.Ny
        self.X = AxisProjection('half', p.Qx, Nx)
        self.Y = AxisProjection('full', p.Qy, Ny)
        self.V = 2 * p.Qx * p.Qy
        px, py = np.meshgrid(self.X.nodes, self.Y.nodes, indexing='ij')
        self.px, self.py = px.ravel(), py.ravel()
        self.grid = sv.Grid(p.S, p.A)
        self.dx = self.grid.widths()
        idx = np.arange(self.V).reshape(2 * p.Qx, p.Qy)
        self.mirror = idx[::-1, ::-1].ravel()
        self.pos, self.neg = self.px > 0, self.px < 0
        self.g_wall = self.phi_eq(1.0, 0.0, p.u_w, p.T_w)
        self.wall_den = np.sum(self.px[self.neg] * self.g_wall[self.neg])
        self.extrap = {}
        for s in (p.S + 1, p.S + 2):
            xs = self.grid.x(s)
            x1, x2, x3 = self.grid.x(s - 1), self.grid.x(s - 2), self.grid.x(s - 3)
            self.extrap[s] = ((xs - x2) * (xs - x3) / ((x1 - x2) * (x1 - x3)),
                              (xs - x1) * (xs - x3) / ((x2 - x1) * (x2 - x3)),
                              (xs - x1) * (xs - x2) / ((x3 - x1) * (x3 - x2)))

    def phi_eq(self, n, ux, uy, T):
        gx = self.X.factor(ux, T)
        gy = self.Y.factor(uy, T)
        n = np.asarray(n, dtype=np.float64)
        prod = n[..., None, None] * gx[..., :, None] * gy[..., None, :]
        return prod.reshape(prod.shape[:-2] + (self.V,))

    def moments(self, phi, chi):
        n = phi.sum(-1)
        ux = (phi * self.px).sum(-1) / n
        uy = (phi * self.py).sum(-1) / n
        xx = self.px - ux[:, None]
        xy = self.py - uy[:, None]
        P = {'xx': (phi * xx * xx).sum(-1), 'yy': (phi * xy * xy).sum(-1), 'xy': (phi * xx * xy).sum(-1),
             'zz': chi.sum(-1)}
        T = (P['xx'] + P['yy'] + P['zz']) / (3 * n)
        r2 = xx * xx + xy * xy
        qx = 0.5 * ((phi * r2 * xx).sum(-1) + (chi * xx).sum(-1))
        qy = 0.5 * ((phi * r2 * xy).sum(-1) + (chi * xy).sum(-1))
        return n, ux, uy, T, P, qx, qy, xx, xy

    def targets(self, phi, chi):
        n, ux, uy, T, P, qx, qy, xx, xy = self.moments(phi, chi)
        feq = self.phi_eq(n, ux, uy, T)
        r2 = xx * xx + xy * xy
        coef = (1 - self.p.pr) / (n * T * T)
        qxi = qx[:, None] * xx + qy[:, None] * xy
        S_phi = coef[:, None] * (r2 / (5 * T[:, None]) - 0.8) * qxi
        S_chi = coef[:, None] * (r2 / (5 * T[:, None]) - 0.4) * qxi
        tau = sv.relaxation_time(n, T, self.p)
        return feq * (1 + S_phi), T[:, None] * feq * (1 + S_chi), tau

    def ghosts(self, F, wall_scale, n_w):
        S = self.p.S
        G = np.full((S + 6, self.V), np.nan)
        G[3:S + 3] = F
        for k in (1, 2, 3):
            G[3 - k] = F[k - 1][self.mirror]
        for s in (S + 1, S + 2):
            c1, c2, c3 = self.extrap[s]
            G[s + 2, self.pos] = c1 * G[s + 1, self.pos] + c2 * G[s, self.pos] + c3 * G[s - 1, self.pos]
        if n_w is None:
            phi_wall = sv.stencil_fluxes(G[:, self.pos], self.px[self.pos], self.p.scheme, S, S)[0]
            n_w = -np.sum(phi_wall) / self.wall_den
        for s in (S + 1, S + 2, S + 3):
            G[s + 2, self.neg] = wall_scale * n_w * self.g_wall[self.neg]
        return G, n_w

    def rhs(self, state):
        phi, chi = state
        p = self.p
        Gp, n_w = self.ghosts(phi, 1.0, None)
        Gc, _ = self.ghosts(chi, p.T_w, n_w)
        out = []
        FS = self.targets(phi, chi) if not p.collisionless else None
        for k, (F, G) in enumerate(((phi, Gp), (chi, Gc))):
            flux = sv.stencil_fluxes(G, self.px, p.scheme, 0, p.S)
            D = (flux[1:] - flux[:-1]) / self.dx[:, None]
            if FS is None:
                out.append(-D)
            else:
                out.append(-D - (F - FS[k]) / FS[2][:, None])
        return np.stack(out)

    def step(self, state):
        return sv.rk3(state, self.rhs, self.p.dt)

    def equilibrium_state(self):
        f = self.phi_eq(self.p.n0, 0.0, 0.0, self.p.T_w)
        phi = np.tile(f, (self.p.S, 1))
        return np.stack([phi, self.p.T_w * phi])
