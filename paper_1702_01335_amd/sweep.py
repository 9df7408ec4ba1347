"""Ragged parameter sweeps: sample instances, group them by shape, run them as one batch.

A sweep instance varies the rarefaction kn (log-uniform), the wall speed u_w (uniform), the
viscosity index omega, the half-range order Qx and the node count S.  Instances that share
(Qx, S) form one group (one Solver); all groups advance together in a Batch.  Each
instance's time step follows the Courant condition dt = courant * dx_min / max|p_x| of its
own velocity set and grid.  run_to_steady retires instances whose residual falls below the
tolerance and reports the steps each one needed.
"""
import time

import numpy as np

from . import hrlb, inputs


def sample(n, seed, kn_range=(0.01, 100.0), uw_range=(0.05, 0.6), omegas=(0.5, 0.72, 0.81, 1.0),
           qx=(4, 8, 16, 32), nodes=(64, 128, 256)):
    """n instance descriptions drawn with numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        out.append(dict(kn=float(10 ** rng.uniform(np.log10(kn_range[0]), np.log10(kn_range[1]))),
                        u_w=float(rng.uniform(*uw_range)), omega=float(rng.choice(omegas)),
                        Qx=int(rng.choice(qx)), S=int(rng.choice(nodes))))
    return out


class Sweep:
    """Groups of sampled instances on the GPU, advanced as one Batch."""

    def __init__(self, instances, Qy=5, Qz=5, scheme='upwind2', pr=2.0 / 3.0, A=0.0, courant=0.5, cells=16, waves=1,
                 device='cuda', seed_perturb=None, eps=0.0):
        self.instances = list(instances)
        self.QyQz = Qy * Qz
        keys = sorted({(d['Qx'], d['S']) for d in self.instances})
        self.groups = []        # (key, [instance indices], Solver)
        self.order = []         # concatenated batch order -> instance index
        for key in keys:
            idx = [i for i, d in enumerate(self.instances) if (d['Qx'], d['S']) == key]
            Qx, S = key
            q = hrlb.Quadrature(Qx, Qy, Qz)
            px, _ = q.nodes(0)
            dx = 1.0 / (2 * S)   # equidistant half channel
            params = []
            for i in idx:
                d = self.instances[i]
                dt = courant * dx / float(np.abs(px).max())
                d['dt'] = dt
                params.append(hrlb.make_params(kn=d['kn'], u_w=d['u_w'], omega=d['omega'], pr=pr, A=A, dt=dt))
            r = None
            if seed_perturb is not None:
                import torch
                r = torch.from_numpy(np.stack([inputs.perturbation(seed_perturb + i, (S, q.V)) for i in idx])).to(device)
            solver = hrlb.Solver(q, S, scheme, params, device=device, perturb=r, eps=eps)
            self.groups.append((key, idx, solver))
            self.order.extend(idx)
        self.batch = hrlb.Batch([g[2] for g in self.groups], cells, waves)
        self.B = len(self.order)

    def pairs(self, active=None):
        tot = 0
        for k, i in enumerate(self.order):
            if active is None or active[k]:
                d = self.instances[i]
                tot += d['S'] * 2 * d['Qx'] * self.QyQz
        return tot

    def run_to_steady(self, tol, max_steps, check_every=200):
        """Step until every instance's residual is below tol (retiring converged ones) or the
        step budget is spent.  Returns per-instance steps (-1 if not converged), the final
        residuals and the wall time."""
        steps = np.full(self.B, -1)
        active = np.ones(self.B, dtype=np.int32)
        done = 0
        t0 = time.perf_counter()
        R = np.full(self.B, np.inf)
        while done < max_steps and active.any():
            n = min(check_every, max_steps - done)
            self.batch.step(n)
            done += n
            R = self.batch.residual()
            newly = (R < tol) & (active == 1)
            if newly.any():
                steps[newly] = done
                active[newly] = 0
                if active.any():
                    self.batch.set_active(active)
        wall = time.perf_counter() - t0
        return steps, R, wall
