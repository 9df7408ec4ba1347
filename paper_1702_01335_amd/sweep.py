"""Ragged parameter sweeps: sample instances, group them by shape, run them as one batch.

A sweep instance varies the rarefaction kn (log-uniform), the wall speed u_w (uniform), the
viscosity index omega, the half-range order Qx and the node count S.  Instances that share
(Qx, S) form one group (one Solver); all groups advance together in a Batch.  Each
instance's time step follows the Courant condition dt = courant * dx_min / max|p_x| of its
own velocity set and grid.  run_to_steady retires instances whose residual falls below the
tolerance and reports the steps each one needed; run_plain drives the same instances one at
a time, each with its own graph-captured step, as the unbatched comparison.
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
        self.Qy, self.Qz, self.QyQz = Qy, Qz, Qy * Qz
        self.scheme, self.pr, self.A, self.courant = scheme, pr, A, courant
        self.device, self.seed_perturb, self.eps = device, seed_perturb, eps
        self._quads = {}
        keys = sorted({(d['Qx'], d['S']) for d in self.instances})
        self.groups = []        # (key, [instance indices], Solver)
        self.order = []         # concatenated batch order -> instance index
        for key in keys:
            idx = [i for i, d in enumerate(self.instances) if (d['Qx'], d['S']) == key]
            self.groups.append((key, idx, self._solver(key, idx)))
            self.order.extend(idx)
        self.cells, self.waves = cells, waves
        self.batch = hrlb.Batch([g[2] for g in self.groups], cells, waves)
        self.B = len(self.order)

    def _quad(self, Qx):
        if Qx not in self._quads:
            self._quads[Qx] = hrlb.Quadrature(Qx, self.Qy, self.Qz)
        return self._quads[Qx]

    def _solver(self, key, idx):
        """One Solver over the instances idx, which all have shape key = (Qx, S)."""
        Qx, S = key
        q = self._quad(Qx)
        px, _ = q.nodes(0)
        dx = 1.0 / (2 * S)   # equidistant half channel
        params = []
        for i in idx:
            d = self.instances[i]
            d['dt'] = self.courant * dx / float(np.abs(px).max())
            params.append(hrlb.make_params(kn=d['kn'], u_w=d['u_w'], omega=d['omega'], pr=self.pr, A=self.A,
                                           dt=d['dt']))
        r = None
        if self.seed_perturb is not None:
            import torch
            r = torch.from_numpy(np.stack([inputs.perturbation(self.seed_perturb + i, (S, q.V)) for i in idx]))
            r = r.to(self.device)
        return hrlb.Solver(q, S, self.scheme, params, device=self.device, perturb=r, eps=self.eps)

    def pairs(self, active=None):
        tot = 0
        for k, i in enumerate(self.order):
            if active is None or active[k]:
                d = self.instances[i]
                tot += d['S'] * 2 * d['Qx'] * self.QyQz
        return tot

    def autotune(self, cells=(4, 8, 16, 32, 64), waves=(1, 2, 4), probe_steps=10):
        """Time probe_steps batched steps for each (cells, waves) candidate, keep the fastest
        as self.batch and put every group's state back where it was.  Returns
        (cells, waves, ms per step)."""
        import torch
        saved = [g[2].get_state().clone() for g in self.groups]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        best = None
        for c in cells:
            for w in waves:
                b = hrlb.Batch([g[2] for g in self.groups], c, w)
                b.step(2)
                e0.record()
                b.step(probe_steps)
                e1.record()
                e1.synchronize()
                ms = e0.elapsed_time(e1) / probe_steps
                del b
                if best is None or ms < best[2]:
                    best = (c, w, ms)
        for g, F in zip(self.groups, saved):
            g[2].set_state(F)
        self.cells, self.waves, ms = best
        self.batch = hrlb.Batch([g[2] for g in self.groups], self.cells, self.waves)
        torch.cuda.synchronize()
        return self.cells, self.waves, ms

    def run_to_steady(self, tol, max_steps, check_every=200):
        """Step until every instance's residual is below tol (retiring converged ones) or the
        step budget is spent.  Returns per-instance steps in batch order (-1 if not
        converged), the final residuals and the wall time."""
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

    def run_plain(self, tol, max_steps, check_every=200):
        """The same instances, in batch order, each alone in its own Solver with a
        graph-captured step, stepped to the same tolerance with the same residual checks.
        Returns per-instance steps (-1 if not converged), final residuals and the summed
        wall time (set-up excluded)."""
        steps = np.full(self.B, -1)
        R = np.full(self.B, np.inf)
        wall = 0.0
        for k, i in enumerate(self.order):
            d = self.instances[i]
            s = self._solver((d['Qx'], d['S']), [i])
            s.set_graph(True)
            s.synchronize()
            done = 0
            t0 = time.perf_counter()
            while done < max_steps:
                n = min(check_every, max_steps - done)
                s.step(n)
                done += n
                R[k] = s.residual()[0]
                if R[k] < tol:
                    steps[k] = done
                    break
            wall += time.perf_counter() - t0
            del s
        return steps, R, wall
