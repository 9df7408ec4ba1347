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


def smallest_cell(S, A):
    """Width of the smallest of S cells on the half channel: the equidistant 1/(2S), or on
    the tanh grid of Eq. stretch (x = tanh(eta) / 2A, eta_s = (s - 1/2) artanh(A) / S) the
    cell at the wall, whose interfaces sit at eta = artanh(A) (S -+ 1/2 -+ 1/2) / S."""
    if A == 0.0:
        return 1.0 / (2 * S)
    e = np.arctanh(A) / S
    return (np.tanh(S * e) - np.tanh((S - 1) * e)) / (2 * A)


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
        dx = smallest_cell(S, self.A)
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

    def autotune(self, cells=(4, 8, 16, 32, 64), waves=(1, 2, 4), probe_steps=10, active=None):
        """Time probe_steps batched steps for each (cells, waves) candidate, keep the fastest
        as self.batch and put every group's state back where it was.  active (batch order),
        if given, holds the instances still stepping: the probes time only those, and the
        kept batch has the same set active.  Returns (cells, waves, ms per step)."""
        import torch
        saved = [g[2].get_state().clone() for g in self.groups]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        best = None
        for c in cells:
            for w in waves:
                b = hrlb.Batch([g[2] for g in self.groups], c, w)
                if active is not None:
                    b.set_active(active)
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
        if active is not None:
            self.batch.set_active(active)
        torch.cuda.synchronize()
        return self.cells, self.waves, ms

    def run_to_steady(self, tol, max_steps, check_every=200, progress=None, retune=False):
        """Step until every instance's residual is below tol (retiring converged ones) or the
        step budget is spent.  Returns per-instance steps in batch order (-1 if not
        converged), the residuals (each retired instance's at its retirement, the others'
        at the last check) and the wall time.  progress, if given, is called
        after every residual check with (steps done, instances still active).  With retune,
        the launch shape is timed again for the instances left whenever their number has
        halved since the last tuning (a shape tuned for many instances leaves few tiles, and
        long ones, to the last few); the tuning time counts in the wall time.  A new shape
        sums in another order, so step counts can then differ from an untuned run's by a
        residual check at the threshold."""
        steps = np.full(self.B, -1)
        active = np.ones(self.B, dtype=np.int32)
        tuned_for = self.B
        done = 0
        t0 = time.perf_counter()
        R = np.full(self.B, np.inf)
        R_out = np.full(self.B, np.inf)
        while done < max_steps and active.any():
            n = min(check_every, max_steps - done)
            self.batch.step(n)
            done += n
            R = self.batch.residual()
            newly = (R < tol) & (active == 1)
            if newly.any():
                steps[newly] = done
                R_out[newly] = R[newly]
                active[newly] = 0
                if active.any():
                    self.batch.set_active(active)
                    if retune and active.sum() <= tuned_for // 2:
                        self.autotune(cells=(8, 16, 32, 64), waves=(1, 2, 4), probe_steps=5, active=active)
                        tuned_for = int(active.sum())
            if progress is not None:
                progress(done, int(active.sum()))
        wall = time.perf_counter() - t0
        R_out[active == 1] = R[active == 1]
        return steps, R_out, wall

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


def main():
    """Run a sampled sweep to steady state as one batch and report the per-instance steps.
    The one-instance-at-a-time time is estimated from each instance's step count and the
    measured step time of one instance of its shape (HIP graph, autotuned launch)."""
    import argparse
    import json

    import torch

    ap = argparse.ArgumentParser(description=main.__doc__.split('\n')[0])
    ap.add_argument('--instances', type=int, default=256)
    ap.add_argument('--seed', type=int, default=20170204)
    ap.add_argument('--tol', type=float, default=1e-10)
    ap.add_argument('--max-steps', type=int, default=2000000)
    ap.add_argument('--check-every', type=int, default=1000)
    ap.add_argument('--out', default=None)
    a = ap.parse_args()
    sw = Sweep(sample(a.instances, a.seed))
    c, w, _ = sw.autotune(probe_steps=3)
    print(json.dumps({'groups': [[k[0], k[1], len(i)] for k, i, _ in sw.groups], 'launch': [c, w]}), flush=True)
    t_last = [time.perf_counter()]

    def progress(done, n_active):
        if time.perf_counter() - t_last[0] > 20.0:
            t_last[0] = time.perf_counter()
            print(json.dumps({'steps': done, 'active': n_active}), flush=True)

    steps, R, wall = sw.run_to_steady(a.tol, a.max_steps, a.check_every, progress, retune=True)
    print(json.dumps({'batched_wall_s': wall, 'converged': int((steps > 0).sum())}), flush=True)
    # single-instance step time per shape
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_shape = {}
    for key, idx, _ in sw.groups:
        s = sw._solver(key, [idx[0]])
        s.autotune(probe_steps=3)
        s.set_graph(True)
        s.step(5)
        e0.record()
        s.step(50)
        e1.record()
        e1.synchronize()
        t_shape[key] = e0.elapsed_time(e1) / 50 / 1e3
        del s
    plain = 0.0
    for k, i in enumerate(sw.order):
        d = sw.instances[i]
        n = steps[k] if steps[k] > 0 else a.max_steps
        plain += n * t_shape[(d['Qx'], d['S'])]
    res = dict(instances=a.instances, seed=a.seed, tol=a.tol, check_every=a.check_every, launch=[c, w],
               final_launch=[sw.cells, sw.waves],
               converged=int((steps > 0).sum()), batched_wall_s=wall, plain_estimate_s=plain,
               speedup_estimate=plain / wall, steps_max=int(steps.max()), steps_median=float(np.median(steps)),
               single_step_ms={f"Qx{k[0]}_S{k[1]}": v * 1e3 for k, v in t_shape.items()},
               steps=[int(x) for x in steps], max_residual=float(R.max()))
    print(json.dumps({k: v for k, v in res.items() if k != 'steps'}), flush=True)
    if a.out:
        with open(a.out, 'w') as f:
            json.dump(res, f, indent=1)


if __name__ == '__main__':
    main()
