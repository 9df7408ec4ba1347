"""Learned warm start of sweep instances.

1. collect: a sweep of instances is run to steady state as one batch; every node of every
   converged instance gives a training row, inputs (log10 kn, u_w, omega, Pr, x / (L/2))
   and targets (n, u_y, T, P_xx, P_xy, P_yy, q_x, q_y) from the library's moments.
2. train: the profile network (network.Network) is fitted on the GPU by its own kernels,
   AdamW on minibatches drawn with torch's generator, cosine learning-rate decay.
3. seed: the network's predicted moment table seeds each instance through
   hrlb_seed_state (Shakhov-form reconstruction, scaled to the mass of the equilibrium
   start since the scheme conserves mass; instances whose prediction is not a valid state
   fall back to the equilibrium at rest).
4. guard: after seeding, one RK3 step of each instance is compared with one step from the
   equilibrium start; where the seeded start has the larger residual the instance is
   started from the equilibrium instead, so the plain start is both the fallback and the
   yardstick of the prediction.
5. compare: the same held-out instances are run to the same residual from the
   equilibrium start and from the warm start; steps, wall time and the converged moments
   are compared.

The node position enters as the fraction (s - 1/2) / S of the half channel, which is
x / (L/2) on the equidistant grid the sweeps use.  The inputs carry no discretisation
parameter, so the steady states a network learns from and the instances it seeds share
one velocity set and grid (by default Qx = 8, Qy = Qz = 5, S = 64): otherwise the targets
would not be a function of the inputs.
"""
import math
import time

import numpy as np

from . import network
from .sweep import Sweep, sample

CHANNELS = (0, 2, 4, 5, 8, 6, 11, 12)   # n, u_y, T, P_xx, P_xy, P_yy, q_x, q_y in the moment table


def instance_features(d, S, pr):
    x = (np.arange(S) + 0.5) / S
    f = np.empty((S, network.IN), dtype=np.float32)
    f[:, 0] = math.log10(d['kn'])
    f[:, 1] = d['u_w']
    f[:, 2] = d['omega']
    f[:, 3] = pr
    f[:, 4] = x
    return f


def group_features(sw, g):
    key, idx, solver = sw.groups[g]
    return np.concatenate([instance_features(sw.instances[i], key[1], sw.pr) for i in idx])


def steady_rows(sw, converged):
    """Training rows (inputs, targets) of the converged instances of a sweep, in batch order."""
    X, Y = [], []
    k = 0
    for g, (key, idx, solver) in enumerate(sw.groups):
        mom = solver.moments().cpu().numpy()          # [B][S][14]
        for b, i in enumerate(idx):
            if converged[k + b]:
                X.append(instance_features(sw.instances[i], key[1], sw.pr))
                Y.append(mom[b][:, CHANNELS].astype(np.float32))
        k += len(idx)
    return np.concatenate(X), np.concatenate(Y)


def collect(n, seed, tol=1e-10, max_steps=400000, check_every=1000, qx=(8,), nodes=(64,), kn_range=(0.01, 100.0),
            **kw):
    sw = Sweep(sample(n, seed, kn_range=kn_range, qx=qx, nodes=nodes), **kw)
    sw.autotune(probe_steps=3)
    steps, R, wall = sw.run_to_steady(tol, max_steps, check_every)
    X, Y = steady_rows(sw, steps > 0)
    info = dict(instances=n, converged=int((steps > 0).sum()), rows=int(X.shape[0]), wall_s=wall,
                steps_max=int(steps.max()), pairs=sw.pairs())
    del sw
    return X, Y, info


def fit_norm(X, Y):
    mx, sx = X.mean(0), X.std(0)
    my, sy = Y.mean(0), Y.std(0)
    sx = np.where(sx > 0, sx, 1.0)
    sy = np.where(sy > 0, sy, 1.0)
    return network.norm_vector(mx, sx, my, sy)


def train(X, Y, steps=10000, batch=4096, lr=2e-3, lr_min=1e-5, wd=1e-4, seed=0, device='cuda', log_every=500):
    """Fit a fresh network; returns it with the loss log [(step, loss)] and the wall time."""
    import torch
    net = network.Network(batch, fit_norm(X, Y), seed=seed, device=device)
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(device)
    Yd = torch.from_numpy(np.ascontiguousarray(Y, dtype=np.float32)).to(device)
    gen = torch.Generator(device=device).manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float32, device=device)
    log = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(steps):
        idx = torch.randint(0, X.shape[0], (min(batch, X.shape[0]),), device=device, dtype=torch.int32, generator=gen)
        a = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * it / steps))
        net.train_step(Xd, Yd, idx, a, wd, loss)
        if it % log_every == 0 or it == steps - 1:
            log.append((it, float(loss.item())))
    torch.cuda.synchronize()
    return net, log, time.perf_counter() - t0


def predicted_tables(sw, net):
    import torch
    out = []
    for g, (key, idx, solver) in enumerate(sw.groups):
        f = torch.from_numpy(group_features(sw, g)).to(solver.device)
        out.append(net.predict_table(f).reshape(len(idx), key[1], 14))
    return out


def _one_step_residual(s):
    s.step(1)
    return s.residual()


def seed(sw, net, guard=True):
    """Seed every group of the sweep from the network.  With guard, one step from the seed
    and one from the equilibrium start are compared per instance and the equilibrium start
    is kept where it does better.  Returns per-instance flags in batch order: 0 warm,
    1 invalid prediction (fallback), 2 rejected by the guard; and the steps spent probing."""
    import torch
    tables = predicted_tables(sw, net)
    flags = np.zeros(sw.B, dtype=np.int32)
    probe = 0
    if guard:
        R_eq = np.concatenate([_one_step_residual(s) for _, _, s in sw.groups])
        probe += 1
    k = 0
    for (key, idx, s), t in zip(sw.groups, tables):
        fb = s.seed_state(t)
        flags[k:k + len(idx)] = fb
        k += len(idx)
    if guard:
        R_w = np.concatenate([_one_step_residual(s) for _, _, s in sw.groups])
        probe += 1
        reject = (R_w >= R_eq) & (flags == 0)
        flags[reject] = 2
        k = 0
        for (key, idx, s), t in zip(sw.groups, tables):
            t = t.clone()
            f = flags[k:k + len(idx)]
            t[torch.from_numpy(f != 0).to(t.device)] = float('nan')   # selects the equilibrium start
            s.seed_state(t)
            k += len(idx)
    return flags, probe


def compare(net, n, seed_value, tol=1e-10, max_steps=400000, check_every=1000, qx=(8,), nodes=(64,),
            kn_range=(0.01, 100.0), guard=True, **kw):
    """Held-out instances run to tol from the equilibrium start and from the warm start."""
    import torch
    inst = sample(n, seed_value, kn_range=kn_range, qx=qx, nodes=nodes)
    plain = Sweep([dict(d) for d in inst], **kw)
    c, w, _ = plain.autotune(probe_steps=3)
    st_p, R_p, wall_p = plain.run_to_steady(tol, max_steps, check_every)
    mom_p = [s.moments().cpu().numpy() for _, _, s in plain.groups]
    del plain
    warm = Sweep([dict(d) for d in inst], cells=c, waves=w, **kw)
    # profile error of the start: equilibrium start vs network prediction, against the converged state
    eq_tab = [s.moments().cpu().numpy() for _, _, s in warm.groups]
    pred = [t.cpu().numpy() for t in predicted_tables(warm, net)]
    err_eq, err_nn = [], []
    for mp, me, mn in zip(mom_p, eq_tab, pred):
        for b in range(mp.shape[0]):
            ref = mp[b][:, CHANNELS]
            scale = np.abs(ref).max(axis=0) + 1e-30
            err_eq.append((np.abs(me[b][:, CHANNELS] - ref) / scale).max())
            err_nn.append((np.abs(mn[b][:, CHANNELS] - ref) / scale).max())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flags, probe = seed(warm, net, guard)
    torch.cuda.synchronize()
    t_seed = time.perf_counter() - t0
    st_w, R_w, wall_w = warm.run_to_steady(tol, max_steps, check_every)
    mom_w = [s.moments().cpu().numpy() for _, _, s in warm.groups]
    dmax = max(float(np.abs(a - b).max() / np.abs(a).max()) for a, b in zip(mom_p, mom_w))
    ok_p, ok_w = st_p > 0, st_w > 0
    both = ok_p & ok_w
    return dict(instances=n, tol=tol, check_every=check_every, launch=dict(cells=c, waves=w),
                converged_plain=int(ok_p.sum()), converged_warm=int(ok_w.sum()),
                steps_plain_total=int(st_p[both].sum()), steps_warm_total=int(st_w[both].sum() + probe * both.sum()),
                steps_plain_median=float(np.median(st_p[both])), steps_warm_median=float(np.median(st_w[both])),
                steps_plain_max=int(st_p.max()), steps_warm_max=int(st_w.max()),
                steps_plain=st_p.tolist(), steps_warm=st_w.tolist(),
                step_ratio=float((st_w[both].sum() + probe * both.sum()) / st_p[both].sum()),
                wall_plain_s=wall_p, wall_warm_s=wall_w + t_seed, seed_s=t_seed,
                wall_ratio=(wall_w + t_seed) / wall_p,
                fallback=int((flags == 1).sum()), rejected_by_guard=int((flags == 2).sum()),
                start_error_equilibrium_median=float(np.median(err_eq)),
                start_error_network_median=float(np.median(err_nn)),
                converged_moment_diff=dmax, max_residual=float(max(R_p.max(), R_w.max())))


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description=__doc__.split('\n')[0])
    ap.add_argument('--train-instances', type=int, default=2000)
    ap.add_argument('--heldout', type=int, default=200)
    ap.add_argument('--train-steps', type=int, default=10000)
    ap.add_argument('--out', default=None)
    a = ap.parse_args()
    X, Y, info = collect(a.train_instances, 20170205)
    print(json.dumps({'collect': info}), flush=True)
    net, log, t_train = train(X, Y, steps=a.train_steps)
    print(json.dumps({'train': {'wall_s': t_train, 'loss': log[-1][1], 'loss_first': log[0][1]}}), flush=True)
    res = compare(net, a.heldout, 20170206)
    out = dict(collect=info, train=dict(steps=a.train_steps, wall_s=t_train, log=log), heldout=res)
    print(json.dumps({'heldout': res}), flush=True)
    if a.out:
        with open(a.out, 'w') as f:
            json.dump(out, f, indent=1)


if __name__ == '__main__':
    main()
