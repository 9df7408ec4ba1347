"""Learned warm start end to end on a small sweep: steady states collected by the batched
solver train the network on the GPU; seeded held-out instances reach the same residual in
fewer steps than from the equilibrium start, and converge to the same moments.  Two more
held-out instances, started from the network, are run to R < 1e-10 and compared with the
oracle's steady states (tests/golden/warm_start_s16_steady.json, written by
tests/golden/make_oracle_golden.py from the oracle alone, run to 1e-12): the stopping rule
brackets the steady state to about (1e-10 + 1e-12) / lambda, lambda the decay rate of the
oracle's residual, as in the steady-state test of the first workload."""
import json
import os

import numpy as np
import pytest

from paper_1702_01335_amd import warmstart as ws
from paper_1702_01335_amd.sweep import Sweep

pytestmark = pytest.mark.gpu

# Qy = Qz = 4: the Shakhov term conserves mass only with full-range orders N >= 3
SMALL = dict(qx=(4,), nodes=(16,), kn_range=(0.05, 5.0), Qy=4, Qz=4, check_every=200)


def test_warm_start_saves_steps_on_held_out_instances():
    X, Y, info = ws.collect(96, 101, tol=1e-9, max_steps=100000, **SMALL)
    print(f"[warm] collect {info}", flush=True)
    assert info['converged'] == 96 and X.shape == (96 * 16, 5) and Y.shape == (96 * 16, 8)
    net, log, t = ws.train(X, Y, steps=600, batch=1024, lr=3e-3, log_every=100)
    print(f"[warm] train loss {log[0][1]:.3e} -> {log[-1][1]:.3e} in {t:.2f}s", flush=True)
    assert log[-1][1] < 0.05 * log[0][1]
    res = ws.compare(net, 16, 202, tol=1e-9, max_steps=100000, **SMALL)
    print(f"[warm] {res}", flush=True)
    assert res['converged_plain'] == 16 and res['converged_warm'] == 16
    assert res['fallback'] == 0
    assert res['start_error_network_median'] < 0.2 * res['start_error_equilibrium_median']
    assert res['steps_warm_total'] < res['steps_plain_total']
    # both starts reach the same steady state: the difference is bounded by tol / decay rate
    assert res['converged_moment_diff'] < 1e-6

    # warm-started held-out instances against the oracle's steady states
    gold = json.load(open(os.path.join(os.path.dirname(__file__), 'golden', 'warm_start_s16_steady.json')))
    gr = gold['grid']
    inst = [dict(d, Qx=gr['Qx'], S=gr['S']) for d in gold['instances']]
    sw = Sweep(inst, Qy=gr['Qy'], Qz=gr['Qz'], scheme=gr['scheme'], pr=gr['pr'], A=gr['A'], courant=gr['courant'])
    flags, _ = ws.seed(sw, net, guard=True)
    tol = 1e-10
    steps, R, _ = sw.run_to_steady(tol, 100000, gold['check_every'])
    assert (steps > 0).all(), (steps, R)
    (_, idx, solver), = sw.groups
    mom = solver.moments().cpu().numpy()
    for b, i in enumerate(idx):
        ref = np.array(gold['moments'][i])
        bound = 10.0 * (tol + gold['tol']) / gold['decay_rate_per_time'][i]
        scale = np.maximum(np.abs(ref).max(axis=0), gold['instances'][i]['u_w'])
        err = (np.abs(mom[b] - ref) / scale).max()
        print(f"[warm] held-out {gold['instances'][i]}: start flag {flags[b]}, {steps[b]} steps "
              f"(oracle from rest: {gold['steps'][i]}), largest moment difference from the oracle's "
              f"steady state {err:.2e} of the bound {bound:.2e}", flush=True)
        assert err <= bound
    assert (flags == 0).any()  # at least one of the two started from the network
