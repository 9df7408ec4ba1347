"""Learned warm start end to end on a small sweep: steady states collected by the batched
solver train the network on the GPU; seeded held-out instances reach the same residual in
fewer steps than from the equilibrium start, and converge to the same moments."""
import numpy as np
import pytest

from paper_1702_01335_amd import warmstart as ws

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
