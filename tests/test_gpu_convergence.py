"""Quadrature-order convergence in the transition regime, as in Sec. VI (the figure of the
departures of nu, Pi and T_0 obtained with HHLB(6;Qx) x HLB(6;7) on 16 stretched nodes from
the converged values of HHLB(6;100) x HLB(6;7) on 32 nodes; argon, Sutherland law,
u_w = sqrt 2, delta = 0.1, 1, 10).  Every model runs in one ragged batch: one group per
(Qx, S), one instance per delta.  The paper prints no values for the figure, but states
two numbers for it: with Qx = 7, T_0 lies within 0.1 % of the converged value, and Pi within
0.2 % of the tabulated LB values (Tables V and VI; tests/golden/paper_tables.json).

Time steps keep the Courant number max|p_x| dt / dx_min below one on every model:
dt = 1.25e-4 on 16 nodes (0.83 at Qx = 100), 6.25e-5 on 32 (0.89).  The full study (nine
orders Qx = 4 .. 100, 960 000 steps: 60 time units for the reference, 120 for the 16-node
models, about three minutes on the GPU) runs when HRLB_LONG=1 is set; the default one
takes the orders 7 and 30 against the reference at delta = 0.1 and 1 over the same 960 000
steps (the slow half-range velocities of delta = 0.1 are still settling at 480 000), about
40 s."""
import json
import math
import os

import numpy as np
import pytest

from oracle import diagnostics as dg
from oracle import solver as sv
from paper_1702_01335_amd import hrlb

pytestmark = pytest.mark.gpu
LONG = os.environ.get('HRLB_LONG') == '1'


GOLD = json.load(open(os.path.join(os.path.dirname(__file__), 'golden', 'paper_tables.json')))
FULL = dict(qx=(4, 5, 7, 10, 14, 21, 30, 50, 100), deltas=('0.1', '1', '10'), steps=960000, chunk=120000,
            settled=1e-5)
TRIMMED = dict(qx=(7, 30), deltas=('0.1', '1'), steps=960000, chunk=120000, settled=1e-5)


def _diagnostics(sims, uw, MODELS, DELTAS):
    out = {}
    for (Qx, S, _), s in zip(MODELS, sims):
        mom = s.moments().cpu().numpy()
        x = sv.Grid(S, 0.98).x(np.arange(1, S + 1))
        for b, d in enumerate(DELTAS):
            uy, T, Pxy = mom[b, :, 2], mom[b, :, 4], mom[b, :, 8]
            out[(Qx, S, d)] = np.array([dg.velocity_gradient(x, uy, uw),
                                        dg.reduced_shear_stress(dg.mean_shear_stress(Pxy, 0.98), uw),
                                        dg.centre_value(x, T)])
    return out


@pytest.mark.parametrize("study", [pytest.param(TRIMMED, id='qx7-30'),
                                   pytest.param(FULL, id='qx4-100', marks=pytest.mark.skipif(
                                       not LONG, reason='about three minutes of GPU time: set HRLB_LONG=1 to run'))])
def test_quadrature_order_convergence_transition_regime(study):
    QX, DELTAS, STEPS, CHUNK = study['qx'], study['deltas'], study['steps'], study['chunk']
    MODELS = [(q, 16, 1.25e-4) for q in QX] + [(100, 32, 6.25e-5)]
    uw = math.sqrt(2)
    sims = []
    for Qx, S, dt in MODELS:
        q = hrlb.Quadrature(Qx, 7, 5)
        plist = [hrlb.make_params(kn=1 / (float(d) * math.sqrt(2)), dt=dt, u_w=uw, pr=2 / 3, law='sutherland',
                                  suth_S=GOLD['sutherland_S']['Ar'], A=0.98) for d in DELTAS]
        sims.append(hrlb.Solver(q, S, 'weno5', plist))
    bt = hrlb.Batch(sims, 16, 1)
    prev = None
    for k in range(STEPS // CHUNK):
        bt.step(CHUNK)
        assert np.all(np.isfinite(bt.residual()))
        cur = _diagnostics(sims, uw, MODELS, DELTAS)
        change = max(float(np.abs(cur[key] - prev[key]).max()) for key in cur) if prev else float('nan')
        print(f"[convergence] {(k + 1) * CHUNK} steps, largest change of nu, Pi, T0 since the last check {change:.1e}",
              flush=True)
        prev_change, prev = change, cur
    assert prev_change < study['settled']  # steady to well below the departures measured
    bad = []
    for d in DELTAS:
        conv = cur[(100, 32, d)]
        print(f"[convergence] delta {d}: converged nu {conv[0]:.5f}, Pi {conv[1]:.6f}, T0 {conv[2]:.5f}", flush=True)
        for Qx in QX:
            v = cur[(Qx, 16, d)]
            print(f"[convergence]   Qx {Qx:3d}: nu - nu_conv {v[0] - conv[0]:+.5f}, Pi/Pi_conv - 1 {v[1] / conv[1] - 1:+.2e}, "
                  f"T0/T0_conv - 1 {v[2] / conv[2] - 1:+.2e}", flush=True)
        v7 = cur[(7, 16, d)]
        if abs(v7[2] / conv[2] - 1) >= 1e-3:
            bad.append((d, 'T0(Qx=7) vs converged', v7[2] / conv[2] - 1))
        if abs(v7[1] / GOLD['Pi_uw_sqrt2']['Ar'][d] - 1) >= 2e-3:
            bad.append((d, 'Pi(Qx=7) vs table', v7[1] / GOLD['Pi_uw_sqrt2']['Ar'][d] - 1))
    assert not bad, bad
