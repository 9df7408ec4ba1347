"""The linearised (low Mach) Couette flow of Sec. IV on the GPU: BGK (Pr = 1), tau = k/sqrt 2
(Eq. knLuo), u_w = 1e-5, HHLB(N_x;Q_x) x HLB(1;2) on the phi function alone (Q_z = 1), nodes
stretched with A = 0.98, WENO-5, the Table I models for k = 0.03 (Q_x = 4, S = 64), 0.1
(Q_x = 7, S = 32) and 1 (Q_x = 21, S = 32); k = 10 needs Q_x = 80 and about 10^6 steps.
The paper compares these runs with linearised-Boltzmann benchmark data that is not at hand
here.  What holds without it, and is checked:
  * linear response: the observables divided by u_w agree at u_w = 1e-5 and 2e-5;
  * the limits the observables of Eqs. uslip, ud0_extra, mflow and Txy approach, and their
    order in k: the slip u_slip / u_w is positive and grows with k; L u'_y(0) / 2u_w and
    mdot / mdot_hydro lie below their hydrodynamic value 1 and fall as k grows; T_xy /
    T_xy^bal lies below its ballistic value 1 and grows with k.
About 30 s of GPU time."""
import numpy as np
import pytest

from oracle import diagnostics as dg
from oracle import solver as sv
from paper_1702_01335_amd import hrlb

pytestmark = pytest.mark.gpu

# (k, Q_x, S, dt): Table I; dt keeps max|p_x| dt / dx_min near 0.45 on each grid
CASES = [(0.03, 4, 64, 1e-4), (0.1, 7, 32, 1.5e-4), (1.0, 21, 32, 7.5e-5)]
UW = (1e-5, 2e-5)
STEPS, CHUNK = 400000, 50000


def _observables(sims):
    out = {}
    for (k, Qx, S, _), s in zip(CASES, sims):
        mom = s.moments().cpu().numpy()
        x = sv.Grid(S, 0.98).x(np.arange(1, S + 1))
        for b, uw in enumerate(UW):
            n, uy, Pxy = mom[b, :, 0], mom[b, :, 2], mom[b, :, 8]
            out[(k, uw)] = np.array([dg.u_slip(x, uy, uw) / uw,
                                     dg.centre_derivative(x, uy) / (2 * uw),
                                     dg.mass_flow(n, uy, 0.98) / dg.mass_flow_hydro(1.0, uw),
                                     dg.mean_shear_stress(Pxy, 0.98) / dg.ballistic_shear_stress(1.0, uw)])
    return out


def test_linearised_couette_flow_limits_and_linear_response():
    sims = []
    for k, Qx, S, dt in CASES:
        q = hrlb.Quadrature(Qx, 2, 1)
        plist = [hrlb.make_params(kn=k, dt=dt, u_w=uw, pr=1.0, law='lowmach', A=0.98) for uw in UW]
        sims.append(hrlb.Solver(q, S, 'weno5', plist))
    bt = hrlb.Batch(sims, 16, 1)
    prev = None
    for c in range(STEPS // CHUNK):
        bt.step(CHUNK)
        assert np.all(np.isfinite(bt.residual()))
        cur = _observables(sims)
        change = max(float(np.abs(cur[key] - prev[key]).max()) for key in cur) if prev else float('nan')
        print(f"[lowmach] {(c + 1) * CHUNK} steps, largest change since the last check {change:.1e}", flush=True)
        prev_change, prev = change, cur
    assert prev_change < 1e-5
    rows = [cur[(k, UW[0])] for k, _, _, _ in CASES]
    for (k, _, _, _), r in zip(CASES, rows):
        print(f"[lowmach] k = {k}: u_slip/u_w {r[0]:.5f}, L u'(0)/2u_w {r[1]:.5f}, mdot/mdot_hydro {r[2]:.5f}, "
              f"T_xy/T_xy^bal {r[3]:.5f}", flush=True)
        # linear response: u_w = 2e-5 gives the same normalised observables.  Exactly so in
        # exact arithmetic (the epsilon-free WENO weights are ratios of indicators that scale
        # together); in FP64 the indicators are differences of O(1) populations that differ by
        # O(u_w), and the centre-line velocities are ~1e-7, so rounding enters at ~1e-9 relative
        # and the nonlinear weights amplify it (measured 6e-6): 1e-4 relative is the check
        np.testing.assert_allclose(cur[(k, UW[1])], r, rtol=1e-4, atol=1e-9)
    slip, grad, mflow, txy = (np.array([r[i] for r in rows]) for i in range(4))
    assert np.all(slip > 0) and np.all(np.diff(slip) > 0)
    assert np.all(grad < 1) and np.all(np.diff(grad) < 0)
    assert np.all(mflow < 1) and np.all(np.diff(mflow) < 0)
    assert np.all(txy > 0) and np.all(txy < 1) and np.all(np.diff(txy) > 0)
