"""The C ABI from plain C: tests/capi_c/couette_c.c sets up and advances a BGK Couette instance
through include/hrlb.h alone (hipMalloc'd buffers, its own HIP stream, no Python or torch in
its process; built by __graft_entry__.build()).  The moment table and residual it prints
must match the oracle's for the same instance."""
import os
import subprocess

import numpy as np
import pytest

from oracle import solver as sv

from parity import make_wl, oracle_run

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), 'capi_c', 'couette_c')


@pytest.mark.parametrize("scheme,code", [('upwind2', 0), ('weno5', 1)])
def test_plain_c_program_matches_oracle(scheme, code):
    assert os.path.exists(EXE), "tests/capi_c/couette_c is not built (python __graft_entry__.py build)"
    wl = make_wl(4, 4, 4, 24, scheme, pr=1.0, kn=0.1, u_w=0.1, omega=1.0, A=0.5, dt=5e-4)
    steps = 100
    p = wl['params']
    args = [EXE, str(wl['Qx']), str(wl['Qy']), str(wl['Qz']), str(wl['S']), str(code)] + \
        [repr(float(p[k])) for k in ('kn', 'u_w', 'pr', 'omega', 'A', 'dt')] + [str(steps)]
    print("[capi_c]", ' '.join(args[1:]), flush=True)
    out = subprocess.run(args, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    lines = out.stdout.strip().split('\n')
    R = float(lines[0].split()[1])
    mom = np.array([[float(x) for x in line.split()] for line in lines[1:]])
    Fo, m, Ro = oracle_run(wl, steps)   # the equilibrium start, as the program's
    ref = sv.moments(Fo, m).table()
    assert mom.shape == ref.shape
    # per column relative to its magnitude; columns that vanish by the flow's symmetry
    # (u_x, u_z, P_xz, P_yz, q_z) hold rounding noise and are held to 1e-14 absolute
    scale = np.maximum(np.abs(ref).max(axis=0), 1e-3)
    err = np.abs(mom - ref).max(axis=0) / scale
    print("[capi_c] worst column", int(np.argmax(err)), "relative error", float(err.max()), flush=True)
    assert np.all(err <= 1e-11)
    assert R == pytest.approx(Ro, rel=1e-8)
