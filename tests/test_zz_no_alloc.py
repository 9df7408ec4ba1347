"""hrlb_step_noalloc, whose work memory is the library's fixed per-GPU array, against the
entry points with a caller work buffer (hrlb_init_state, hrlb_step, hrlb_moments) on the same
populations: two calls in a row, the second with a smaller batch, fewer nodes and another
velocity set, each equal to the work-buffer path bit for bit (the same kernels in the same
launch shape), and one instance of each also against the oracle."""
import numpy as np
import pytest

from paper_1702_01335_amd import hrlb, inputs

from parity import assert_parity, make_wl, oracle_run

pytestmark = pytest.mark.gpu

# (label, workload, batch, steps): the first call larger than the second
CASES = [
    ('shakhov-weno5-v800', make_wl(16, 5, 5, 40, 'weno5', A=0.9, dt=2e-5), 6, 7),
    ('bgk-upwind2-v90', make_wl(5, 3, 3, 13, 'upwind2', pr=1.0, omega=1.0), 2, 4),
]


def run_case(label, wl, B, steps):
    import torch
    q = hrlb.Quadrature(wl['Qx'], wl['Qy'], wl['Qz'])
    S, V = wl['S'], q.V
    seeds = [500 + b for b in range(B)]
    plist = [dict(wl['params'], u_w=wl['params']['u_w'] * (1 + 0.2 * b)) for b in range(B)]
    params = [hrlb.make_params(**p) for p in plist]
    r = torch.from_numpy(np.stack([inputs.perturbation(sd, (S, V)) for sd in seeds])).cuda()
    # the work-buffer path
    s = hrlb.Solver(q, S, wl['scheme'], params, perturb=r, eps=0.05)
    F0 = s.get_state().clone()
    s.step(steps)
    F_ref = s.get_state()
    mom_ref = s.moments()
    s.synchronize()
    # the fixed-array path on a fresh state buffer holding the same populations
    sb, wb = hrlb.state_bytes(q.handle, S, B)
    assert wb <= hrlb.SCRATCH_BYTES
    state = torch.zeros(sb, dtype=torch.uint8, device='cuda')
    n = B * S * V
    state[:8 * n].view(torch.float64).copy_(F0.reshape(-1))
    mom = torch.full((B, S, 14), float('nan'), dtype=torch.float64, device='cuda')
    print(f"[noalloc] {label}: B={B} S={S} V={V} steps={steps} work bytes {wb}", flush=True)
    hrlb.step_noalloc(q.handle, S, hrlb.SCHEMES[wl['scheme']], params, state, steps, mom,
                      torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    F = state[:8 * n].view(torch.float64).reshape(B, S, V)
    assert torch.equal(F, F_ref), label
    assert torch.equal(mom, mom_ref), label
    Fo, m, _ = oracle_run(wl, steps, seed=seeds[-1], params=plist[-1])
    assert_parity(F[-1].cpu().numpy(), Fo, m, f"noalloc {label}, instance {B - 1}")


def test_noalloc_equals_work_buffer_path_twice():
    for case in CASES:
        run_case(*case)
