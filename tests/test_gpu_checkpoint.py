"""Checkpoint and resume: N steps equal N/2 steps, a save to disk, a fresh solver restored
from the file, and N/2 more steps, bit for bit (eager and graph-captured steps, explicit and
reduced velocity sets); a file from another discretisation or other parameters is refused."""
import numpy as np
import pytest

from paper_1702_01335_amd import checkpoint, hrlb, inputs

from parity import make_wl

pytestmark = pytest.mark.gpu


def solver(wl, quad, B=2, graph=False, **over):
    import torch
    r = torch.from_numpy(np.stack([inputs.perturbation(70 + b, (wl['S'], quad.V)) for b in range(B)])).cuda()
    plist = [hrlb.make_params(**dict(wl['params'], u_w=0.2 + 0.1 * b, **over)) for b in range(B)]
    s = hrlb.Solver(quad, wl['S'], wl['scheme'], plist, perturb=r, eps=0.05)
    s.set_graph(graph)
    return s


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("reduced", [False, True])
def test_resume_equals_uninterrupted_run(tmp_path, graph, reduced):
    wl = make_wl(6, 5, 3, 21, 'weno5', A=0.9, dt=1e-4)
    quad = hrlb.ReducedQuadrature(6, 5) if reduced else hrlb.Quadrature(6, 5, 3)
    a = solver(wl, quad, graph=graph)
    a.step(40)
    Fa, Ra = a.get_state().cpu().numpy(), a.residual()
    b = solver(wl, quad, graph=graph)
    b.step(20)
    path = str(tmp_path / 'ck.npz')
    checkpoint.save(b, path, 20)
    del b
    c = solver(wl, quad, graph=graph)
    assert checkpoint.load(c, path) == 20
    c.step(20)
    assert np.array_equal(c.get_state().cpu().numpy(), Fa)
    assert np.array_equal(c.residual(), Ra)


def test_checkpoint_of_another_discretisation_is_refused(tmp_path):
    wl = make_wl(6, 5, 3, 21, 'weno5', A=0.9, dt=1e-4)
    a = solver(wl, hrlb.Quadrature(6, 5, 3))
    path = str(tmp_path / 'ck.npz')
    checkpoint.save(a, path, 0)
    with pytest.raises(ValueError):
        checkpoint.load(solver(wl, hrlb.Quadrature(6, 5, 4)), path)
    with pytest.raises(ValueError):
        checkpoint.load(solver(wl, hrlb.Quadrature(6, 5, 3), kn=0.3), path)
