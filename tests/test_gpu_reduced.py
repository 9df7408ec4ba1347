"""The paper's reduced model on the GPU (Sec. III: phi = int f dp_z, chi = int f p_z^2 dp_z of
Eq. reduced_def, evolved by Eq. boltz_red with phi^eq of Eq. phieq, chi^eq = T phi^eq and the
reduced Shakhov factors of Eq. sred_def; chi_w = T_w phi_w at the wall, App. A.4) against the
oracle's literal implementation of those equations (oracle/reduced.py), element by element
at equal step counts from the same seeded start, and against the explicit-z path: for a
scheme linear in F and N_z >= 4 the z-sums of the explicit populations are phi and chi."""
import numpy as np
import pytest

from oracle import reduced as rd
from oracle import solver as sv
from paper_1702_01335_amd import hrlb, inputs

from parity import COL_TOL, NORM_TOL, make_wl, oracle_params

pytestmark = pytest.mark.gpu


def gpu_reduced(wl, steps, seed, eps=0.05, launch=None, graph=False):
    import torch
    q = hrlb.ReducedQuadrature(wl['Qx'], wl['Qy'], wl.get('Nx'), wl.get('Ny'))
    r = torch.from_numpy(inputs.perturbation(seed, (wl['S'], q.V))[None]).cuda()
    s = hrlb.Solver(q, wl['S'], wl['scheme'], [hrlb.make_params(**wl['params'])], perturb=r, eps=eps)
    if launch:
        s.set_launch(*launch)
    s.set_graph(graph)
    s.step(steps)
    return s.get_state().cpu().numpy()[0], s.moments().cpu().numpy()[0], s.residual()[0]


def oracle_reduced(wl, steps, seed, eps=0.05):
    """The oracle's reduced model from the same seeded start: the GPU's column
    (i Qy + j) 2 + c is the oracle's phi (c = 0) or chi (c = 1) at velocity i Qy + j."""
    rm = rd.ReducedModel(oracle_params(wl))
    st = rm.equilibrium_state()
    r = inputs.perturbation(seed, (wl['S'], 2 * rm.V))
    st = st * (1.0 + eps * np.stack([r[:, 0::2], r[:, 1::2]]))
    prev = st
    for _ in range(steps):
        prev = st
        st = rm.step(st)
    F = np.empty((wl['S'], 2 * rm.V))
    F[:, 0::2], F[:, 1::2] = st[0], st[1]
    Fp = np.empty_like(F)
    Fp[:, 0::2], Fp[:, 1::2] = prev[0], prev[1]
    R = np.sqrt(np.sum((F - Fp) ** 2)) / (rm.p.dt * np.sqrt(np.sum(Fp ** 2))) if steps else 0.0
    return F, rm, R


def check(Fg, Fo, label):
    err = np.abs(Fg - Fo)
    norm = err.max() / np.abs(Fo).max()
    col = (err.max(axis=0) / np.abs(Fo).max(axis=0)).max()
    print(f"[reduced] {label}: normwise {norm:.2e}, column {col:.2e}", flush=True)
    assert norm <= NORM_TOL and col <= COL_TOL


# shapes spanning several blocks with ragged tails: V = 4 Qx Qy
CASES = [
    ('weno5-shakhov-stretched', make_wl(5, 4, 1, 13, 'weno5', A=0.9, dt=1e-4)),
    ('upwind2-bgk', make_wl(6, 5, 1, 11, 'upwind2', pr=1.0, omega=1.0)),
    ('weno5-sutherland', make_wl(4, 7, 1, 12, 'weno5', law='sutherland', suth_S=0.5239, kn=0.05, u_w=1.0)),
    ('weno5-collisionless', make_wl(6, 4, 1, 9, 'weno5', collisionless=True, u_w=0.5)),
    ('minimal-S3', make_wl(2, 3, 1, 3, 'weno5', dt=1e-4)),
]


@pytest.mark.parametrize("label,wl", CASES, ids=[c[0] for c in CASES])
def test_reduced_small_shapes_match_oracle(label, wl):
    Fg, mom, R = gpu_reduced(wl, 6, seed=17)
    Fo, rm, Ro = oracle_reduced(wl, 6, seed=17)
    check(Fg, Fo, label)
    assert R == pytest.approx(Ro, rel=1e-9)
    # moments: the phi, chi forms of Eq. qdef (u_z, q_z and the off-diagonal z stresses vanish)
    n, ux, uy, T, P, qx, qy, _, _ = rm.moments(Fo[:, 0::2], Fo[:, 1::2])
    ref = np.stack([n, ux, uy, 0 * n, T, P['xx'], P['yy'], P['zz'], P['xy'], 0 * n, 0 * n, qx, qy, 0 * n], axis=-1)
    scale = np.maximum(np.abs(ref).max(axis=0), 1e-3)
    assert (np.abs(mom - ref) / scale).max() <= 1e-11


@pytest.mark.parametrize("cells,waves", [(1, 1), (4, 2), (16, 3), (64, 4)])
def test_reduced_launch_shapes(cells, waves):
    wl = CASES[0][1]
    Fg, _, _ = gpu_reduced(wl, 3, seed=23, launch=(cells, waves), graph=True)
    Fo, _, _ = oracle_reduced(wl, 3, seed=23)
    check(Fg, Fo, f"cells={cells} waves={waves}")


@pytest.mark.parametrize("steps", [1, 100])
def test_reduced_paper_shape(steps):
    """The paper's own runs of Sec. VI: HHLB(6;7) x HLB(6;7) reduced (196 populations per
    node), 16 nodes with A = 0.98, Sutherland (argon, delta = 1), u_w = sqrt 2, dt = 5e-4."""
    wl = make_wl(7, 7, 1, 16, 'weno5', law='sutherland', suth_S=0.5239, kn=1 / np.sqrt(2), u_w=np.sqrt(2),
                 A=0.98, dt=5e-4)
    Fg, _, R = gpu_reduced(wl, steps, seed=29)
    Fo, _, Ro = oracle_reduced(wl, steps, seed=29)
    check(Fg, Fo, f"paper shape, {steps} steps")
    assert R == pytest.approx(Ro, rel=1e-8)


def test_reduced_second_workload_shape():
    """The second workload's velocity set and grid with p_z integrated out: HHLB(6;16) x
    HLB(4;5) reduced (320 populations per node), 256 nodes, A = 0.98, Shakhov Pr = 2/3,
    mu ~ T^(1/2), Kn = 1, u_w = 0.4, WENO-5, dt = 1e-5, 10 steps."""
    wl = make_wl(16, 5, 1, 256, 'weno5', kn=1.0, u_w=0.4, omega=0.5, A=0.98, dt=1e-5)
    Fg, _, R = gpu_reduced(wl, 10, seed=31)
    Fo, _, Ro = oracle_reduced(wl, 10, seed=31)
    check(Fg, Fo, "second workload shape, 10 steps")
    assert R == pytest.approx(Ro, rel=1e-8)


@pytest.mark.parametrize("pr", [2 / 3, 1.0])
def test_explicit_z_sums_equal_the_reduced_model(pr):
    """Upwind-2 (linear in F), N_z = 4: the explicit path's z-sums are the reduced path's phi
    and chi, both on the GPU, from the equilibrium start."""
    import torch
    wl = make_wl(5, 6, 5, 10, 'upwind2', kn=0.15, u_w=0.6, pr=pr, omega=0.5, A=0.5, dt=2e-4)
    qe, qr = hrlb.Quadrature(5, 6, 5), hrlb.ReducedQuadrature(5, 6)
    p = [hrlb.make_params(**wl['params'])]
    se = hrlb.Solver(qe, 10, 'upwind2', p)
    sr = hrlb.Solver(qr, 10, 'upwind2', p)
    se.step(60)
    sr.step(60)
    Fe = se.get_state().cpu().numpy()[0].reshape(10, 10, 6, 5)
    Fr = sr.get_state().cpu().numpy()[0].reshape(10, 10, 6, 2)
    pz, _ = qe.nodes(2)
    phi, chi = Fe.sum(-1), (Fe * pz ** 2).sum(-1)
    scale = np.abs(Fr[..., 0]).max()
    assert np.abs(phi - Fr[..., 0]).max() / scale < 1e-13
    assert np.abs(chi - Fr[..., 1]).max() / scale < 1e-13
    assert np.abs(se.moments().cpu().numpy()[0, :, 2]).max() > 1e-2


def test_reduced_largest_velocity_set():
    """The paper's largest model, HHLB(6;100) on x, with HLB(15;16) on y (2 x 200 x 16
    populations per node), 13 nodes, 5 steps from a seeded start."""
    wl = make_wl(100, 16, 1, 13, 'weno5', dt=1e-3, kn=1.0, u_w=0.3, omega=0.5)
    wl.update(Nx=6, Ny=15)
    Fg, _, _ = gpu_reduced(wl, 5, seed=77)
    Fo, _, _ = oracle_reduced(wl, 5, seed=77)
    err = np.abs(Fg - Fo)
    norm = err.max() / np.abs(Fo).max()
    col = (err.max(axis=0) / np.abs(Fo).max(axis=0)).max()
    print(f"[reduced] HHLB(6;100) x HLB(15;16): normwise {norm:.2e}, column {col:.2e}", flush=True)
    # per column: twice the measured 1.9e-8; the x factors of HHLB(6;100) are off the exact
    # (mpmath) ones by up to 3.5e-9 per column on both sides, so 1e-10 is out of reach
    assert norm <= NORM_TOL and col <= 4e-8
