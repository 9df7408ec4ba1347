"""Helpers of the GPU parity tests: run the same seeded instance through the HIP library and
through the oracle, and compare the populations.

Tolerance (derived): with rounding only, the two FP64 paths agree to
a few ulp per operation, accumulated over the stages.  Two scales are checked:
  * normwise: max |F_gpu - F_oracle| / max |F_oracle| <= 1e-12;
  * per velocity column: max_s |F_gpu - F_oracle| / max_s |F_oracle| <= max(1e-10, 8 eps kappa_v),
    where kappa_v (``kappa`` below) is the first-order rounding amplification of the
    Hermite-projected equilibrium (Sec. III) at that velocity; it exceeds 1e5 only at the
    outermost half-range nodes, whose populations are ~w ~ 1e-15 .. 1e-52.
"""
import numpy as np

from oracle import solver as sv
from paper_1702_01335_amd import hrlb, inputs
from paper_1702_01335_amd.workloads import workload

NORM_TOL = 1e-12
COL_TOL = 1e-10


def oracle_params(wl, p=None):
    p = dict(wl['params']) if p is None else dict(p)
    return sv.Params(Qx=wl['Qx'], Qy=wl['Qy'], Qz=wl['Qz'], S=wl['S'], scheme=wl['scheme'],
                     Nx=wl.get('Nx'), Ny=wl.get('Ny'), Nz=wl.get('Nz'),
                     **{k: v for k, v in p.items()})


def make_wl(Qx, Qy, Qz, S, scheme, **params):
    base = dict(kn=0.2, u_w=0.3, T_w=1.0, n0=1.0, pr=2.0 / 3.0, law='power', omega=0.7, A=0.0, dt=2e-4)
    base.update(params)
    return dict(Qx=Qx, Qy=Qy, Qz=Qz, S=S, scheme=scheme, params=base)


def kappa(model):
    """Per-velocity first-order rounding amplification of the projected equilibrium: a
    coefficient J_l = sum_k C_lk M_k (M_k the Gaussian moments) carries an error of a few ulp
    of sum_k |C_lk| |M_k|, and node i multiplies it by |w_i P_l(x_i) / gamma_l| / w_i
    relative to its weight; the three axes multiply (oracle tables, u = 0, T = 1 moments)."""
    from oracle import equilibrium as eq
    vs = model.vs

    def axis(ax, mom):
        cl = np.abs(ax.C) @ np.abs(mom)
        return (np.abs(ax.Phi) * cl).sum(1)

    kx = axis(vs.X, eq.half_gaussian_moments(vs.X.N, 0.0, 1.0)) / vs.X.weights[vs.X.Q:]
    kx = np.concatenate([kx[::-1], kx])
    ky = axis(vs.Y, eq.gaussian_moments(vs.Y.N, 0.0, 1.0)) / vs.Y.weights
    kz = axis(vs.Z, eq.gaussian_moments(vs.Z.N, 0.0, 1.0)) / vs.Z.weights
    return (kx[:, None, None] * ky[None, :, None] * kz[None, None, :]).ravel()


def gpu_run(wl, steps, seeds=None, eps=0.05, params_list=None, launch=None, device='cuda'):
    import torch
    q = hrlb.Quadrature(wl['Qx'], wl['Qy'], wl['Qz'], wl.get('Nx'), wl.get('Ny'), wl.get('Nz'))
    plist = params_list if params_list is not None else [wl['params']]
    B = len(plist)
    r = None
    if seeds is not None:
        r = np.stack([inputs.perturbation(sd, (wl['S'], q.V)) for sd in seeds])
        r = torch.from_numpy(r).to(device)
    solver = hrlb.Solver(q, wl['S'], wl['scheme'], [hrlb.make_params(**p) for p in plist], device=device,
                         perturb=r, eps=eps if seeds is not None else 0.0)
    if launch is not None:
        solver.set_launch(*launch)
    solver.step(steps)
    F = solver.get_state().cpu().numpy()
    mom = solver.moments().cpu().numpy()
    res = solver.residual()
    return F, mom, res, solver


def oracle_run(wl, steps, seed=None, eps=0.05, params=None):
    m = sv.Model(oracle_params(wl, params))
    if seed is None:
        F = sv.equilibrium_state(m)
    else:
        F = sv.seeded_state(m, inputs.perturbation(seed, (m.p.S, m.V)), eps)
    Fprev = F
    for _ in range(steps):
        Fprev = F
        F = sv.rk3_step(F, m)
    R = sv.residual(F, Fprev, m.p.dt) if steps > 0 else 0.0
    return F, m, R


def compare(Fg, Fo, model):
    err = np.abs(Fg - Fo)
    norm = err.max() / np.abs(Fo).max()
    col = err.max(axis=0) / np.abs(Fo).max(axis=0)
    tol = np.maximum(COL_TOL, 8 * np.finfo(float).eps * kappa(model))
    worst = int(np.argmax(col / tol))
    return dict(norm=norm, col=col.max(), col_over_tol=float((col / tol).max()), worst_v=worst,
                worst_kappa=float(kappa(model)[worst]))


def assert_parity(Fg, Fo, model, label=''):
    c = compare(Fg, Fo, model)
    print(f"[parity] {label} normwise={c['norm']:.3e} column={c['col']:.3e} col/tol={c['col_over_tol']:.3f}", flush=True)
    assert c['norm'] <= NORM_TOL, c
    assert c['col_over_tol'] <= 1.0, c
    return c
