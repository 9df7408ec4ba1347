"""Checkpoint and resume of a Solver: the populations [B][S][V] (float64, read back with
hrlb_get_state and restored with hrlb_set_state), the step counter, the per-instance
parameters and a fingerprint of the discretisation (expansion orders, the velocity set's
nodes and weights, node count, scheme) in one .npz file.  Loading refuses a file written by
another discretisation or other parameters.  The restored run continues bit for bit: the
moment partials are recomputed from the populations in the solver's launch shape, as the
step's own epilogue computes them."""
import hashlib

import numpy as np

from . import hrlb

PARAM_FIELDS = [name for name, _ in hrlb.Params._fields_]


def fingerprint(solver):
    q = solver.quad
    h = hashlib.sha256()
    for axis in ((0, 1) if getattr(q, 'reduced', False) else (0, 1, 2)):
        p, w = q.nodes(axis)
        h.update(p.tobytes())
        h.update(w.tobytes())
    head = dict(Qx=q.Qx, Nx=q.Nx, Qy=q.Qy, Ny=q.Ny, Qz=q.Qz, Nz=q.Nz, reduced=int(getattr(q, 'reduced', False)),
                S=solver.S, V=solver.V, B=solver.B, scheme=int(solver.scheme))
    return head, h.hexdigest()


def params_array(solver):
    return np.array([[float(getattr(p, f)) for f in PARAM_FIELDS] for p in solver.params])


def save(solver, path, step):
    """Write the solver's current state and `step` to path (.npz)."""
    head, digest = fingerprint(solver)
    F = solver.get_state().cpu().numpy()
    np.savez(path, F=F, step=np.int64(step), params=params_array(solver), digest=np.array(digest),
             **{k: np.int64(v) for k, v in head.items()})


def load(solver, path):
    """Restore the state saved in path into `solver` (same discretisation and parameters);
    returns the saved step counter."""
    d = np.load(path, allow_pickle=False)
    head, digest = fingerprint(solver)
    for k, v in head.items():
        if int(d[k]) != v:
            raise ValueError(f"checkpoint {path}: {k} = {int(d[k])}, the solver has {v}")
    if str(d['digest']) != digest:
        raise ValueError(f"checkpoint {path}: written with another velocity set")
    if not np.array_equal(d['params'], params_array(solver)):
        raise ValueError(f"checkpoint {path}: written with other instance parameters")
    import torch
    solver.set_state(torch.from_numpy(d['F']).to(solver.device))
    return int(d['step'])
