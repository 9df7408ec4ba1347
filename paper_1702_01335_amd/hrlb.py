"""Python binding of libhrlb (C ABI in include/hrlb.h): argument marshalling only.

Every step of the solver runs in the library's HIP kernels; this module allocates the
caller-owned device buffers with torch, passes torch's current HIP stream, and converts
arguments.  It fails loudly (ImportError / RuntimeError) when the compiled library is
missing or a call returns an error; there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, 'libhrlb.so')

HRLB_OK, HRLB_EINVAL, HRLB_ENOMEM, HRLB_EHIP, HRLB_ENUMERIC = 0, -1, -2, -3, -4
LAW_POWER, LAW_SUTHERLAND, LAW_LOWMACH = 0, 1, 2
SCHEME_UPWIND2, SCHEME_WENO5, SCHEME_LINEAR5 = 0, 1, 2
SCHEMES = {'upwind2': SCHEME_UPWIND2, 'weno5': SCHEME_WENO5, 'linear5': SCHEME_LINEAR5}
LAWS = {'power': LAW_POWER, 'sutherland': LAW_SUTHERLAND, 'lowmach': LAW_LOWMACH}
MOMENT_NAMES = ('n', 'ux', 'uy', 'uz', 'T', 'Pxx', 'Pyy', 'Pzz', 'Pxy', 'Pxz', 'Pyz', 'qx', 'qy', 'qz')

EXPORTS = ('hrlb_last_error', 'hrlb_init_quadrature', 'hrlb_quad_free', 'hrlb_quad_size', 'hrlb_quad_nodes',
           'hrlb_state_bytes', 'hrlb_init_state', 'hrlb_sim_free', 'hrlb_step', 'hrlb_moments', 'hrlb_residual',
           'hrlb_get_state', 'hrlb_set_state', 'hrlb_set_launch', 'hrlb_get_launch', 'hrlb_autotune', 'hrlb_set_graph',
           'hrlb_set_timing', 'hrlb_get_timing', 'hrlb_batch_bytes', 'hrlb_batch_create', 'hrlb_batch_step',
           'hrlb_batch_residual', 'hrlb_batch_set_active', 'hrlb_batch_info', 'hrlb_batch_free', 'hrlb_seed_state',
           'hrlb_step_noalloc', 'hrlb_free_molecular_state', 'hrlb_get_stage_timing',
           'hrlb_init_quadrature_reduced', 'hrlb_trace_status')
SCRATCH_BYTES = 32 << 20  # HRLB_SCRATCH_BYTES


class HrlbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libhrlb error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    """Mirror of struct hrlb_params."""
    _fields_ = [('kn', ctypes.c_double), ('u_w', ctypes.c_double), ('T_w', ctypes.c_double),
                ('n0', ctypes.c_double), ('pr', ctypes.c_double), ('omega', ctypes.c_double),
                ('suth_S', ctypes.c_double), ('A', ctypes.c_double), ('dt', ctypes.c_double),
                ('law', ctypes.c_int), ('collisionless', ctypes.c_int)]


def make_params(kn, dt, u_w=0.0, T_w=1.0, n0=1.0, pr=1.0, law='power', omega=1.0, suth_S=0.0, A=0.0,
                collisionless=False):
    return Params(kn=kn, u_w=u_w, T_w=T_w, n0=n0, pr=pr, omega=omega, suth_S=suth_S, A=A, dt=dt,
                  law=LAWS[law] if isinstance(law, str) else int(law), collisionless=int(bool(collisionless)))


_lib = None


def load():
    """Load libhrlb.so (built in-tree by paper_1702_01335_amd.build); raises if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1702_01335_amd.build`")
    # torch brings its own HIP runtime; loading it first makes the library bind to that same
    # runtime instead of a second copy that would not share torch's device context
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, dp, ip, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int), ctypes.c_size_t
    lib.hrlb_last_error.restype = ctypes.c_char_p
    lib.hrlb_last_error.argtypes = []
    lib.hrlb_trace_status.argtypes = [ip]
    lib.hrlb_init_quadrature.argtypes = [ctypes.c_int] * 6 + [ctypes.POINTER(vp)]
    lib.hrlb_init_quadrature_reduced.argtypes = [ctypes.c_int] * 4 + [ctypes.POINTER(vp)]
    lib.hrlb_quad_free.argtypes = [vp]
    lib.hrlb_quad_free.restype = None
    lib.hrlb_quad_size.argtypes = [vp, ip]
    lib.hrlb_quad_nodes.argtypes = [vp, ctypes.c_int, dp, dp]
    lib.hrlb_state_bytes.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(sz), ctypes.POINTER(sz)]
    lib.hrlb_init_state.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Params), ctypes.c_int, vp, sz, vp, sz,
                                    vp, vp, ctypes.c_double, ctypes.POINTER(vp)]
    lib.hrlb_sim_free.argtypes = [vp]
    lib.hrlb_sim_free.restype = None
    lib.hrlb_step.argtypes = [vp, ctypes.c_int]
    lib.hrlb_moments.argtypes = [vp, vp]
    lib.hrlb_residual.argtypes = [vp, dp]
    lib.hrlb_get_state.argtypes = [vp, vp]
    lib.hrlb_set_state.argtypes = [vp, vp]
    lib.hrlb_seed_state.argtypes = [vp, vp, ctypes.c_int, ip]
    lib.hrlb_free_molecular_state.argtypes = [vp]
    lib.hrlb_set_launch.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    lib.hrlb_get_launch.argtypes = [vp, ip, ip]
    lib.hrlb_autotune.argtypes = [vp, ctypes.c_int, ctypes.c_char_p, ip, ip, dp]
    lib.hrlb_set_graph.argtypes = [vp, ctypes.c_int]
    lib.hrlb_set_timing.argtypes = [vp, ctypes.c_int]
    lib.hrlb_get_timing.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_longlong)]
    lib.hrlb_get_stage_timing.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_longlong)]
    lib.hrlb_batch_bytes.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(sz)]
    lib.hrlb_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, sz, vp,
                                      ctypes.POINTER(vp)]
    lib.hrlb_batch_step.argtypes = [vp, ctypes.c_int]
    lib.hrlb_batch_residual.argtypes = [vp, dp]
    lib.hrlb_batch_set_active.argtypes = [vp, ip]
    lib.hrlb_batch_info.argtypes = [vp, ip, ip, ip, ip]
    lib.hrlb_batch_free.argtypes = [vp]
    lib.hrlb_batch_free.restype = None
    lib.hrlb_step_noalloc.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Params), ctypes.c_int, vp, sz,
                                      ctypes.c_int, vp, vp]
    for name in EXPORTS:
        if name not in ('hrlb_last_error', 'hrlb_quad_free', 'hrlb_sim_free', 'hrlb_batch_free'):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc != HRLB_OK:
        raise HrlbError(rc, load().hrlb_last_error().decode())
    return rc


# ---- the C ABI under its own names -----------------------------------------------------

def trace_status():
    """True when the library emits roctx ranges (HRLB_TRACE set when it was first used)."""
    on = ctypes.c_int(0)
    _check(load().hrlb_trace_status(ctypes.byref(on)))
    return bool(on.value)


def init_quadrature(Qx, Nx, Qy, Ny, Qz, Nz):
    h = ctypes.c_void_p()
    _check(load().hrlb_init_quadrature(Qx, Nx, Qy, Ny, Qz, Nz, ctypes.byref(h)))
    return h


def init_quadrature_reduced(Qx, Nx, Qy, Ny):
    h = ctypes.c_void_p()
    _check(load().hrlb_init_quadrature_reduced(Qx, Nx, Qy, Ny, ctypes.byref(h)))
    return h


def state_bytes(quad, S, batch):
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    _check(load().hrlb_state_bytes(quad, S, batch, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def init_state(quad, S, scheme, params, state, work, stream, perturb=None, eps=0.0):
    arr = (Params * len(params))(*params)
    h = ctypes.c_void_p()
    _check(load().hrlb_init_state(quad, S, scheme, arr, len(params), ctypes.c_void_p(state.data_ptr()), state.numel(),
                                  ctypes.c_void_p(work.data_ptr()), work.numel(), ctypes.c_void_p(stream),
                                  ctypes.c_void_p(perturb.data_ptr() if perturb is not None else 0), eps,
                                  ctypes.byref(h)))
    return h


def step(sim, nsteps):
    _check(load().hrlb_step(sim, nsteps))


def moments(sim, out):
    _check(load().hrlb_moments(sim, ctypes.c_void_p(out.data_ptr())))


def step_noalloc(quad, S, scheme, params, state, nsteps, moments_out, stream):
    """hrlb_step_noalloc: state is a device uint8 tensor of the state size; its first
    [B][S][V] float64 array is advanced in place; moments_out is None or a device float64
    tensor [B][S][14]."""
    arr = (Params * len(params))(*params)
    _check(load().hrlb_step_noalloc(quad, S, scheme, arr, len(params), ctypes.c_void_p(state.data_ptr()),
                                    state.numel(), nsteps,
                                    ctypes.c_void_p(moments_out.data_ptr() if moments_out is not None else 0),
                                    ctypes.c_void_p(stream)))


def residual(sim, batch):
    out = np.zeros(batch)
    rc = load().hrlb_residual(sim, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return rc, out


# ---- convenience wrappers ----------------------------------------------------------------

class Quadrature:
    """HHLB(Nx;Qx) x HLB(Ny;Qy) x HLB(Nz;Qz) velocity set (host tables in the library)."""

    def __init__(self, Qx, Qy, Qz, Nx=None, Ny=None, Nz=None):
        self.Qx, self.Qy, self.Qz = Qx, Qy, Qz
        self.Nx = min(6, Qx - 1) if Nx is None else Nx
        self.Ny = Qy - 1 if Ny is None else Ny
        self.Nz = Qz - 1 if Nz is None else Nz
        self.handle = init_quadrature(Qx, self.Nx, Qy, self.Ny, Qz, self.Nz)
        v = ctypes.c_int()
        _check(load().hrlb_quad_size(self.handle, ctypes.byref(v)))
        self.V = v.value

    reduced = False

    def nodes(self, axis):
        n = {0: 2 * self.Qx, 1: self.Qy, 2: self.Qz}[axis]
        p, w = np.zeros(n), np.zeros(n)
        _check(load().hrlb_quad_nodes(self.handle, axis, p.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return p, w

    def __del__(self):
        if getattr(self, 'handle', None) and _lib is not None:
            _lib.hrlb_quad_free(self.handle)
            self.handle = None


class ReducedQuadrature(Quadrature):
    """The paper's HHLB(Nx;Qx) x HLB(Ny;Qy) with p_z integrated out: populations phi and chi
    (Eq. reduced_def) per velocity, flat index (i Qy + j) 2 + c, c = 0 phi, 1 chi."""

    reduced = True

    def __init__(self, Qx, Qy, Nx=None, Ny=None):
        self.Qx, self.Qy, self.Qz = Qx, Qy, 2
        self.Nx = min(6, Qx - 1) if Nx is None else Nx
        self.Ny = Qy - 1 if Ny is None else Ny
        self.Nz = 0
        self.handle = init_quadrature_reduced(Qx, self.Nx, Qy, self.Ny)
        v = ctypes.c_int()
        _check(load().hrlb_quad_size(self.handle, ctypes.byref(v)))
        self.V = v.value


class Solver:
    """A batch of Couette instances sharing a velocity set, node count and scheme.

    Device buffers are torch uint8 tensors on ``device``; the library enqueues on the
    torch stream current at construction.  ``perturb`` (torch float64 [B, S, V] on the
    device) and ``eps`` seed the initial state F = n0 F^eq_rest (1 + eps r)."""

    def __init__(self, quad, S, scheme, params, device='cuda', perturb=None, eps=0.0):
        import torch
        self.torch = torch
        self.quad, self.S, self.B, self.V = quad, S, len(params), quad.V
        self.scheme = SCHEMES[scheme] if isinstance(scheme, str) else scheme
        sb, wb = state_bytes(quad.handle, S, self.B)
        self.state = torch.empty(sb, dtype=torch.uint8, device=device)
        self.work = torch.empty(wb, dtype=torch.uint8, device=device)
        self.device = self.state.device
        self.stream = torch.cuda.current_stream(self.device)
        if perturb is not None:
            perturb = perturb.to(device=self.device, dtype=torch.float64).contiguous()
            assert tuple(perturb.shape) == (self.B, S, self.V)
        self._perturb = perturb
        self.params = list(params)
        self.handle = init_state(quad.handle, S, self.scheme, self.params, self.state, self.work,
                                 self.stream.cuda_stream, perturb, eps)

    def step(self, nsteps=1):
        step(self.handle, nsteps)

    def moments(self):
        out = self.torch.empty((self.B, self.S, 14), dtype=self.torch.float64, device=self.device)
        moments(self.handle, out)
        return out

    def residual(self, raise_on_fault=True):
        rc, out = residual(self.handle, self.B)
        if rc != HRLB_OK and raise_on_fault:
            _check(rc)
        return out if raise_on_fault else (rc, out)

    def get_state(self):
        out = self.torch.empty((self.B, self.S, self.V), dtype=self.torch.float64, device=self.device)
        _check(load().hrlb_get_state(self.handle, ctypes.c_void_p(out.data_ptr())))
        return out

    def set_state(self, F):
        F = F.to(device=self.device, dtype=self.torch.float64).contiguous()
        assert tuple(F.shape) == (self.B, self.S, self.V)
        self._staged = F
        _check(load().hrlb_set_state(self.handle, ctypes.c_void_p(F.data_ptr())))

    def seed_state(self, table, preserve_mass=True):
        """Warm start from a moment table (torch float64 [B, S, 14] on the device, the
        column order of moments()), scaled to the mass of the equilibrium start unless
        preserve_mass is False.  Returns the per-instance fallback flags (1 where the table
        was invalid and the equilibrium at rest was used)."""
        t = table.to(device=self.device, dtype=self.torch.float64).contiguous()
        assert tuple(t.shape) == (self.B, self.S, 14)
        fb = np.zeros(self.B, dtype=np.int32)
        _check(load().hrlb_seed_state(self.handle, ctypes.c_void_p(t.data_ptr()), 1 if preserve_mass else 0,
                                      fb.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
        return fb

    def free_molecular_state(self):
        """Overwrite the state with the free-molecular steady state of the diffuse walls."""
        _check(load().hrlb_free_molecular_state(self.handle))

    def set_launch(self, cells, waves):
        _check(load().hrlb_set_launch(self.handle, cells, waves))

    def get_launch(self):
        c, w = ctypes.c_int(), ctypes.c_int()
        _check(load().hrlb_get_launch(self.handle, ctypes.byref(c), ctypes.byref(w)))
        return c.value, w.value

    def autotune(self, probe_steps=5, cache_path=None):
        c, w, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        path = cache_path.encode() if cache_path else None
        _check(load().hrlb_autotune(self.handle, probe_steps, path, ctypes.byref(c), ctypes.byref(w), ctypes.byref(ms)))
        return c.value, w.value, ms.value

    def set_graph(self, on):
        _check(load().hrlb_set_graph(self.handle, int(bool(on))))

    def set_timing(self, on):
        _check(load().hrlb_set_timing(self.handle, int(bool(on))))

    def get_timing(self):
        ms = (ctypes.c_double * 2)()
        n = (ctypes.c_longlong * 2)()
        _check(load().hrlb_get_timing(self.handle, ms, n))
        return {'stage_ms': ms[0], 'stage_launches': n[0], 'closure_ms': ms[1], 'closure_launches': n[1]}

    def get_stage_timing(self):
        """Device time (ms) and launch counts of the stage kernel per RK3 stage and of the
        closure kernel, accumulated since set_timing(True)."""
        ms = (ctypes.c_double * 4)()
        n = (ctypes.c_longlong * 4)()
        _check(load().hrlb_get_stage_timing(self.handle, ms, n))
        return {'stage_ms': [ms[0], ms[1], ms[2]], 'stage_launches': [n[0], n[1], n[2]], 'closure_ms': ms[3],
                'closure_launches': n[3]}

    def synchronize(self):
        self.stream.synchronize()

    def __del__(self):
        if getattr(self, 'handle', None) and _lib is not None:
            try:
                self.stream.synchronize()
            except Exception:
                pass
            _lib.hrlb_sim_free(self.handle)
            self.handle = None


class Batch:
    """Several Solvers (groups of instances that differ in velocity set, node count or
    scheme) advanced together by one launch per kernel per stage, graph-captured.
    All solvers must use the torch stream current at construction."""

    def __init__(self, solvers, cells, waves):
        import torch
        self.torch = torch
        self.solvers = list(solvers)
        arr = (ctypes.c_void_p * len(self.solvers))(*[s.handle for s in self.solvers])
        self._arr = arr
        nbytes = ctypes.c_size_t()
        _check(load().hrlb_batch_bytes(arr, len(arr), cells, waves, ctypes.byref(nbytes)))
        dev = self.solvers[0].device
        self.work = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=dev)
        self.stream = torch.cuda.current_stream(dev)
        h = ctypes.c_void_p()
        _check(load().hrlb_batch_create(arr, len(arr), cells, waves, ctypes.c_void_p(self.work.data_ptr()),
                                        self.work.numel(), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.handle = h
        self.B = sum(s.B for s in self.solvers)

    def step(self, nsteps=1):
        _check(load().hrlb_batch_step(self.handle, nsteps))

    def residual(self, raise_on_fault=True):
        out = np.zeros(self.B)
        rc = load().hrlb_batch_residual(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        if raise_on_fault:
            _check(rc)
            return out
        return rc, out

    def set_active(self, active):
        a = np.ascontiguousarray(np.asarray(active, dtype=np.int32))
        assert a.shape == (self.B,)
        _check(load().hrlb_batch_set_active(self.handle, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))

    def info(self):
        v = [ctypes.c_int() for _ in range(4)]
        _check(load().hrlb_batch_info(self.handle, *[ctypes.byref(x) for x in v]))
        return dict(zip(('tiles', 'closure_items', 'grid_stage', 'grid_closure'), [x.value for x in v]))

    def __del__(self):
        if getattr(self, 'handle', None) and _lib is not None:
            try:
                self.stream.synchronize()
            except Exception:
                pass
            _lib.hrlb_batch_free(self.handle)
            self.handle = None
