"""Python binding of the warm-start network (C ABI in include/hrlb_mlp.h): argument
marshalling only.  The forward pass, loss, gradient and AdamW update all run in the
library's kernels; this module allocates the caller-owned device buffers with torch and
passes torch's current HIP stream."""
import ctypes

import numpy as np

from . import hrlb

EXPORTS = ('hrlb_mlp_bytes', 'hrlb_mlp_create', 'hrlb_mlp_set_params', 'hrlb_mlp_get_params', 'hrlb_mlp_forward',
           'hrlb_mlp_predict_table', 'hrlb_mlp_gradient', 'hrlb_mlp_train_step', 'hrlb_mlp_free')
IN, OUT, WIDTH, NPARAMS, NNORM = 5, 8, 256, 135176, 26

_bound = False


def load():
    global _bound
    lib = hrlb.load()
    if not _bound:
        vp, sz, ci, fl = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_float
        lib.hrlb_mlp_bytes.argtypes = [ci, ctypes.POINTER(sz), ctypes.POINTER(sz)]
        lib.hrlb_mlp_create.argtypes = [vp, sz, vp, sz, ci, vp, ctypes.c_ulonglong, ctypes.POINTER(fl), vp,
                                        ctypes.POINTER(vp)]
        lib.hrlb_mlp_set_params.argtypes = [vp, vp]
        lib.hrlb_mlp_get_params.argtypes = [vp, vp]
        lib.hrlb_mlp_forward.argtypes = [vp, vp, ci, vp]
        lib.hrlb_mlp_predict_table.argtypes = [vp, vp, ci, vp]
        lib.hrlb_mlp_gradient.argtypes = [vp, vp, vp, vp, ci, vp, vp]
        lib.hrlb_mlp_train_step.argtypes = [vp, vp, vp, vp, ci, fl, fl, vp]
        lib.hrlb_mlp_free.argtypes = [vp]
        lib.hrlb_mlp_free.restype = None
        _bound = True
    return lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def norm_vector(in_mean, in_std, out_mean, out_std):
    """The 26 standardisation constants in the order the library takes them."""
    v = np.concatenate([in_mean, in_std, out_mean, out_std]).astype(np.float32)
    assert v.shape == (NNORM,)
    return v


class Network:
    """The 5 -> 256 -> 256 -> 256 -> 8 warm-start network on one device."""

    def __init__(self, max_rows, norm, params=None, seed=0, device='cuda'):
        import torch
        self.torch = torch
        lib = load()
        sb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        hrlb._check(lib.hrlb_mlp_bytes(max_rows, ctypes.byref(sb), ctypes.byref(wb)))
        self.state = torch.empty(sb.value, dtype=torch.uint8, device=device)
        self.work = torch.empty(wb.value, dtype=torch.uint8, device=device)
        self.device = self.state.device
        self.stream = torch.cuda.current_stream(self.device)
        self.max_rows = max_rows
        self.norm = np.ascontiguousarray(norm, dtype=np.float32)
        p = self._dev(params) if params is not None else None
        h = ctypes.c_void_p()
        hrlb._check(lib.hrlb_mlp_create(_ptr(self.state), sb.value, _ptr(self.work), wb.value, max_rows, _ptr(p), seed,
                                        self.norm.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                        ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.handle = h

    def _dev(self, a, dtype=None):
        torch = self.torch
        if not isinstance(a, torch.Tensor):
            a = torch.from_numpy(np.ascontiguousarray(a))
        return a.to(device=self.device, dtype=dtype or torch.float32).contiguous()

    def set_params(self, params):
        p = self._dev(params)
        assert p.numel() == NPARAMS
        self._keep = p
        hrlb._check(load().hrlb_mlp_set_params(self.handle, _ptr(p)))

    def get_params(self):
        out = self.torch.empty(NPARAMS, dtype=self.torch.float32, device=self.device)
        hrlb._check(load().hrlb_mlp_get_params(self.handle, _ptr(out)))
        return out

    def _rows(self, fn, x, out):
        # the library takes at most max_rows rows per call; larger inputs go in slices
        for r0 in range(0, x.shape[0], self.max_rows):
            n = min(self.max_rows, x.shape[0] - r0)
            hrlb._check(fn(self.handle, _ptr(x[r0:r0 + n]), n, _ptr(out[r0:r0 + n])))
        return out

    def forward(self, x):
        x = self._dev(x)
        out = self.torch.empty((x.shape[0], OUT), dtype=self.torch.float32, device=self.device)
        return self._rows(load().hrlb_mlp_forward, x, out)

    def predict_table(self, x):
        x = self._dev(x)
        out = self.torch.empty((x.shape[0], 14), dtype=self.torch.float64, device=self.device)
        return self._rows(load().hrlb_mlp_predict_table, x, out)

    def gradient(self, x, t, idx=None, rows=None):
        """(gradient [NPARAMS], loss [1]) on device for the selected rows."""
        x, t = self._dev(x), self._dev(t)
        idx = self._dev(idx, self.torch.int32) if idx is not None else None
        rows = rows if rows is not None else (idx.numel() if idx is not None else x.shape[0])
        g = self.torch.empty(NPARAMS, dtype=self.torch.float32, device=self.device)
        loss = self.torch.empty(1, dtype=self.torch.float32, device=self.device)
        hrlb._check(load().hrlb_mlp_gradient(self.handle, _ptr(x), _ptr(t), _ptr(idx), rows, _ptr(g), _ptr(loss)))
        return g, loss

    def train_step(self, x, t, idx, lr, wd, loss=None):
        """One AdamW step on the rows idx (device int32) of the device arrays x, t; the loss
        goes to loss (device float32 [1]) if given."""
        hrlb._check(load().hrlb_mlp_train_step(self.handle, _ptr(x), _ptr(t), _ptr(idx), idx.numel(), float(lr),
                                               float(wd), _ptr(loss)))

    def __del__(self):
        if getattr(self, 'handle', None) and hrlb is not None and hrlb._lib is not None:
            try:
                self.stream.synchronize()
            except Exception:
                pass
            hrlb._lib.hrlb_mlp_free(self.handle)
            self.handle = None
