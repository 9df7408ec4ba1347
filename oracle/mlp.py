"""Oracle of the warm-start network (test infrastructure only; see ``oracle/__init__``).

A plain numpy definition of the fully connected network that predicts steady Couette
profiles, its mean-squared-error loss, the loss gradient by the chain rule, and the AdamW
update.  Everything is computed in float64.  With ``quant=True`` the values are rounded
to bfloat16 at the points where the GPU kernels store bfloat16 operands:

* the weight matrices (the kernels multiply with a bfloat16 copy of the fp32 master
  weights; biases stay fp32 and are added to the fp32 accumulator),
* the network input and every hidden activation h = silu(z),
* every backward signal dZ that feeds a matrix product (dZ of the output layer included).

Pre-activations z, the output y, the loss, bias gradients (summed from the bfloat16 dZ)
and weight gradients are not rounded.  With ``quant=False`` nothing is rounded and the
gradient is the exact float64 gradient of the float64 network.

Network (layer widths ``DIMS``): y = W3 s(W2 s(W1 s(W0 x + b0) + b1) + b2) + b3 with
s = silu, silu(z) = z / (1 + exp(-z)).  Weights are stored W_l[out][in].

Pins (tests/test_oracle_mlp.py): bfloat16 rounding equals torch's float -> bfloat16
conversion; forward and gradient with quant=False equal torch's float64 autograd of the
same network and central differences of the loss; the AdamW update equals
torch.optim.AdamW over several steps.
"""
import numpy as np

DIMS = (5, 256, 256, 256, 8)
NLAYERS = len(DIMS) - 1


def bf16(x):
    """Round to the nearest bfloat16 value, ties to even (via float32), returned as float64.
    Inputs are finite and within the float32 range."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    """d silu / dz = s (1 + z (1 - s)), s = 1 / (1 + exp(-z))."""
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(seed, dims=DIMS):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases from numpy's
    default_rng(seed), in layer order W0, b0, W1, b1, ..."""
    rng = np.random.default_rng(seed)
    params = []
    for l in range(len(dims) - 1):
        a = 1.0 / np.sqrt(dims[l])
        params.append(rng.uniform(-a, a, size=(dims[l + 1], dims[l])))
        params.append(rng.uniform(-a, a, size=(dims[l + 1],)))
    return params


def forward(params, X, quant=True):
    """Output y[M][8] and the cache (layer inputs h_l, pre-activations z_l, the weights
    used) for the backward pass."""
    r = bf16 if quant else (lambda a: np.asarray(a, dtype=np.float64))
    h = r(X)
    hs, zs, Ws = [h], [], []
    nl = len(params) // 2
    for l in range(nl):
        W = r(params[2 * l])
        b = np.asarray(params[2 * l + 1], dtype=np.float64)
        z = h @ W.T + b
        zs.append(z)
        Ws.append(W)
        if l < nl - 1:
            h = r(silu(z))
            hs.append(h)
        else:
            h = z
    return h, dict(h=hs, z=zs, W=Ws)


def loss(y, T):
    """Mean of (y - T)^2 over rows and channels."""
    return float(np.mean((y - T) ** 2))


def loss_and_grad(params, X, T, quant=True):
    """Loss and its gradient with respect to every parameter, in the order of params."""
    r = bf16 if quant else (lambda a: a)
    y, c = forward(params, X, quant)
    M = y.shape[0]
    nl = len(params) // 2
    g = [None] * len(params)
    dz = r(2.0 * (y - T) / y.size)
    for l in range(nl - 1, -1, -1):
        g[2 * l] = dz.T @ c['h'][l]
        g[2 * l + 1] = dz.sum(axis=0)
        if l > 0:
            dh = dz @ c['W'][l]
            dz = r(dh * silu_grad(c['z'][l - 1]))
    assert M == X.shape[0]
    return loss(y, T), g


class AdamW:
    """Decoupled weight decay (Loshchilov and Hutter) with bias-corrected moments, in the
    form torch.optim.AdamW uses: theta <- theta (1 - lr wd), then
    theta <- theta - lr m_hat / (sqrt(v_hat) + eps)."""

    def __init__(self, params, lr=1e-3, betas=(0.9, 0.999), eps=1e-8, weight_decay=1e-2):
        self.lr, self.b1, self.b2, self.eps, self.wd = lr, betas[0], betas[1], eps, weight_decay
        self.m = [np.zeros_like(p) for p in params]
        self.v = [np.zeros_like(p) for p in params]
        self.t = 0

    def step(self, params, grads, lr=None):
        lr = self.lr if lr is None else lr
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        out = []
        for k, (p, gk) in enumerate(zip(params, grads)):
            self.m[k] = self.b1 * self.m[k] + (1.0 - self.b1) * gk
            self.v[k] = self.b2 * self.v[k] + (1.0 - self.b2) * gk * gk
            p = p * (1.0 - lr * self.wd)
            p = p - lr * (self.m[k] / c1) / (np.sqrt(self.v[k] / c2) + self.eps)
            out.append(p)
        return out


def standardize_fit(A):
    """Per-column mean and standard deviation (1 where a column is constant)."""
    mu = A.mean(axis=0)
    sd = A.std(axis=0)
    sd = np.where(sd > 0, sd, 1.0)
    return mu, sd
