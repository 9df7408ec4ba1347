"""Pins of the warm-start network oracle against library routines and calculus:
bfloat16 rounding against torch's conversion, forward and gradient against torch's float64
autograd of the same network, the gradient against central differences of the loss, and
AdamW against torch.optim.AdamW."""
import numpy as np
import pytest
import torch

from oracle import mlp

DIMS_SMALL = (5, 12, 9, 7, 8)


def data(M, seed, dims=mlp.DIMS):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(M, dims[0])), rng.normal(size=(M, dims[-1]))


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.uniform(-30, 30, size=4000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -9, 65504.0, 3.4e38]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x), ref)
    # ties go to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    assert mlp.bf16(1.0 + 2 ** -8) == 1.0
    assert mlp.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6


def torch_net(params, dims):
    layers = []
    for l in range(len(dims) - 1):
        lin = torch.nn.Linear(dims[l], dims[l + 1], dtype=torch.float64)
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(params[2 * l]))
            lin.bias.copy_(torch.from_numpy(params[2 * l + 1]))
        layers.append(lin)
        if l < len(dims) - 2:
            layers.append(torch.nn.SiLU())
    return torch.nn.Sequential(*layers)


@pytest.mark.parametrize("dims", [DIMS_SMALL, mlp.DIMS])
def test_forward_and_gradient_match_torch_autograd(dims):
    params = mlp.init_params(3, dims)
    X, T = data(37, 4, dims)
    y, _ = mlp.forward(params, X, quant=False)
    L, g = mlp.loss_and_grad(params, X, T, quant=False)
    net = torch_net(params, dims)
    yt = net(torch.from_numpy(X))
    lt = torch.mean((yt - torch.from_numpy(T)) ** 2)
    lt.backward()
    assert np.allclose(y, yt.detach().numpy(), rtol=1e-13, atol=1e-14)
    assert abs(L - lt.item()) <= 1e-13 * abs(L)
    tg = []
    for mod in net:
        if isinstance(mod, torch.nn.Linear):
            tg += [mod.weight.grad.numpy(), mod.bias.grad.numpy()]
    for a, b in zip(g, tg):
        assert a.shape == b.shape
        assert np.abs(a - b).max() <= 1e-12 * max(np.abs(b).max(), 1e-300)


def test_gradient_matches_central_differences():
    params = mlp.init_params(5, DIMS_SMALL)
    X, T = data(23, 6, DIMS_SMALL)
    _, g = mlp.loss_and_grad(params, X, T, quant=False)
    rng = np.random.default_rng(7)
    h = 1e-6
    for k, p in enumerate(params):
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in p.shape)
            pp = [q.copy() for q in params]
            pm = [q.copy() for q in params]
            pp[k][idx] += h
            pm[k][idx] -= h
            fd = (mlp.loss(mlp.forward(pp, X, False)[0], T) - mlp.loss(mlp.forward(pm, X, False)[0], T)) / (2 * h)
            assert abs(fd - g[k][idx]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g[k]).max())


def test_quantized_gradient_is_close_to_exact():
    params = mlp.init_params(8, mlp.DIMS)
    X, T = data(64, 9)
    _, g = mlp.loss_and_grad(params, X, T, quant=False)
    _, gq = mlp.loss_and_grad(params, X, T, quant=True)
    for a, b in zip(g, gq):
        assert np.linalg.norm(a - b) <= 3e-2 * np.linalg.norm(a)


def test_adamw_matches_torch():
    params = mlp.init_params(10, DIMS_SMALL)
    X, T = data(16, 11, DIMS_SMALL)
    opt = mlp.AdamW(params, lr=3e-3, weight_decay=0.05)
    net = torch_net(params, DIMS_SMALL)
    topt = torch.optim.AdamW(net.parameters(), lr=3e-3, weight_decay=0.05, betas=(0.9, 0.999), eps=1e-8)
    for _ in range(5):
        _, g = mlp.loss_and_grad(params, X, T, quant=False)
        params = opt.step(params, g)
        topt.zero_grad()
        torch.mean((net(torch.from_numpy(X)) - torch.from_numpy(T)) ** 2).backward()
        topt.step()
    tp = [p.detach().numpy() for p in net.parameters()]
    for a, b in zip(params, tp):
        assert np.abs(a - b).max() <= 1e-12
