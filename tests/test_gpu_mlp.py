"""The warm-start network's kernels against the oracle network (oracle/mlp.py, float64 with
the same bfloat16 rounding points): forward pass, loss and gradient of every parameter,
the AdamW update, row gathering, ragged row counts and the Couette moment table; and the
warm-start seed kernel against the oracle seed (oracle/warmstart.py)."""
import numpy as np
import pytest
import torch

from oracle import mlp as om
from oracle import solver as sv
from oracle import warmstart as ows
from paper_1702_01335_amd import hrlb, network

from parity import assert_parity, compare, make_wl, oracle_params

pytestmark = pytest.mark.gpu

IDENT = network.norm_vector(np.zeros(5), np.ones(5), np.zeros(8), np.ones(8))


def flat(params):
    return np.concatenate([p.ravel() for p in params]).astype(np.float32)


def unflat(v):
    out, o = [], 0
    for l in range(len(om.DIMS) - 1):
        n, k = om.DIMS[l + 1], om.DIMS[l]
        out.append(np.asarray(v[o:o + n * k], dtype=np.float64).reshape(n, k))
        o += n * k
        out.append(np.asarray(v[o:o + n], dtype=np.float64))
        o += n
    assert o == network.NPARAMS
    return out


def f32(params):
    """Parameters as the GPU holds them (fp32 master copy)."""
    return [p.astype(np.float32).astype(np.float64) for p in params]


def data(M, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(M, 5)).astype(np.float32)
    T = (0.5 * rng.normal(size=(M, 8))).astype(np.float32)
    return X, T


def rel(a, b):
    return np.linalg.norm(np.asarray(a, dtype=np.float64) - b) / np.linalg.norm(b)


@pytest.mark.parametrize("M", [1, 37, 64, 200, 1000])
def test_forward_matches_oracle(M):
    params = f32(om.init_params(1))
    net = network.Network(1024, IDENT, params=flat(params))
    X, _ = data(M, 2)
    y = net.forward(X).cpu().numpy()
    yo, _ = om.forward(params, X.astype(np.float64), quant=True)
    err = rel(y, yo)
    print(f"[mlp] forward M={M} rel err {err:.2e}", flush=True)
    assert err <= 1e-2
    assert np.abs(y - yo).max() <= 2e-2 * np.abs(yo).max()


@pytest.mark.parametrize("M", [64, 333, 2048])
def test_gradient_matches_oracle(M):
    params = f32(om.init_params(3))
    net = network.Network(4096, IDENT, params=flat(params))
    X, T = data(M, 4)
    g, loss = net.gradient(X, T)
    g = unflat(g.cpu().numpy())
    Lo, go = om.loss_and_grad(params, X.astype(np.float64), T.astype(np.float64), quant=True)
    print(f"[mlp] M={M} loss gpu {loss.item():.6e} oracle {Lo:.6e}", flush=True)
    assert abs(loss.item() - Lo) <= 1e-3 * Lo
    for k, (a, b) in enumerate(zip(g, go)):
        err = rel(a, b)
        # element by element, against the tensor's largest entry: the two sides round to
        # bfloat16 at the same points but accumulate in different orders (float32 on the
        # matrix cores, float64 in the oracle), so a rounded product can land one bfloat16
        # step (2^-8 relative) apart and carry that into the sums downstream
        emax = np.abs(np.asarray(a, dtype=np.float64) - b).max() / np.abs(b).max()
        print(f"[mlp]   param {k} {b.shape}: rel err {err:.2e}, largest entry difference {emax:.2e}", flush=True)
        assert err <= 1e-2, k
        assert emax <= 1e-2, k
    # and close to the exact float64 gradient (bfloat16 rounding only)
    _, ge = om.loss_and_grad(params, X.astype(np.float64), T.astype(np.float64), quant=False)
    for a, b in zip(g, ge):
        assert rel(a, b) <= 5e-2


def test_forward_in_slices_beyond_max_rows():
    params = f32(om.init_params(2))
    net = network.Network(64, IDENT, params=flat(params))
    X, _ = data(200, 3)
    y = net.forward(X).cpu().numpy()
    big = network.Network(256, IDENT, params=flat(params))
    assert np.array_equal(y, big.forward(X).cpu().numpy())
    assert np.array_equal(net.predict_table(X).cpu().numpy(), big.predict_table(X).cpu().numpy())


def test_gradient_gathers_rows_by_index():
    params = f32(om.init_params(5))
    net = network.Network(512, IDENT, params=flat(params))
    X, T = data(300, 6)
    idx = np.random.default_rng(7).permutation(300)[:129].astype(np.int32)
    g1, l1 = net.gradient(X, T, idx=idx)
    g2, l2 = net.gradient(X[idx], T[idx])
    assert torch.equal(g1, g2) and torch.equal(l1, l2)


def test_standardisation_is_applied():
    params = f32(om.init_params(8))
    rng = np.random.default_rng(9)
    im, isd = rng.normal(size=5), rng.uniform(0.5, 2.0, 5)
    omu, osd = rng.normal(size=8), rng.uniform(0.5, 2.0, 8)
    norm = network.norm_vector(im, isd, omu, osd)
    net = network.Network(256, norm, params=flat(params))
    X, T = data(100, 10)
    y = net.forward(X).cpu().numpy()
    Xs = (X.astype(np.float32) - norm[:5]) / norm[5:10]
    yo, _ = om.forward(params, Xs.astype(np.float64), quant=True)
    assert rel(y, yo * norm[18:26] + norm[10:18]) <= 1e-2
    tab = net.predict_table(X).cpu().numpy()
    y64 = y.astype(np.float64)
    n, T_ = y64[:, 0], y64[:, 2]
    assert np.array_equal(tab[:, [0, 2, 4, 5, 8, 6, 11, 12]], y64)
    assert np.all(tab[:, [1, 3, 9, 10, 13]] == 0)
    assert np.allclose(tab[:, 7], 3 * n * T_ - y64[:, 3] - y64[:, 5], rtol=1e-12, atol=1e-12)


def test_adamw_step_matches_oracle_update():
    params = f32(om.init_params(11))
    net = network.Network(512, IDENT, params=flat(params))
    X, T = data(256, 12)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    idx = torch.arange(256, dtype=torch.int32, device='cuda')
    opt = om.AdamW(params, lr=2e-3, weight_decay=0.01)
    cur = params
    for _ in range(3):
        g, _ = net.gradient(Xd, Td, idx=idx)
        net.train_step(Xd, Td, idx, 2e-3, 0.01)
        cur = opt.step(cur, unflat(g.cpu().numpy()))
    got = unflat(net.get_params().cpu().numpy())
    for a, b in zip(got, cur):
        assert np.abs(a - b).max() <= 1e-6 * max(np.abs(b).max(), 1.0)


def test_training_fits_a_smooth_map():
    rng = np.random.default_rng(13)
    X = rng.uniform(-1, 1, size=(4096, 5)).astype(np.float32)
    W = rng.normal(size=(5, 8))
    T = np.tanh(X @ W).astype(np.float32)
    mu, sd = om.standardize_fit(T)
    norm = network.norm_vector(np.zeros(5), np.ones(5), mu, sd)
    net = network.Network(4096, norm, seed=1)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    loss = torch.zeros(1, device='cuda')
    g = torch.Generator(device='cuda').manual_seed(0)
    first = None
    for it in range(300):
        idx = torch.randint(0, 4096, (512,), device='cuda', dtype=torch.int32, generator=g)
        net.train_step(Xd, Td, idx, 2e-3, 1e-4, loss)
        if it == 0:
            first = loss.item()
    _, L = net.gradient(Xd, Td)
    print(f"[mlp] training loss {first:.3e} -> {L.item():.3e}", flush=True)
    assert L.item() < 0.05 * first


def test_initialisation_range():
    net = network.Network(64, IDENT, seed=42)
    p = unflat(net.get_params().cpu().numpy())
    for l in range(4):
        a = 1.0 / np.sqrt(om.DIMS[l])
        for t in (p[2 * l], p[2 * l + 1]):
            assert np.abs(t).max() <= a
            if t.size >= 256:
                assert np.abs(t).max() > 0.95 * a and abs(t.mean()) < 0.2 * a
    q = unflat(network.Network(64, IDENT, seed=42).get_params().cpu().numpy())
    assert all(np.array_equal(a, b) for a, b in zip(p, q))


# ---- warm-start seed -------------------------------------------------------------------

SEED_CASES = [make_wl(5, 3, 3, 13, 'weno5', A=0.9, dt=1e-4), make_wl(7, 7, 7, 6, 'upwind2', dt=1e-4)]


def random_tables(rng, B, S):
    n = rng.uniform(0.8, 1.2, (B, S))
    uy = rng.uniform(-0.3, 0.3, (B, S))
    T = rng.uniform(0.9, 1.1, (B, S))
    P = [n * T * (1 + rng.uniform(-0.05, 0.05, (B, S))) for _ in range(2)]
    small = [rng.uniform(-0.05, 0.05, (B, S)) for _ in range(3)]
    prof = np.stack([n, uy, T, P[0], small[0], P[1], small[1], small[2]], axis=-1)
    tab = ows.table_from_profiles(prof)
    tab[..., 1] = rng.uniform(-0.05, 0.05, (B, S))   # exercise every column
    tab[..., 13] = rng.uniform(-0.02, 0.02, (B, S))
    return tab


@pytest.mark.parametrize("case", range(len(SEED_CASES)))
def test_seed_matches_oracle(case):
    wl = SEED_CASES[case]
    q = hrlb.Quadrature(wl['Qx'], wl['Qy'], wl['Qz'])
    B = 3
    s = hrlb.Solver(q, wl['S'], wl['scheme'], [hrlb.make_params(**wl['params'])] * B)
    tab = random_tables(np.random.default_rng(20 + case), B, wl['S'])
    fb = s.seed_state(torch.from_numpy(tab).cuda(), preserve_mass=False)
    assert not fb.any()
    F = s.get_state().cpu().numpy()
    m = sv.Model(oracle_params(wl))
    for b in range(B):
        Fo = ows.seed(tab[b], m.vs)
        res = compare(F[b], Fo, m)
        print(f"[seed] case {case} instance {b}: {res}", flush=True)
        assert_parity(F[b], Fo, m, f"seed instance {b}")
    # the seeded state steps like the oracle seeded the same way
    s.step(3)
    F3 = s.get_state().cpu().numpy()
    Fo = sv.run(ows.seed(tab[1], m.vs), m, 3)
    assert_parity(F3[1], Fo, m, "seeded state after 3 steps")


def test_mass_preserving_seed_matches_oracle():
    # with full-range orders >= 3 the correction terms carry no mass, so the seed's mass is
    # the scaled table's
    wl = make_wl(5, 4, 4, 13, 'weno5', A=0.9, dt=1e-4)
    q = hrlb.Quadrature(wl['Qx'], wl['Qy'], wl['Qz'])
    B = 2
    p = dict(wl['params'])
    p['n0'] = 1.2
    s = hrlb.Solver(q, wl['S'], wl['scheme'], [hrlb.make_params(**p)] * B)
    tab = random_tables(np.random.default_rng(40), B, wl['S'])
    s.seed_state(torch.from_numpy(tab).cuda(), preserve_mass=True)
    F = s.get_state().cpu().numpy()
    m = sv.Model(oracle_params(wl, p))
    for b in range(B):
        Fo = ows.seed(ows.mass_preserving(tab[b], m.dx, 1.2), m.vs)
        assert_parity(F[b], Fo, m, f"mass-preserving seed {b}")
        assert abs(np.sum(F[b].sum(axis=1) * m.dx) - 1.2 * np.sum(m.dx)) <= 1e-13


def test_seed_falls_back_to_equilibrium_for_invalid_tables():
    wl = SEED_CASES[0]
    q = hrlb.Quadrature(wl['Qx'], wl['Qy'], wl['Qz'])
    B = 4
    params = [hrlb.make_params(**wl['params'])] * B
    s = hrlb.Solver(q, wl['S'], wl['scheme'], params)
    F_eq = s.get_state().cpu().numpy()
    tab = random_tables(np.random.default_rng(30), B, wl['S'])
    tab[1, 3, 4] = -1.0          # T <= 0
    tab[2, 0, 7] = np.nan        # not finite
    tab[3, 5, 0] = 0.0           # n <= 0
    fb = s.seed_state(torch.from_numpy(tab).cuda())
    assert fb.tolist() == [0, 1, 1, 1]
    F = s.get_state().cpu().numpy()
    for b in (1, 2, 3):
        assert np.array_equal(F[b], F_eq[b])
    assert not np.array_equal(F[0], F_eq[0])
    s.step(2)
    assert np.all(np.isfinite(s.residual()))


def test_gradient_with_many_rows_matches_oracle():
    """Long reductions (split K slices, many bias-gradient row slices) at 20000 rows."""
    params = f32(om.init_params(14))
    net = network.Network(20000, IDENT, params=flat(params))
    X, T = data(20000, 15)
    g, loss = net.gradient(X, T)
    g = unflat(g.cpu().numpy())
    Lo, go = om.loss_and_grad(params, X.astype(np.float64), T.astype(np.float64), quant=True)
    assert abs(loss.item() - Lo) <= 1e-3 * Lo
    for k, (a, b) in enumerate(zip(g, go)):
        assert rel(a, b) <= 1e-2, k
