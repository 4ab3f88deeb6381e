"""The learned warm start's network on the GPU (BF16 MFMA, FP32 accumulation)
against the FP64 CPU oracle (oracle/mlp.py).

Bars: forward RMS error <= 2e-2 of the RMS output (BF16 weights and
activations through three layers) and every output within its per-sample
BF16 error bound (oracle/mlp.py, 6 standard deviations); gradient cosine similarity >= 0.98 for the
whole vector and for each weight matrix; Adam step to FP32 rounding;
gradients bitwise reproducible."""
import ctypes as C

import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2510_12011_amd import sim
    return sim.Simulation(0)


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda:0")


def _p(t):
    return C.c_void_p(t.data_ptr())


def _forward(ctx, theta, X):
    import torch
    from paper_2510_12011_amd import _lib as L
    P, Xd = _t(theta), _t(X)
    y = torch.empty(X.shape[0], dtype=torch.float32, device="cuda:0")
    ctx._check(L.lib().mdx_mlp_forward(ctx._h, _p(P), X.shape[0], _p(Xd), _p(y)))
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64)


def _grad(ctx, theta, X, T):
    import torch
    from paper_2510_12011_amd import _lib as L
    n = X.shape[0]
    P, Xd, Td = _t(theta), _t(X), _t(T)
    g = torch.empty(mlp.N_PARAM, dtype=torch.float32, device="cuda:0")
    loss = torch.empty(1, dtype=torch.float32, device="cuda:0")
    nb = L.lib().mdx_mlp_grad_scratch(n)
    scratch = torch.empty(nb // 4 + 64, dtype=torch.float32, device="cuda:0")
    ctx._check(L.lib().mdx_mlp_grad(ctx._h, _p(P), n, _p(Xd), _p(Td), _p(g), _p(loss),
                                    _p(scratch), nb))
    torch.cuda.synchronize()
    return float(loss.item()), g.cpu().numpy().astype(np.float64)


def _cos(a, b):
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


def test_nparams(ctx):
    from paper_2510_12011_amd import _lib as L
    assert L.lib().mdx_mlp_nparams() == mlp.N_PARAM


@pytest.mark.parametrize("n", [1, 31, 33, 1000, 1100, 70000])
def test_forward_matches_oracle(ctx, n):
    rng = np.random.default_rng(n)
    theta = mlp.init_params(7)
    theta[mlp.N_PARAM - 1] = 0.3
    X = rng.normal(size=(n, 4))
    y_ref = mlp.forward(theta, X)
    y = _forward(ctx, theta, X)
    # scale of the network's outputs: RMS over a reference population (a
    # single output can sit near zero while its BF16 error follows the size
    # of the intermediate sums)
    rms = np.sqrt(np.mean(mlp.forward(theta, np.random.default_rng(0).normal(size=(4096, 4))) ** 2))
    err = np.sqrt(np.mean((y - y_ref) ** 2))
    bound = mlp.bf16_error_bound(theta, X)
    worst = float(np.max(np.abs(y - y_ref) / bound))
    print(f"  n={n}: forward RMS error / RMS = {err / rms:.2e}, worst node at "
          f"{worst:.2f} of its BF16 bound", flush=True)
    assert err <= 2e-2 * rms
    assert worst <= 1.0


def test_gradient_matches_oracle(ctx):
    rng = np.random.default_rng(3)
    theta = mlp.init_params(11)
    n = 4099
    X = rng.normal(size=(n, 4))
    T = np.sin(X[:, 0]) + X[:, 1] * X[:, 2]
    L_ref, g_ref = mlp.loss_and_grad(theta, X, T)
    L_gpu, g = _grad(ctx, theta, X, T)
    assert L_gpu == pytest.approx(L_ref, rel=2e-2)
    cos = _cos(g, g_ref)
    print(f"  loss {L_gpu:.4f} vs {L_ref:.4f}; gradient cosine {cos:.5f}", flush=True)
    assert cos >= 0.98
    G, Gr = mlp.unpack(g), mlp.unpack(g_ref)
    for name in ("W1", "b1", "W2", "b2", "W3", "b3", "W4"):
        c = _cos(G[name].ravel(), Gr[name].ravel())
        assert c >= 0.98, (name, c)
    assert G["b4"][0] == pytest.approx(Gr["b4"][0], rel=2e-2, abs=1e-3)


def test_gradient_deterministic(ctx):
    rng = np.random.default_rng(4)
    theta = mlp.init_params(5)
    X = rng.normal(size=(10000, 4))
    T = rng.normal(size=10000)
    _, g1 = _grad(ctx, theta, X, T)
    _, g2 = _grad(ctx, theta, X, T)
    assert np.array_equal(g1, g2)


def test_adam_matches_oracle(ctx):
    import torch
    from paper_2510_12011_amd import _lib as L
    rng = np.random.default_rng(6)
    theta = rng.normal(size=mlp.N_PARAM)
    m = rng.normal(size=mlp.N_PARAM) * 0.1
    v = rng.uniform(0, 0.1, mlp.N_PARAM)
    g = rng.normal(size=mlp.N_PARAM)
    P, Md, Vd, Gd = _t(theta), _t(m), _t(v), _t(g)
    ctx._check(L.lib().mdx_mlp_adam(ctx._h, _p(P), _p(Md), _p(Vd), _p(Gd), 3, 1e-3, 0.9, 0.999,
                                    1e-8))
    torch.cuda.synchronize()
    mlp.adam_step(theta, m, v, g, 3, lr=1e-3)
    np.testing.assert_allclose(P.cpu().numpy(), theta, rtol=1e-6, atol=1e-6)


def test_training_on_gpu_reduces_loss(ctx):
    """200 Adam steps on the GPU (forward + backward + Adam kernels) fit a
    smooth target; the GPU-trained network's loss, evaluated by the FP64
    oracle, falls below 10% of the initial loss."""
    import torch
    from paper_2510_12011_amd import _lib as L
    rng = np.random.default_rng(8)
    n = 8192
    X = rng.normal(size=(n, 4))
    T = X[:, 0] - 0.5 * X[:, 1] + X[:, 2] * X[:, 3]
    theta0 = mlp.init_params(9)
    P, Xd, Td = _t(theta0), _t(X), _t(T)
    Md = torch.zeros_like(P)
    Vd = torch.zeros_like(P)
    g = torch.empty_like(P)
    nb = L.lib().mdx_mlp_grad_scratch(n)
    scratch = torch.empty(nb // 4 + 64, dtype=torch.float32, device="cuda:0")
    for t in range(1, 201):
        ctx._check(L.lib().mdx_mlp_grad(ctx._h, _p(P), n, _p(Xd), _p(Td), _p(g), None,
                                        _p(scratch), nb))
        ctx._check(L.lib().mdx_mlp_adam(ctx._h, _p(P), _p(Md), _p(Vd), _p(g), t, 3e-3, 0.9,
                                        0.999, 1e-8))
    torch.cuda.synchronize()
    theta = P.cpu().numpy().astype(np.float64)
    L0 = np.mean((mlp.forward(theta0, X) - T) ** 2)
    L1 = np.mean((mlp.forward(theta, X) - T) ** 2)
    print(f"  loss {L0:.4f} -> {L1:.4f}", flush=True)
    assert L1 < 0.1 * L0


def test_samples_gather_raw_and_standardised(ctx):
    """mdx_mlp_samples, the training batches' gather: the rows an index list
    picks, raw (bitwise) and standardised as the network trains on them (the
    same FP32 operations written out in numpy: (x - mean) * (1/std), target
    (dV - x1) / out_scale), and a zero row with a NaN target for an index
    outside the rows."""
    import torch
    from paper_2510_12011_amd import _lib as L
    rng = np.random.default_rng(5)
    n, k = 5000, 777
    X = rng.normal(size=(n, 4)).astype(np.float32)
    dV = rng.normal(size=n).astype(np.float32)
    idx = rng.integers(0, n, k).astype(np.int64)
    idx[5] = n + 3
    norm = np.array([0.1, -0.2, 0.3, 0.0, 1.5, 0.7, 2.0, 1.1, 0.25])
    Xd, dVd = _t(X), _t(dV)
    idxd = torch.from_numpy(idx).to("cuda:0")
    Xo = torch.empty((k, 4), dtype=torch.float32, device="cuda:0")
    To = torch.empty(k, dtype=torch.float32, device="cuda:0")
    ok = np.arange(k) != 5
    ctx._check(L.lib().mdx_mlp_samples(ctx._h, k, _p(idxd), n, _p(Xd), _p(dVd), None, _p(Xo),
                                       _p(To)))
    torch.cuda.synchronize()
    xo, to = Xo.cpu().numpy(), To.cpu().numpy()
    assert np.array_equal(xo[ok], X[idx[ok]]) and np.array_equal(to[ok], dV[idx[ok]])
    assert not xo[5].any() and np.isnan(to[5])
    nm = norm.ctypes.data_as(C.c_void_p)
    ctx._check(L.lib().mdx_mlp_samples(ctx._h, k, _p(idxd), n, _p(Xd), _p(dVd), nm, _p(Xo),
                                       _p(To)))
    torch.cuda.synchronize()
    xo, to = Xo.cpu().numpy(), To.cpu().numpy()
    mean = norm[:4].astype(np.float32)
    inv = (1.0 / norm[4:8]).astype(np.float32)
    want_x = (X[idx[ok]] - mean) * inv
    want_t = (dV[idx[ok]] - X[idx[ok], 1]) / np.float32(norm[8])
    np.testing.assert_allclose(xo[ok], want_x, rtol=2e-7, atol=1e-7)
    np.testing.assert_allclose(to[ok], want_t, rtol=2e-7, atol=1e-7)
    assert not xo[5].any() and np.isnan(to[5])
    bad = norm.copy()
    bad[5] = 0.0
    assert L.lib().mdx_mlp_samples(ctx._h, k, _p(idxd), n, _p(Xd), _p(dVd),
                                   bad.ctypes.data_as(C.c_void_p), _p(Xo),
                                   _p(To)) == L.MDX_ERR_INVALID_ARG
