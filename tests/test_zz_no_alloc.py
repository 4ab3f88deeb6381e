"""mdx_mlp_grad_noalloc (the gradient entry point that allocates nothing:
its partials live in the library's own device array) against mdx_mlp_grad
with a caller-allocated scratch, through the C ABI.

Three calls in a row on one context: a large batch (more workgroups than the
array holds, so the samples are split differently: equal to FP32 summation
order), then two smaller ones (the same partition as mdx_mlp_grad: bitwise
equal), the last smaller than the one before."""
import ctypes as C

import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda:0")


def _p(t):
    return C.c_void_p(t.data_ptr())


def _both(sim, theta, X, T):
    import torch
    from paper_2510_12011_amd import _lib as L
    n = X.shape[0]
    P, Xd, Td = _t(theta), _t(X), _t(T)
    g_ref = torch.empty(mlp.N_PARAM, dtype=torch.float32, device="cuda:0")
    l_ref = torch.empty(1, dtype=torch.float32, device="cuda:0")
    nb = L.lib().mdx_mlp_grad_scratch(n)
    scratch = torch.empty(nb // 4 + 64, dtype=torch.float32, device="cuda:0")
    sim._check(L.lib().mdx_mlp_grad(sim._h, _p(P), n, _p(Xd), _p(Td), _p(g_ref), _p(l_ref),
                                    _p(scratch), nb))
    g = torch.full((mlp.N_PARAM,), float("nan"), dtype=torch.float32, device="cuda:0")
    loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda:0")
    sim._check(L.lib().mdx_mlp_grad_noalloc(sim._h, _p(P), n, _p(Xd), _p(Td), _p(g), _p(loss)))
    torch.cuda.synchronize()
    return (g_ref.cpu().numpy(), float(l_ref.item()), g.cpu().numpy(), float(loss.item()))


def test_noalloc_gradient_matches_allocating_entry_point():
    from paper_2510_12011_amd import sim as S
    sim = S.Simulation(0)
    theta = mlp.init_params(5)
    for n, bitwise in ((100_000, False), (8000, True), (3000, True)):
        rng = np.random.default_rng(n)
        X = rng.normal(size=(n, 4))
        T = rng.normal(size=n) * 0.1
        print(f"  noalloc gradient n={n}", flush=True)
        g_ref, l_ref, g, loss = _both(sim, theta, X, T)
        assert np.all(np.isfinite(g)) and np.isfinite(loss)
        if bitwise:
            assert np.array_equal(g, g_ref), np.abs(g - g_ref).max()
            assert loss == l_ref
        else:
            # FP32 sums of the same per-sample terms in another grouping
            scale = np.abs(g_ref).max()
            assert np.allclose(g, g_ref, rtol=1e-4, atol=1e-5 * scale), np.abs(g - g_ref).max()
            assert abs(loss - l_ref) <= 1e-5 * abs(l_ref)


def test_noalloc_rejects_bad_sizes():
    from paper_2510_12011_amd import _lib as L
    from paper_2510_12011_amd import sim as S
    sim = S.Simulation(0)
    P = _t(mlp.init_params(1))
    X = _t(np.zeros((32, 4)))
    T = _t(np.zeros(32))
    g = _t(np.zeros(mlp.N_PARAM))
    assert L.lib().mdx_mlp_grad_noalloc(sim._h, _p(P), 0, _p(X), _p(T), _p(g), None) == -1
    assert L.lib().mdx_mlp_grad_noalloc(sim._h, _p(P), 2**31, _p(X), _p(T), _p(g), None) == -1
