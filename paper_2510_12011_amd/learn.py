"""Learned warm start: record training data from the plain solver, train the
per-node network on the GPU with the library's own kernels (mdx_mlp_grad,
mdx_mlp_adam), install it (mdx_set_mlp) and measure what it saves.

Torch is used here only for device memory and copies; the selection of
recorded samples, their standardisation statistics and the epochs'
permutations are host (numpy) work, and the batches' gather and
standardisation (mdx_mlp_samples), the network's forward pass, gradient and
optimiser step are the library's kernels (BF16 MFMA for the network).
"""
from __future__ import annotations

import ctypes as C
import time

import numpy as np

from . import _lib as L

N_PARAM = 8705
_SHAPES = [((64, 4), 4), ((64,), 0), ((64, 64), 64), ((64,), 0), ((64, 64), 64), ((64,), 0),
           ((64,), 64), ((1,), 0)]


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases, FP32, in the
    library's parameter layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape, fan_in in _SHAPES:
        if fan_in:
            lim = np.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-lim, lim, shape).ravel())
        else:
            parts.append(np.zeros(int(np.prod(shape))))
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.shape[0] == N_PARAM
    return theta


def _p(t):
    return C.c_void_p(t.data_ptr())


def _device_copy(a, dev, dtype=None):
    """Host numpy array -> new device tensor (a copy, no device arithmetic)."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to(dev)


def concat(parts):
    """Device tensors joined along their first axis, by copies."""
    import torch
    total = sum(int(t.shape[0]) for t in parts)
    out = torch.empty((total,) + tuple(parts[0].shape[1:]), dtype=parts[0].dtype,
                      device=parts[0].device)
    o = 0
    for t in parts:
        out[o:o + t.shape[0]].copy_(t)
        o += int(t.shape[0])
    return out


def record(sim, n_steps: int, every: int = 10, front: float = 0.02, frac: float = 0.05,
           seed: int = 0, cap: int | None = None):
    """Advance `sim` by n_steps; on every `every`-th step record (raw
    features, V^{n+1} - V^n) of all nodes whose increment exceeds `front` mV
    plus a random `frac` of the others (at most `cap` of them per recorded
    step, drawn at random).  The selection is made on the host from the
    step's increments; the library's mdx_mlp_samples gathers the chosen rows
    on the device.  Returns device tensors X [N, 4], dV [N]."""
    import torch
    dev = f"cuda:{sim.device}"
    n = sim.n
    Xr = torch.empty((n, 4), dtype=torch.float32, device=dev)
    dVr = torch.empty(n, dtype=torch.float32, device=dev)
    rng = np.random.default_rng(seed)
    chunks = []
    done = 0
    while done < n_steps:
        skip = min(every - 1, n_steps - done - 1)
        if skip > 0:
            sim.run(skip)
        sim._check(L.lib().mdx_set_recorder(sim._h, _p(Xr), _p(dVr), None))
        sim.run(1)
        sim._check(L.lib().mdx_set_recorder(sim._h, None, None, None))
        d = dVr.cpu().numpy()                     # waits for the step
        keep = np.flatnonzero((np.abs(d) > front) | (rng.random(n) < frac))
        if cap is not None and keep.size > cap:
            keep = np.sort(rng.choice(keep, size=cap, replace=False))
        if keep.size:
            idx = _device_copy(keep, dev, np.int64)
            Xc = torch.empty((keep.size, 4), dtype=torch.float32, device=dev)
            dc = torch.empty(keep.size, dtype=torch.float32, device=dev)
            sim._check(L.lib().mdx_mlp_samples(sim._h, keep.size, _p(idx), n, _p(Xr), _p(dVr),
                                               None, _p(Xc), _p(dc)))
            chunks.append((Xc, dc))
        done += skip + 1
    if not chunks:
        return (torch.empty((0, 4), dtype=torch.float32, device=dev),
                torch.empty(0, dtype=torch.float32, device=dev))
    return concat([c[0] for c in chunks]), concat([c[1] for c in chunks])


def fit(sim, X, dV, epochs: int = 10, batch: int = 8192, lr: float = 2e-3, seed: int = 0,
        theta0: np.ndarray | None = None, log=None):
    """Train on (X, dV): the network's target is the standardised departure
    of V^{n+1} from the extrapolation 2V^n - V^{n-1}, i.e. the increment
    V^{n+1} - V^n less the previous one (feature 1).  The standardisation
    (FP64 mean and standard deviation of the samples, computed on the host)
    and the per-epoch permutation are host work; every batch is gathered and
    standardised by mdx_mlp_samples, and the gradient and Adam step are the
    library's kernels.  Returns (params float32 [8705], norm float64 [9],
    per-epoch mean loss)."""
    import torch
    dev = X.device
    Xh = X.cpu().numpy().astype(np.float64)
    dh = dV.cpu().numpy().astype(np.float64)
    n = Xh.shape[0]
    mean = Xh.mean(0)
    std = np.maximum(Xh.std(0, ddof=1), 1e-6)
    out_scale = max(float((dh - Xh[:, 1]).std(ddof=1)), 1e-6)
    norm = np.concatenate([mean, std, [out_scale]])
    del Xh, dh
    P = _device_copy(init_params(seed) if theta0 is None else theta0, dev, np.float32)
    M = _device_copy(np.zeros(N_PARAM), dev, np.float32)
    Vm = _device_copy(np.zeros(N_PARAM), dev, np.float32)
    G = torch.empty_like(P)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    nb = L.lib().mdx_mlp_grad_scratch(batch)
    scratch = torch.empty(nb // 4 + 64, dtype=torch.float32, device=dev)
    Xb = torch.empty((batch, 4), dtype=torch.float32, device=dev)
    Tb = torch.empty(batch, dtype=torch.float32, device=dev)
    nm = np.ascontiguousarray(norm, np.float64)
    nm_p = nm.ctypes.data_as(C.c_void_p)
    rng = np.random.default_rng(seed)
    t = 0
    history = []
    for ep in range(epochs):
        perm = _device_copy(rng.permutation(n), dev, np.int64)
        tot, cnt = 0.0, 0
        for s in range(0, n - batch + 1, batch):
            t += 1
            sim._check(L.lib().mdx_mlp_samples(sim._h, batch, C.c_void_p(perm.data_ptr() + 8 * s),
                                               n, _p(X), _p(dV), nm_p, _p(Xb), _p(Tb)))
            sim._check(L.lib().mdx_mlp_grad(sim._h, _p(P), batch, _p(Xb), _p(Tb), _p(G),
                                            _p(loss), _p(scratch), nb))
            sim._check(L.lib().mdx_mlp_adam(sim._h, _p(P), _p(M), _p(Vm), _p(G), t, lr, 0.9,
                                            0.999, 1e-8))
            if cnt % 16 == 0:
                tot += float(loss.item())
            cnt += 1
        history.append(tot / max(1, (cnt + 15) // 16))
        if log:
            log(f"epoch {ep}: loss {history[-1]:.4f}")
    return P.cpu().numpy(), norm, history


def install(sim, params: np.ndarray, norm: np.ndarray):
    p = np.ascontiguousarray(params, np.float32)
    nm = np.ascontiguousarray(norm, np.float64)
    sim._check(L.lib().mdx_set_mlp(sim._h, p.ctypes.data_as(C.c_void_p),
                                   nm.ctypes.data_as(C.c_void_p)))


def timed_run(sim, n_steps: int):
    """Run n_steps; returns (seconds, iterations per step, fallbacks)."""
    import torch
    f0 = sim.stats()["fallbacks"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(n_steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return el, sim.iterations(n_steps), sim.stats()["fallbacks"] - f0


def save(path: str, params: np.ndarray, norm: np.ndarray, **meta):
    """Network and standardisation to an .npz (meta: scalars describing the
    training run and the mesh it belongs to)."""
    np.savez(path, params=np.asarray(params, np.float32), norm=np.asarray(norm, np.float64),
             **{k: np.asarray(v) for k, v in meta.items()})


def load(path: str):
    """(params, norm, meta dict) from save()'s file."""
    z = np.load(path, allow_pickle=False)
    meta = {k: z[k].item() for k in z.files if k not in ("params", "norm")}
    return z["params"].astype(np.float32), z["norm"].astype(np.float64), meta
