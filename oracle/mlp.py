"""CPU oracle of the learned warm start's network.  TEST INFRASTRUCTURE ONLY
(tests, smoke check, benchmark CPU baseline).

A per-node multilayer perceptron 4 -> 64 -> 64 -> 64 -> 1 with ReLU
activations maps node-local features of the monodomain step to one
normalised output (the learned warm start uses it as the departure of
V^{n+1} from the extrapolation 2V^n - V^{n-1}); it is trained by
mean-squared error with Adam (Kingma & Ba, ICLR 2015).  Plain FP64 numpy: forward pass,
hand-written backward pass (chain rule, no autograd), Adam.  Pinned in the
CPU tests against central finite differences and hand-computed Adam steps.

Parameter vector (flat, 8,705 values; the HIP kernels use the same layout):
    W1[64][4] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[64] b4[1]
(W[out][in], so layer l computes z = W h + b).
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 4, 64
SHAPES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_H, N_H)), ("b3", (N_H,)), ("W4", (N_H,)), ("b4", (1,))]
N_PARAM = sum(int(np.prod(s)) for _, s in SHAPES)   # 8705


def unpack(theta):
    """Views of the flat parameter vector by name."""
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = theta[o:o + k].reshape(shape)
        o += k
    return out


def init_params(seed=0):
    """He-uniform weights (fan-in), zero biases."""
    rng = np.random.default_rng(seed)
    theta = np.zeros(N_PARAM)
    p = unpack(theta)
    for name, shape in SHAPES:
        if name.startswith("W"):
            fan_in = shape[-1] if len(shape) == 2 else N_H
            lim = np.sqrt(6.0 / fan_in)
            p[name][...] = rng.uniform(-lim, lim, shape)
    return theta


def forward(theta, X, keep=False):
    """y[n] for features X[n, 4]; with keep=True also the pre-activations."""
    p = unpack(np.asarray(theta, np.float64))
    X = np.asarray(X, np.float64)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ p["W3"].T + p["b3"]
    h3 = np.maximum(z3, 0.0)
    y = h3 @ p["W4"] + p["b4"][0]
    if keep:
        return y, (X, z1, h1, z2, h2, z3, h3)
    return y


def loss_and_grad(theta, X, T):
    """L = mean (y - T)^2 and dL/dtheta (flat), by the chain rule."""
    y, (X, z1, h1, z2, h2, z3, h3) = forward(theta, X, keep=True)
    p = unpack(np.asarray(theta, np.float64))
    n = X.shape[0]
    r = y - np.asarray(T, np.float64)
    L = float(np.mean(r * r))
    dy = 2.0 * r / n                          # dL/dy
    g = np.zeros(N_PARAM)
    G = unpack(g)
    G["W4"][...] = dy @ h3
    G["b4"][0] = dy.sum()
    dz3 = np.outer(dy, p["W4"]) * (z3 > 0)
    G["W3"][...] = dz3.T @ h2
    G["b3"][...] = dz3.sum(axis=0)
    dz2 = (dz3 @ p["W3"]) * (z2 > 0)
    G["W2"][...] = dz2.T @ h1
    G["b2"][...] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"]) * (z1 > 0)
    G["W1"][...] = dz1.T @ X
    G["b1"][...] = dz1.sum(axis=0)
    return L, g


def adam_step(theta, m, v, g, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place (t is the 1-based step count)."""
    m *= beta1
    m += (1.0 - beta1) * g
    v *= beta2
    v += (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    theta -= lr * mhat / (np.sqrt(vhat) + eps)
    return theta


BF16_U = 2.0 ** -8   # unit roundoff of bfloat16 (8 significand bits)


def bf16_error_bound(theta, X, k=6.0):
    """Per-sample bound on |y_bf16 - y| for an evaluation of the network with
    BF16 inputs, weights and activations and FP32 accumulation: each rounding
    is an independent relative error of at most BF16_U, propagated through
    the layers in root-sum-square with this network's own activations
    (var_0 = (u x)^2, var_l = (var_{l-1} + 2 (u h_{l-1})^2) W_l^2 elementwise
    squared, ReLU 1-Lipschitz); k standard deviations per sample."""
    p = unpack(np.asarray(theta, np.float64))
    _, (X, z1, h1, z2, h2, z3, h3) = forward(theta, X, keep=True)
    u = BF16_U
    var = (u * X) ** 2
    for W, h in ((p["W1"], X), (p["W2"], h1), (p["W3"], h2)):
        var = (var + 2 * (u * h) ** 2) @ (W ** 2).T
    var = (var + 2 * (u * h3) ** 2) @ (p["W4"] ** 2)
    return k * np.sqrt(var) + 1e-6
