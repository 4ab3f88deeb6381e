"""Pins of the MLP oracle: parameter count, a hand-computed forward pass,
central finite differences of the loss, and hand-computed Adam steps."""
import numpy as np
import pytest

from oracle import mlp


def test_parameter_count():
    # 4*64 + 64 + 2*(64*64 + 64) + 64 + 1
    assert mlp.N_PARAM == 8705


def test_forward_hand_computed():
    """With W2 = W3 = identity, a single active path gives y by hand."""
    theta = np.zeros(mlp.N_PARAM)
    p = mlp.unpack(theta)
    p["W1"][0] = [1.0, -2.0, 0.5, 0.0]
    p["b1"][0] = 0.25
    p["W2"][...] = np.eye(64)
    p["W3"][...] = np.eye(64)
    p["W4"][0] = 3.0
    p["b4"][0] = -1.0
    x = np.array([[2.0, 0.5, 4.0, 9.0], [0.0, 1.0, 0.0, 0.0]])
    y = mlp.forward(theta, x)
    # row 0: z = 2 - 1 + 2 + 0.25 = 3.25 -> 3 * 3.25 - 1; row 1: z = -2 + .25 < 0 -> -1
    np.testing.assert_allclose(y, [3 * 3.25 - 1.0, -1.0], rtol=1e-15)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = mlp.init_params(1) * 0.5
    X = rng.normal(size=(37, 4))
    T = rng.normal(size=37)
    L, g = mlp.loss_and_grad(theta, X, T)
    idx = np.concatenate([rng.choice(mlp.N_PARAM, 200, replace=False),
                          [0, 255, 256, 8639, 8640, 8703, 8704]])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        Lp = np.mean((mlp.forward(tp, X) - T) ** 2)
        Lm = np.mean((mlp.forward(tm, X) - T) ** 2)
        fd = (Lp - Lm) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-6, abs=1e-9), i


def test_adam_hand_computed():
    """First Adam step moves every coordinate by lr * sign(g) (bias-corrected
    m/sqrt(v) = g/|g|); second step with gradient g2 from the recurrences."""
    theta = np.array([1.0, -2.0, 0.0])
    m, v = np.zeros(3), np.zeros(3)
    g = np.array([0.5, -3.0, 1e-3])
    mlp.adam_step(theta, m, v, g, 1, lr=0.1, eps=0.0)
    np.testing.assert_allclose(theta, [0.9, -1.9, -0.1], rtol=1e-12)
    g2 = np.array([0.5, 1.0, 0.0])
    mlp.adam_step(theta, m, v, g2, 2, lr=0.1, eps=0.0)
    m_ref = 0.9 * 0.1 * g + 0.1 * g2
    v_ref = 0.999 * 0.001 * g * g + 0.001 * g2 * g2
    step = 0.1 * (m_ref / (1 - 0.81)) / np.sqrt(v_ref / (1 - 0.999 ** 2))
    np.testing.assert_allclose(theta, np.array([0.9, -1.9, -0.1]) - step, rtol=1e-12)


def test_training_reduces_loss_on_a_smooth_target():
    """Sanity of the whole loop: fitting y = x0 - 0.5 x1 + x2 x3 lowers the loss."""
    rng = np.random.default_rng(2)
    X = rng.normal(size=(512, 4))
    T = X[:, 0] - 0.5 * X[:, 1] + X[:, 2] * X[:, 3]
    theta = mlp.init_params(3)
    m, v = np.zeros_like(theta), np.zeros_like(theta)
    L0, _ = mlp.loss_and_grad(theta, X, T)
    for t in range(1, 201):
        L, g = mlp.loss_and_grad(theta, X, T)
        mlp.adam_step(theta, m, v, g, t, lr=3e-3)
    assert L < 0.1 * L0


def _bf16(a):
    """Round to bfloat16 (nearest, ties to even), returned as float32."""
    b = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def test_bf16_error_bound_holds_for_an_emulated_bf16_evaluation():
    """The per-sample bound the GPU tests use: a numpy evaluation with BF16
    inputs, weights and activations and FP32 sums and biases stays within
    it at every sample, and the bound is not vacuous (its median ratio to
    the actual error is within two orders of magnitude)."""
    rng = np.random.default_rng(9)
    theta = mlp.init_params(7)
    theta[mlp.N_PARAM - 1] = 0.3
    X = rng.normal(size=(20000, 4))
    p = mlp.unpack(theta)
    h = _bf16(X)
    for W, b in (("W1", "b1"), ("W2", "b2"), ("W3", "b3")):
        z = h @ _bf16(p[W]).T + p[b].astype(np.float32)
        h = _bf16(np.maximum(z, 0.0))
    y = h @ _bf16(p["W4"]) + np.float32(p["b4"][0])
    err = np.abs(y.astype(np.float64) - mlp.forward(theta, X))
    bound = mlp.bf16_error_bound(theta, X)
    assert np.all(err <= bound)
    assert np.median(err / bound) > 1e-2
