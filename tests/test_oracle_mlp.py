"""Pins of the FP64 surrogate reference (oracle/mlp.py) against definitions
it does not itself use: finite differences, closed forms of GELU and Adam,
and torch's own float32 -> bfloat16 conversion."""
import math

import numpy as np

from oracle import mlp
from paper_2403_11167_amd import inputs


def norm4():
    return dict(x_shift=np.array([0.5, 0.725, 5.0, 1.25]),
                x_scale=np.array([2.0, 2 / 0.45, 1 / 3, 2 / 1.5]),
                y_shift=np.array([-1.0, -4.0, -5.0, 1.5]),
                y_scale=np.array([0.2, 1.0, 0.7, 0.3]))


def data(n, seed):
    rng = np.random.default_rng(seed)
    x = np.stack([rng.integers(0, 2, n), rng.uniform(0.5, 0.95, n), rng.uniform(2, 8, n),
                  rng.uniform(0.5, 2, n)], axis=1).astype(np.float64)
    y = np.exp(np.stack([-1 + 0.2 * rng.standard_normal(n), -4 + rng.standard_normal(n),
                         -5 + 0.7 * rng.standard_normal(n), 1.5 + 0.3 * rng.standard_normal(n)],
                        axis=1))
    return x, y


def test_parameter_count_and_layout():
    assert mlp.NPARAMS == 34180
    assert inputs.mlp_initial_params(0).size == mlp.NPARAMS
    offs = [w for w, _, _, _ in mlp.LAYOUT]
    assert offs == [0, 640, 17152, 33664]


def test_bf16_round_matches_torch_conversion():
    import torch
    rng = np.random.default_rng(1)
    v = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        # exact ties: bfloat16 value plus half an ulp
                        (np.arange(1, 200, dtype=np.float32) * 2 ** -7 + 1.0) + 2 ** -8,
                        np.array([0.0, -0.0, 1.0, -2.5, 3.0e38])]).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    got = mlp.bf16_round(v)
    assert np.array_equal(got, ref)


def test_gelu_closed_forms():
    phi1 = 0.5 * (1 + math.erf(1 / math.sqrt(2)))
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert abs(mlp.gelu(np.array([1.0]))[0] - phi1) < 1e-16
    assert abs(mlp.gelu(np.array([-1.0]))[0] + (1 - phi1)) < 1e-16
    z = np.linspace(-6, 6, 101)
    # x Phi(x) - (-x) Phi(-x) = x
    assert np.max(np.abs(mlp.gelu(z) - mlp.gelu(-z) - z)) < 1e-14
    h = 1e-5
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_prime(z))) < 1e-9


def test_gradient_matches_finite_differences():
    x, y = data(24, 2)
    theta = inputs.mlp_initial_params(3).astype(np.float64)
    theta += 0.05 * np.random.default_rng(4).standard_normal(theta.size)  # nonzero biases
    nm = norm4()
    _, g = mlp.loss_and_grad(theta, x, y, nm)
    rng = np.random.default_rng(5)
    picks = np.concatenate([np.arange(0, 640, 7), rng.integers(640, 33664, 300),
                            np.arange(33664, mlp.NPARAMS)])
    h = 1e-6
    for p in picks:
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        fd = (mlp.loss_and_grad(tp, x, y, nm)[0] - mlp.loss_and_grad(tm, x, y, nm)[0]) / (2 * h)
        assert abs(fd - g[p]) <= 1e-7 * max(1.0, abs(g[p])) + 1e-9, (p, fd, g[p])


def test_perfect_targets_give_zero_loss_and_gradient():
    x, _ = data(10, 6)
    theta = inputs.mlp_initial_params(7).astype(np.float64)
    nm = norm4()
    y = mlp.predict(theta, x, nm)
    loss, g = mlp.loss_and_grad(theta, x, y, nm)
    assert loss < 1e-28 and np.max(np.abs(g)) < 1e-14


def test_adam_constant_gradient_closed_form():
    # with a constant gradient g: m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2,
    # so every bias-corrected step moves theta by -lr g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    theta = np.array([1.0, 2.0, 3.0, 4.0])
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 0.01, 1e-8
    th = theta.copy()
    for t in range(1, 6):
        th, m, v = mlp.adam(th, m, v, g, t, lr, eps=eps)
        assert np.allclose(m, (1 - 0.9 ** t) * g, rtol=1e-14, atol=0)
        assert np.allclose(v, (1 - 0.999 ** t) * g * g, rtol=1e-13, atol=0)
    step = -lr * g / (np.abs(g) + eps)
    assert np.allclose(th, theta + 5 * step, rtol=1e-12, atol=1e-15)


def test_training_by_reference_reduces_loss():
    x, y = data(64, 8)
    theta = inputs.mlp_initial_params(9).astype(np.float64)
    nm = norm4()
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = mlp.loss_and_grad(theta, x, y, nm)[0]
    for t in range(1, 151):
        _, g = mlp.loss_and_grad(theta, x, y, nm)
        theta, m, v = mlp.adam(theta, m, v, g, t, 3e-3)
    assert mlp.loss_and_grad(theta, x, y, nm)[0] < 0.2 * l0
