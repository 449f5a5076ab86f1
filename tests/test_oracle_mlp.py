"""Pins of the surrogate-network oracle (oracle/mlp.py): BF16 rounding
against the bit-level definition, the exact GELU and its derivative, the
FP64 backward pass against central finite differences, Adam's first steps
in closed form, and that training lowers the loss on a learnable map."""
import math

import numpy as np
import pytest

from oracle import mlp as M
from paper_2609_15043_amd import workloads as W


def _bits_bf16(x32):
    """BF16 of FP32 values through their bit patterns: add 0x7FFF plus the
    lowest kept bit, drop the low 16 bits."""
    u = np.asarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def test_bf16_rounding():
    rng = np.random.default_rng(1)
    x = (rng.normal(size=200_000) * np.exp(rng.uniform(-20, 20, 200_000))).astype(np.float32)
    assert np.array_equal(M.bf16(x.astype(np.float64)), _bits_bf16(x))
    # ties go to the even neighbour
    assert M.bf16(1 + 2 ** -8) == 1.0
    assert M.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6
    assert M.bf16(-(1 + 2 ** -8)) == -1.0
    assert M.bf16(0.0) == 0.0


def test_gelu_and_derivative():
    z = np.linspace(-6, 6, 1201)
    assert abs(M.gelu(np.array(0.0))) == 0.0
    assert abs(M.gelu_grad(np.array(0.0)) - 0.5) < 1e-15
    # GELU(z) - GELU(-z) = z and GELU -> relu in the tails
    assert np.max(np.abs(M.gelu(z) - M.gelu(-z) - z)) < 1e-14
    assert abs(M.gelu(np.array(8.0)) - 8.0) < 1e-12
    h = 1e-5
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - M.gelu_grad(z))) < 1e-9


def test_fp64_backward_matches_finite_differences():
    H, n_in, n_out, B = 64, 29, 20, 16
    theta = W.mlp_init_params(seed=3, hidden=H).astype(np.float64)
    rng = np.random.default_rng(4)
    # non-zero biases so their gradients are exercised
    p = M.unpack(theta, H)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.normal(0, 0.1, p[k].shape)
    p["b4"][:n_out] = rng.normal(0, 0.1, n_out)
    theta = M.pack(p, H)
    net = M.MLP(theta, H, n_in, n_out, bf16_storage=False)
    x = rng.normal(size=(B, n_in))
    t = rng.normal(size=(B, n_out))
    loss, g = net.loss_and_grad(x, t)
    idx = rng.choice(np.nonzero(theta != 0)[0], 60, replace=False)
    idx = np.concatenate([idx, np.nonzero(np.abs(g) > 0)[0][-20:]])
    def f(i, d):
        th = theta.copy()
        th[i] += d
        return net.loss_and_grad(x, t, th)[0]

    for i in idx:
        # fourth-order central difference
        h = 1e-4 * max(1.0, abs(theta[i]))
        fd = (8 * (f(i, h) - f(i, -h)) - (f(i, 2 * h) - f(i, -2 * h))) / (12 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(abs(g[i]), 1e-3 * np.max(np.abs(g))), (i, fd, g[i])
    # padding stays out of the gradient
    gp = M.unpack(g, H)
    assert np.all(gp["W1"][:, n_in:] == 0) and np.all(gp["W4"][n_out:] == 0) and np.all(gp["b4"][n_out:] == 0)


def test_adam_first_steps_closed_form():
    H = 64
    theta = W.mlp_init_params(seed=5, hidden=H).astype(np.float64)
    net = M.MLP(theta, H, 29, 20)
    g = np.random.default_rng(6).normal(size=theta.size)
    g[::7] = 0.0
    lr = 1e-3
    net.adam_step(g, lr)
    # first step: mhat = g, vhat = g^2, so the step is lr g / (|g| + eps)
    np.testing.assert_allclose(net.theta, theta - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    th1 = net.theta.copy()
    net.adam_step(g, lr)
    # same gradient again: the bias-corrected moments are unchanged
    np.testing.assert_allclose(net.theta, th1 - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_training_lowers_the_loss():
    H, n_in, n_out = 64, 29, 20
    rng = np.random.default_rng(7)
    A = rng.normal(size=(n_in, n_out)) / math.sqrt(n_in)
    x = rng.normal(size=(512, n_in))
    t = np.tanh(x @ A)
    net = M.MLP(W.mlp_init_params(seed=8, hidden=H), H, n_in, n_out)
    l0 = net.loss_and_grad(x, t)[0]
    for _ in range(60):
        net.train_step(x, t, 3e-3)
    l1 = net.loss_and_grad(x, t)[0]
    assert l1 < 0.2 * l0, (l0, l1)
