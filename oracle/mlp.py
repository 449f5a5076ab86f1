"""Plain FP64 CPU oracle of the surrogate network (TEST INFRASTRUCTURE ONLY:
only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s
``cpu_baseline`` leg may use it; it shares no code with the HIP path).

The network maps standardised circuit state and plasma moments to
standardised load responses: three hidden layers of width H with the exact
(erf) GELU, a linear output layer, mean-squared error, Adam (Kingma & Ba,
ICLR 2015) on FP32-master / BF16-compute weights.

With ``bf16=True`` every value the GPU kernels store in BF16 is rounded to
BF16 (round to nearest, ties to even) at the same point: the network input,
the weight copies used by the products, the hidden activations, and the
output- and pre-activation gradients entering the backward products.  All
other arithmetic is FP64.  With ``bf16=False`` the same code is the exact
FP64 network whose gradient is checked against finite differences.

Parameter vector (flat, padded: inputs and outputs to P = 32 columns):
  W1 [H x P], b1 [H], W2 [H x H], b2 [H], W3 [H x H], b3 [H], W4 [P x H], b4 [P]
(W row-major, rows = outputs).  Padded input columns and output rows stay
zero.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

PAD = 32


def bf16(x):
    """Round to the nearest BF16 value (8 significant bits), ties to even."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                 # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0), e - 8)


def gelu(z):
    return 0.5 * z * (1.0 + special.erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + special.erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def layout(H):
    """[(name, shape)] of the flat parameter vector."""
    return [("W1", (H, PAD)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)), ("b3", (H,)),
            ("W4", (PAD, H)), ("b4", (PAD,))]


def unpack(theta, H):
    out, o = {}, 0
    for name, shape in layout(H):
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(p, H):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in layout(H)])


def n_params(H):
    return sum(int(np.prod(s)) for _, s in layout(H))


class MLP:
    """Forward, backward and Adam of the surrogate network."""

    def __init__(self, theta, H, n_in, n_out, bf16_storage=True, norm=None):
        self.H, self.n_in, self.n_out = H, n_in, n_out
        self.theta = np.asarray(theta, dtype=np.float64).copy()
        self.bf = bf16_storage
        self.m = np.zeros_like(self.theta)
        self.v = np.zeros_like(self.theta)
        self.t = 0
        if norm is None:
            norm = (np.zeros(n_in), np.ones(n_in), np.zeros(n_out), np.ones(n_out))
        self.in_mean, self.in_std, self.out_mean, self.out_std = (np.asarray(a, dtype=np.float64) for a in norm)

    def _r(self, x):
        return bf16(x) if self.bf else x

    def _input(self, x):
        B = x.shape[0]
        X = np.zeros((B, PAD))
        X[:, :self.n_in] = (x - self.in_mean) / self.in_std
        return self._r(X)

    def forward_std(self, x, theta=None):
        """Standardised outputs and the stored intermediates."""
        p = unpack(self.theta if theta is None else theta, self.H)
        W = {k: self._r(p[k]) for k in ("W1", "W2", "W3", "W4")}
        A0 = self._input(x)
        Z1 = A0 @ W["W1"].T + p["b1"]
        A1 = self._r(gelu(Z1))
        Z2 = A1 @ W["W2"].T + p["b2"]
        A2 = self._r(gelu(Z2))
        Z3 = A2 @ W["W3"].T + p["b3"]
        A3 = self._r(gelu(Z3))
        Y = A3 @ W["W4"].T + p["b4"]
        return Y, (W, A0, Z1, A1, Z2, A2, Z3, A3)

    def predict(self, x):
        """De-standardised outputs (n_out columns)."""
        Y, _ = self.forward_std(np.atleast_2d(x))
        return Y[:, :self.n_out] * self.out_std + self.out_mean

    def loss_and_grad(self, x, t, theta=None):
        """Mean-squared error over B x n_out standardised targets and its
        gradient with respect to the flat parameters."""
        x = np.atleast_2d(np.asarray(x, dtype=np.float64))
        t = np.atleast_2d(np.asarray(t, dtype=np.float64))
        B = x.shape[0]
        Y, (W, A0, Z1, A1, Z2, A2, Z3, A3) = self.forward_std(x, theta)
        T = np.zeros((B, PAD))
        T[:, :self.n_out] = (t - self.out_mean) / self.out_std
        D = np.zeros((B, PAD))
        D[:, :self.n_out] = Y[:, :self.n_out] - T[:, :self.n_out]
        loss = float(np.sum(D * D)) / (B * self.n_out)
        dY = 2.0 * D / (B * self.n_out)
        g = {}
        G4 = self._r(dY)
        g["W4"] = G4.T @ A3
        g["b4"] = G4.sum(axis=0)
        dZ3 = (G4 @ W["W4"]) * gelu_grad(Z3)
        G3 = self._r(dZ3)
        g["W3"] = G3.T @ A2
        g["b3"] = G3.sum(axis=0)
        dZ2 = (G3 @ W["W3"]) * gelu_grad(Z2)
        G2 = self._r(dZ2)
        g["W2"] = G2.T @ A1
        g["b2"] = G2.sum(axis=0)
        dZ1 = (G2 @ W["W2"]) * gelu_grad(Z1)
        G1 = self._r(dZ1)
        g["W1"] = G1.T @ A0
        g["b1"] = G1.sum(axis=0)
        return loss, pack(g, self.H)

    def adam_step(self, grad, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        """theta -= lr mhat / (sqrt(vhat) + eps) with bias-corrected moments."""
        self.t += 1
        self.m = beta1 * self.m + (1 - beta1) * grad
        self.v = beta2 * self.v + (1 - beta2) * grad * grad
        mhat = self.m / (1 - beta1 ** self.t)
        vhat = self.v / (1 - beta2 ** self.t)
        self.theta = self.theta - lr * mhat / (np.sqrt(vhat) + eps)

    def train_step(self, x, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        loss, g = self.loss_and_grad(x, t)
        self.adam_step(g, lr, beta1, beta2, eps)
        return loss, g
