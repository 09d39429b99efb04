"""FP64 reference of the warm-start network — TEST INFRASTRUCTURE ONLY.

A plain multilayer perceptron: h_0 = x; z_l = h_l W_l + b_l; h_{l+1} =
GELU(z_l) (exact form x Phi(x)) for every layer but the last, whose z is
the output.  Loss: mean squared error over the batch and output
coordinates.  Optimiser: Adam with bias correction.

With ``bf16=True`` the same values are rounded to bfloat16 (round to nearest
even) where the GPU stores them in bfloat16: the input, the weight copies
used by the products, the hidden activations, and the output-side
gradients used as product operands.  Everything else is FP64.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np
from scipy.special import erf

SQRT2 = np.sqrt(2.0)
INV_SQRT_2PI = 1.0 / np.sqrt(2.0 * np.pi)


def bf16_round(x) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) via FP32; returns FP64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * INV_SQRT_2PI * np.exp(-0.5 * z * z)


Params = List[Tuple[np.ndarray, np.ndarray]]


def forward(params: Params, x, bf16: bool = True):
    r = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    hs = [r(x)]
    zs = []
    Ws = [r(W) for W, _ in params]
    L = len(params)
    for l in range(L):
        z = hs[-1] @ Ws[l] + np.asarray(params[l][1], np.float64)
        zs.append(z)
        if l < L - 1:
            hs.append(r(gelu(z)))
    return zs[-1], (hs, zs, Ws)


def loss_and_grads(params: Params, x, y, bf16: bool = True):
    """MSE loss and gradients (dW_l, db_l) for every layer."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    out, (hs, zs, Ws) = forward(params, x, bf16)
    B, k = out.shape
    diff = out - np.asarray(y, np.float64)
    loss = float((diff * diff).sum() / (B * k))
    g = 2.0 * diff / (B * k)
    grads = [None] * len(params)
    for l in reversed(range(len(params))):
        gb = r(g)
        grads[l] = (hs[l].T @ gb, g.sum(axis=0))
        if l > 0:
            g = (gb @ Ws[l].T) * gelu_grad(zs[l - 1])
    return loss, grads, out


class Adam:
    """Adam with bias correction, FP64 state."""

    def __init__(self, params: Params, b1=0.9, b2=0.999, eps=1e-8):
        self.b1, self.b2, self.eps = b1, b2, eps
        self.t = 0
        self.m = [(np.zeros_like(W, dtype=np.float64), np.zeros_like(b, dtype=np.float64))
                  for W, b in params]
        self.v = [(np.zeros_like(W, dtype=np.float64), np.zeros_like(b, dtype=np.float64))
                  for W, b in params]

    def step(self, params: Params, grads, lr: float) -> Params:
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        out = []
        for l, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
            new = []
            for j, (p, g) in enumerate(((W, gW), (b, gb))):
                m = self.m[l][j] * self.b1 + (1 - self.b1) * g
                v = self.v[l][j] * self.b2 + (1 - self.b2) * g * g
                self.m[l] = tuple(m if q == j else self.m[l][q] for q in range(2))
                self.v[l] = tuple(v if q == j else self.v[l][q] for q in range(2))
                new.append(np.asarray(p, np.float64) - lr * (m / c1) / (np.sqrt(v / c2) + self.eps))
            out.append((new[0], new[1]))
        return out


def feature_stats(raw, min_sd: float):
    """Input standardisation: per-column mean and 1 / max(sample SD, min_sd)
    (the SD with N - 1 in the denominator), FP64."""
    r = np.asarray(raw, np.float64)
    mu = r.mean(axis=0)
    sd = r.std(axis=0, ddof=1) if r.shape[0] > 1 else np.zeros(r.shape[1])
    return mu, 1.0 / np.maximum(sd, min_sd)


def consensus(Y):
    """Mean of each object's m points (Y: k x m x d)."""
    return np.asarray(Y, np.float64).mean(axis=1)


def init_params(dims, seed: int) -> Params:
    """He-normal weights (std sqrt(2/fan_in)), zero biases, FP32."""
    rng = np.random.default_rng(seed)
    out = []
    for a, b in zip(dims[:-1], dims[1:]):
        out.append(((rng.standard_normal((a, b)) * np.sqrt(2.0 / a)).astype(np.float32),
                    np.zeros(b, np.float32)))
    return out
