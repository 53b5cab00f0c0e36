"""Float64 multilayer perceptron -- the oracle of the surrogate network.

Test infrastructure only (see ``oracle/__init__``).

Network with layer widths d_0, ..., d_L:
    h_0 = x,   z_l = W_l h_{l-1} + b_l   (W_l: d_l x d_{l-1}),
    h_l = GELU(z_l) for l < L,   y = z_L,
GELU(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2, GELU'(z) = Phi(z) + z phi(z).
Loss: mean over the batch and the outputs of (y - t)^2.

``bf16=True`` reproduces the rounding points of the library's kernels (the
values themselves stay float64 here): every operand of a matrix product --
the input x, the hidden activations h_l, the weights W_l, and in the
backward pass the gradients with respect to z_l -- is rounded to bfloat16
(round to nearest, ties to even, from float32); biases, pre-activations,
the loss and the gradient sums are not rounded.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) via float32; returns float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _erf(z: np.ndarray) -> np.ndarray:
    return np.vectorize(math.erf, otypes=[np.float64])(z)


def gelu(z: np.ndarray) -> np.ndarray:
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z: np.ndarray) -> np.ndarray:
    phi = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * phi


class MLP:
    def __init__(self, widths: Sequence[int], params: np.ndarray, bf16: bool = False):
        self.widths = list(widths)
        self.bf16 = bf16
        self.W: List[np.ndarray] = []
        self.b: List[np.ndarray] = []
        p = np.asarray(params, dtype=np.float64)
        off = 0
        for l in range(1, len(widths)):
            n_out, n_in = widths[l], widths[l - 1]
            self.W.append(p[off: off + n_out * n_in].reshape(n_out, n_in))
            off += n_out * n_in
            self.b.append(p[off: off + n_out].copy())
            off += n_out
        assert off == p.size

    def _r(self, a):
        return bf16_round(a) if self.bf16 else a

    def forward(self, x: np.ndarray) -> Tuple[np.ndarray, list]:
        h = self._r(np.asarray(x, dtype=np.float64))
        cache = []
        L = len(self.W)
        for l in range(L):
            z = h @ self._r(self.W[l]).T + self.b[l]
            cache.append((h, z))
            h = z if l == L - 1 else self._r(gelu(z))
        return h, cache

    def backward_from(self, cache: list, gy: np.ndarray):
        """Gradients of sum(gy * y) with respect to the parameters and the input."""
        L = len(self.W)
        gW = [None] * L
        gb = [None] * L
        g = np.asarray(gy, dtype=np.float64)
        dx = None
        for l in range(L - 1, -1, -1):
            h, z = cache[l]
            gr = self._r(g)
            gW[l] = gr.T @ h
            gb[l] = g.sum(axis=0)
            da = gr @ self._r(self.W[l])
            if l > 0:
                g = da * gelu_grad(cache[l - 1][1])
            else:
                dx = da
        flat = np.concatenate([np.concatenate([gW[l].ravel(), gb[l]]) for l in range(L)])
        return flat, dx

    def loss_and_grad(self, x: np.ndarray, t: np.ndarray):
        y, cache = self.forward(x)
        n = y.size
        loss = float(np.sum((y - t) ** 2) / n)
        grad, dx = self.backward_from(cache, 2.0 * (y - t) / n)
        return loss, grad, dx
