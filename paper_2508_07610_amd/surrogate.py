"""Binding of the surrogate network (``mpdo_mlp_*`` in include/mpdo.h).

Argument marshalling only: forward, backward and Adam run in the library's
HIP kernels on torch-allocated device buffers.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

from . import mpdo as M

# C5 surrogate: 144 ansatz angles + 24 noise strengths -> GHZ fidelity and 11 <Z_i Z_i+1>
C5_WIDTHS = (168, 256, 256, 256, 12)


def init_params(widths: Sequence[int], rng: np.random.Generator) -> np.ndarray:
    """W_l ~ N(0, 1/d_{l-1}), b_l = 0, packed W_1, b_1, W_2, b_2, ..."""
    parts = []
    for l in range(1, len(widths)):
        parts.append(rng.normal(scale=1.0 / np.sqrt(widths[l - 1]), size=widths[l] * widths[l - 1]))
        parts.append(np.zeros(widths[l]))
    return np.concatenate(parts).astype(np.float32)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class MLP:
    def __init__(self, widths: Sequence[int], max_batch: int, params: Optional[np.ndarray] = None,
                 seed: int = 0, stream=None):
        import torch
        self.widths = [int(w) for w in widths]
        self.max_batch = int(max_batch)
        w = (ctypes.c_int32 * len(self.widths))(*self.widths)
        self._h = ctypes.c_void_p()
        M.check(M.lib().mpdo_mlp_create(w, len(self.widths) - 1, self.max_batch, M.stream_handle(stream),
                                        ctypes.byref(self._h)))
        n = ctypes.c_int64()
        M.check(M.lib().mpdo_mlp_info(self._h, ctypes.byref(n)))
        self.nparams = n.value
        self._torch = torch
        if params is None:
            params = init_params(self.widths, np.random.default_rng(seed))
        self.set_params(params)

    def close(self) -> None:
        if self._h:
            M.lib().mpdo_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p: np.ndarray) -> None:
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.nparams
        M.check(M.lib().mpdo_mlp_set_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def get_params(self) -> np.ndarray:
        p = np.zeros(self.nparams, dtype=np.float32)
        M.check(M.lib().mpdo_mlp_get_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return p

    def _check(self, x):
        torch = self._torch
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and x.shape[1] == self.widths[0]
        assert 1 <= x.shape[0] <= self.max_batch

    def forward(self, x):
        self._check(x)
        y = self._torch.empty((x.shape[0], self.widths[-1]), dtype=self._torch.float32, device=x.device)
        M.check(M.lib().mpdo_mlp_forward(self._h, x.data_ptr(), x.shape[0], y.data_ptr()))
        return y

    def backward(self, x, t=None, gy=None, want_grad=False, want_dx=False, want_loss=True):
        """Returns (y, grad or None, dx or None, loss or None)."""
        torch = self._torch
        self._check(x)
        B = x.shape[0]
        y = torch.empty((B, self.widths[-1]), dtype=torch.float32, device=x.device)
        g = torch.empty(self.nparams, dtype=torch.float32, device=x.device) if want_grad else None
        dx = torch.empty_like(x) if want_dx else None
        loss = ctypes.c_float()
        M.check(M.lib().mpdo_mlp_backward(self._h, x.data_ptr(), _ptr(t), _ptr(gy), B, y.data_ptr(), _ptr(g),
                                          _ptr(dx), ctypes.byref(loss) if want_loss else None))
        return y, g, dx, (loss.value if want_loss else None)

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
        M.check(M.lib().mpdo_mlp_adam(self._h, lr, beta1, beta2, eps))

    def train_step(self, x, t, lr: float, want_loss: bool = True):
        _, _, _, loss = self.backward(x, t=t, want_loss=want_loss)
        self.adam(lr)
        return loss

    def fit(self, x, t, steps: int, batch: int, lr: float, cosine: bool = False, seed: int = 0,
            want_loss: bool = False):
        """`steps` Adam steps on minibatches of `batch` rows drawn on the
        device (SplitMix64 from `seed`) from the dataset (x, t), in one call;
        returns the last step's loss if want_loss."""
        torch = self._torch
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and x.shape[1] == self.widths[0]
        assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.shape == (x.shape[0], self.widths[-1])
        loss = ctypes.c_float()
        M.check(M.lib().mpdo_mlp_fit(self._h, x.data_ptr(), t.data_ptr(), x.shape[0], int(batch), int(steps),
                                     float(lr), 1 if cosine else 0, int(seed) & ((1 << 64) - 1),
                                     ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def ascend(self, x0, nfree: int, steps: int, lr: float, out_index: int = 0, beta1: float = 0.9,
               beta2: float = 0.999, eps: float = 1e-8, reset: bool = True):
        """Adam ascent of output `out_index` over the first `nfree` inputs
        from the row x0 (d_0 floats on the device); returns the (steps, d_0)
        rows after each step.  The moments persist between calls unless reset."""
        torch = self._torch
        assert x0.is_cuda and x0.dtype == torch.float32 and x0.is_contiguous() and x0.numel() == self.widths[0]
        xs = torch.empty((max(int(steps), 1), self.widths[0]), dtype=torch.float32, device=x0.device)
        M.check(M.lib().mpdo_mlp_ascend(self._h, x0.data_ptr(), int(nfree), int(out_index), int(steps), float(lr),
                                        float(beta1), float(beta2), float(eps), 1 if reset else 0, xs.data_ptr()))
        return xs[: int(steps)]
