"""Variational GHZ preparation with the MPDO as the judge, and its
surrogate-assisted form.

The objective is the GHZ fidelity of the noisy RY/CZ ansatz (2 n depth RY
angles, a process-tomography channel after every gate).  The plain optimizer
ascends it with exact parameter-shift gradients: for an RY angle, followed
by a channel that does not depend on it, dF/dtheta_k =
[F(theta + pi/2 e_k) - F(theta - pi/2 e_k)] / 2, so one step is one
``mpdo_batch_run`` over 2P + 1 parameter rows.  The surrogate-assisted
optimizer trains the MLP (``surrogate.MLP``) on every MPDO evaluation it has
made, proposes a step by ascending the network's prediction, and accepts it
only if one MPDO evaluation confirms an improvement; otherwise it falls back
to a parameter-shift step.  Every accepted point is an MPDO-verified value.

Noise inputs (the 2n = 24 strengths of the surrogate's input at n = 12):
n per-qubit scales of the 1q channel, n - 1 per-bond scales of the 2q
channel and one global scale; a gate's channel strength is its scale times
the global scale, quantised to a log grid of 33 levels on [1/4, 4]
(``workloads.gate_noise_levels``).
"""
from __future__ import annotations

import ctypes
import math
import time
from typing import List, Optional

import numpy as np

from . import mpdo as M
from . import workloads as W

LEVELS = W.NOISE_LEVELS


def n_noise(n: int) -> int:
    return 2 * n


class AnsatzEvaluator:
    """GHZ fidelity and <Z_i Z_i+1> of the noisy ansatz for many (theta, noise) rows, one batch_run per call."""

    def __init__(self, n: int, depth: int, chi_max: int = 32, kappa_max: int = 4, prec: int = M.C128,
                 svd_cutoff: float = 1e-10, kappa_cutoff: float = 1e-10):
        self.n, self.depth = n, depth
        self.P = 2 * n * depth
        self.kw = dict(chi_max=chi_max, kappa_max=kappa_max, max_kraus=16, svd_cutoff=svd_cutoff,
                       kappa_cutoff=kappa_cutoff, prec=prec)
        self.chans = ([M.Channel(W.chi_1q_default(W.noise_level_scale(i)), 1) for i in range(LEVELS)]
                      + [M.Channel(W.chi_2q_default(W.noise_level_scale(i)), 2) for i in range(LEVELS)])
        self._chan_arr = (ctypes.c_void_p * len(self.chans))(*[c.handle.value for c in self.chans])
        fixed = np.zeros((1, 4, 4), dtype=np.complex128)
        fixed[0] = W.CZ
        self._fixed = M._cplx(fixed)
        obs = []
        for i in range(n - 1):
            o = np.stack([np.eye(2, dtype=np.complex128)] * n)
            o[i] = o[i + 1] = np.diag([1.0, -1.0])
            obs.append(o)
        for m in (np.diag([1.0, 0.0]), np.diag([0.0, 1.0]), np.array([[0.0, 1.0], [0.0, 0.0]])):
            obs.append(np.stack([m.astype(np.complex128)] * n))
        self.nobs = len(obs)
        self._obs = M._cplx(np.stack(obs))
        self._ops_cache = {}
        self.evaluations = 0

    def _ops(self, noise: Optional[np.ndarray]):
        n = self.n
        eff1, eff2 = W.gate_noise_levels(n, noise)
        key = (eff1.tobytes(), eff2.tobytes())
        ops = self._ops_cache.get(key)
        if ops is not None:
            return ops
        count = self.depth * (2 * n + (n // 2) + ((n - 1) // 2))
        ops = (M.mpdo_op * count)()
        j = k = 0
        for _ in range(self.depth):
            for parity in (0, 1):
                for q in range(n):
                    o = ops[j]
                    o.q, o.site, o.kind, o.param, o.scale, o.chan, o.fixed = 1, q, M.G_RY, k, 1.0, int(eff1[q]), 0
                    j += 1
                    k += 1
                for q in range(parity, n - 1, 2):
                    o = ops[j]
                    o.q, o.site, o.kind, o.param, o.scale, o.chan, o.fixed = 2, q, M.G_FIXED, -1, 1.0, \
                        LEVELS + int(eff2[q]), 0
                    j += 1
        assert j == count
        if len(self._ops_cache) > 4096:
            self._ops_cache.clear()
        self._ops_cache[key] = ops
        return ops

    def __call__(self, thetas, noises: Optional[np.ndarray] = None):
        """thetas: (K, P) array (numpy or torch); noises: (K, 2n) or None (all ones).
        Returns numpy (K, n): column 0 the GHZ fidelity, then <Z_i Z_i+1>."""
        import torch
        th = torch.as_tensor(thetas, dtype=torch.float64, device="cuda").contiguous()
        K = th.shape[0]
        progs = (M.mpdo_program * K)()
        keep = []
        for b in range(K):
            ops = self._ops(None if noises is None else np.asarray(noises[b]))
            keep.append(ops)
            progs[b].n = self.n
            progs[b].nops = len(ops)
            progs[b].ops = ops
            progs[b].nobs = self.nobs
            progs[b].obs = M._dptr(self._obs)
        out = torch.empty(K * self.nobs, dtype=torch.complex128, device="cuda")
        cfg = M.mpdo_config(0, self.kw["chi_max"], self.kw["kappa_max"], self.kw["max_kraus"],
                            self.kw["svd_cutoff"], self.kw["kappa_cutoff"], self.kw["prec"])
        M.check(M.lib().mpdo_batch_run(ctypes.byref(cfg), progs, K, th.data_ptr(), self.P, M._dptr(self._fixed), 1,
                                       self._chan_arr, len(self.chans), out.data_ptr(), 0, None))
        r = out.view(K, self.nobs).cpu().numpy()
        self.evaluations += K
        res = np.empty((K, self.n))
        res[:, 0] = 0.5 * (r[:, -3].real + r[:, -2].real + 2 * r[:, -1].real)
        res[:, 1:] = r[:, : self.n - 1].real
        return res


class Adam:
    def __init__(self, dim: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.m = np.zeros(dim)
        self.v = np.zeros(dim)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, x: np.ndarray, g: np.ndarray) -> np.ndarray:
        """One ascent step along g."""
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return x + self.lr * mh / (np.sqrt(vh) + self.eps)


def shift_rows(theta: np.ndarray) -> np.ndarray:
    P = theta.size
    rows = np.repeat(theta[None, :], 2 * P + 1, axis=0)
    idx = np.arange(P)
    rows[1 + idx, idx] += math.pi / 2
    rows[1 + P + idx, idx] -= math.pi / 2
    return rows


def parameter_shift(ev: AnsatzEvaluator, theta: np.ndarray):
    """F(theta), its exact gradient, and all 2P + 1 evaluated rows with their outputs."""
    rows = shift_rows(theta)
    out = ev(rows)
    P = theta.size
    F = out[:, 0]
    grad = 0.5 * (F[1: 1 + P] - F[1 + P:])
    return F[0], grad, rows, out


def plain_optimize(ev: AnsatzEvaluator, theta0: np.ndarray, target: float, max_steps: int = 200,
                   lr: float = 0.05, time_limit: float = 600.0) -> dict:
    """Parameter-shift gradient ascent (Adam) until the MPDO-verified F reaches target."""
    theta = theta0.copy()
    opt = Adam(theta.size, lr)
    t0 = time.perf_counter()
    hist: List[tuple] = []
    best = -1.0
    for step in range(max_steps):
        F, g, _, _ = parameter_shift(ev, theta)
        best = max(best, F)
        hist.append((time.perf_counter() - t0, F, ev.evaluations))
        if F >= target or time.perf_counter() - t0 > time_limit:
            break
        theta = opt.step(theta, g)
    reached = best >= target
    return {"reached": reached, "time": hist[-1][0] if reached else None, "best": best, "steps": len(hist),
            "history": hist, "theta": theta, "evaluations": ev.evaluations}


def encode(thetas: np.ndarray, noises: np.ndarray) -> np.ndarray:
    """Network input: angles reduced to [-pi, pi) and divided by pi, then the noise scales."""
    th = np.mod(thetas + math.pi, 2 * math.pi) / math.pi - 1.0
    return np.concatenate([th, noises], axis=1).astype(np.float32)


def generate_dataset(ev: AnsatzEvaluator, count: int, rng: np.random.Generator, batch: int = 256):
    """(theta ~ U[0, 2 pi), noise scales ~ U[0.5, 2]) -> MPDO outputs."""
    X, Y = [], []
    for a in range(0, count, batch):
        k = min(batch, count - a)
        th = rng.uniform(0, 2 * math.pi, size=(k, ev.P))
        nz = rng.uniform(0.5, 2.0, size=(k, n_noise(ev.n)))
        out = ev(th, nz)
        X.append(encode(th, nz))
        Y.append(out.astype(np.float32))
    return np.concatenate(X), np.concatenate(Y)


def surrogate_optimize(ev: AnsatzEvaluator, net, theta0: np.ndarray, target: float, max_steps: int = 200,
                       lr: float = 0.05, fit_steps: int = 150, fit_lr: float = 2e-3,
                       scales=(1.0, 2.0, 3.0, 4.0, 6.0, 8.0), window: int = 4096, time_limit: float = 600.0,
                       rng: Optional[np.random.Generator] = None) -> dict:
    """Surrogate-assisted ascent.  Each iteration computes the parameter-shift
    gradient (2P + 1 MPDO rows, which also label the network's training data
    around the iterate), refits the network on the samples seen so far, and
    lets it choose the length of the Adam step: the candidates
    theta + a * delta (delta the plain Adam step, a in `scales`) are ranked by
    the predicted fidelity, and the MPDO evaluates the network's choice next to
    the plain step (a = 1); the better verified point is taken.  With a = 1
    always chosen this is the plain optimizer, so the network can only change
    which MPDO-verified point is kept.  Returns the plain_optimize record plus
    the choices and the network's error on the verified points."""
    import torch
    rng = rng or np.random.default_rng(0)
    theta = theta0.copy()
    opt = Adam(theta.size, lr)
    noise = np.ones((1, n_noise(ev.n)))
    X = np.zeros((0, ev.P + n_noise(ev.n)), np.float32)
    Y = np.zeros((0, ev.n), np.float32)
    t0 = time.perf_counter()
    hist: List[tuple] = []
    picks, errs = [], []
    best = -1.0
    for step in range(max_steps):
        F, g, rows, out = parameter_shift(ev, theta)
        X = np.concatenate([X, encode(rows, np.repeat(noise, rows.shape[0], 0))])[-window:]
        Y = np.concatenate([Y, out.astype(np.float32)])[-window:]
        best = max(best, F)
        hist.append((time.perf_counter() - t0, F, ev.evaluations))
        if F >= target or time.perf_counter() - t0 > time_limit:
            break
        delta = opt.step(theta, g) - theta
        # refit on the samples seen so far
        xd = torch.tensor(X, device="cuda")
        yd = torch.tensor(Y, device="cuda")
        nb = min(net.max_batch, X.shape[0])
        for _ in range(fit_steps):
            idx = torch.randint(0, X.shape[0], (nb,), device="cuda")
            net.train_step(xd[idx].contiguous(), yd[idx].contiguous(), fit_lr, want_loss=False)
        cands = np.stack([theta + a * delta for a in scales])
        pred = net.forward(torch.tensor(encode(cands, np.repeat(noise, len(scales), 0)), device="cuda"))
        pred = pred.cpu().numpy()[:, 0]
        pick = int(np.argmax(pred))
        picks.append(scales[pick])
        if pick == 0:
            theta = cands[0]
            continue
        ver = ev(np.stack([cands[0], cands[pick]]))[:, 0]
        errs.append(abs(float(pred[pick]) - float(ver[1])))
        theta = cands[pick] if ver[1] > ver[0] else cands[0]
    reached = best >= target
    return {"reached": reached, "time": hist[-1][0] if reached else None, "best": best, "steps": len(hist),
            "history": hist, "theta": theta, "evaluations": ev.evaluations, "proposals": len(picks),
            "longer_steps_chosen": int(sum(1 for p in picks if p != 1.0)),
            "surrogate_abs_err": float(np.mean(errs)) if errs else None}
