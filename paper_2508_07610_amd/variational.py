"""Variational GHZ preparation with the MPDO as the verifier, and its
surrogate-assisted form.

The objective is the GHZ fidelity of the noisy RY/CZ ansatz (2 n depth RY
angles, a process-tomography channel after every gate).  The plain optimizer
ascends it with exact parameter-shift gradients: for an RY angle, followed
by a channel that does not depend on it, dF/dtheta_k =
[F(theta + pi/2 e_k) - F(theta - pi/2 e_k)] / 2, so one step is one
``mpdo_batch_run`` over 2P + 1 parameter rows.  The surrogate (``surrogate.MLP``)
is first trained on MPDO-generated (theta, noise) -> observables data
(``generate_dataset``, ``pretrain``); in the variational loop it is refit on
the MPDO rows around the iterate and proposes steps by ascending its own
prediction, and the MPDO verifies every proposal (``surrogate_optimize``);
every accepted point is an MPDO-verified value and the plain parameter-shift
step is the fallback.

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
    e0 = ev.evaluations
    hist: List[tuple] = []
    best = -1.0
    for step in range(max_steps):
        F, g, _, _ = parameter_shift(ev, theta)
        best = max(best, F)
        hist.append((time.perf_counter() - t0, F, ev.evaluations - e0))
        if F >= target or time.perf_counter() - t0 > time_limit:
            break
        theta = opt.step(theta, g)
    reached = best >= target
    tr = next((h[0] for h in hist if h[1] >= target), None)
    rr = next((h[2] for h in hist if h[1] >= target), None)
    return {"reached": reached, "time": tr, "rows_to_target": rr, "best": best, "steps": len(hist),
            "history": hist, "theta": theta, "evaluations": ev.evaluations - e0}


def encode(thetas: np.ndarray, noises: np.ndarray, center: Optional[np.ndarray] = None) -> np.ndarray:
    """Network input: each angle's offset from `center` (0 if None) reduced to
    [-pi, pi) and divided by pi, then the noise strengths."""
    d = thetas if center is None else thetas - center
    th = np.mod(d + math.pi, 2 * math.pi) / math.pi - 1.0
    return np.concatenate([th, noises], axis=1).astype(np.float32)


def generate_dataset(ev: AnsatzEvaluator, count: int, rng: np.random.Generator, batch: int = 2048):
    """The surrogate's data: (theta ~ U[0, 2 pi)^P, noise strengths ~ U[0.5, 2]^2n)
    -> MPDO outputs (GHZ fidelity, <Z_i Z_i+1>), `batch` rows per mpdo_batch_run."""
    X, Y = [], []
    for a in range(0, count, batch):
        k = min(batch, count - a)
        th = rng.uniform(0, 2 * math.pi, size=(k, ev.P))
        nz = rng.uniform(0.5, 2.0, size=(k, n_noise(ev.n)))
        out = ev(th, nz)
        X.append(encode(th, nz))
        Y.append(out.astype(np.float32))
    return np.concatenate(X), np.concatenate(Y)


def pretrain(net, X: np.ndarray, Y: np.ndarray, steps: int, batch: int = 512, lr: float = 1e-3,
             holdout: float = 0.1, rng: Optional[np.random.Generator] = None) -> dict:
    """Train on (X, Y) with the library's kernels (cosine learning-rate
    decay); report the held-out mean absolute error and R^2 per output
    group (fidelity; correlators)."""
    import torch
    rng = rng or np.random.default_rng(0)
    nv = int(len(X) * holdout)
    perm = rng.permutation(len(X))
    va, tr = perm[:nv], perm[nv:]
    xd = torch.tensor(X[tr], device="cuda")
    yd = torch.tensor(Y[tr], device="cuda")
    b = min(batch, net.max_batch, len(tr))
    t0 = time.perf_counter()
    # one library call: minibatches drawn on the device, cosine decay of lr
    net.fit(xd, yd, steps, b, lr, cosine=True, seed=int(rng.integers(1 << 62)))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    xv = torch.tensor(X[va], device="cuda")
    pv = np.concatenate([net.forward(xv[a: a + net.max_batch].contiguous()).cpu().numpy()
                         for a in range(0, nv, net.max_batch)])
    yv = Y[va]
    mae = np.abs(pv - yv).mean(0)
    r2 = 1 - ((pv - yv) ** 2).mean(0) / np.maximum(yv.var(0), 1e-30)
    return {"train_seconds": dt, "steps": steps, "holdout": nv, "mae_fidelity": float(mae[0]),
            "mae_correlators": float(mae[1:].mean()), "r2_fidelity": float(r2[0]),
            "r2_correlators": float(r2[1:].mean()), "fidelity_mean": float(yv[:, 0].mean()),
            "fidelity_max": float(yv[:, 0].max())}


def surrogate_optimize(ev: AnsatzEvaluator, net, theta0: np.ndarray, target: float, max_rows: int = 20000,
                       lr: float = 0.05, fit_steps: int = 150, fit_lr: float = 1e-3, fit_batch: int = 512,
                       window: int = 4,
                       inner: int = 30, inner_lr: float = 0.04, cand_at=(3, 6, 10, 15, 22, 30),
                       out_scale: float = 10.0, time_limit: float = 600.0) -> dict:
    """Surrogate-assisted ascent: the network proposes steps, the MPDO verifies them.

    Every parameter-shift evaluation (2P + 1 rows: the exact gradient, which
    also labels data around the iterate) is added to a buffer.  The network is
    refit on the buffer's last `window` gradient evaluations in coordinates
    centred on the iterate (inputs: angle offsets, outputs: the change of
    fidelity, scaled), then its input gradient is ascended from the iterate
    on the device (Adam, `inner` steps); the points reached after the steps
    in `cand_at`, and the plain Adam step, are evaluated together by one
    MPDO batch.  The best verified point is taken if it beats the iterate;
    when it is one of the network's points, the network proposes again from
    there without a new gradient, otherwise the next iteration starts with a
    parameter-shift evaluation.  The network is refit only after a gradient
    evaluation; a proposal round that continues from an accepted point of the
    network keeps ascending in the same coordinates.  Every accepted point is
    an MPDO value; the plain step is the fallback.  The refit (``MLP.fit``)
    and the ascent (``MLP.ascend``, on the network input u = offset / pi with
    lr / pi and eps pi: the same Adam path as in the offsets) each run as one
    library call.  Returns the record of plain_optimize plus the surrogate's
    proposal statistics and its error on verified points."""
    import torch
    P = ev.P
    nn_ = n_noise(ev.n)
    noise = np.ones((1, nn_))
    opt = Adam(P, lr)
    theta = theta0.copy()
    Xr = np.zeros((0, P))
    Yr = np.zeros((0,))
    t0 = time.perf_counter()
    hist: List[tuple] = []
    counts = {"gradients": 0, "proposal_rounds": 0, "surrogate_accepted": 0, "plain_accepted": 0}
    errs = []
    best = -1.0
    need_grad = True
    Fc = -1.0
    plain_next = theta
    nz_t = torch.tensor(noise.astype(np.float32), device="cuda")
    rows_per_grad = 2 * P + 1
    e0 = ev.evaluations
    while ev.evaluations - e0 < max_rows:
        if need_grad:
            F, g, rows, out = parameter_shift(ev, theta)
            counts["gradients"] += 1
            Xr = np.concatenate([Xr, rows])[-window * rows_per_grad * 2:]
            Yr = np.concatenate([Yr, out[:, 0]])[-window * rows_per_grad * 2:]
            Fc = F
            best = max(best, F)
            hist.append((time.perf_counter() - t0, F, ev.evaluations - e0))
            if F >= target or time.perf_counter() - t0 > time_limit:
                break
            plain_next = opt.step(theta, g)
        if need_grad:
            # refit around the iterate (inputs: offsets from it; output: the
            # change of fidelity); the ascent starts there
            center, Fref = theta.copy(), Fc
            xd = torch.tensor(encode(Xr, np.repeat(noise, len(Xr), 0), center), device="cuda")
            yt = np.zeros((len(Xr), net.widths[-1]), np.float32)
            yt[:, 0] = (Yr - Fref) * out_scale
            yd = torch.tensor(yt, device="cuda")
            nb = min(net.max_batch, len(Xr), fit_batch)
            net.fit(xd, yd, fit_steps, nb, fit_lr, seed=7919 * counts["gradients"] + 17)
            x0 = torch.cat([torch.zeros((1, P), dtype=torch.float32, device="cuda"), nz_t], dim=1).view(-1)
            reset = True
        # ascend the network on the device from the last accepted point
        rows_all = net.ascend(x0.contiguous(), P, inner, inner_lr / math.pi, eps=1e-8 * math.pi, reset=reset)
        cands = rows_all[[t - 1 for t in cand_at if t <= inner]].contiguous()
        xs = cands[:, :P].double().cpu().numpy() * math.pi
        pred = net.forward(cands).cpu().numpy()[:, 0] / out_scale + Fref
        C = center[None, :] + xs
        if need_grad:
            C = np.concatenate([C, plain_next[None, :]])
        out = ev(C)
        counts["proposal_rounds"] += 1
        errs.extend(np.abs(pred - out[: len(cands), 0]).tolist())
        Xr = np.concatenate([Xr, C])[-window * rows_per_grad * 2:]
        Yr = np.concatenate([Yr, out[:, 0]])[-window * rows_per_grad * 2:]
        b = int(np.argmax(out[:, 0]))
        if out[b, 0] > Fc:
            theta, Fc = C[b], float(out[b, 0])
            best = max(best, Fc)
            hist.append((time.perf_counter() - t0, Fc, ev.evaluations - e0))
            if b < len(cands):
                counts["surrogate_accepted"] += 1
                need_grad = False
                x0 = cands[b].clone()   # continue from the accepted point (same moments)
                reset = False
            else:
                counts["plain_accepted"] += 1
                need_grad = True
            if Fc >= target:
                break
        else:
            if need_grad:
                theta = plain_next   # the plain step is taken as the fallback
                counts["plain_accepted"] += 1
            need_grad = True
        if time.perf_counter() - t0 > time_limit:
            break
    reached = best >= target
    tr = next((h[0] for h in hist if h[1] >= target), None)
    rr = next((h[2] for h in hist if h[1] >= target), None)
    return {"reached": reached, "time": tr, "rows_to_target": rr, "best": best, "history": hist,
            "theta": theta, "evaluations": ev.evaluations - e0, **counts,
            "surrogate_abs_err": float(np.mean(errs)) if errs else None}
