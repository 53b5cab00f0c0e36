"""The truncation study of Sec. IV.C (Fig. `exp1_fig`): random one-dimensional
circuits (a layer of random RX / RY / RZ, then a CNOT layer, m - 1 times,
then a final single-qubit layer; Fig. `randomCirc_fig`(a)) with QPT-style
noise after every gate and a crosstalk rotation RZ(alpha), alpha uniform in
(1e-5 pi, 1e-3 pi], on the nearest neighbour of every CNOT (Fig.
`randomCirc_fig`(b)); the Uhlmann fidelity of Sec. IV.C between the state
simulated without truncation and with bond / inner limits (chi, kappa),
averaged over many circuits.

The crosstalk rotation acts on a qubit the CNOT does not touch, so it is
applied as a unitary on that qubit right after the CNOT (the same map as the
three-qubit gate of Fig. `randomCirc_fig`(b)).  Every simulation runs on the
device; the fidelity is a host-side measurement (NumPy eigendecompositions)
of the dense results (n <= 12).

``run_batched`` is the study at the paper's scale: all circuits of one
(Q, depth) point and one (chi, kappa) limit in one ``mpdo_batch_run_dense``
call (the reference at chi = kappa = 64, the largest limits, is one more such
call; it is lossless only to within its own discarded weight), the
paper's 1,000 circuits per point."""
from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import mpdo as M
from . import workloads as W
from .crosstalk import uhlmann_fidelity


def circuit(q: int, depth: int, rng: np.random.Generator) -> "W.Program":
    """One random circuit of the study (depth = number of CNOT layers m - 1
    plus the final single-qubit layer, as in the paper's construction)."""
    gates = (W.rx, W.ry, W.rz)
    chis = [W.chi_1q_default(), W.chi_2q_default()]
    ops: List[W.Op] = []

    def one_q_layer():
        for s in range(q):
            g = gates[int(rng.integers(0, 3))]
            ops.append(W.Op((s,), g(float(2 * math.pi - rng.uniform(0, 2 * math.pi))), 0, "r"))

    for d in range(depth):
        one_q_layer()
        for a in range(d % 2, q - 1, 2):
            for _, sites, U in W.cnot_compiled():
                ops.append(W.Op(tuple(a + t for t in sites), U, 1 if len(sites) == 2 else -1, "cnot"))
            nb = a + 2 if a + 2 < q else a - 1  # the neighbour of the pair
            if 0 <= nb < q:
                alpha = math.pi * (1e-5 + (1e-3 - 1e-5) * (1.0 - rng.random()))
                ops.append(W.Op((nb,), W.rz(alpha), -1, "xtalk"))
    one_q_layer()
    return W.Program(q, ops, chis, depth)


def run(q: int, depth: int, limits: Sequence[Tuple[int, int]], ncirc: int, seed: int = 0,
        full: Tuple[int, int] = (64, 64)) -> Dict:
    """Fidelity of each (chi, kappa) in `limits` against the run with the
    `full` limits (the largest the library takes; not exactly lossless: its
    own discarded weight, ~1e-7 at Q = 3 depth 4, bounds how close to 1 a
    fidelity is resolved), averaged over `ncirc` circuits; FP64 path, svd and
    inner cutoffs at 1e-14."""
    rng = W.rng_for(4500 + seed)
    chans = None
    fid = {lim: [] for lim in limits}
    for _ in range(ncirc):
        prog = circuit(q, depth, rng)
        if chans is None:
            chans = [M.Channel(prog.chis[0], 1), M.Channel(prog.chis[1], 2)]

        def dense(chi, kap):
            st = M.MPDO(q, chi_max=chi, kappa_max=kap, max_kraus=16, svd_cutoff=1e-14, kappa_cutoff=1e-14)
            M.run_program(prog, st, chans)
            r = st.to_dense()
            st.close()
            return r / np.trace(r).real

        rho = dense(*full)
        for lim in limits:
            fid[lim].append(uhlmann_fidelity(rho, dense(*lim)))
    for ch in chans or []:
        ch.close()
    return {f"chi={c},kappa={k}": {"mean": float(np.mean(v)), "std": float(np.std(v)), "min": float(np.min(v))}
            for (c, k), v in fid.items()}


def uhlmann_batch(rho: np.ndarray, sigma: np.ndarray) -> np.ndarray:
    """Eq. (23) for stacks (B, d, d) of density matrices (normalised here):
    F = (tr sqrt(sqrt(rho) sigma sqrt(rho)))^2, by two batched Hermitian
    eigendecompositions on the host.  Eigenvalues below 1e-12 of each
    matrix's largest are rounding and are set to zero (their square roots,
    ~1e-8 each, would otherwise add up in the trace of a rank-deficient
    product)."""
    rho = rho / np.trace(rho, axis1=1, axis2=2).real[:, None, None]
    sigma = sigma / np.trace(sigma, axis1=1, axis2=2).real[:, None, None]
    rho = 0.5 * (rho + np.conj(np.swapaxes(rho, 1, 2)))
    sigma = 0.5 * (sigma + np.conj(np.swapaxes(sigma, 1, 2)))
    w, v = np.linalg.eigh(rho)
    w = np.where(w > 1e-12 * w.max(axis=1, keepdims=True), w, 0.0)
    sq = (v * np.sqrt(w)[:, None, :]) @ np.conj(np.swapaxes(v, 1, 2))
    m = sq @ sigma @ sq
    m = 0.5 * (m + np.conj(np.swapaxes(m, 1, 2)))
    ev = np.linalg.eigvalsh(m)
    ev = np.where(ev > 1e-12 * ev.max(axis=1, keepdims=True), ev, 0.0)
    return np.sum(np.sqrt(ev), axis=1) ** 2


def circuits(q: int, depth: int, ncirc: int, seed: int = 0) -> List["W.Program"]:
    """The seeded circuits of one (q, depth) point of run_batched."""
    rng = W.rng_for(4500 + 100 * q + depth + 10000 * seed)
    return [circuit(q, depth, rng) for _ in range(ncirc)]


def run_batched(q: int, depth: int, limits: Sequence[Tuple[int, int]], ncirc: int = 1000, seed: int = 0,
                full: Tuple[int, int] = (64, 64), prec: int = M.C128, per_circuit: bool = False) -> Dict:
    """The Sec. IV.C study at scale: `ncirc` seeded circuits of one (q, depth)
    point, each (chi, kappa) of `limits` and the reference `full` limits run
    as one batch each; returns per limit the mean, standard deviation and
    minimum of the Uhlmann fidelity against the reference state (and every
    circuit's value with per_circuit), and the device seconds of the
    batches."""
    import time
    import torch
    progs = circuits(q, depth, ncirc, seed)
    chans = [M.Channel(progs[0].chis[0], 1), M.Channel(progs[0].chis[1], 2)]
    plan = M.BatchPlan(progs, [np.zeros((0,))] * ncirc, use_params=False)
    kw = dict(max_kraus=16, svd_cutoff=1e-14, kappa_cutoff=1e-14, prec=prec)
    t = {}

    def dense(chi, kap):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mats = M.batch_run_dense(plan, None, chans, chi_max=chi, kappa_max=kap, **kw)
        torch.cuda.synchronize()
        t[f"chi={chi},kappa={kap}"] = time.perf_counter() - t0
        return torch.stack(mats).cpu().numpy()

    rho = dense(*full)
    out = {}
    for lim in limits:
        f = uhlmann_batch(rho, dense(*lim))
        out[f"chi={lim[0]},kappa={lim[1]}"] = {"mean": float(np.mean(f)), "std": float(np.std(f)),
                                               "min": float(np.min(f))}
        if per_circuit:
            out[f"chi={lim[0]},kappa={lim[1]}"]["all"] = f.tolist()
    for ch in chans:
        ch.close()
    return {"fidelity": out, "device_seconds": t, "circuits": ncirc}


if __name__ == "__main__":
    import json
    import sys
    lims = [(2, 2), (4, 4), (8, 8), (16, 4), (16, 16)]
    res = {}
    for q in (3, 6):
        for depth in (2, 4, 6, 8, 10):
            res[f"Q={q},depth={depth}"] = run_batched(q, depth, lims, ncirc=int(sys.argv[1]) if len(sys.argv) > 1
                                                      else 1000)
            print(f"Q={q} depth={depth}", json.dumps(res[f"Q={q},depth={depth}"]["fidelity"]), flush=True)
