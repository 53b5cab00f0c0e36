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
device; the fidelity is a host-side measurement of the dense results
(n <= 12)."""
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
    `full` limits (large enough to be lossless at these sizes), averaged over
    `ncirc` circuits; FP64 path, svd and inner cutoffs at 1e-14."""
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
