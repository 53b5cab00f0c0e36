"""Error mitigation by the inverse of the noisy process (Sec. V), on the GPU.

The output of a noisy circuit N_L U_L .. N_1 U_1 (Eq. (8): every gate
followed by its channel) is taken as an MPO of local density tensors
(Eq. (6)) and mapped by the inverse of the process under a noise model N^
followed by the ideal circuit: N^_L^-1, U_L^-1, .., N^_2^-1, U_2^-1, N^_1^-1
(U_1^-1 and the replayed U_1 cancel), then U_2 .. U_L.  With the exact model
the result is the noiseless state; with a mismatched model (e.g. a standard
noise model in place of the process-tomography channels) the residual
measures the model's error.  Every map runs through the mpdo_mpo_* entry
points; this module only orders the calls."""
from __future__ import annotations

from typing import Sequence

import numpy as np

from . import mpdo as M


def mitigate(prog, state: "M.MPDO", model: Sequence["M.Channel"], d_max: int = 256,
             cutoff: float = 0.0) -> "M.MPO":
    """MPO of the mitigated state of `state` (the output of `prog`); model[c]
    is the noise model of the program's channel c (q <= 2)."""
    m = state.to_mpo(d_max, cutoff)
    try:
        ops = prog.ops
        for k in range(len(ops) - 1, -1, -1):
            op = ops[k]
            if op.chan >= 0:
                m.apply_channel(op.sites[0], model[op.chan], inverse=True)
            if k > 0:
                m.apply_gate(op.sites[0], op.U, inverse=True)
        for op in ops[1:]:
            m.apply_gate(op.sites[0], op.U)
    except Exception:
        m.close()
        raise
    return m


def ghz_fidelity(m: "M.MPO") -> float:
    """<GHZ| rho |GHZ> / Tr(rho) of an MPO state: (rho_00 + rho_11) / 2 +
    Re rho_01 over the all-zero and all-one strings, by three product
    operators and the identity."""
    n = m.n
    P0 = np.diag([1.0, 0.0]).astype(np.complex128)
    P1 = np.diag([0.0, 1.0]).astype(np.complex128)
    F10 = np.array([[0.0, 0.0], [1.0, 0.0]], dtype=np.complex128)   # |1><0|: Tr(|1..1><0..0| rho) = rho_(0..0),(1..1)
    ops = np.stack([np.stack([x] * n) for x in (P0, P1, F10, np.eye(2, dtype=np.complex128))])
    v = m.expect_products(ops)
    return float(np.real(0.5 * (v[0] + v[1]) + np.real(v[2])) / np.real(v[3]))


def expect_normalised(m: "M.MPO", ops: np.ndarray) -> np.ndarray:
    """Tr(O rho) / Tr(rho) for product operators ops (nops, n, 2, 2)."""
    ops = np.asarray(ops, dtype=np.complex128)
    ident = np.stack([np.eye(2, dtype=np.complex128)] * m.n)[None]
    v = m.expect_products(np.concatenate([ops, ident]))
    return v[:-1] / v[-1]
