"""Error mitigation by the inverse of the noisy process, as a matrix product
operator (Sec. V of the paper: mitigation through an MPO inverse of noisy
processes) -- the oracle.

Test infrastructure only (see ``oracle/__init__``).  Plain NumPy, complex128.

Superoperators.  A channel rho -> sum_j K_j rho K_j^dagger acts on the
row-major vectorisation |rho>> (index (p, p')) as S = sum_j K_j (x) conj(K_j);
a q-qubit S acts on the pair indices (p_1 p_1', ..., p_q p_q') after the
reordering of that vector from (p_1 .. p_q, p_1' .. p_q').  Its inverse S^-1
(the map that undoes the channel; not completely positive) is the matrix
inverse.  A unitary gate U has S = U (x) conj(U), S^-1 = U^dagger (x) U^T.

Mitigation of a noisy circuit Phi = N_L U_L ... N_1 U_1 (each gate followed
by its channel, Eq. (8)) with a noise model N^_g: the output rho_out is
mapped by Phi_ideal Phi^-1 = U_L .. U_2 (N^_1^-1 U_2^-1 N^_2^-1 .. U_L^-1
N^_L^-1), i.e. the circuit is unwound gate by gate (inverse channel, then
inverse gate) back to after the first gate, and the ideal gates are replayed
forward.  With the exact model the result is the ideal state
U_L .. U_1 rho_0 U_1^dagger .. U_L^dagger.

MPO form.  rho as the chain of the paper's local density tensors (Eq. (6)):
R_i[(l l'), (p p'), (r r')] = sum_n T_i[l, p, n, r] conj(T_i[l', p', n, r']),
rho = contraction of the R_i (Eq. (7)).  A one-site superoperator acts on
(p p') of one tensor; a two-site one on the contracted pair, which is split
again by an SVD (bond kept by the discarded-weight rule).  Tr(O rho) is the
contraction of every R_i with O_i (linear in rho).
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np


def superop(kraus: Sequence[np.ndarray]) -> np.ndarray:
    """S = sum_j K_j (x) conj(K_j) on |rho>> in the pair order (p_1 p_1', ...)."""
    K = [np.asarray(k, dtype=np.complex128) for k in kraus]
    d = K[0].shape[0]
    q = int(round(np.log2(d)))
    S = sum(np.kron(k, k.conj()) for k in K)          # index (p, p'), p = (p_1..p_q)
    if q == 1:
        return S
    # reorder (p_1 .. p_q, p_1' .. p_q') -> (p_1 p_1', ..., p_q p_q') on both sides
    perm = [x for t in range(q) for x in (t, q + t)]
    S = S.reshape([2] * (4 * q))
    S = S.transpose(perm + [2 * q + x for x in perm])
    return S.reshape(4 ** q, 4 ** q)


def inverse_superop(kraus: Sequence[np.ndarray]) -> np.ndarray:
    return np.linalg.inv(superop(kraus))


def apply_superop_dense(rho: np.ndarray, S: np.ndarray, first: int, n: int) -> np.ndarray:
    """Apply a q-site superoperator (pair order) to a dense rho on sites first..first+q-1."""
    q = int(round(np.log(S.shape[0]) / np.log(4)))
    t = rho.reshape([2] * (2 * n))
    # move (p_s, p_s') pairs of the acted sites to the front, in pair order
    axes = []
    for s in range(first, first + q):
        axes += [s, n + s]
    rest = [a for a in range(2 * n) if a not in axes]
    t = t.transpose(axes + rest).reshape(4 ** q, -1)
    t = (S @ t).reshape([2] * (2 * q) + [2] * (2 * n - 2 * q))
    inv = np.argsort(axes + rest)
    return t.transpose(inv).reshape(rho.shape)


class MPO:
    """rho as local density tensors R_i[a, 4, b] (Eq. (6)), FP64, untruncated
    unless d_max / cutoff say otherwise."""

    def __init__(self, R: List[np.ndarray], d_max: int = 1 << 30, cutoff: float = 0.0):
        self.R = [np.asarray(r, dtype=np.complex128) for r in R]
        self.n = len(R)
        self.d_max = d_max
        self.cutoff = cutoff
        self.discarded = 0.0

    @staticmethod
    def from_mpdo(T: Sequence[np.ndarray], **kw) -> "MPO":
        """R[(l l'), (p p'), (r r')] = sum_n T[l, p, n, r] conj(T[l', p', n, r'])."""
        R = []
        for t in T:
            l, _, k, r = t.shape
            x = np.einsum("apnb,cqnd->acpqbd", t, t.conj())
            R.append(x.reshape(l * l, 4, r * r))
        return MPO(R, **kw)

    def apply1(self, i: int, S: np.ndarray) -> None:
        self.R[i] = np.einsum("xy,ayb->axb", S, self.R[i])

    def apply2(self, i: int, S: np.ndarray) -> None:
        A, B = self.R[i], self.R[i + 1]
        a, _, _ = A.shape
        _, _, c = B.shape
        th = np.einsum("axb,byc->axyc", A, B).reshape(a, 16, c)
        th = np.einsum("zw,awc->azc", S, th).reshape(a * 4, 4 * c)
        U, s, Vh = np.linalg.svd(th, full_matrices=False)
        w = s ** 2
        W = w.sum()
        tail = np.concatenate([np.cumsum(w[::-1])[::-1], [0.0]])
        r = next((k for k in range(1, len(w) + 1) if tail[k] <= self.cutoff * W), len(w))
        r = max(1, min(r, self.d_max))
        self.discarded += float(tail[r] / W) if W > 0 else 0.0
        self.R[i] = U[:, :r].reshape(a, 4, r)
        self.R[i + 1] = (s[:r, None] * Vh[:r]).reshape(r, 4, c)

    def apply(self, first: int, S: np.ndarray) -> None:
        if S.shape[0] == 4:
            self.apply1(first, S)
        else:
            self.apply2(first, S)

    def expect(self, ops: Sequence[np.ndarray]) -> complex:
        """Tr(O rho) for O = (x)_i ops[i]: R_i contracted with O_i^T on (p p')."""
        v = np.ones(1, dtype=np.complex128)
        for R, O in zip(self.R, ops):
            o = np.asarray(O, dtype=np.complex128).T.reshape(4)   # O[p', p] at (p p')
            v = v @ np.einsum("axb,x->ab", R, o)
        return complex(v[0])

    def to_dense(self) -> np.ndarray:
        n = self.n
        t = np.ones((1, 1), dtype=np.complex128)      # (pairs so far, bond)
        for R in self.R:
            t = np.einsum("Pa,axb->Pxb", t, R).reshape(-1, R.shape[2])
        t = t[:, 0].reshape([2] * (2 * n))            # (p_1 p_1' p_2 p_2' ...)
        perm = [2 * s for s in range(n)] + [2 * s + 1 for s in range(n)]
        return t.transpose(perm).reshape(2 ** n, 2 ** n)


def mitigation_sequence(prog, kraus_model) -> List[tuple]:
    """The superoperators that map a noisy circuit's output to the mitigated
    state (see the module docstring), in order: (first site, S).
    kraus_model[c] is the noise model's Kraus list of channel c."""
    seq = []
    ops = prog.ops
    for k in range(len(ops) - 1, -1, -1):
        op = ops[k]
        if op.chan >= 0:
            seq.append((op.sites[0], inverse_superop(kraus_model[op.chan])))
        if k > 0:
            U = op.U
            seq.append((op.sites[0], superop([U.conj().T])))
    for op in ops[1:]:
        seq.append((op.sites[0], superop([op.U])))
    return seq
