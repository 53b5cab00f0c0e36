"""CPU matrix product density operator, complex128 -- the oracle of the MPDO path.

Test infrastructure only (see ``oracle/__init__``).  Plain NumPy: every
decomposition is a full ``numpy.linalg.svd`` / ``eigh`` / ``qr`` of the
matrix the paper names, with no blocking or reduced forms.

State (Sec. II.C, Eq. (5)).  Site i holds T_i[l, p, n, r]: left bond l,
physical p in {0, 1}, noise (inner) index n < kappa_i, right bond r.  The
density matrix is rho = sum_n |Psi_n><Psi_n| over all inner indices (Eqs.
(6)-(7)): the tensors form a purification MPS whose "physical" leg is (p, n)
and whose conjugate copy is never stored.  The chain starts in |0...0>.

Gauge.  Tensors are kept right-orthonormal (sum over p, n, r of T T^* = 1 on
the left bond) together with bond weights lambda_i on every bond (the
Schmidt values of the purification).  The environment of any site or pair of
neighbouring sites is then diag(lambda_{left}^2) on the left and the identity
on the right, which is the canonical form Sec. II.D asks for before an SVD
truncation, maintained gate by gate.  ``truncate_sweep`` performs the
paper's explicit procedure -- QR from left to right, then SVD from right to
left.  It leaves every tensor but the first right-orthonormal; each bond's
weights are its singular values when it was cut, which are the Schmidt
values of the result when nothing further left is cut (always for bond 0).

Noisy gates (Eq. (8), Fig. fig_mpdoSingle).  A gate on q adjacent sites with
ideal unitary U and channel {K_j} acts through the fused operators
G_j = K_j U.  The new noise index j is attached to the inner index of the
leftmost site (q = 1, 2) or of the middle site (q = 3).

Inner truncation (Eqs. (9)-(11)).  T ~= U Sigma V^dagger over (p, l, r) x n,
the SVD taken of T with its left bond weighted by lambda (the environment of
the site in canonical form); the new tensor is T V_kappa.  The SVD is taken
of the matrix itself, not of a Gram matrix, so weights far below the
largest are resolved.

Bond truncation (Sec. II.D, Fig. fig_svdTruncate (b)).  The two-site block is
split by an SVD of lambda_left * Theta; the right factor V^dagger becomes the
new right tensor, the singular values the new bond weights, and Theta V the
new left tensor.

Truncation rule for both kinds of index (a reading: the paper fixes no rule):
with eta the squared singular values (descending) and W their sum, keep the
smallest r >= 1 with sum_{i >= r} eta_i <= cutoff * W, capped at the maximum
dimension; then rescale so the kept weight is 1 (Tr rho = 1).  There is no
other floor: the cutoff alone decides what is numerically zero.
"""
from __future__ import annotations

import math
from typing import List, Optional, Sequence

import numpy as np


TIE_REL = 1e-9     # weights closer than this (relative) form one multiplet
TIE_FLOOR = 1e-11  # ... unless they carry less than this fraction of the total


def select_rank(eta: np.ndarray, max_dim: int, cutoff: float) -> int:
    """Smallest r >= 1 with sum_{i>=r} eta_i <= cutoff * W, capped at max_dim.
    eta (squared singular values) is in descending order; negative values
    count as zero.

    A degenerate multiplet straddling the cut is dropped as a whole (r is
    lowered until eta_{r-1} and eta_r differ), so the kept subspace -- and
    with it the truncated state -- is unique; multiplets below TIE_FLOOR of
    the total weight are left as they fall."""
    e = np.clip(np.asarray(eta, dtype=np.float64), 0.0, None)
    W = e.sum()
    if W <= 0:
        return 1
    # tail[r] = sum_{i >= r} e_i
    tail = np.concatenate([np.cumsum(e[::-1])[::-1], [0.0]])
    r = len(e)
    for cand in range(1, len(e) + 1):
        if tail[cand] <= cutoff * W:
            r = cand
            break
    r = int(max(1, min(r, max_dim)))
    r0 = r
    while 1 < r < len(e) and e[r - 1] > TIE_FLOOR * W and e[r - 1] - e[r] <= TIE_REL * e[r - 1]:
        r -= 1
    if r == 1 and len(e) > 1 and e[0] - e[1] <= TIE_REL * e[0]:
        r = r0   # the leading multiplet itself straddles the cut: keep the plain rank
    return r


def _svd(M: np.ndarray):
    """Thin SVD M = U diag(S) Vh, singular values descending.  NumPy's
    divide-and-conquer driver (gesdd) occasionally reports non-convergence on
    matrices with many tiny singular values; the same decomposition is then
    taken with the one-sided QR-iteration driver (gesvd)."""
    try:
        return np.linalg.svd(M, full_matrices=False)
    except np.linalg.LinAlgError:
        import scipy.linalg
        return scipy.linalg.svd(M, full_matrices=False, lapack_driver="gesvd")


class MPDO:
    def __init__(self, n: int, chi_max: int = 1 << 30, kappa_max: int = 1 << 30,
                 svd_cutoff: float = 1e-14, kappa_cutoff: float = 1e-14):
        self.n = n
        self.chi_max = chi_max
        self.kappa_max = kappa_max
        self.svd_cutoff = svd_cutoff
        self.kappa_cutoff = kappa_cutoff
        self.T: List[np.ndarray] = []
        for _ in range(n):
            t = np.zeros((1, 2, 1, 1), dtype=np.complex128)
            t[0, 0, 0, 0] = 1.0
            self.T.append(t)
        self.lam: List[np.ndarray] = [np.ones(1) for _ in range(n - 1)]
        self.discarded = 0.0   # summed discarded weight of all truncations
        self.cuts: List[float] = []   # discarded fraction of every bond cut, in order

    # -- helpers ----------------------------------------------------------------
    def lam_left(self, i: int) -> np.ndarray:
        return self.lam[i - 1] if i > 0 else np.ones(1)

    def bond_dims(self) -> List[int]:
        return [t.shape[3] for t in self.T[:-1]]

    def inner_dims(self) -> List[int]:
        return [t.shape[2] for t in self.T]

    # -- inner (noise) truncation, Eqs. (9)-(11) ---------------------------------
    def _compress_inner(self, Tp: np.ndarray, inner_axis: int, lam_l: np.ndarray):
        """Tp has the left bond on axis 0 and the inner index on `inner_axis`.
        Returns Tp V_kappa (the inner axis replaced by the kept directions),
        rescaled so the kept weight is 1."""
        moved = np.moveaxis(Tp, inner_axis, -1)
        shape = moved.shape
        M = (lam_l.reshape((-1,) + (1,) * (moved.ndim - 1)) * moved).reshape(-1, shape[-1])
        _, S, Vh = _svd(M)
        eta = S ** 2
        k = select_rank(eta, self.kappa_max, self.kappa_cutoff)
        W = eta.sum()
        kept = eta[:k].sum()
        out = moved.reshape(-1, shape[-1]) @ Vh[:k].conj().T
        out = out.reshape(shape[:-1] + (k,)) / math.sqrt(kept)
        self.discarded += float((W - kept) / W) if W > 0 else 0.0
        return np.moveaxis(out, -1, inner_axis)

    # -- noisy gates (Eq. (8)) -------------------------------------------------------
    def apply_1q(self, i: int, G: Sequence[np.ndarray]) -> None:
        """T'[l, s, (k j), r] = sum_t G_j[s, t] T[l, t, k, r], then inner truncation."""
        G = np.asarray(G, dtype=np.complex128).reshape(-1, 2, 2)
        T = self.T[i]
        l, _, k, r = T.shape
        m = G.shape[0]
        Tp = np.einsum("jst,ltkr->lskjr", G, T).reshape(l, 2, k * m, r)
        if m == 1:           # a unitary leaves the inner spectrum unchanged
            self.T[i] = Tp
            return
        self.T[i] = self._compress_inner(Tp, 2, self.lam_left(i))

    def apply_2q(self, i: int, G: Sequence[np.ndarray]) -> None:
        """Two-site noisy gate on (i, i+1): contract the pair, apply every G_j,
        truncate the inner index (k_i, j) of site i, split by SVD."""
        G = np.asarray(G, dtype=np.complex128).reshape(-1, 4, 4)
        A, B = self.T[i], self.T[i + 1]
        l, _, k1, _ = A.shape
        _, _, k2, r = B.shape
        m = G.shape[0]
        theta = np.einsum("lakc,cbdr->lakbdr", A, B)               # l t1 k1 t2 k2 r
        Gr = G.reshape(m, 2, 2, 2, 2)                              # j s1 s2 t1 t2
        thp = np.einsum("jxyab,lakbdr->lxkjydr", Gr, theta)
        thp = thp.reshape(l, 2, k1 * m, 2, k2, r)
        lam_l = self.lam_left(i)
        if m > 1:
            thp = self._compress_inner(thp, 2, lam_l)
        kp = thp.shape[2]
        self._split(i, thp.reshape(l * 2 * kp, 2 * k2 * r), (l, 2, kp), (2, k2, r), lam_l)

    def _split(self, i: int, theta: np.ndarray, lshape, rshape, lam_l: np.ndarray) -> None:
        """SVD of lambda_left * Theta; right factor -> T_{i+1}, Theta V -> T_i."""
        wl = np.repeat(lam_l, theta.shape[0] // lam_l.shape[0])
        U, S, Vh = _svd(wl[:, None] * theta)
        eta = S ** 2
        rr = select_rank(eta, self.chi_max, self.svd_cutoff)
        W = eta.sum()
        kept = eta[:rr].sum()
        self.discarded += float((W - kept) / W) if W > 0 else 0.0
        self.cuts.append(float((W - kept) / W) if W > 0 else 0.0)
        s = 1.0 / math.sqrt(kept)
        self.T[i + 1] = Vh[:rr].reshape((rr,) + tuple(rshape))
        self.T[i] = (theta @ Vh[:rr].conj().T).reshape(tuple(lshape) + (rr,)) * s
        self.lam[i] = S[:rr] * s

    def apply_3q(self, i: int, G: Sequence[np.ndarray]) -> None:
        """Three-site noisy gate on (i, i+1, i+2), written as contract-apply-split
        on the full three-site block: the three tensors are contracted, every
        G_j is applied to the physical indices with the new noise index j joined
        to the inner index of the middle site, that inner index is truncated
        (Eqs. (9)-(11)), and the block is split by two SVDs, first at bond i
        (left site off), then at bond i+1 with the new weights of bond i."""
        G = np.asarray(G, dtype=np.complex128).reshape(-1, 8, 8)
        A, B, C = self.T[i], self.T[i + 1], self.T[i + 2]
        l, _, k1, _ = A.shape
        _, _, k2, _ = B.shape
        _, _, k3, r = C.shape
        m = G.shape[0]
        blk = np.einsum("lakc,cbde,efgr->lakbdfgr", A, B, C)       # l t1 k1 t2 k2 t3 k3 r
        Gr = G.reshape(m, 2, 2, 2, 2, 2, 2)                        # j s1 s2 s3 t1 t2 t3
        blk = np.einsum("jxyzabf,lakbdfgr->lxkydjzgr", Gr, blk)    # l s1 k1 s2 (k2 j) s3 k3 r
        blk = blk.reshape(l, 2, k1, 2, k2 * m, 2, k3, r)
        lam_l = self.lam_left(i)
        if m > 1:
            blk = self._compress_inner(blk, 4, lam_l)
        k2p = blk.shape[4]
        # split off site i
        self._split(i, blk.reshape(l * 2 * k1, 2 * k2p * 2 * k3 * r), (l, 2, k1),
                    (2, k2p, 2, k3, r), lam_l)
        # the right factor (now T[i+1] with shape (rr, 2, k2p, 2, k3, r)) is split again
        rest = self.T[i + 1]
        rr = rest.shape[0]
        lam_m = self.lam[i]
        self._split(i + 1, rest.reshape(rr * 2 * k2p, 2 * k3 * r), (rr, 2, k2p), (2, k3, r), lam_m)

    # -- the paper's truncation sweep (Sec. II.D) ------------------------------------
    def truncate_sweep(self, chi_max: Optional[int] = None, kappa_max: Optional[int] = None,
                       cutoff: Optional[float] = None) -> float:
        """QR from left to right to canonical form (on the purification, without
        the conjugate copy), then SVD from right to left truncating every bond,
        then inner truncation of every site.  Returns the discarded weight."""
        chi_max = self.chi_max if chi_max is None else chi_max
        kappa_max = self.kappa_max if kappa_max is None else kappa_max
        cutoff = self.svd_cutoff if cutoff is None else cutoff
        before = self.discarded
        self.bond_sweep(chi_max, cutoff)
        saved = self.kappa_max
        self.kappa_max = kappa_max
        for i in range(self.n):
            T = self.T[i]
            if T.shape[2] > 1:
                self.T[i] = self._compress_inner(T, 2, self.lam_left(i))
        self.kappa_max = saved
        return self.discarded - before

    def bond_sweep(self, chi_max: int, cutoff: float) -> None:
        """The bond part of the sweep: QR left to right, then SVD right to left
        with every bond truncated by the rank rule; the state is renormalised
        once at the end, each cut's discarded fraction is logged in ``cuts``."""
        n = self.n
        for i in range(n - 1):
            T = self.T[i]
            l, _, k, r = T.shape
            Q, R = np.linalg.qr(T.reshape(l * 2 * k, r))
            self.T[i] = Q.reshape(l, 2, k, Q.shape[1])
            self.T[i + 1] = np.einsum("ab,bskr->askr", R, self.T[i + 1])
        for i in range(n - 1, 0, -1):
            T = self.T[i]
            l, _, k, r = T.shape
            U, S, Vh = np.linalg.svd(T.reshape(l, 2 * k * r), full_matrices=False)
            eta = S ** 2
            rr = select_rank(eta, chi_max, cutoff)
            W, kept = eta.sum(), eta[:rr].sum()
            self.discarded += float((W - kept) / W) if W > 0 else 0.0
            self.cuts.append(float((W - kept) / W) if W > 0 else 0.0)
            self.T[i] = Vh[:rr].reshape(rr, 2, k, r)
            self.T[i - 1] = np.einsum("lskb,bc->lskc", self.T[i - 1], U[:, :rr] * S[:rr])
            self.lam[i - 1] = S[:rr] / math.sqrt(kept)
        t0 = self.T[0]
        self.T[0] = t0 / np.linalg.norm(t0)

    # -- observables (Eqs. (6)-(7)) -------------------------------------------------
    def expect_product(self, ops: Sequence[np.ndarray]) -> complex:
        """Tr(O rho) for O = (x)_i ops[i], by the transfer matrices
        E'[r, r'] = sum E[l, l'] T[l, s, k, r] O[s', s] conj(T[l', s', k, r'])."""
        E = np.ones((1, 1), dtype=np.complex128)
        for T, O in zip(self.T, ops):
            E = np.einsum("ab,askr,ts,btkc->rc", E, T, np.asarray(O, dtype=np.complex128), T.conj())
        return complex(E[0, 0])

    def trace(self) -> float:
        return float(np.real(self.expect_product([np.eye(2)] * self.n)))

    def expect_pauli(self, s: str) -> complex:
        mats = {"I": np.eye(2), "X": np.array([[0, 1], [1, 0]]),
                "Y": np.array([[0, -1j], [1j, 0]]), "Z": np.diag([1.0, -1.0])}
        return self.expect_product([mats[c] for c in s]) / self.trace()

    def fidelity_ghz(self) -> float:
        """<GHZ| rho |GHZ> / Tr rho = (rho_00 + rho_11 + 2 Re rho_01) / 2."""
        n = self.n
        p0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
        p1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)
        up = np.array([[0, 0], [1, 0]], dtype=np.complex128)   # |1><0|
        r00 = self.expect_product([p0] * n)
        r11 = self.expect_product([p1] * n)
        r01 = self.expect_product([up] * n)                    # Tr(|1..1><0..0| rho) = rho_{0..0,1..1}
        return float(np.real(r00 + r11 + 2 * r01) / 2 / self.trace())

    def to_dense(self) -> np.ndarray:
        """Full rho = sum_n |Psi_n><Psi_n| (Eq. (7)); n <= 10."""
        if self.n > 10:
            raise ValueError("to_dense is for n <= 10")
        psi = np.ones((1, 1, 1), dtype=np.complex128)      # (phys, anc, bond)
        for T in self.T:
            psi = np.einsum("pab,bskr->psakr", psi, T)
            P, _, A, K, R = psi.shape
            psi = psi.reshape(P * 2, A * K, R)
        psi = psi[:, :, 0]
        return psi @ psi.conj().T


def run_program(prog, mpdo: MPDO, kraus_of_chan) -> MPDO:
    """Apply a workloads.Program to an oracle MPDO.  kraus_of_chan[c] is the
    Kraus list of channel c (from ``oracle.channels.kraus_from_chi``)."""
    for op in prog.ops:
        U = op.U
        if op.chan >= 0:
            G = [K @ U for K in kraus_of_chan[op.chan]]
        else:
            G = [U]
        q = len(op.sites)
        if q == 1:
            mpdo.apply_1q(op.sites[0], G)
        elif q == 2:
            mpdo.apply_2q(op.sites[0], G)
        else:
            mpdo.apply_3q(op.sites[0], G)
    return mpdo


def run_program_dense(prog, sim, kraus_of_chan):
    for op in prog.ops:
        if op.chan >= 0:
            G = [K @ op.U for K in kraus_of_chan[op.chan]]
        else:
            G = [op.U]
        sim.apply_kraus(op.sites, G)
    return sim
