"""chi-matrix -> Kraus operators, written from Sec. III of the paper.

Test infrastructure only (see ``oracle/__init__``).

Steps, in the paper's order and notation:

1. The process matrix chi is given in an operator basis {sigma_m}
   (Eq. (12)): eps(rho) = sum_mn chi_mn sigma_m rho sigma_n^dagger.  Here the
   basis is the unnormalised Pauli products, order I, X, Y, Z, site 0 most
   significant (a reading: the paper does not fix the normalisation or order).
2. Change of basis to the "Choi" matrix Lambda = sum_mn chi_mn
   |sigma_m>><<sigma_n| (Eqs. (13)-(14)), with |A>> the row-major
   vectorisation of A.
3. Eigendecomposition Lambda = sum_i eta_i |psi_i><psi_i| (Eq. (15)),
   eigenvalues in descending order.
4. K_i = sqrt(eta_i) A_i with |A_i>> = |psi_i> (Eq. (16)); the number of
   Kraus operators is the rank of Lambda.  Negative eigenvalues (a map that
   is not completely positive) are clipped to zero.
5. Pruning "by descending eigenvalue magnitude" (Sec. III): operators whose
   weight w_i = eta_i / sum_j eta_j is below eps are dropped; the remaining
   set is not renormalised.
"""
from __future__ import annotations

import numpy as np


def _pauli_basis(q):
    paulis = [np.eye(2, dtype=np.complex128),
              np.array([[0, 1], [1, 0]], dtype=np.complex128),
              np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
              np.array([[1, 0], [0, -1]], dtype=np.complex128)]
    basis = [np.ones((1, 1), dtype=np.complex128)]
    for _ in range(q):
        basis = [np.kron(b, p) for b in basis for p in paulis]
    return basis


def choi_from_chi(chi: np.ndarray) -> np.ndarray:
    """Lambda = sum_mn chi_mn |sigma_m>><<sigma_n|  (Eqs. (13)-(14))."""
    chi = np.asarray(chi, dtype=np.complex128)
    d2 = chi.shape[0]
    q = int(round(np.log2(d2) / 2))
    vecs = np.array([s.reshape(-1) for s in _pauli_basis(q)])  # row m = |sigma_m>>
    lam = np.zeros((d2, d2), dtype=np.complex128)
    for m in range(d2):
        for n in range(d2):
            lam += chi[m, n] * np.outer(vecs[m], vecs[n].conj())
    return lam


def kraus_from_chi(chi: np.ndarray, eps: float = 0.0, rank_tol: float = 1e-13):
    """Kraus operators K_i = sqrt(eta_i) unvec(psi_i) of the channel chi.

    Returns (kraus list [d x d], eigenvalues eta in descending order (before
    clipping), weights of the kept operators).  Eigenvalues at or below
    rank_tol * max(eta) count as zero (rank of Lambda, Eq. (16))."""
    lam = choi_from_chi(chi)
    lam = (lam + lam.conj().T) / 2
    eta, psi = np.linalg.eigh(lam)
    order = np.argsort(-eta, kind="stable")
    eta, psi = eta[order], psi[:, order]
    d = int(round(np.sqrt(lam.shape[0])))
    pos = np.clip(eta, 0.0, None)
    total = pos.sum()
    kraus, weights = [], []
    for i in range(len(eta)):
        if pos[i] <= rank_tol * pos[0]:
            continue
        w = pos[i] / total
        if w < eps:
            continue
        kraus.append(np.sqrt(pos[i]) * psi[:, i].reshape(d, d))
        weights.append(w)
    return kraus, eta, np.array(weights)


def apply_channel_dense(kraus, rho):
    """eps(rho) = sum_i K_i rho K_i^dagger  (Eq. (1))."""
    return sum(K @ rho @ K.conj().T for K in kraus)


def apply_chi_dense(chi, rho):
    """eps(rho) = sum_mn chi_mn sigma_m rho sigma_n^dagger evaluated literally
    (Eq. (12)); used to pin the Kraus conversion."""
    d2 = chi.shape[0]
    q = int(round(np.log2(d2) / 2))
    basis = _pauli_basis(q)
    out = np.zeros_like(rho, dtype=np.complex128)
    for m in range(d2):
        for n in range(d2):
            if chi[m, n] != 0:
                out += chi[m, n] * basis[m] @ rho @ basis[n].conj().T
    return out


def completeness_error(kraus) -> float:
    """|| sum_i K_i^dagger K_i - I ||_max."""
    d = kraus[0].shape[0]
    s = sum(K.conj().T @ K for K in kraus)
    return float(np.abs(s - np.eye(d)).max())
