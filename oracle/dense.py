"""Dense density-matrix simulator (n <= 12), complex128.

Test infrastructure only (see ``oracle/__init__``).  This is the plain
definition the MPDO approximates: rho is a 2^n x 2^n matrix, a noisy gate on
adjacent sites applies rho -> sum_i K_i rho K_i^dagger (Eq. (1)) with K_i the
fused noisy operator N_i K~ (Eq. (8)) embedded on those sites, and
observables are traces.  Qubit 0 is the most significant bit of the dense
index (the |p_0 ... p_{N-1}> ordering of Eq. (7)).
"""
from __future__ import annotations

import numpy as np


class DenseSim:
    def __init__(self, n: int):
        if n > 12:
            raise ValueError("dense oracle is limited to n <= 12")
        self.n = n
        self.rho = np.zeros((2 ** n, 2 ** n), dtype=np.complex128)
        self.rho[0, 0] = 1.0

    # -- channels -------------------------------------------------------------
    def _embed_apply(self, K: np.ndarray, first: int, rho: np.ndarray) -> np.ndarray:
        """K rho for K acting on sites first..first+q-1 (row index only)."""
        n = self.n
        q = int(round(np.log2(K.shape[0])))
        a, b = 2 ** first, 2 ** (n - first - q)
        r = rho.reshape(a, 2 ** q, b, -1)
        return np.einsum("st,atbc->asbc", K, r).reshape(rho.shape)

    def apply_kraus(self, sites, kraus) -> None:
        sites = tuple(sites)
        if list(sites) != list(range(sites[0], sites[0] + len(sites))):
            raise ValueError("sites must be ascending and adjacent")
        out = np.zeros_like(self.rho)
        for K in kraus:
            t = self._embed_apply(K, sites[0], self.rho)          # K rho
            t = self._embed_apply(K.conj(), sites[0], t.T).T      # (K rho) K^dagger
            out += t
        self.rho = out

    def apply_unitary(self, sites, U) -> None:
        self.apply_kraus(sites, [U])

    # -- observables ----------------------------------------------------------
    def trace(self) -> complex:
        return complex(np.trace(self.rho))

    def expect_pauli(self, s: str) -> complex:
        P = pauli_matrix(s)
        return complex(np.trace(P @ self.rho) / np.trace(self.rho))

    def fidelity_pure(self, psi: np.ndarray) -> float:
        psi = np.asarray(psi, dtype=np.complex128)
        return float(np.real(psi.conj() @ self.rho @ psi) / np.real(np.trace(self.rho)))

    def purity(self) -> float:
        r = self.rho / np.trace(self.rho)
        return float(np.real(np.trace(r @ r)))


def pauli_matrix(s: str) -> np.ndarray:
    mats = {"I": np.eye(2), "X": np.array([[0, 1], [1, 0]]),
            "Y": np.array([[0, -1j], [1j, 0]]), "Z": np.diag([1, -1])}
    out = np.ones((1, 1), dtype=np.complex128)
    for c in s:
        out = np.kron(out, np.asarray(mats[c], dtype=np.complex128))
    return out


def ghz_state(n: int) -> np.ndarray:
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[0] = psi[-1] = 1 / np.sqrt(2)
    return psi


def _psd_sqrt(a: np.ndarray) -> np.ndarray:
    a = (a + a.conj().T) / 2
    w, v = np.linalg.eigh(a)
    return (v * np.sqrt(np.clip(w, 0.0, None))) @ v.conj().T


def uhlmann_fidelity(rho: np.ndarray, sigma: np.ndarray) -> float:
    """F(rho, sigma) = (tr sqrt(sqrt(rho) sigma sqrt(rho)))^2  (Eq. (23)),
    both arguments normalised to unit trace first."""
    rho = rho / np.trace(rho)
    sigma = sigma / np.trace(sigma)
    s = _psd_sqrt(rho)
    m = s @ sigma @ s
    m = (m + m.conj().T) / 2
    w = np.clip(np.linalg.eigvalsh(m), 0.0, None)
    return float(np.sum(np.sqrt(w)) ** 2)


def jsd(p: np.ndarray, q: np.ndarray) -> float:
    """Jensen-Shannon divergence (Eq. (18)), natural log, 0 ln 0 = 0."""
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    m = (p + q) / 2

    def kl(a, b):
        mask = a > 0
        return float(np.sum(a[mask] * np.log(a[mask] / b[mask])))

    return 0.5 * (kl(p, m) + kl(q, m))
