"""Pins of the chi -> Kraus conversion (Sec. III, Eqs. (12)-(16)) against
closed forms and the defining equation, independent of the conversion code."""
import math

import numpy as np
import pytest

from oracle import channels, dense
from paper_2508_07610_amd import workloads as W


def _rand_rho(d, rng):
    a = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    r = a @ a.conj().T
    return r / np.trace(r)


def _rand_kraus(d, m, rng):
    As = [rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d)) for _ in range(m)]
    S = sum(A.conj().T @ A for A in As)
    w, v = np.linalg.eigh(S)
    Sih = (v / np.sqrt(w)) @ v.conj().T
    return [A @ Sih for A in As]


@pytest.mark.parametrize("p", [0.0, 1e-3, 0.03, 0.5, 1.0])
def test_depolarizing_chi_gives_eq3(p):
    """Eq. (3): chi = diag(1-3p/4, p/4, p/4, p/4); the Kraus set must act as
    (1-p) rho + p I/2 and be complete."""
    chi = np.diag([1 - 3 * p / 4, p / 4, p / 4, p / 4]).astype(complex)
    ks, eta, _ = channels.kraus_from_chi(chi)
    assert channels.completeness_error(ks) < 1e-14
    rng = np.random.default_rng(1)
    rho = _rand_rho(2, rng)
    want = (1 - p) * rho + p * np.eye(2) / 2
    assert np.abs(channels.apply_channel_dense(ks, rho) - want).max() < 1e-14
    # Choi eigenvalues in the unnormalised Pauli basis are 2 * (1-3p/4, p/4, p/4, p/4)
    want_eta = sorted([2 * (1 - 3 * p / 4)] + [2 * p / 4] * 3, reverse=True)
    assert np.allclose(np.sort(eta)[::-1], want_eta, atol=1e-14)
    # number of Kraus operators = rank of the Choi matrix (Eq. (16))
    assert len(ks) == (1 if p == 0 else 4)


@pytest.mark.parametrize("q,m", [(1, 3), (2, 5), (3, 4)])
def test_kraus_reproduces_eq12(q, m):
    """The Kraus set must reproduce eps(rho) = sum chi_mn sigma_m rho sigma_n^dag
    evaluated term by term, for a random CPTP map (chi built from random Kraus)."""
    rng = np.random.default_rng(10 + q)
    d = 2 ** q
    chi = W.chi_from_kraus(_rand_kraus(d, m, rng))
    ks, _, _ = channels.kraus_from_chi(chi)
    assert len(ks) == m
    assert channels.completeness_error(ks) < 1e-12
    rho = _rand_rho(d, rng)
    assert np.abs(channels.apply_channel_dense(ks, rho) - channels.apply_chi_dense(chi, rho)).max() < 1e-12


def test_identity_and_unitary_chi():
    """Identity chi = e0 e0^T leaves rho unchanged with one Kraus operator;
    a rank-one chi = v v^dag with U = sum v_m sigma_m gives exactly U (up to phase)."""
    chi = np.zeros((4, 4), complex)
    chi[0, 0] = 1
    ks, _, _ = channels.kraus_from_chi(chi)
    assert len(ks) == 1
    rng = np.random.default_rng(3)
    rho = _rand_rho(2, rng)
    assert np.abs(channels.apply_channel_dense(ks, rho) - rho).max() < 1e-15
    U = W.rx(0.7) @ W.rz(1.3)
    ks, _, _ = channels.kraus_from_chi(W.chi_from_kraus([U]))
    assert len(ks) == 1
    K = ks[0]
    phase = np.vdot(K.reshape(-1), U.reshape(-1))
    phase /= abs(phase)
    assert np.abs(K * phase - U).max() < 1e-14


def test_amplitude_damping_population():
    """P(1) = (1-gamma)^k after k applications of amplitude damping to |1>."""
    g = 0.07
    ks, _, _ = channels.kraus_from_chi(W.chi_from_kraus(W.kraus_amplitude_damping(g)))
    rho = np.diag([0.0, 1.0]).astype(complex)
    for k in range(1, 6):
        rho = channels.apply_channel_dense(ks, rho)
        assert abs(rho[1, 1].real - (1 - g) ** k) < 1e-14


def test_pruning_weights():
    """Pruning keeps operators in descending weight order with w_i = eta_i / sum eta."""
    chi = W.chi_2q_default()
    ks0, eta, w0 = channels.kraus_from_chi(chi, eps=0.0)
    assert len(ks0) == 16
    assert abs(w0.sum() - 1) < 1e-12
    assert np.all(np.diff(w0) <= 1e-15)
    ks1, _, w1 = channels.kraus_from_chi(chi, eps=1e-3)
    assert len(ks1) == int(np.sum(w0 >= 1e-3))


def test_uhlmann_and_jsd_special_cases():
    rng = np.random.default_rng(5)
    rho = _rand_rho(4, rng)
    assert abs(dense.uhlmann_fidelity(rho, rho) - 1) < 1e-10
    a = rng.normal(size=4) + 1j * rng.normal(size=4)
    b = rng.normal(size=4) + 1j * rng.normal(size=4)
    a /= np.linalg.norm(a)
    b /= np.linalg.norm(b)
    f = dense.uhlmann_fidelity(np.outer(a, a.conj()), np.outer(b, b.conj()))
    # sqrt of a rank-one matrix through eigh carries ~sqrt(eps) error
    assert abs(f - abs(np.vdot(a, b)) ** 2) < 1e-7
    p = np.array([0.1, 0.2, 0.3, 0.4])
    q = np.array([0.4, 0.3, 0.2, 0.1])
    f = dense.uhlmann_fidelity(np.diag(p).astype(complex), np.diag(q).astype(complex))
    assert abs(f - np.sum(np.sqrt(p * q)) ** 2) < 1e-12
    assert dense.jsd(p, p) == 0.0
    assert abs(dense.jsd(np.array([1.0, 0.0]), np.array([0.0, 1.0])) - math.log(2)) < 1e-15
