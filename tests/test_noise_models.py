"""The standard noise models of the circuit model (thermal relaxation,
depolarizing on the target only, read-out flips; Sec. II.B, Fig.
`fig_unifiedNoise`), generated as Pauli chi-matrices, against the physics
they must reproduce (closed forms on the dense oracle)."""
import math

import numpy as np
import pytest

from oracle import channels, dense
from paper_2508_07610_amd import distributions as D
from paper_2508_07610_amd import workloads as W


def _dense_after(n, rho0, sites, chi):
    sim = dense.DenseSim(n)
    sim.rho = rho0.astype(np.complex128)
    sim.apply_kraus(sites, channels.kraus_from_chi(chi)[0])
    return sim.rho


@pytest.mark.parametrize("t,T1,T2", [(0.05, 1.0, 0.7), (0.3, 2.0, 4.0), (1.0, 0.5, 0.2)])
def test_thermal_relaxation_closed_forms(t, T1, T2):
    """P(1) of |1> decays as exp(-t/T1), the coherence of |+> as exp(-t/T2);
    the Kraus set is trace preserving."""
    ks = W.kraus_thermal_relaxation(t, T1, T2)
    assert np.allclose(sum(k.conj().T @ k for k in ks), np.eye(2), atol=1e-15)
    chi = W.chi_from_kraus(ks)
    one = np.diag([0.0, 1.0])
    assert abs(_dense_after(1, one, (0,), chi)[1, 1].real - math.exp(-t / T1)) < 1e-14
    plus = np.full((2, 2), 0.5)
    assert abs(abs(_dense_after(1, plus, (0,), chi)[0, 1]) - 0.5 * math.exp(-t / T2)) < 1e-14


def test_thermal_relaxation_rejects_t2_above_2t1():
    with pytest.raises(ValueError):
        W.kraus_thermal_relaxation(0.1, 1.0, 2.5)


def test_unified_model_depolarizes_the_target_only():
    """On |11>: <Z_control> = 1 - 2 exp(-t/T1) (relaxation only) and
    <Z_target> = (1 - p)(1 - 2 exp(-t/T1)); swapping the target swaps them.
    The general model depolarizes both."""
    p, t, T1, T2 = 0.03, 0.2, 1.0, 1.2
    rho = np.zeros((4, 4)); rho[3, 3] = 1.0
    zc = np.kron(W.Z, np.eye(2)); zt = np.kron(np.eye(2), W.Z)
    r = 1 - 2 * math.exp(-t / T1)
    out = _dense_after(2, rho, (0, 1), W.chi_unified_2q(p, t, T1, T2, target=1))
    assert abs(np.trace(zc @ out).real - r) < 1e-14
    assert abs(np.trace(zt @ out).real - (1 - p) * r) < 1e-14
    out = _dense_after(2, rho, (0, 1), W.chi_unified_2q(p, t, T1, T2, target=0))
    assert abs(np.trace(zc @ out).real - (1 - p) * r) < 1e-14
    assert abs(np.trace(zt @ out).real - r) < 1e-14
    out = _dense_after(2, rho, (0, 1), W.chi_ideal_noisy_2q(p, t, T1, T2))
    assert abs(np.trace(zc @ out).real - (1 - p) * r) < 1e-14
    assert abs(np.trace(zt @ out).real - (1 - p) * r) < 1e-14


def _superop(ks):
    return sum(np.kron(k, k.conj()) for k in ks)


def test_standard_1q_is_relaxation_then_depolarizing():
    """chi_standard_1q is thermal relaxation followed by depolarizing: on |1>,
    <Z> = (1 - p)(1 - 2 exp(-t/T1)); its superoperator through the oracle's
    chi -> Kraus route equals that of the composed Kraus set."""
    p, t, T1, T2 = 0.02, 0.1, 1.0, 0.8
    chi = W.chi_standard_1q(p, t, T1, T2)
    out = _dense_after(1, np.diag([0.0, 1.0]), (0,), chi)
    assert abs((out[0, 0] - out[1, 1]).real - (1 - p) * (1 - 2 * math.exp(-t / T1))) < 1e-14
    ref = _superop(W.compose(W.kraus_thermal_relaxation(t, T1, T2), W.kraus_depolarizing(p)))
    got = _superop(channels.kraus_from_chi(chi)[0])
    assert np.abs(ref - got).max() < 1e-14


def test_measurement_flip_against_brute_force():
    """Independent read-out flips: the Kronecker product of the 2 x 2 flip
    matrices applied to the distribution (qubit 0 = most significant bit)."""
    rng = np.random.default_rng(9)
    n, pm = 3, 0.07
    P = rng.random(1 << n); P /= P.sum()
    F = np.array([[1 - pm, pm], [pm, 1 - pm]])
    ref = np.kron(np.kron(F, F), F) @ P
    assert np.abs(D.measurement_flip(P, n, pm) - ref).max() < 1e-15
    # one qubit, |0>: P(1) = pm
    assert np.allclose(D.measurement_flip(np.array([1.0, 0.0]), 1, pm), [1 - pm, pm])
