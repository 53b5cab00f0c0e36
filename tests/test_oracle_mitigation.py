"""Pins of the mitigation oracle (Sec. V: error mitigation through an MPO
inverse of the noisy process) against the dense simulator and closed forms."""
import math

import numpy as np
import pytest

from oracle import channels as OC
from oracle import dense as OD
from oracle import mitigation as MI
from oracle import mpdo as OM
from paper_2508_07610_amd import workloads as W


def _kraus(prog):
    return [OC.kraus_from_chi(c)[0] for c in prog.chis]


def _rand_rho(d, rng):
    a = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    r = a @ a.conj().T
    return r / np.trace(r)


@pytest.mark.parametrize("which", ["1q", "2q"])
def test_superoperator_is_the_channel(which):
    """S = sum K (x) conj(K) in pair order applied to a dense rho equals the
    channel's Kraus form (Eq. (1)) on random states and sites."""
    rng = np.random.default_rng(3)
    n = 4
    kr = OC.kraus_from_chi(W.chi_1q_default(3.0) if which == "1q" else W.chi_2q_default(3.0))[0]
    for first in range(n - (0 if which == "1q" else 1)):
        rho = _rand_rho(2 ** n, rng)
        got = MI.apply_superop_dense(rho, MI.superop(kr), first, n)
        sim = OD.DenseSim(n)
        sim.rho = rho.copy()
        sim.apply_kraus(tuple(range(first, first + (1 if which == "1q" else 2))), kr)
        assert np.abs(got - sim.rho).max() < 1e-14


@pytest.mark.parametrize("q,p", [(1, 0.03), (2, 0.05)])
def test_inverse_depolarizing_closed_form(q, p):
    """The inverse of D(rho) = (1-p) rho + p Tr(rho) I / d (Eq. (3)) is
    rho -> (rho - p Tr(rho) I / d) / (1 - p)."""
    rng = np.random.default_rng(4)
    d = 2 ** q
    kr = W.kraus_depolarizing(p) if q == 1 else W.kraus_depolarizing2(p)
    rho = _rand_rho(d, rng)
    got = MI.apply_superop_dense(rho, MI.inverse_superop(kr), 0, q)
    want = (rho - p * np.trace(rho) * np.eye(d) / d) / (1 - p)
    assert np.abs(got - want).max() < 1e-13


def _ghz_noisy(n, scale):
    """H and compiled CNOTs with the QPT-style channels after every gate."""
    chis = [W.chi_1q_default(scale), W.chi_2q_default(scale)]
    ops = [W.Op((0,), W.H, 0, "h")]
    for q in range(n - 1):
        for name, loc, U in W.cnot_compiled():
            ops.append(W.Op(tuple(q + s for s in loc), U, 0 if len(loc) == 1 else 1, name))
    return W.Program(n, ops, chis, 0)


@pytest.mark.parametrize("n", [3, 5])
def test_mitigation_with_the_exact_model_recovers_the_ideal_state(n):
    """Unwinding the noisy GHZ circuit with the exact channels' inverses and
    replaying the ideal gates gives the pure GHZ state: fidelity 1,
    <Z_i Z_i+1> = 1 (closed forms), while the noisy state is below."""
    prog = _ghz_noisy(n, 3.0)
    kr = _kraus(prog)
    sim = OM.run_program_dense(prog, OD.DenseSim(n), kr)
    f_noisy = sim.fidelity_pure(OD.ghz_state(n))
    assert f_noisy < 0.95
    rho = sim.rho
    for first, S in MI.mitigation_sequence(prog, kr):
        rho = MI.apply_superop_dense(rho, S, first, n)
    g = OD.ghz_state(n)
    assert abs(np.real(g.conj() @ rho @ g) - 1) < 1e-12
    assert abs(np.trace(rho) - 1) < 1e-12
    for s in W.zz_strings(n):
        assert abs(np.trace(OD.pauli_matrix(s) @ rho) - 1) < 1e-12


def test_mpo_of_the_mpdo_is_its_density_matrix():
    """R_i = sum_n T_i conj(T_i) (Eq. (6)) contracted along the chain (Eq. (7))
    is the MPDO's rho; superoperators applied to the MPO (two-site ones with
    an SVD split, lossless) equal their dense application."""
    n = 4
    prog = W.ghz_ansatz(n, 1, W.ansatz_params(n, 1, 6))
    kr = _kraus(prog)
    m = OM.run_program(prog, OM.MPDO(n, 1 << 20, 1 << 20, 1e-15, 1e-15), kr)
    mpo = MI.MPO.from_mpdo(m.T)
    rho = m.to_dense()
    assert np.abs(mpo.to_dense() - rho).max() < 1e-14
    rng = np.random.default_rng(5)
    for first, q in [(1, 2), (0, 1), (2, 2), (3, 1), (0, 2)]:
        X = rng.normal(size=(4 ** q, 4 ** q)) + 1j * rng.normal(size=(4 ** q, 4 ** q))
        mpo.apply(first, X)
        rho = MI.apply_superop_dense(rho, X, first, n)
    assert np.abs(mpo.to_dense() - rho).max() < 1e-11 * max(1.0, np.abs(rho).max())
    ops = [np.diag([1.0, -1.0]), np.array([[0, 1], [1, 0]]), np.eye(2), np.array([[0, -1j], [1j, 0]])]
    want = np.trace(np.kron(np.kron(np.kron(ops[0], ops[1]), ops[2]), ops[3]) @ rho)
    assert abs(mpo.expect(ops) - want) < 1e-10 * max(1.0, abs(want))


def test_mitigation_with_a_mismatched_model_is_not_exact():
    """With the standard (unified) noise model in place of the QPT-style
    channels the inverse maps are still trace preserving (Tr rho stays 1)
    but the result is not the ideal state: the residual measures the model's
    error; an inverse of the wrong channel can over-correct, so the mitigated
    matrix need not be positive."""
    n = 4
    prog = _ghz_noisy(n, 3.0)
    kr = _kraus(prog)
    sim = OM.run_program_dense(prog, OD.DenseSim(n), kr)
    model = [OC.kraus_from_chi(W.chi_standard_1q(3e-3, 0.03, 30.0, 20.0))[0],
             OC.kraus_from_chi(W.chi_unified_2q(3e-2, 0.3, 30.0, 20.0))[0]]
    rho = sim.rho
    for first, S in MI.mitigation_sequence(prog, model):
        rho = MI.apply_superop_dense(rho, S, first, n)
    g = OD.ghz_state(n)
    ideal = np.outer(g, g.conj())
    assert abs(np.trace(rho) - 1) < 1e-12
    assert np.abs(rho - ideal).max() > 1e-3
    assert np.abs(rho - sim.rho).max() > 1e-3
