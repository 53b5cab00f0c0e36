"""GPU MPDO (through the C ABI) against the CPU oracle and closed forms.

Tolerances: complex128 path 1e-10 on observables; complex64 contractions
with FP64 truncation 1e-5 (the stated accuracy targets of the two paths)."""
import math

import numpy as np
import pytest

from oracle import channels as OC
from oracle import dense as OD
from oracle import mpdo as OM
from paper_2508_07610_amd import mpdo as M
from paper_2508_07610_amd import workloads as W
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu

TOL = {M.C128: 1e-10, M.C64_MIXED: 1e-5}


def _superop(kraus):
    return sum(np.kron(K, K.conj()) for K in kraus)


@pytest.mark.parametrize("which", ["dep", "ad", "1q_default", "2q_default", "rand2", "rand3"])
def test_channel_from_chi_matches_oracle(which):
    """chi -> Kraus on the GPU gives the same channel (superoperator) and the
    same Kraus count (rank of the Choi matrix) as the oracle."""
    require_gpu()
    rng = np.random.default_rng(11)
    if which == "dep":
        chi, q = W.chi_from_kraus(W.kraus_depolarizing(0.03)), 1
    elif which == "ad":
        chi, q = W.chi_from_kraus(W.kraus_amplitude_damping(0.2)), 1
    elif which == "1q_default":
        chi, q = W.chi_1q_default(), 1
    elif which == "2q_default":
        chi, q = W.chi_2q_default(), 2
    elif which == "rand2":
        ks = [rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4)) for _ in range(5)]
        S = sum(K.conj().T @ K for K in ks)
        w, v = np.linalg.eigh(S)
        ks = [K @ (v / np.sqrt(w)) @ v.conj().T for K in ks]
        chi, q = W.chi_from_kraus(ks), 2
    else:
        chi, q = W.random_cptp_near_identity_3q(rng), 3
    ch = M.Channel(chi, q)
    kg = ch.info()
    ko, _, _ = OC.kraus_from_chi(chi)
    assert len(kg) == len(ko)
    assert np.abs(_superop(kg) - _superop(ko)).max() < 1e-12
    for eps in (1e-4, 1e-3):
        ko_e, _, _ = OC.kraus_from_chi(chi, eps=eps)
        assert M.Channel(chi, q, eps=eps).nkraus == len(ko_e)


def test_channel_rejects_non_trace_preserving():
    require_gpu()
    chi = np.diag([0.5, 0.1, 0.1, 0.1]).astype(complex)
    with pytest.raises(M.MPDOError) as e:
        M.Channel(chi, 1)
    assert e.value.status == M.ENOTCPTP


def _gpu_run(prog, chis_eps=0.0, **kw):
    chans = [M.Channel(c, int(round(math.log(c.shape[0], 4))), eps=chis_eps) for c in prog.chis]
    st = M.MPDO(prog.n, **kw)
    M.run_program(prog, st, chans)
    return st


def _oracle_run(prog, chi_max, kappa_max, svd_cutoff, kappa_cutoff):
    kr = [OC.kraus_from_chi(c)[0] for c in prog.chis]
    return OM.run_program(prog, OM.MPDO(prog.n, chi_max, kappa_max, svd_cutoff, kappa_cutoff), kr)


@pytest.mark.parametrize("prec", [M.C128, M.C64_MIXED])
def test_lossless_small_circuit_equals_dense(prec):
    """n = 5, one noisy ansatz layer, no effective truncation: GPU observables
    equal the dense density matrix."""
    require_gpu()
    n = 5
    prog = W.ghz_ansatz(n, 1, W.ansatz_params(n, 1, 3))
    kr = [OC.kraus_from_chi(c)[0] for c in prog.chis]
    sim = OM.run_program_dense(prog, OD.DenseSim(n), kr)
    st = _gpu_run(prog, chi_max=64, kappa_max=32, max_kraus=16, svd_cutoff=1e-15, kappa_cutoff=1e-15, prec=prec)
    tol = TOL[prec]
    assert abs(st.trace() - 1) < tol
    for s in W.zz_strings(n) + ["XYZIX", "ZZZZZ", "IYIYI"]:
        assert abs(st.expect(s) - sim.expect_pauli(s)) < tol, s
    assert abs(st.fidelity_ghz() - sim.fidelity_pure(OD.ghz_state(n))) < tol


@pytest.mark.parametrize("n,p", [(4, 0.05), (7, 0.02)])
def test_ghz_local_depolarizing_closed_form(n, p):
    """GHZ by H + compiled CNOTs (ideal gates), then local depolarizing p:
    F = [(2-p)^n + p^n]/2^(n+1) + (1-p)^n/2 and <Z_i Z_{i+1}> = (1-p)^2."""
    require_gpu()
    dep = M.Channel(W.chi_from_kraus(W.kraus_depolarizing(p)), 1)
    st = M.MPDO(n, chi_max=16, kappa_max=8, max_kraus=4)
    st.apply_gate([0], W.H)
    for q in range(n - 1):
        for _, loc, U in W.cnot_compiled():
            st.apply_gate([q + s for s in loc], U)
    for q in range(n):
        st.apply_channel([q], dep)
    F = ((2 - p) ** n + p ** n) / 2 ** (n + 1) + (1 - p) ** n / 2
    assert abs(st.fidelity_ghz() - F) < 1e-12
    for s in W.zz_strings(n):
        assert abs(st.expect(s).real - (1 - p) ** 2) < 1e-12
    bonds, inner, disc = st.dims()
    assert max(bonds) == 2 and max(inner) <= 4 and disc < 1e-12


@pytest.mark.parametrize("prec", [M.C128, M.C64_MIXED])
@pytest.mark.parametrize("n,depth,chi,kap,tag", [(6, 3, 16, 4, 0), (8, 2, 16, 4, 1), (10, 3, 32, 8, 2)])
def test_truncated_ansatz_matches_oracle(prec, n, depth, chi, kap, tag):
    """The noisy RY/CZ ansatz with QPT channels under active chi / kappa
    truncation: the GPU follows the same algorithm as the oracle, so bond
    dimensions, inner dimensions, the discarded weight and the observables
    agree (observables to the tolerance of the precision)."""
    require_gpu()
    prog = W.ghz_ansatz(n, depth, W.ansatz_params(n, depth, tag))
    o = _oracle_run(prog, chi, kap, 1e-10, 1e-10)
    st = _gpu_run(prog, chi_max=chi, kappa_max=kap, max_kraus=16, svd_cutoff=1e-10, kappa_cutoff=1e-10, prec=prec)
    bonds, inner, disc = st.dims()
    tol = TOL[prec]
    if prec == M.C128:
        assert bonds == o.bond_dims()
        assert inner == o.inner_dims()
    assert abs(disc - o.discarded) < 1e3 * tol
    for s in W.zz_strings(n) + ["X" * n, "Y" + "Z" * (n - 1)]:
        assert abs(st.expect(s) - o.expect_pauli(s)) < tol, s
    assert abs(st.fidelity_ghz() - o.fidelity_ghz()) < tol
    if prec == M.C128:
        for b in range(n - 1):
            lam = st.bond_weights(b)
            assert np.abs(lam - o.lam[b]).max() < 1e-9


@pytest.mark.parametrize("prec", [M.C128, M.C64_MIXED])
@pytest.mark.parametrize("n,depth,chi,kap", [(10, 3, 32, 8), (8, 3, 80, 4)])
def test_right_factor_basis_routes_agree_with_oracle(prec, n, depth, chi, kap):
    """The two-site update's basis of the right factor from the
    eigendecomposition of E = F F^H and from its pivoted Cholesky
    factorisation (the default; E in LDS for 2 chi <= 128, in global memory
    up to 256): both write F = L_F Q with orthonormal rows Q, an exact change
    of basis, so either route matches the oracle's truncations and
    observables."""
    require_gpu()
    prog = W.ghz_ansatz(n, depth, W.ansatz_params(n, depth, 2))
    o = _oracle_run(prog, chi, kap, 1e-10, 1e-10)
    tol = TOL[prec]
    obs = {}
    for chol in (False, True):
        prev = M.e_cholesky(chol)
        try:
            st = _gpu_run(prog, chi_max=chi, kappa_max=kap, max_kraus=16, svd_cutoff=1e-10, kappa_cutoff=1e-10,
                          prec=prec)
            bonds, inner, disc = st.dims()
            if prec == M.C128:
                assert bonds == o.bond_dims() and inner == o.inner_dims(), chol
            vals = [st.expect(s) for s in W.zz_strings(n)] + [st.fidelity_ghz()]
            ref = [o.expect_pauli(s) for s in W.zz_strings(n)] + [o.fidelity_ghz()]
            assert np.abs(np.array(vals) - np.array(ref)).max() < tol, chol
            obs[chol] = np.array(vals)
        finally:
            M.e_cholesky(prev)
    assert np.abs(obs[True] - obs[False]).max() < tol


def test_invalid_sites_rejected():
    require_gpu()
    st = M.MPDO(4, chi_max=8, kappa_max=2, max_kraus=4)
    with pytest.raises(M.MPDOError) as e:
        st.apply_gate([1, 3], W.CZ)
    assert e.value.status == M.EINVAL
    with pytest.raises(M.MPDOError):
        st.apply_gate([3, 4], W.CZ)
    dep2 = M.Channel(W.chi_2q_default(), 2)
    with pytest.raises(M.MPDOError):
        st.apply_channel([0, 1], dep2)      # 16 Kraus operators > max_kraus = 4
