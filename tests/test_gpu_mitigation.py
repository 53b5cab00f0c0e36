"""Error mitigation by the inverse of the noisy process (Sec. V) on the GPU,
through the mpdo_mpo_* entry points, against oracle/mitigation.py and the
closed forms it is pinned to.

Tolerance.  The two-site maps split the contracted pair through the Gram
matrix of one side (FP64), which resolves singular values down to about
sqrt(eps_64) ~ 1.5e-8 of the largest; rho is linear in the MPO tensors, so a
lossless split agrees with the oracle's SVD to that level relative to the
largest entry of rho.  TOL = 1e-8 (relative) is that bound."""
import math

import numpy as np
import pytest

from oracle import channels as OC
from oracle import dense as OD
from oracle import mitigation as MI
from oracle import mpdo as OM
from paper_2508_07610_amd import mitigation as GM
from paper_2508_07610_amd import mpdo as M
from paper_2508_07610_amd import workloads as W
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu

TOL = 1e-8
LOSSLESS = dict(chi_max=64, kappa_max=64, max_kraus=16, svd_cutoff=1e-14, kappa_cutoff=1e-14)


def _channels(prog):
    return [M.Channel(c, int(round(math.log(c.shape[0], 4)))) for c in prog.chis]


def _ghz_noisy(n, scale):
    chis = [W.chi_1q_default(scale), W.chi_2q_default(scale)]
    ops = [W.Op((0,), W.H, 0, "h")]
    for q in range(n - 1):
        for name, loc, U in W.cnot_compiled():
            ops.append(W.Op(tuple(q + s for s in loc), U, 0 if len(loc) == 1 else 1, name))
    return W.Program(n, ops, chis, 0)


def _gpu_state(prog, chans, prec=M.C128, **kw):
    """The program on the GPU; LOSSLESS limits by default (exact for the
    GHZ circuits here; a cap of 64 can still cut deeper circuits)."""
    st = M.MPDO(prog.n, prec=prec, **(kw or LOSSLESS))
    M.run_program(prog, st, chans)
    return st


@pytest.mark.parametrize("prec", [M.C128, M.C64_MIXED])
def test_mpo_of_the_state_is_its_density_matrix(prec):
    """R_i = sum_n B_i conj(B_i) (Eq. (6)) contracted along the chain (Eq. (7))
    equals the state's rho: its dense form on the GPU, and the oracle's
    truncated MPDO at the same limits (chi = 64, kappa = 16, cutoffs 1e-10)."""
    require_gpu()
    n = 5
    kw = dict(chi_max=64, kappa_max=16, max_kraus=16, svd_cutoff=1e-10, kappa_cutoff=1e-10)
    prog = W.ghz_ansatz(n, 2, W.ansatz_params(n, 2, 3))
    chans = _channels(prog)
    st = _gpu_state(prog, chans, prec, **kw)
    with st.to_mpo() as m:
        rho_m = m.to_dense()
    rho_s = st.to_dense()
    kr = [OC.kraus_from_chi(c)[0] for c in prog.chis]
    rho_o = OM.run_program(prog, OM.MPDO(n, 64, 16, 1e-10, 1e-10), kr).to_dense()
    err_s = np.abs(rho_m - rho_s).max()
    err_o = np.abs(rho_m - rho_o).max()
    print(f"prec {prec}: |MPO - state| = {err_s:.2e}, |MPO - oracle| = {err_o:.2e}")
    assert err_s < 1e-13
    assert err_o < (1e-10 if prec == M.C128 else 1e-5)
    st.close()
    for c in chans:
        c.close()


def test_maps_equal_dense_superoperators():
    """Gates, channels and their inverses on one and two sites (the two-site
    ones split again, lossless) equal the oracle's superoperators applied to
    the dense rho."""
    require_gpu()
    n = 4
    rng = np.random.default_rng(11)
    prog = W.ghz_ansatz(n, 1, W.ansatz_params(n, 1, 6))
    chans = _channels(prog)
    st = _gpu_state(prog, chans)
    kr = [OC.kraus_from_chi(c)[0] for c in prog.chis]
    rho = OM.run_program_dense(prog, OD.DenseSim(n), kr).rho
    m = st.to_mpo()
    model = [M.Channel(W.chi_standard_1q(3e-3, 0.03, 30.0, 20.0), 1),
             M.Channel(W.chi_unified_2q(3e-2, 0.3, 30.0, 20.0), 2)]
    mk = [OC.kraus_from_chi(W.chi_standard_1q(3e-3, 0.03, 30.0, 20.0))[0],
          OC.kraus_from_chi(W.chi_unified_2q(3e-2, 0.3, 30.0, 20.0))[0]]
    steps = [("gate", 1, 0, False), ("gate", 2, 1, False), ("chan", 1, 2, True), ("chan", 2, 0, True),
             ("gate", 2, 2, True), ("chan", 1, 3, False), ("chan", 2, 1, False), ("gate", 1, 3, True)]
    for kind, q, site, inv in steps:
        if kind == "gate":
            a = rng.normal(size=(2 ** q, 2 ** q)) + 1j * rng.normal(size=(2 ** q, 2 ** q))
            U = np.linalg.qr(a)[0]
            m.apply_gate(site, U, inverse=inv)
            S = MI.superop([U.conj().T if inv else U])
        else:
            m.apply_channel(site, model[q - 1], inverse=inv)
            S = MI.inverse_superop(mk[q - 1]) if inv else MI.superop(mk[q - 1])
        rho = MI.apply_superop_dense(rho, S, site, n)
        err = np.abs(m.to_dense() - rho).max()
        print(f"{kind} q={q} site={site} inverse={inv}: max |GPU - oracle| = {err:.2e}")
        assert err < TOL * np.abs(rho).max()
    ops = np.stack([np.stack([W.Z, W.X, np.eye(2), W.Y]).astype(np.complex128)])
    want = np.trace(np.kron(np.kron(np.kron(W.Z, W.X), np.eye(2)), W.Y) @ rho)
    got = m.expect_products(ops)[0]
    assert abs(got - want) < TOL * max(1.0, abs(want))
    m.close()
    st.close()
    for c in chans + model:
        c.close()


@pytest.mark.parametrize("n", [3, 5, 8])
def test_exact_model_mitigation_recovers_the_ghz_state(n):
    """With the circuit's own channels as the model, unwinding the noisy GHZ
    circuit and replaying the ideal gates gives the pure GHZ state: fidelity
    1 and <Z_i Z_i+1> = 1 (closed forms), from a noisy fidelity below 0.95."""
    require_gpu()
    prog = _ghz_noisy(n, 3.0)
    chans = _channels(prog)
    st = _gpu_state(prog, chans)
    f_noisy = st.fidelity_ghz()
    with GM.mitigate(prog, st, chans) as m:
        f = GM.ghz_fidelity(m)
        zz = GM.expect_normalised(m, np.stack([W.pauli_ops(s) for s in W.zz_strings(n)]))
        bonds, disc = m.dims()
    print(f"n={n}: noisy F = {f_noisy:.6f}, mitigated F = {f:.12f}, max |ZZ - 1| = "
          f"{np.abs(zz - 1).max():.2e}, bonds {bonds}, discarded {disc:.1e}")
    assert f_noisy < 0.95
    assert abs(f - 1) < TOL
    assert np.abs(zz - 1).max() < TOL
    st.close()
    for c in chans:
        c.close()


def test_mismatched_model_matches_the_oracle():
    """A standard noise model in place of the circuit's channels: the GPU's
    mitigated rho equals the oracle's (dense superoperators, lossless), keeps
    trace 1 and is not the ideal state."""
    require_gpu()
    n = 4
    prog = _ghz_noisy(n, 3.0)
    chans = _channels(prog)
    c1, c2 = W.chi_standard_1q(3e-3, 0.03, 30.0, 20.0), W.chi_unified_2q(3e-2, 0.3, 30.0, 20.0)
    model = [M.Channel(c1, 1), M.Channel(c2, 2)]
    st = _gpu_state(prog, chans)
    with GM.mitigate(prog, st, model) as m:
        got = m.to_dense()
    kr = [OC.kraus_from_chi(c)[0] for c in prog.chis]
    rho = OM.run_program_dense(prog, OD.DenseSim(n), kr).rho
    for first, S in MI.mitigation_sequence(prog, [OC.kraus_from_chi(c1)[0], OC.kraus_from_chi(c2)[0]]):
        rho = MI.apply_superop_dense(rho, S, first, n)
    err = np.abs(got - rho).max()
    g = OD.ghz_state(n)
    print(f"mismatched model: max |GPU - oracle| = {err:.2e}, F = {np.real(g.conj() @ got @ g):.6f}")
    assert err < TOL * np.abs(rho).max()
    assert abs(np.trace(got) - 1) < TOL
    assert np.abs(got - np.outer(g, g.conj())).max() > 1e-3
    st.close()
    for c in chans + model:
        c.close()


@pytest.mark.parametrize("d_max,cutoff", [(10, 0.0), (20, 0.0), (256, 1e-6), (256, 1e-3)])
def test_truncated_mitigation_matches_the_oracle_mpo(d_max, cutoff):
    """With bond limits that cut, the GPU's splits keep what the oracle's SVD
    keeps: the same bonds, summed discarded weight and observables (random
    circuit with the default channels, mismatched standard model, n = 6).

    A split of a non-canonical MPO is not an optimal truncation of the whole
    state, and a cap that lands in a cluster of singular values makes the
    result depend on rounding: here d_max = 12 moves the oracle's own
    observables by 1e-3 under a 1e-13 perturbation of its input.  The limits
    below are ones where the oracle's result is stable under such a
    perturbation (spread <= 4e-11)."""
    require_gpu()
    n = 6
    prog = W.random_circuit(n, 3, W.rng_for(77), chi2=W.chi_2q_default(2.0))
    chans = _channels(prog)
    c2 = W.chi_unified_2q(3e-2, 0.3, 30.0, 20.0)
    model = [M.Channel(c2, 2)]
    st = _gpu_state(prog, chans)
    kr = [OC.kraus_from_chi(c)[0] for c in prog.chis]
    om = OM.run_program(prog, OM.MPDO(n, 64, 64, 1e-14, 1e-14), kr)
    ref = MI.MPO.from_mpdo(om.T, d_max=d_max, cutoff=cutoff)
    for first, S in MI.mitigation_sequence(prog, [OC.kraus_from_chi(c2)[0]]):
        ref.apply(first, S)
    obs = np.stack([W.pauli_ops(s) for s in W.zz_strings(n)] + [W.pauli_ops("X" * n), W.pauli_ops("I" * n)])
    want = np.array([ref.expect(o) for o in obs])
    with GM.mitigate(prog, st, model, d_max=d_max, cutoff=cutoff) as m:
        got = m.expect_products(obs)
        bonds, disc = m.dims()
    err = np.abs(got - want).max()
    print(f"d_max={d_max} cutoff={cutoff}: bonds {bonds} vs {[r.shape[2] for r in ref.R[:-1]]}, "
          f"discarded {disc:.3e} vs {ref.discarded:.3e}, max |GPU - oracle| = {err:.2e}")
    assert ref.discarded > 1e-9
    assert bonds == [r.shape[2] for r in ref.R[:-1]]
    assert abs(disc - ref.discarded) < 1e-7 * max(1.0, ref.discarded)
    assert err < 1e-7 * max(1.0, np.abs(want).max())
    st.close()
    for c in chans + model:
        c.close()


def test_mpo_argument_and_error_paths():
    """Rejected arguments leave the MPO usable; the inverse of the fully
    depolarizing channel (a singular superoperator) is ENOTCONV; three-site
    channels are EUNSUPPORTED."""
    require_gpu()
    n = 3
    prog = _ghz_noisy(n, 1.0)
    chans = _channels(prog)
    st = _gpu_state(prog, chans)
    for dm, cut in [(0, 0.0), (257, 0.0), (8, 1.0), (8, -1.0)]:
        with pytest.raises(M.MPDOError) as e:
            st.to_mpo(dm, cut)
        assert e.value.status == M.EINVAL
    m = st.to_mpo()
    with pytest.raises(M.MPDOError) as e:
        m.apply_gate(2, np.eye(4))
    assert e.value.status == M.EINVAL
    with pytest.raises(M.MPDOError) as e:
        m.apply_gate(0, np.eye(8))
    assert e.value.status == M.EINVAL
    c3 = M.Channel(W.chi_from_kraus([np.eye(8, dtype=np.complex128)]), 3)
    with pytest.raises(M.MPDOError) as e:
        m.apply_channel(0, c3)
    assert e.value.status == M.EUNSUPPORTED
    f_before = GM.ghz_fidelity(m)
    full = M.Channel(W.chi_from_kraus(W.kraus_depolarizing(1.0)), 1)
    m.apply_channel(1, full)                     # forward: allowed
    with pytest.raises(M.MPDOError) as e:
        m.apply_channel(1, full, inverse=True)   # no inverse
    assert e.value.status == M.ENOTCONV
    assert 0.4 < f_before <= 1.0 + 1e-12
    m.close()
    st.close()
    for c in chans + [c3, full]:
        c.close()
