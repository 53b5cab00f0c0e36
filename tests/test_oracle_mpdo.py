"""Pins of the CPU MPDO oracle against the dense simulator, closed forms and
invariants (Secs. II.C-II.D, Eqs. (1), (5)-(11), (19)-(22))."""
import copy
import math

import numpy as np
import pytest

from oracle import channels, dense, mpdo
from paper_2508_07610_amd import workloads as W


def _kraus(prog):
    return [channels.kraus_from_chi(c)[0] for c in prog.chis]


def _lossless(n):
    return mpdo.MPDO(n, 1 << 20, 1 << 20, 1e-15, 1e-15)


def _ghz_prep_ops(n):
    """H on qubit 0, then CNOT(q, q+1) compiled as RY(-pi/2)_t CZ RY(pi/2)_t."""
    ops = [((0,), W.H)]
    for q in range(n - 1):
        for name, loc, U in W.cnot_compiled():
            ops.append((tuple(q + s for s in loc), U))
    return ops


def _apply(sim_or_mpdo, sites, G):
    if isinstance(sim_or_mpdo, dense.DenseSim):
        sim_or_mpdo.apply_kraus(sites, G)
    elif len(sites) == 1:
        sim_or_mpdo.apply_1q(sites[0], G)
    else:
        sim_or_mpdo.apply_2q(sites[0], G)


def test_untruncated_mpdo_equals_dense():
    """Noisy RY/CZ ansatz with QPT-style channels, n = 5, one layer: the
    lossless MPDO reproduces the dense rho entrywise."""
    n = 5
    prog = W.ghz_ansatz(n, 1, W.ansatz_params(n, 1, 3))
    kr = _kraus(prog)
    m = mpdo.run_program(prog, _lossless(n), kr)
    sim = mpdo.run_program_dense(prog, dense.DenseSim(n), kr)
    rho = m.to_dense()
    assert abs(np.trace(rho) - 1) < 1e-12
    assert np.abs(rho - sim.rho).max() < 1e-12
    assert np.abs(rho - rho.conj().T).max() < 1e-14            # Hermitian
    assert np.linalg.eigvalsh(rho).min() > -1e-13              # positive (Eq. (6) form)
    for s in W.zz_strings(n) + ["XYZIX", "ZZZZZ"]:
        assert abs(m.expect_pauli(s) - sim.expect_pauli(s)) < 1e-12
    assert abs(m.fidelity_ghz() - sim.fidelity_pure(dense.ghz_state(n))) < 1e-12


@pytest.mark.parametrize("n,p", [(3, 0.05), (5, 0.02), (6, 0.1)])
def test_ghz_local_depolarizing_closed_form(n, p):
    """GHZ_n then local depolarizing p on every qubit:
    F = [(2-p)^n + p^n]/2^(n+1) + (1-p)^n/2,
    purity = [(1+q)^n + (1-q)^n]/2^(n+1) + q^n/2 with q = (1-p)^2,
    <Z_i Z_j> = (1-p)^2."""
    dep = channels.kraus_from_chi(W.chi_from_kraus(W.kraus_depolarizing(p)))[0]
    sim, m = dense.DenseSim(n), _lossless(n)
    for sites, U in _ghz_prep_ops(n):
        _apply(sim, sites, [U])
        _apply(m, sites, [U])
    for qb in range(n):
        _apply(sim, (qb,), dep)
        _apply(m, (qb,), dep)
    F = ((2 - p) ** n + p ** n) / 2 ** (n + 1) + (1 - p) ** n / 2
    q = (1 - p) ** 2
    pur = ((1 + q) ** n + (1 - q) ** n) / 2 ** (n + 1) + q ** n / 2
    assert abs(sim.fidelity_pure(dense.ghz_state(n)) - F) < 1e-14
    assert abs(sim.purity() - pur) < 1e-14
    assert abs(m.fidelity_ghz() - F) < 1e-13
    for s in W.zz_strings(n):
        assert abs(m.expect_pauli(s).real - (1 - p) ** 2) < 1e-13
        assert abs(sim.expect_pauli(s).real - (1 - p) ** 2) < 1e-14
    # the inner index of every site holds at most the 4 Kraus branches
    assert max(m.inner_dims()) <= 4


def test_amplitude_damping_on_mpdo():
    """<Z> = 1 - 2 (1-gamma)^k after X and k amplitude-damping channels."""
    g = 0.05
    ad = channels.kraus_from_chi(W.chi_from_kraus(W.kraus_amplitude_damping(g)))[0]
    m = _lossless(3)
    m.apply_1q(1, [W.X])
    for k in range(1, 5):
        m.apply_1q(1, ad)
        assert abs(m.expect_pauli("IZI").real - (1 - 2 * (1 - g) ** k)) < 1e-13


def _qaoa_p1(edges, n, gamma, beta):
    """Closed form of <C_uv> for p = 1 MaxCut QAOA (Wang, Hadfield, Jiang,
    Rieffel, PRA 97, 022304): 1/2 + 1/4 sin4b sing (cos^(du-1) g + cos^(dv-1) g)
    - 1/4 sin^2(2b) cos^(du+dv-2-2l) g (1 - cos^l 2g), l = triangles on (u,v)."""
    adj = {i: set() for i in range(n)}
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    out = {}
    for u, v in edges:
        du, dv = len(adj[u]) , len(adj[v])
        lam = len(adj[u] & adj[v])
        g, b = gamma, beta
        c = (0.5 + 0.25 * math.sin(4 * b) * math.sin(g) * (math.cos(g) ** (du - 1) + math.cos(g) ** (dv - 1))
             - 0.25 * math.sin(2 * b) ** 2 * math.cos(g) ** (du + dv - 2 - 2 * lam) * (1 - math.cos(2 * g) ** lam))
        out[(u, v)] = c
    return out


@pytest.mark.parametrize("n,seed", [(6, 0), (8, 1)])
def test_qaoa_p1_closed_form(n, seed):
    """Noiseless QAOA p = 1 through the SWAP network on a random 3-regular graph:
    <C_uv> = (1 - <Z_u Z_v>)/2 (Eq. (20)) matches the closed form for every edge."""
    rng = W.rng_for(100 + seed)
    edges = W.random_3_regular(n, rng)
    gamma, beta = 0.63, 0.27
    prog, pos = W.qaoa_swap_network(n, edges, [gamma], [beta], noisy=False)
    m = mpdo.run_program(prog, _lossless(n), [])
    where = {lq: s for s, lq in enumerate(pos)}
    want = _qaoa_p1(edges, n, gamma, beta)
    for (u, v), c in want.items():
        s = W.pauli_string(n, {where[u]: "Z", where[v]: "Z"})
        got = 0.5 * (1 - m.expect_pauli(s).real)
        assert abs(got - c) < 1e-12, (u, v, got, c)
    # gamma = beta = 0 gives <C> = |E|/2
    prog0, pos0 = W.qaoa_swap_network(n, edges, [0.0], [0.0], noisy=False)
    m0 = mpdo.run_program(prog0, _lossless(n), [])
    w0 = {lq: s for s, lq in enumerate(pos0)}
    tot = sum(0.5 * (1 - m0.expect_pauli(W.pauli_string(n, {w0[u]: "Z", w0[v]: "Z"})).real) for u, v in edges)
    assert abs(tot - len(edges) / 2) < 1e-12


def _purification(m):
    psi = np.ones((1, 1), dtype=np.complex128)
    for T in m.T:
        psi = np.einsum("ab,bpkr->apkr", psi, T).reshape(-1, T.shape[3])
    return psi[:, 0]


def test_bond_truncation_eckart_young():
    """Eq. (10): truncating one bond of a state in canonical form to rank r
    changes the purification by exactly the discarded weight
    (||Psi - sqrt(kept) Psi_r||^2 = 1 - kept)."""
    n = 4
    prog = W.ghz_ansatz(n, 1, W.ansatz_params(n, 1, 9))
    kr = _kraus(prog)
    m0 = mpdo.run_program(prog, _lossless(n), kr)
    U = W.CZ @ np.kron(W.ry(0.4), W.rx(1.1))
    m1 = copy.deepcopy(m0)
    m1.apply_2q(1, [U])
    full = m1.lam[1].shape[0]
    assert full >= 3
    m2 = copy.deepcopy(m0)
    m2.chi_max = full - 2
    m2.apply_2q(1, [U])
    s = m1.lam[1]
    kept = float(np.sum(s[: full - 2] ** 2) / np.sum(s ** 2))
    psi1, psi2 = _purification(m1), _purification(m2)
    assert abs(np.vdot(psi1, psi1) - 1) < 1e-12
    err = np.linalg.norm(psi1 - math.sqrt(kept) * psi2) ** 2
    assert abs(err - (1 - kept)) < 1e-12
    assert abs(m2.discarded - (1 - kept)) < 1e-12


def test_truncate_sweep_lossless_and_canonical():
    """The QR / SVD sweep at no truncation leaves rho unchanged and produces
    right-orthonormal tensors whose bond weights are the Schmidt values."""
    n = 5
    prog = W.ghz_ansatz(n, 1, W.ansatz_params(n, 1, 4))
    kr = _kraus(prog)
    m = mpdo.run_program(prog, _lossless(n), kr)
    before = m.to_dense()
    d = m.truncate_sweep()
    assert d < 1e-14
    assert np.abs(m.to_dense() - before).max() < 1e-12
    for i in range(1, n):
        T = m.T[i]
        M = T.reshape(T.shape[0], -1)
        assert np.abs(M @ M.conj().T - np.eye(T.shape[0])).max() < 1e-12
    psi = _purification(m)
    # Schmidt values of the purification across bond 1|2 are lambda_1
    left = 2 * m.T[0].shape[2] * 2 * m.T[1].shape[2]
    sv = np.linalg.svd(psi.reshape(left, -1), compute_uv=False)
    r = m.lam[1].shape[0]
    assert np.abs(sv[:r] - m.lam[1]).max() < 1e-12
    assert abs(np.sum(m.lam[1] ** 2) - 1) < 1e-12


def test_rank_selection_rule():
    eta = np.array([0.5, 0.3, 0.15, 0.04, 0.01])
    assert mpdo.select_rank(eta, 10, 0.0) == 5
    assert mpdo.select_rank(eta, 10, 0.01) == 4
    assert mpdo.select_rank(eta, 10, 0.05) == 3
    assert mpdo.select_rank(eta, 2, 0.0) == 2
    assert mpdo.select_rank(np.array([1.0, -1e-18]), 5, 1e-14) == 1
    # a multiplet straddling the cut is dropped whole
    e = np.array([5.0, 3.0, 2.0, 2.0, 2.0, 1.0])
    assert mpdo.select_rank(e, 3, 0.0) == 2
    assert mpdo.select_rank(e, 5, 0.0) == 5
    assert mpdo.select_rank(np.array([1.0, 1.0, 1.0]), 2, 0.0) == 2   # leading multiplet: plain rank


def test_degenerate_cut_result_is_unique(monkeypatch):
    """With the multiplet rule the truncated state does not depend on which
    basis of a degenerate singular subspace the SVD returns: rotating every
    degenerate block (U_blk Q, Q^H Vh_blk: the same matrix) by a random
    unitary leaves the result unchanged."""
    n, depth, chi, kap, tag = 6, 2, 16, 4, 0
    prog = W.ghz_ansatz(n, depth, W.ansatz_params(n, depth, tag))
    kr = _kraus(prog)
    ref = mpdo.run_program(prog, mpdo.MPDO(n, chi, kap, 1e-10, 1e-10), kr)
    rng = np.random.default_rng(0)
    plain = mpdo._svd
    hits = [0]

    def scrambled(M):
        U, S, Vh = plain(M)
        U, Vh = U.copy(), Vh.copy()
        i = 0
        while i < len(S):
            j = i + 1
            while j < len(S) and abs(S[j] ** 2 - S[i] ** 2) <= 1e-12 * S[0] ** 2:
                j += 1
            if j - i > 1 and S[i] ** 2 > 1e-10 * S[0] ** 2:
                hits[0] += 1
                g = rng.normal(size=(j - i, j - i)) + 1j * rng.normal(size=(j - i, j - i))
                q, _ = np.linalg.qr(g)
                U[:, i:j] = U[:, i:j] @ q
                Vh[i:j] = q.conj().T @ Vh[i:j]
            i = j
        return U, S, Vh

    monkeypatch.setattr(mpdo, "_svd", scrambled)
    alt = mpdo.run_program(prog, mpdo.MPDO(n, chi, kap, 1e-10, 1e-10), kr)
    assert hits[0] > 0
    assert alt.bond_dims() == ref.bond_dims()
    assert alt.inner_dims() == ref.inner_dims()
    for s in W.zz_strings(n):
        assert abs(alt.expect_pauli(s) - ref.expect_pauli(s)) < 1e-12
    assert abs(alt.fidelity_ghz() - ref.fidelity_ghz()) < 1e-12


def _normalised(rho):
    return rho / np.trace(rho)


def _crosstalk_prog(n, depth, tag, n3=2):
    rng = W.rng_for(900 + tag)
    chi3 = [W.random_cptp_near_identity_3q(rng) for _ in range(n3)]
    return W.random_circuit(n, depth, W.rng_for(950 + tag), chi2=W.chi_2q_default(), chi3=chi3)


def _kraus_eps(prog, eps3):
    qs = [int(round(math.log(c.shape[0], 4))) for c in prog.chis]
    return [channels.kraus_from_chi(c, eps3 if q == 3 else 0.0)[0] for c, q in zip(prog.chis, qs)]


def _random_tp_3q(rng, m):
    """m Ginibre operators on three qubits made trace preserving,
    K_i = A_i S^(-1/2) with S = sum A_i^H A_i, as a Pauli chi-matrix."""
    As = [rng.normal(size=(8, 8)) + 1j * rng.normal(size=(8, 8)) for _ in range(m)]
    S = sum(A.conj().T @ A for A in As)
    w, v = np.linalg.eigh(S)
    return W.chi_from_kraus([A @ (v / np.sqrt(w)) @ v.conj().T for A in As])


@pytest.mark.parametrize("n,depth,tag,m3", [(4, 1, 0, 64), (3, 2, 1, 64), (4, 1, 2, 6)])
def test_lossless_three_site_channels_equal_dense(n, depth, tag, m3):
    """Random circuits with 2q channels and trace-preserving 3-site channels
    (the near-identity crosstalk maps with 64 Kraus operators, or strongly
    mixing maps with 6) on neighbouring triples: the lossless MPDO (apply_3q:
    contract, apply, two SVD splits) reproduces the dense rho entrywise."""
    if m3 == 64:
        prog = _crosstalk_prog(n, depth, tag)
    else:
        rng = W.rng_for(970 + tag)
        prog = W.random_circuit(n, depth, rng, chi2=W.chi_2q_default(),
                                chi3=[_random_tp_3q(rng, m3) for _ in range(2)])
    kr = _kraus_eps(prog, 0.0)
    assert len(kr[1]) == m3 and len(kr[2]) == m3
    m = mpdo.run_program(prog, _lossless(n), kr)
    sim = mpdo.run_program_dense(prog, dense.DenseSim(n), kr)
    assert abs(np.trace(sim.rho) - 1) < 1e-12                  # trace preserving
    assert np.abs(m.to_dense() - sim.rho).max() < 1e-12
    for s in W.zz_strings(n) + ["X" * n, "Y" + "Z" * (n - 1)]:
        assert abs(m.expect_pauli(s) - sim.expect_pauli(s)) < 1e-12


def test_lossless_unitary_three_site_gate_equals_dense():
    n = 5
    rng = np.random.default_rng(9)
    U, _ = np.linalg.qr(rng.normal(size=(8, 8)) + 1j * rng.normal(size=(8, 8)))
    prog = W.ghz_ansatz(n, 1, W.ansatz_params(n, 1, 5))
    prog.ops.append(W.Op((1, 2, 3), U, -1, "u3"))
    prog.ops.append(W.Op((0, 1, 2), U.conj().T, -1, "u3"))
    kr = _kraus(prog)
    m = mpdo.run_program(prog, _lossless(n), kr)
    sim = mpdo.run_program_dense(prog, dense.DenseSim(n), kr)
    assert np.abs(m.to_dense() - sim.rho).max() < 1e-12


@pytest.mark.parametrize("eps", [1e-4, 1e-3])
def test_lossless_pruned_three_site_channels_equal_dense(eps):
    """Kraus sets pruned by weight (Sec. III) are no longer trace preserving;
    the lossless MPDO still reproduces the dense rho once both are
    normalised (Tr rho is rescaled at every truncation, reading R14)."""
    n = 4
    prog = _crosstalk_prog(n, 2, 3, n3=1)
    kr = _kraus_eps(prog, eps)
    assert len(kr[1]) < 64
    m = mpdo.run_program(prog, _lossless(n), kr)
    sim = mpdo.run_program_dense(prog, dense.DenseSim(n), kr)
    assert abs(np.trace(sim.rho) - 1) > 1e-8                  # not trace preserving
    assert np.abs(_normalised(m.to_dense()) - _normalised(sim.rho)).max() < 1e-12


def _purification_vec(m):
    psi = np.ones((1, 1), dtype=np.complex128)
    for T in m.T:
        psi = np.einsum("ab,bpkr->apkr", psi, T).reshape(-1, T.shape[3])
    return psi[:, 0]


def _site_leg_sizes(m):
    return [2 * T.shape[2] for T in m.T]


def test_sweep_single_cut_is_the_best_rank_r_approximation():
    """Eq. (10): when the sweep cuts one bond only, its result (before
    renormalisation) is the best rank-r approximation of the purification
    across that bond: equal entrywise to U_r S_r V_r^H of the purification's
    SVD, at the distance sqrt(sum of the dropped squared singular values)."""
    n = 5
    prog = W.ghz_ansatz(n, 1, W.ansatz_params(n, 1, 12))
    m = mpdo.run_program(prog, _lossless(n), _kraus(prog))
    for a in (0.3, 1.1):                     # widen bond 2 only (to 16)
        m.apply_2q(2, [W.CZ @ np.kron(W.ry(a), W.rx(2 * a))])
    dims = m.bond_dims()
    b = int(np.argmax(dims))
    r = dims[b] - 5
    assert r >= 2 and sorted(dims)[-2] <= r        # only bond b exceeds r
    psi = _purification_vec(m)
    legs = _site_leg_sizes(m)
    left = int(np.prod(legs[: b + 1]))
    U, S, Vh = np.linalg.svd(psi.reshape(left, -1), full_matrices=False)
    best = (U[:, :r] * S[:r]) @ Vh[:r]
    m.cuts = []
    m.bond_sweep(r, 0.0)
    kept = 1 - sum(m.cuts)
    assert sum(1 for c in m.cuts if c > 0) == 1
    got = math.sqrt(kept) * _purification_vec(m)
    assert np.abs(got.reshape(left, -1) - best).max() < 1e-12
    assert abs(np.linalg.norm(psi - got) ** 2 - float(np.sum(S[r:] ** 2))) < 1e-12
    assert abs((1 - kept) - float(np.sum(S[r:] ** 2))) < 1e-12


def test_sweep_several_cuts_discard_the_product_of_kept_weights():
    """With every bond cut, the sweep is a product of nested projections
    (each keeps a subspace of the right part that the next one refines), so
    the unnormalised result is an orthogonal projection of Psi:
    ||Psi - sqrt(K) Psi_hat||^2 = 1 - K and <Psi|Psi_hat> = sqrt(K), with
    K the product of the kept fractions of the cuts."""
    n = 6
    prog = W.ghz_ansatz(n, 2, W.ansatz_params(n, 2, 13))
    m = mpdo.run_program(prog, mpdo.MPDO(n, 16, 2, 1e-12, 1e-12), _kraus(prog))
    psi = _purification_vec(m)
    psi /= np.linalg.norm(psi)          # inner truncations leave Tr rho near 1 only
    m.cuts = []
    m.bond_sweep(3, 0.0)
    assert sum(1 for c in m.cuts if c > 1e-6) >= 3
    K = float(np.prod([1 - c for c in m.cuts]))
    hat = _purification_vec(m)
    assert abs(np.linalg.norm(hat) - 1) < 1e-12
    assert abs(np.linalg.norm(psi - math.sqrt(K) * hat) ** 2 - (1 - K)) < 1e-12
    assert abs(np.vdot(hat, psi) - math.sqrt(K)) < 1e-12
    assert max(m.bond_dims()) <= 3
    # every bond's weights are its singular values at the moment of its cut,
    # renormalised; bond 0 is cut last, so its weights are the Schmidt values
    # of the result
    for b in range(n - 1):
        assert abs(float(np.sum(m.lam[b] ** 2)) - 1) < 1e-12
    sv = np.linalg.svd(hat.reshape(_site_leg_sizes(m)[0], -1), compute_uv=False)
    r = m.lam[0].shape[0]
    assert np.abs(sv[:r] - m.lam[0]).max() < 1e-12 and sv[r:].sum() < 1e-12
    for i in range(1, n):
        T = m.T[i].reshape(m.T[i].shape[0], -1)
        assert np.abs(T @ T.conj().T - np.eye(T.shape[0])).max() < 1e-12


def test_inner_truncation_eckart_young():
    """Eqs. (9)-(11): keeping kappa inner directions of one site changes the
    purification by exactly the discarded weight: the projected tensor
    T V_k V_k^H gives ||Psi - Psi_k||^2 = 1 - kept, and the oracle's new
    tensor is sqrt(kept)^-1 T V_k."""
    n = 4
    prog = W.ghz_ansatz(n, 1, W.ansatz_params(n, 1, 14))
    m = mpdo.run_program(prog, _lossless(n), _kraus(prog))
    site = int(np.argmax(m.inner_dims()))
    T = m.T[site]
    k = T.shape[2] - 2
    assert k >= 1
    psi = _purification_vec(m)
    lam = m.lam_left(site)
    Mw = (lam[:, None, None, None] * T).transpose(0, 1, 3, 2).reshape(-1, T.shape[2])
    _, S, Vh = np.linalg.svd(Mw, full_matrices=False)
    P = Vh[:k].conj().T @ Vh[:k]
    proj = copy.deepcopy(m)
    proj.T[site] = np.einsum("lskr,kq->lsqr", T, P)
    tail = float(np.sum(S[k:] ** 2) / np.sum(S ** 2))
    assert abs(np.linalg.norm(psi - _purification_vec(proj)) ** 2 - tail) < 1e-12
    m2 = copy.deepcopy(m)
    m2.kappa_max = k
    m2.discarded = 0.0
    m2.T[site] = m2._compress_inner(T, 2, lam)
    assert abs(m2.discarded - tail) < 1e-12
    assert np.abs(m2.to_dense() - proj.to_dense() / (1 - tail)).max() < 1e-12


def test_svd_fallback_driver_gives_the_same_decomposition(monkeypatch):
    """When NumPy's gesdd driver reports non-convergence the oracle takes the
    same thin SVD with gesvd: U diag(S) Vh reconstructs M, S descending,
    U and Vh orthonormal, S equal to the singular values of M."""
    rng = np.random.default_rng(9)
    M_ = rng.normal(size=(12, 7)) + 1j * rng.normal(size=(12, 7))
    want = np.linalg.svd(M_, compute_uv=False)
    orig = np.linalg.svd

    def failing(a, full_matrices=True, compute_uv=True, **kw):
        raise np.linalg.LinAlgError("SVD did not converge")

    monkeypatch.setattr(np.linalg, "svd", failing)
    U, S, Vh = mpdo._svd(M_)
    monkeypatch.setattr(np.linalg, "svd", orig)
    assert np.abs(U @ np.diag(S) @ Vh - M_).max() < 1e-13
    assert np.all(np.diff(S) <= 0)
    assert np.abs(U.conj().T @ U - np.eye(7)).max() < 1e-13
    assert np.abs(Vh @ Vh.conj().T - np.eye(7)).max() < 1e-13
    assert np.abs(S - want).max() < 1e-13
