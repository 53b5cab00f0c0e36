"""Three-site noisy gates (crosstalk channels on neighbouring triples) on the
GPU against the oracle MPDO: observables, bond and inner dimensions, bond
weights and discarded weight; a unitary three-site gate; Kraus pruning by
weight against the oracle's counts; batched runs.  The cases include
kappa_max chi_max = 512 (the bond Grams at 4 chi) and a middle inner index of
16 x 64 Kraus operators (a Gamma eigenproblem of size 1024)."""
import math

import numpy as np
import pytest

from oracle import channels as OC
from oracle import mpdo as OM
from paper_2508_07610_amd import mpdo as M
from paper_2508_07610_amd import workloads as W
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu

TOL = {M.C128: 1e-10, M.C64_MIXED: 1e-5}


def _run_both(prog, chi, kap, eps, prec, max_kraus):
    """eps prunes the Kraus sets of the three-site channels only."""
    qs = [int(round(math.log(c.shape[0], 4))) for c in prog.chis]
    kr = [OC.kraus_from_chi(c, eps if q == 3 else 0.0)[0] for c, q in zip(prog.chis, qs)]
    o = OM.run_program(prog, OM.MPDO(prog.n, chi, kap, 1e-10, 1e-10), kr)
    chans = [M.Channel(c, q, eps=eps if q == 3 else 0.0) for c, q in zip(prog.chis, qs)]
    st = M.MPDO(prog.n, chi_max=chi, kappa_max=kap, max_kraus=max_kraus, svd_cutoff=1e-10, kappa_cutoff=1e-10,
                prec=prec)
    M.run_program(prog, st, chans)
    return o, st


@pytest.mark.parametrize("prec", [M.C128, M.C64_MIXED])
@pytest.mark.parametrize("n,depth,chi,kap,eps,tag", [(6, 2, 16, 4, 1e-4, 1), (5, 2, 8, 4, 0.0, 2),
                                                      (7, 3, 16, 8, 1e-3, 3), (5, 2, 64, 8, 1e-4, 4),
                                                      (4, 2, 16, 16, 0.0, 5), (6, 4, 64, 8, 1e-4, 6)])
def test_crosstalk_circuit_matches_oracle(prec, n, depth, chi, kap, eps, tag):
    require_gpu()
    rng = W.rng_for(400 + tag)
    chi3 = [W.random_cptp_near_identity_3q(rng) for _ in range(2)]
    prog = W.random_circuit(n, depth, rng, chi2=W.chi_2q_default(), chi3=chi3)
    o, st = _run_both(prog, chi, kap, eps, prec, max_kraus=64)
    tol = TOL[prec]
    bonds, inner, disc = st.dims()
    if prec == M.C128:
        assert bonds == o.bond_dims()
        assert inner == o.inner_dims()
        for b in range(n - 1):
            assert np.abs(st.bond_weights(b) - o.lam[b]).max() < 1e-9, b
    assert abs(disc - o.discarded) < 1e3 * tol
    for s in W.zz_strings(n) + ["X" * n, "Y" + "Z" * (n - 1), "Z" * n]:
        assert abs(st.expect(s) - o.expect_pauli(s)) < tol, s


def test_unitary_three_site_gate():
    require_gpu()
    n = 5
    rng = np.random.default_rng(9)
    X = rng.normal(size=(8, 8)) + 1j * rng.normal(size=(8, 8))
    U, _ = np.linalg.qr(X)
    prog = W.ghz_ansatz(n, 1, W.ansatz_params(n, 1, 5))
    prog.ops.append(W.Op((1, 2, 3), U, -1, "u3"))
    prog.ops.append(W.Op((0, 1, 2), U.conj().T, -1, "u3"))
    o, st = _run_both(prog, 16, 8, 0.0, M.C128, max_kraus=16)
    for s in W.zz_strings(n) + ["X" * n, "Y" + "X" * (n - 1)]:
        assert abs(st.expect(s) - o.expect_pauli(s)) < 1e-10, s
    assert st.dims()[0] == o.bond_dims()


@pytest.mark.parametrize("eps", [0.0, 1e-4, 1e-3])
def test_kraus_pruning_counts(eps):
    require_gpu()
    chi = W.random_cptp_near_identity_3q(W.rng_for(77))
    ch = M.Channel(chi, 3, eps=eps)
    ko = OC.kraus_from_chi(chi, eps)[0]
    assert ch.nkraus == len(ko)


@pytest.mark.parametrize("prec", [M.C128, M.C64_MIXED])
def test_batch_run_with_crosstalk(prec):
    """Crosstalk circuits of different sizes in one batched run (graph and
    launch by launch) against the oracle, instance by instance."""
    require_gpu()
    rng = W.rng_for(500)
    chi3 = [W.random_cptp_near_identity_3q(rng) for _ in range(2)]
    chis = [W.chi_2q_default()] + chi3
    progs = [W.random_circuit(n, 2, W.rng_for(510 + n), chi2=chis[0], chi3=chi3) for n in (5, 7, 6)]
    obs = []
    for pr in progs:
        n = pr.n
        z = np.zeros((n - 1, n, 2, 2), dtype=np.complex128)
        for k in range(n - 1):
            for s in range(n):
                z[k, s] = np.diag([1.0, -1.0]) if s in (k, k + 1) else np.eye(2)
        obs.append(z)
    chans = [M.Channel(chis[0], 2), M.Channel(chi3[0], 3), M.Channel(chi3[1], 3)]
    kw = dict(chi_max=16, kappa_max=4, max_kraus=64, svd_cutoff=1e-10, kappa_cutoff=1e-10, prec=prec)
    out = M.batch_run(progs, None, chans, obs, use_graph=True, **kw).cpu().numpy()
    out_ng = M.batch_run(progs, None, chans, obs, use_graph=False, **kw).cpu().numpy()
    assert np.array_equal(out, out_ng)
    kr = [OC.kraus_from_chi(c)[0] for c in chis]
    tol = TOL[prec]
    off = 0
    for pr, ob in zip(progs, obs):
        o = OM.run_program(pr, OM.MPDO(pr.n, 16, 4, 1e-10, 1e-10), kr)
        ref = np.array([o.expect_product(list(x)) / o.trace() for x in ob])
        got = out[off: off + len(ob)]
        off += len(ob)
        assert float(np.abs(got - ref).max()) < tol, (pr.n, float(np.abs(got - ref).max()))


@pytest.mark.parametrize("eps", [1e-3, 1e-4])
def test_crosstalk_workload_at_full_bond_and_inner_limits(eps):
    """The crosstalk workload at chi=128, kappa=16 (n=24): both precisions give
    a normalised state (trace 1) and agree on every <Z_i>, <Z_i Z_i+1> to the
    tolerance of the mixed path, 1e-5, or 10 eps / g when that is larger (g
    the smallest relative gap at a cut of the complex128 run, eps = 6e-8 the
    FP32 contraction rounding: a cut that close to a multiplet moves the kept
    subspace by about eps / g); bonds and inner indices respect their limits
    (no oracle at this size: the properties hold at any size)."""
    require_gpu()
    from paper_2508_07610_amd import crosstalk as X
    n, depth = 24, 4
    r64 = X.run(n=n, depth=depth, chi_max=128, kappa_max=16, eps_list=(eps,), prec=M.C64_MIXED)[0]
    r128 = X.run(n=n, depth=depth, chi_max=128, kappa_max=16, eps_list=(eps,), prec=M.C128)[0]
    assert abs(r128["trace"] - 1) < 1e-10
    assert abs(r64["trace"] - 1) < 1e-4
    assert r128["max_bond"] <= 128 and r128["max_inner"] <= 16
    dev = float(np.abs(r64["obs"] - r128["obs"]).max())
    bound = max(1e-5, 10 * 6e-8 / r128["min_gap"])
    print(f"eps {eps}: max |c64 - c128| = {dev:.2e}, smallest gap {r128['min_gap']:.2e}, bound {bound:.2e}")
    assert dev < bound
    assert float(np.abs(r128["obs"]).max()) <= 1 + 1e-12
    assert r128["max_bond"] > 32


@pytest.mark.parametrize("prec", [M.C128, M.C64_MIXED])
def test_crosstalk_batch_equals_per_gate_runs(prec):
    """Seeded crosstalk instances with their own three-site channels in one
    mpdo_batch_run give each instance's per-gate observables."""
    require_gpu()
    from paper_2508_07610_amd import crosstalk as X
    r = X.run_batch(nb=3, n=10, depth=3, chi_max=32, kappa_max=8, eps=1e-4, prec=prec)
    assert r["obs"].shape == (3, 2 * 10 - 1)
    for t in range(3):
        single = X.run(n=10, depth=3, chi_max=32, kappa_max=8, eps_list=(1e-4,), prec=prec, seed_tag=t)[0]["obs"]
        assert float(np.abs(r["obs"][t] - single).max()) < 1e-12, t
