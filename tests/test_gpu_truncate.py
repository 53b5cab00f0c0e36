"""mpdo_truncate (the truncation sweep of Sec. II.D) on the GPU against the
oracle's sweep: same bond and inner dimensions, bond weights, discarded
weight and observables; a sweep that cuts nothing leaves the state as it
was."""
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


def _pair(n, depth, chi, kap, tag, prec):
    prog = W.ghz_ansatz(n, depth, W.ansatz_params(n, depth, tag))
    kr = [OC.kraus_from_chi(c)[0] for c in prog.chis]
    o = OM.run_program(prog, OM.MPDO(n, chi, kap, 1e-10, 1e-10), kr)
    chans = [M.Channel(c, int(round(math.log(c.shape[0], 4)))) for c in prog.chis]
    st = M.MPDO(n, chi_max=chi, kappa_max=kap, max_kraus=16, svd_cutoff=1e-10, kappa_cutoff=1e-10, prec=prec)
    M.run_program(prog, st, chans)
    return o, st


def _observables(n):
    return W.zz_strings(n) + ["X" * n, "Y" + "Z" * (n - 1), "Z" * n]


@pytest.mark.parametrize("prec", [M.C128, M.C64_MIXED])
@pytest.mark.parametrize("n,depth,chi,kap,chi2,kap2,cut,tag", [
    (6, 2, 16, 8, 4, 2, 1e-8, 1),
    (8, 3, 32, 8, 6, 3, 1e-6, 2),
    (7, 2, 16, 4, 16, 1, 1e-10, 3),
])
def test_truncate_matches_oracle(prec, n, depth, chi, kap, chi2, kap2, cut, tag):
    require_gpu()
    o, st = _pair(n, depth, chi, kap, tag, prec)
    d_gpu = st.truncate(chi2, kap2, cut)
    d_or = o.truncate_sweep(chi2, kap2, cut)
    tol = TOL[prec]
    bonds, inner, _ = st.dims()
    if prec == M.C128:
        assert bonds == o.bond_dims()
        assert inner == o.inner_dims()
        for b in range(n - 1):
            assert np.abs(st.bond_weights(b) - o.lam[b]).max() < 1e-9, b
    assert abs(d_gpu - d_or) < 1e3 * tol
    # the inner truncations of the sites are independent renormalised
    # projections, so Tr rho moves away from 1 by about the discarded weight,
    # identically on both sides
    assert abs(st.trace() - o.trace()) < tol
    for s in _observables(n):
        assert abs(st.expect(s) - o.expect_pauli(s)) < tol, s
    assert abs(st.fidelity_ghz() - o.fidelity_ghz()) < tol


def test_truncate_without_cuts_keeps_the_state():
    require_gpu()
    n = 6
    o, st = _pair(n, 2, 32, 16, 4, M.C128)
    before = [st.expect(s) for s in _observables(n)]
    d = st.truncate(32, 16, 0.0)
    after = [st.expect(s) for s in _observables(n)]
    assert d < 1e-12
    assert max(abs(a - b) for a, b in zip(before, after)) < 1e-11


def test_truncate_rejects_bad_limits():
    require_gpu()
    st = M.MPDO(4, chi_max=8, kappa_max=2, max_kraus=4)
    for args in [(0, 1, 0.0), (9, 1, 0.0), (4, 3, 0.0), (4, 1, 1.5)]:
        with pytest.raises(M.MPDOError) as e:
            st.truncate(*args)
        assert e.value.status == M.EINVAL
