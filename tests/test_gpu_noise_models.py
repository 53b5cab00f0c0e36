"""Standard noise models (thermal relaxation + depolarizing, Fig.
`fig_unifiedNoise`) through the device simulator: parity with the oracle on
the bitstring distribution, and the Jensen-Shannon divergence (Eq. (18))
between them and the QPT-style channels."""
import math

import numpy as np
import pytest

from oracle import channels as OC
from oracle import dense as OD
from oracle import mpdo as OM
from oracle import sampling as OS
from paper_2508_07610_amd import distributions as D
from paper_2508_07610_amd import mpdo as M
from paper_2508_07610_amd import workloads as W
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu
T1, T2, T_1Q, T_2Q, P1, P2 = 30.0, 20.0, 0.03, 0.3, 1e-3, 1e-2  # microseconds


def _probs(prog, prec=M.C128):
    qs = [int(round(math.log(c.shape[0], 4))) for c in prog.chis]
    st = M.MPDO(prog.n, chi_max=32, kappa_max=8, max_kraus=64, svd_cutoff=1e-10, kappa_cutoff=1e-10, prec=prec)
    M.run_program(prog, st, [M.Channel(c, q) for c, q in zip(prog.chis, qs)])
    p = st.probabilities(D.all_bitstrings(prog.n))
    st.close()
    return p


@pytest.mark.parametrize("model", ["unified", "ideal"])
def test_standard_models_match_oracle(model):
    require_gpu()
    n, depth = 6, 2
    base = W.ghz_ansatz(n, depth, W.ansatz_params(n, depth, 90))
    c2 = W.chi_unified_2q(P2, T_2Q, T1, T2) if model == "unified" else W.chi_ideal_noisy_2q(P2, T_2Q, T1, T2)
    prog = W.with_channels(base, W.chi_standard_1q(P1, T_1Q, T1, T2), c2)
    kr = [OC.kraus_from_chi(c)[0] for c in prog.chis]
    o = OM.run_program(prog, OM.MPDO(n, 32, 8, 1e-10, 1e-10), kr)
    ref = OS.basis_probabilities(o.to_dense())
    got = _probs(prog)
    assert float(np.abs(got - ref).max()) < 1e-10


def test_jsd_between_noise_models():
    """The QPT-style channels and the two standard models give distinct
    distributions (JSD > 0, below ln 2); a model against itself gives 0; read-
    out flips move the distribution further."""
    require_gpu()
    n, depth = 6, 2
    base = W.ghz_ansatz(n, depth, W.ansatz_params(n, depth, 91))
    pq = _probs(base)
    pu = _probs(W.with_channels(base, W.chi_standard_1q(P1, T_1Q, T1, T2), W.chi_unified_2q(P2, T_2Q, T1, T2)))
    pi = _probs(W.with_channels(base, W.chi_standard_1q(P1, T_1Q, T1, T2), W.chi_ideal_noisy_2q(P2, T_2Q, T1, T2)))
    assert D.jsd(pq, pq) == 0.0
    for p in (pu, pi):
        j = D.jsd(pq, p)
        assert 0 < j < math.log(2)
        assert abs(j - OD.jsd(pq, p)) < 1e-15
    pm = D.measurement_flip(pu, n, 0.02)
    assert abs(pm.sum() - 1) < 1e-12 and D.jsd(pq, pm) > D.jsd(pq, pu)
