"""The truncation study of Sec. IV.C on the device: the fidelity between the
truncated and the lossless state against the oracle's, and its limits."""
import numpy as np
import pytest

from oracle import channels as OC
from oracle import dense as OD
from oracle import mpdo as OM
from paper_2508_07610_amd import mpdo as M
from paper_2508_07610_amd import truncation_study as TS
from paper_2508_07610_amd import workloads as W
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def test_fidelity_matches_oracle():
    """One Q = 4, depth 3 circuit: the lossless states agree, and F(lossless,
    truncated) from device states equals the oracle's from its own MPDO runs."""
    require_gpu()
    prog = TS.circuit(4, 3, W.rng_for(4600))
    kr = [OC.kraus_from_chi(c)[0] for c in prog.chis]
    chans = [M.Channel(prog.chis[0], 1), M.Channel(prog.chis[1], 2)]

    def dev(chi, kap):
        st = M.MPDO(4, chi_max=chi, kappa_max=kap, max_kraus=16, svd_cutoff=1e-14, kappa_cutoff=1e-14)
        M.run_program(prog, st, chans)
        r = st.to_dense()
        return r / np.trace(r).real

    def ora(chi, kap):
        o = OM.run_program(prog, OM.MPDO(4, chi, kap, 1e-14, 1e-14), kr)
        r = o.to_dense()
        return r / np.trace(r).real

    full_d, full_o = dev(64, 64), ora(64, 64)
    assert float(np.abs(full_d - full_o).max()) < 1e-10
    # kappa = 2 would cut through the nearly degenerate X / Y / Z branches of
    # the depolarizing channels (relative gaps near 1e-6, above the tie rule),
    # where the kept vectors follow rounding: compare at limits whose cuts
    # fall in clear gaps
    for lim in ((4, 4), (8, 4)):
        f_dev = TS.uhlmann_fidelity(full_d, dev(*lim))
        f_ora = OD.uhlmann_fidelity(full_o, ora(*lim))
        assert f_dev < 1 - 1e-4
        assert abs(f_dev - f_ora) < 1e-9, lim


def test_study_limits():
    """Lossless limits give F = 1; every mean lies in (0, 1]; the loosest
    truncation is at least as faithful on average as the tightest."""
    require_gpu()
    r = TS.run(3, 4, [(64, 64), (4, 4), (1, 1)], ncirc=6, seed=1)
    assert abs(r["chi=64,kappa=64"]["mean"] - 1) < 1e-9
    for v in r.values():
        assert 0 < v["min"] <= v["mean"] <= 1 + 1e-9
    assert r["chi=4,kappa=4"]["mean"] >= r["chi=1,kappa=1"]["mean"] - 1e-12


def test_batched_study_equals_per_circuit_runs():
    """run_batched (every circuit of a point in one mpdo_batch_run_dense per
    limit) gives each circuit the fidelity of its own per-gate runs."""
    require_gpu()
    q, depth, lims = 3, 4, [(4, 4), (8, 4)]
    r = TS.run_batched(q, depth, lims, ncirc=6, seed=2, per_circuit=True)
    progs = TS.circuits(q, depth, 6, seed=2)
    chans = [M.Channel(progs[0].chis[0], 1), M.Channel(progs[0].chis[1], 2)]

    def dev(prog, chi, kap):
        st = M.MPDO(q, chi_max=chi, kappa_max=kap, max_kraus=16, svd_cutoff=1e-14, kappa_cutoff=1e-14)
        M.run_program(prog, st, chans)
        x = st.to_dense()
        st.close()
        return x / np.trace(x).real

    for i, prog in enumerate(progs):
        full = dev(prog, 64, 64)
        for lim in lims:
            f = TS.uhlmann_fidelity(full, dev(prog, *lim))
            assert abs(f - r["fidelity"][f"chi={lim[0]},kappa={lim[1]}"]["all"][i]) < 1e-9, (i, lim)
    assert r["circuits"] == 6


@pytest.mark.parametrize("q", [3, 6])
def test_reference_state_against_the_dense_simulator(q):
    """The study's reference (chi = kappa = 64, cutoffs 1e-14) against the
    oracle's dense simulation of the same circuits (Eq. (1) gate by gate):
    the difference in normalised rho is bounded by the reference's own
    discarded weight (mpdo_stats), which is what limits how close to 1 a
    study fidelity can be resolved (the cap kappa * max_kraus <= 1024 keeps
    kappa at 64)."""
    require_gpu()
    for prog in TS.circuits(q, 4, 2, seed=3):
        kr = [OC.kraus_from_chi(c)[0] for c in prog.chis]
        d = OM.run_program_dense(prog, OD.DenseSim(q), kr).rho
        d = d / np.trace(d).real
        chans = [M.Channel(prog.chis[0], 1), M.Channel(prog.chis[1], 2)]
        st = M.MPDO(q, chi_max=64, kappa_max=64, max_kraus=16, svd_cutoff=1e-14, kappa_cutoff=1e-14)
        M.run_program(prog, st, chans)
        r = st.to_dense()
        r = r / np.trace(r).real
        disc = st.stats()["discarded"]
        err = float(np.abs(r - d).max())
        print(f"Q={q}: max |reference - dense| = {err:.2e}, discarded weight {disc:.2e}")
        assert err <= 2 * disc + 1e-12
        st.close()
        for c in chans:
            c.close()
