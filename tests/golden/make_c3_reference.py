"""Writes tests/golden/c3_reference.json: the oracle's truncated MPDO
(complex128, chi = 32, kappa = 4, cutoffs 1e-10) on two instances of the
mixed GHZ / MaxCut batch -- the first ansatz point (n = 12, depth 6) and the
first QAOA p = 2 instance with n = 20 -- with each instance's observables
normalised by the trace, and the smallest relative gap
eta_{r-1} / eta_r - 1 over the truncations that dropped weight above 1e-10
of their total (the conditioning of the truncated result: a cut that close
to a multiplet moves the kept subspace by about eps / gap).  Calls only
oracle/ (inputs from workloads).  Run from the repository root:
python tests/golden/make_c3_reference.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import channels as OC  # noqa: E402
from oracle import mpdo as OM  # noqa: E402
from paper_2508_07610_amd import workloads as W  # noqa: E402

CHI, KAPPA, CUT = 32, 4, 1e-10
GAPS = []
_select = OM.select_rank


def _recording_select(eta, max_dim, cutoff):
    r = _select(eta, max_dim, cutoff)
    if r < len(eta) and eta[r] > 0 and eta[r] > 1e-10 * sum(eta):
        GAPS.append(float(eta[r - 1] / eta[r] - 1))
    return r


OM.select_rank = _recording_select

if __name__ == "__main__":
    progs, P, obs, info = W.maxcut_batch_instances(256, 128)
    picks = [0, next(i for i, x in enumerate(info) if x["kind"] == "qaoa" and x["n"] == 20)]
    kr = [OC.kraus_from_chi(c)[0] for c in (W.chi_1q_default(), W.chi_2q_default())]
    cases = []
    for b in picks:
        t0 = time.perf_counter()
        GAPS.clear()
        o = OM.run_program(progs[b], OM.MPDO(progs[b].n, CHI, KAPPA, CUT, CUT), kr)
        tr = o.trace()
        vals = [o.expect_product(list(ob)) / tr for ob in obs[b]]
        cases.append({"index": b, "kind": info[b]["kind"], "n": progs[b].n,
                      "re": [float(v.real) for v in vals], "im": [float(v.imag) for v in vals],
                      "bond_dims": o.bond_dims(), "min_gap": min(GAPS) if GAPS else None,
                      "oracle_seconds": time.perf_counter() - t0})
    out = {"workload": {"n_ghz": 256, "n_qaoa": 128, "depth": 6, "chi_max": CHI, "kappa_max": KAPPA,
                        "svd_cutoff": CUT, "kappa_cutoff": CUT}, "cases": cases}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_reference.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, [c["oracle_seconds"] for c in cases])
