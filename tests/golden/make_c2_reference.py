"""Writes tests/golden/c2_reference.json: the oracle's truncated MPDO on the
headline workload (n = 16, depth 10 noisy RY/CZ ansatz, chi = 64, kappa = 8,
cutoffs 1e-10, noise strengths x1 and x3, parameter point 0), computed by
oracle/ only (the CPU MPDO of Secs. II.C-II.D in complex128).  Run from the
repository root:  python tests/golden/make_c2_reference.py
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

N, DEPTH, CHI, KAPPA, CUT = 16, 10, 64, 8, 1e-10


def reference(scale: float, tag: int = 0) -> dict:
    prog = W.ghz_ansatz(N, DEPTH, W.ansatz_params(N, DEPTH, tag), noise_scale=scale)
    kr = [OC.kraus_from_chi(c)[0] for c in prog.chis]
    t0 = time.perf_counter()
    m = OM.run_program(prog, OM.MPDO(N, CHI, KAPPA, CUT, CUT), kr)
    dt = time.perf_counter() - t0
    return {
        "noise_scale": scale, "param_tag": tag, "oracle_seconds": dt,
        "zz": [m.expect_pauli(s).real for s in W.zz_strings(N)],
        "ghz_fidelity": m.fidelity_ghz(),
        "trace": m.trace(),
        "bond_dims": m.bond_dims(), "inner_dims": m.inner_dims(),
        "discarded": m.discarded,
        "lam": [list(map(float, l)) for l in m.lam],
    }


if __name__ == "__main__":
    # each case is written as soon as it is done (about half an hour each on
    # four cores); a rerun keeps the cases already in the file
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_reference.json")
    out = {"workload": {"n": N, "depth": DEPTH, "chi_max": CHI, "kappa_max": KAPPA, "svd_cutoff": CUT,
                        "kappa_cutoff": CUT}, "cases": []}
    if os.path.exists(path):
        with open(path) as f:
            old = json.load(f)
        if old["workload"] == out["workload"]:
            out = old
    for scale in (1.0, 3.0):
        if any(c["noise_scale"] == scale for c in out["cases"]):
            continue
        out["cases"].append(reference(scale))
        with open(path + ".tmp", "w") as f:
            json.dump(out, f, indent=1)
        os.replace(path + ".tmp", path)
        print("wrote", path, [c["oracle_seconds"] for c in out["cases"]], flush=True)
