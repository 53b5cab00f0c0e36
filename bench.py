"""Benchmark: MPDO gate-layers/s on the n=16, chi=64, kappa=8 noisy ansatz.

One step = one pass of the whole simulation over one batch of synthetic
input: the depth-10 noisy RY/CZ ansatz (2 RY sublayers + 2 CZ sublayers per
layer, a synthetic QPT channel after every gate) from |0...0>, followed by
the GHZ fidelity and all <Z_i Z_{i+1}>.  gate-layers/s = instances x layers
per second of wall time, inputs resident on the GPU.

Prints one JSON line (see the design doc for the fields).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_QUBITS, DEPTH, CHI, KAPPA = 16, 10, 64, 8
SVD_CUT, KAP_CUT = 1e-10, 1e-14


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", choices=["c128", "c64"], default="c128")
    ap.add_argument("--depth", type=int, default=DEPTH)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-layers", type=int, default=5)
    ap.add_argument("--mode", choices=["batched", "plain"], default="batched")
    ap.add_argument("--batch", type=int, default=32, help="parameter points per step (batched mode)")
    ap.add_argument("--no-graph", action="store_true", help="batched mode without HIP graph capture")
    return ap.parse_args()


def gpu_step(M, W, prog, chans, prec):
    st = M.MPDO(N_QUBITS, chi_max=CHI, kappa_max=KAPPA, max_kraus=16, svd_cutoff=SVD_CUT,
                kappa_cutoff=KAP_CUT, prec=prec)
    M.run_program(prog, st, chans)
    f = st.fidelity_ghz()
    zz = [st.expect(s).real for s in W.zz_strings(N_QUBITS)]
    st.close()
    return f, zz


def cpu_baseline(W, layers):
    """The oracle MPDO as it stands on the first `layers` layers of the same circuit."""
    import numpy as np
    from oracle import channels as OC
    from oracle import mpdo as OM
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    prog = W.ghz_ansatz(N_QUBITS, layers, W.ansatz_params(N_QUBITS, DEPTH, 0))
    kr = [OC.kraus_from_chi(c)[0] for c in prog.chis]
    t0 = time.perf_counter()
    OM.run_program(prog, OM.MPDO(N_QUBITS, CHI, KAPPA, SVD_CUT, KAP_CUT), kr)
    dt = time.perf_counter() - t0
    return {"value": layers / dt, "unit": "gate-layers/s", "cores": threads, "kind": "oracle",
            "sample": f"first {layers} of {DEPTH} layers of the same circuit, one instance, complex128 "
                      f"NumPy/LAPACK ({dt:.1f} s)"}


def observables(W, n):
    """GHZ-fidelity terms and the <Z_i Z_i+1> as product operators."""
    import numpy as np
    ops = []
    for i in range(n - 1):
        o = np.stack([np.eye(2, dtype=np.complex128)] * n)
        o[i] = o[i + 1] = np.diag([1.0, -1.0])
        ops.append(o)
    for m in (np.diag([1.0, 0.0]), np.diag([0.0, 1.0]), np.array([[0.0, 1.0], [0.0, 0.0]])):
        ops.append(np.stack([m.astype(np.complex128)] * n))
    return np.stack(ops)


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only (the MPDO path is not sharded); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2508_07610_amd import mpdo as M
    from paper_2508_07610_amd import workloads as W
    torch.cuda.set_device(0)
    prec = M.C128 if a.prec == "c128" else M.C64_MIXED
    prog = W.ghz_ansatz(N_QUBITS, a.depth, W.ansatz_params(N_QUBITS, DEPTH, 0))
    chans = [M.Channel(prog.chis[0], 1), M.Channel(prog.chis[1], 2)]
    if a.mode == "plain":
        ninst = 1

        def step():
            return gpu_step(M, W, prog, chans, prec)
    else:
        ninst = a.batch
        P = np.stack([W.ansatz_params(N_QUBITS, DEPTH, t) for t in range(ninst)])
        progs = [W.ghz_ansatz(N_QUBITS, a.depth, P[b]) for b in range(ninst)]
        pdev = torch.tensor(P, dtype=torch.float64, device="cuda")
        obs = observables(W, N_QUBITS)
        nobs = obs.shape[0]

        def step():
            r = M.batch_run(progs, pdev, chans, [obs] * ninst, chi_max=CHI, kappa_max=KAPPA, max_kraus=16,
                            svd_cutoff=SVD_CUT, kappa_cutoff=KAP_CUT, prec=prec, use_graph=not a.no_graph)
            r = r.view(ninst, nobs)
            f = 0.5 * (r[0, -3] + r[0, -2] + 2 * r[0, -1]).real.item()
            return f, r[0, : N_QUBITS - 1].real.cpu().tolist()
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        f, zz = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = 1e3 * dt / a.steps
    value = ninst * a.depth * a.steps / dt
    if a.mode == "plain":
        wl = (f"plain MPDO, noisy RY/CZ ansatz n={N_QUBITS} depth={a.depth} chi={CHI} kappa={KAPPA} "
              f"svd_cutoff={SVD_CUT}, per-gate ABI calls, one instance")
    else:
        wl = (f"batched MPDO, {ninst} parameter points of the noisy RY/CZ ansatz n={N_QUBITS} depth={a.depth} "
              f"chi={CHI} kappa={KAPPA} svd_cutoff={SVD_CUT}, one mpdo_batch_run per step"
              + ("" if a.no_graph else " captured in one HIP graph"))
    out = {
        "metric": "MPDO gate-layers/s (n=16,chi=64,kappa=8) plain vs batched; surrogate time-to-fidelity",
        "value": value, "unit": "gate-layers/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c128" if prec == M.C128 else "c64+f64", "data": "synthetic",
        "config": {"workload": wl, "instances": ninst, "ghz_fidelity": f, "zz0": zz[0]},
        "roofline": None,
        "cpu_baseline": None if a.no_cpu else cpu_baseline(W, a.cpu_layers),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
