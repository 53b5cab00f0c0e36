"""Mixed batch of variational GHZ points and QAOA MaxCut instances in one
batched run (Eqs. (20)-(22) for the MaxCut cost; the ansatz of the GHZ
study).

Instances: `n_ghz` parameter points of the noisy RY/CZ ansatz (n = 12,
depth 6) and `n_qaoa` QAOA p = 2 instances on random 3-regular graphs with n
drawn from {8, 10, ..., 20}, edges routed through an odd-even SWAP network,
the same process-tomography channels after every gate.  One
``mpdo_batch_run`` (optionally one HIP graph) evaluates all of them; the
results are the GHZ fidelity terms and <Z_i Z_i+1> of the ansatz points and
<Z_a Z_b> of every graph edge, from which <H_cut> = sum_edges (1 - <Z_a Z_b>)/2.
Argument marshalling only: the simulation runs in the library's kernels.
"""
from __future__ import annotations

import math
import time
from typing import Dict, List

import numpy as np

from . import mpdo as M
from . import workloads as W


def instances(n_ghz: int = 256, n_qaoa: int = 128, depth: int = 6, seed_tag: int = 0):
    """Programs, the parameter matrix, the observables and per-instance info
    (the seeded recipe of workloads.maxcut_batch_instances)."""
    return W.maxcut_batch_instances(n_ghz, n_qaoa, depth, seed_tag)


def run(n_ghz: int = 256, n_qaoa: int = 128, depth: int = 6, chi_max: int = 32, kappa_max: int = 4,
        prec: int = M.C64_MIXED, use_graph: bool = True, repeats: int = 1, seed_tag: int = 0) -> Dict:
    """Build the batch, run it `repeats` times (the first untimed) and return
    the per-instance results and the timing of the timed runs."""
    import torch
    progs, P, obs, info = instances(n_ghz, n_qaoa, depth, seed_tag)
    chans = [M.Channel(W.chi_1q_default(), 1), M.Channel(W.chi_2q_default(), 2)]
    pdev = torch.tensor(P, dtype=torch.float64, device="cuda")
    kw = dict(chi_max=chi_max, kappa_max=kappa_max, max_kraus=16, svd_cutoff=1e-10, kappa_cutoff=1e-10, prec=prec)
    plan = M.BatchPlan(progs, obs, use_params=True)  # the host-side form, built once
    out = M.batch_run(plan, pdev, chans, None, use_graph=use_graph, **kw)
    torch.cuda.synchronize()
    times = []
    for _ in range(max(0, repeats - 1)):
        t0 = time.perf_counter()
        out = M.batch_run(plan, pdev, chans, None, use_graph=use_graph, out=out, **kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    res = out.cpu().numpy()
    off = 0
    per: List[Dict] = []
    raw: List[np.ndarray] = []
    for b, (pr, ob, inf) in enumerate(zip(progs, obs, info)):
        k = ob.shape[0]
        raw.append(res[off: off + k])
        v = res[off: off + k].real
        off += k
        if inf["kind"] == "ghz":
            f = 0.5 * (v[-3] + v[-2] + 2 * v[-1])
            per.append({**inf, "ghz_fidelity": float(f), "zz": v[:11].tolist()})
        else:
            per.append({**inf, "h_cut": float(np.sum((1 - v) / 2)), "zz_edges": v.tolist()})
    return {"instances": per, "raw": raw, "seconds": times, "programs": progs, "params": P, "observables": obs,
            "channels": chans, "config": kw, "gates": sum(len(p.ops) for p in progs)}
