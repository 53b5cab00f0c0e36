"""Benchmark: MPDO gate-layers/s on the n=16, chi=64, kappa=8 noisy ansatz.

One step = one pass of the whole simulation over one batch of synthetic
input: the depth-10 noisy RY/CZ ansatz (per layer two RY sublayers and two CZ
sublayers, the synthetic process-tomography channel after every gate) from
|0...0>, followed by the GHZ-fidelity terms and every <Z_i Z_i+1>.

  batched (default): B parameter points advanced together by one
      mpdo_batch_run call per step;
  plain: one instance through per-gate C-ABI calls.

gate-layers/s = instances x layers / wall time of the timed steps, with the
inputs already resident on the GPU.  During the timed steps the library's
profiler brackets every compute launch with HIP events on its stream and
accumulates the launches' algorithmic work; the kernel class with the largest
summed time is reported as the roofline kernel.  The CPU oracle (the plain
NumPy/LAPACK MPDO) is timed on a bounded sample of the same circuit.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_QUBITS, DEPTH, CHI, KAPPA = 16, 10, 64, 8
SVD_CUT, KAP_CUT = 1e-10, 1e-14
# MI355X published peaks
PEAK = {"f64_mfma": 78.6, "f32_mfma": 157.3, "f64_valu": 78.6, "hbm": 8000.0}


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
    ap.add_argument("--batch", type=int, default=64, help="parameter points per step (batched mode)")
    ap.add_argument("--no-ttf", action="store_true", help="skip the time-to-fidelity leg (C5 variational loop)")
    ap.add_argument("--ttf-steps", type=int, default=30)
    ap.add_argument("--no-maxcut", action="store_true",
                    help="skip the mixed GHZ-ansatz / QAOA MaxCut batch leg")
    ap.add_argument("--no-sampling", action="store_true", help="skip the bitstring sampling leg")
    ap.add_argument("--no-gemm-tiles", action="store_true", help="skip the full-tile GEMM throughput leg")
    ap.add_argument("--no-noise-models", action="store_true", help="skip the standard noise model comparison")
    ap.add_argument("--no-truncation-study", action="store_true", help="skip the truncation study leg")
    ap.add_argument("--no-crosstalk", action="store_true",
                    help="skip the crosstalk leg (three-site channels, Kraus pruning thresholds)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB three times (b.copy_(a), 2^28 float32): the reference run that "
                         "scales the FETCH_SIZE / WRITE_SIZE counters to bytes")
    ap.add_argument("--graph", action="store_true",
                    help="capture each batched step into one HIP graph (the roofline then comes from one "
                         "extra profiled step outside the timed region)")
    return ap.parse_args()


def gpu_step(M, W, prog, chans, prec):
    st = M.MPDO(N_QUBITS, chi_max=CHI, kappa_max=KAPPA, max_kraus=16, svd_cutoff=SVD_CUT,
                kappa_cutoff=KAP_CUT, prec=prec)
    M.run_program(prog, st, chans)
    f = st.fidelity_ghz()
    zz = [st.expect(s).real for s in W.zz_strings(N_QUBITS)]
    st.close()
    return f, zz


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        n = [d.get("num_threads", 0) for d in threadpool_info() if d.get("user_api") == "blas"]
        if n:
            return max(n)
    except Exception:
        pass
    return len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()


def cpu_baseline(W, layers):
    """The oracle MPDO as it stands, on the first `layers` layers of the same circuit."""
    from oracle import channels as OC
    from oracle import mpdo as OM
    prog = W.ghz_ansatz(N_QUBITS, layers, W.ansatz_params(N_QUBITS, DEPTH, 0))
    kr = [OC.kraus_from_chi(c)[0] for c in prog.chis]
    t0 = time.perf_counter()
    OM.run_program(prog, OM.MPDO(N_QUBITS, CHI, KAPPA, SVD_CUT, KAP_CUT), kr)
    dt = time.perf_counter() - t0
    return {"value": layers / dt, "unit": "gate-layers/s", "cores": blas_threads(), "kind": "oracle",
            "sample": f"first {layers} of {DEPTH} layers of the same circuit (parameter point 0), one instance, "
                      f"complex128 NumPy/LAPACK, {dt:.1f} s; the early layers have smaller bonds, so this "
                      f"overstates the CPU rate on the full circuit"}


def observables(n):
    """<Z_i Z_i+1> and the GHZ-fidelity terms as product operators."""
    import numpy as np
    ops = []
    for i in range(n - 1):
        o = np.stack([np.eye(2, dtype=np.complex128)] * n)
        o[i] = o[i + 1] = np.diag([1.0, -1.0])
        ops.append(o)
    for m in (np.diag([1.0, 0.0]), np.diag([0.0, 1.0]), np.array([[0.0, 1.0], [0.0, 0.0]])):
        ops.append(np.stack([m.astype(np.complex128)] * n))
    return np.stack(ops)


# sources that decide a kernel class's code and the shapes it is launched with
KERNEL_SOURCES = {
    "k_gemm": ("gemm.hip", "common.h", "ops.hip", "ops.h", "engine.hip", "engine.h", "kernels.h"),
    "k_heev": ("eigh.hip", "common.h", "ops.hip", "engine.hip", "kernels.h"),
}


def kernel_sources_hash(kernel):
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2508_07610_amd", "csrc")
    key = "k_gemm" if kernel.startswith("k_gemm") else "k_heev"
    for f in KERNEL_SOURCES[key]:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel, launches_per_step):
    """HBM bytes per launch from the committed PMC summary of this kernel, if it
    was taken from the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(kernel)
    if not e or e.get("sources") != kernel_sources_hash(kernel):
        return None
    return e.get("bytes_per_launch")


def roofline(M, prec_c128, steps):
    classes = {}
    for c, name in M.PROF_NAMES.items():
        classes[c] = M.profile_read(c)
    dom = max(classes, key=lambda c: classes[c]["ms"])
    r = classes[dom]
    if dom == M.PROF_GEMM_F64:
        bound, peak = "mfma", PEAK["f64_mfma"]
    elif dom == M.PROF_GEMM_F32:
        bound, peak = "mfma", PEAK["f32_mfma"]
    else:
        bound, peak = "alu", PEAK["f64_valu"]
    achieved = r["flops"] / (r["ms"] * 1e-3) / 1e12 if r["ms"] > 0 else 0.0
    out = {"bound": bound, "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
           "traffic": traffic_for(M.PROF_NAMES[dom], r["launches"] / max(1, steps)),
           "kernel": M.PROF_NAMES[dom], "launches": r["launches"], "avg_launch_ms": r["ms"] / max(1, r["launches"]),
           "flops_per_launch": r["flops"] / max(1, r["launches"]),
           "algorithmic_bytes_per_launch": r["bytes"] / max(1, r["launches"])}
    share = {M.PROF_NAMES[c]: {"ms": v["ms"], "launches": v["launches"],
                               "tflops": (v["flops"] / (v["ms"] * 1e-3) / 1e12) if v["ms"] > 0 else 0.0}
             for c, v in classes.items()}
    return out, share


def ttf_leg(steps):
    """Time to fidelity of the variational GHZ loop (n=12, depth 6, chi=32,
    kappa=4, c128 judge): plain parameter-shift Adam versus the surrogate-
    assisted loop, both from the same start.  The target is 0.9 x the best
    fidelity of the plain run (the 0.9 target itself is out of reach under
    this noise), each time measured from the start of its own optimisation."""
    import numpy as np
    from paper_2508_07610_amd import surrogate as S
    from paper_2508_07610_amd import variational as V
    n, depth = 12, 6
    theta0 = np.random.default_rng(7610).uniform(-0.3, 0.3, size=2 * n * depth)
    ev = V.AnsatzEvaluator(n, depth, chi_max=32, kappa_max=4)
    ev(theta0[None, :])  # warm-up
    plain = V.plain_optimize(ev, theta0, target=2.0, max_steps=steps, lr=0.05)
    f_best = plain["best"]
    target = 0.9 * f_best
    t_plain = next(h[0] for h in plain["history"] if h[1] >= target)
    e_plain = next(h[2] for h in plain["history"] if h[1] >= target)
    ev2 = V.AnsatzEvaluator(n, depth, chi_max=32, kappa_max=4)
    net = S.MLP(list(S.C5_WIDTHS), max_batch=1024, seed=1)
    sur = V.surrogate_optimize(ev2, net, theta0, target=target, max_steps=steps, lr=0.05,
                               time_limit=10 * plain["history"][-1][0])
    return {"workload": "variational GHZ fidelity, noisy RY/CZ ansatz n=12 depth=6 chi=32 kappa=4, c128 MPDO judge, "
                        "parameter-shift gradients (289 rows per step in one mpdo_batch_run)",
            "f_best_plain": f_best, "target": target,
            "plain_seconds": t_plain, "plain_mpdo_rows": e_plain,
            "surrogate_seconds": sur["time"], "surrogate_reached": sur["reached"],
            "surrogate_mpdo_rows": sur["evaluations"] if sur["reached"] else None,
            "surrogate_longer_steps_chosen": sur["longer_steps_chosen"], "surrogate_proposals": sur["proposals"],
            "surrogate_abs_err_on_verified": sur["surrogate_abs_err"],
            "note": "surrogate seconds include its online training; no pre-training data"}


def maxcut_leg():
    """256 GHZ-ansatz points (n=12, depth 6) and 128 QAOA p=2 MaxCut instances
    (n in 8..20) in one graph-captured mpdo_batch_run, chi=32, kappa=4, mixed
    precision: instances per second and the <H_cut> of the QAOA instances."""
    import numpy as np
    from paper_2508_07610_amd import maxcut as MC
    r = MC.run(n_ghz=256, n_qaoa=128, repeats=4)
    t = float(np.median(r["seconds"]))
    cuts = [p["h_cut"] / p["edges"] for p in r["instances"] if p["kind"] == "qaoa"]
    return {"workload": "one graph-captured mpdo_batch_run: 256 noisy RY/CZ ansatz points n=12 depth=6 + 128 QAOA "
                        "p=2 MaxCut instances on random 3-regular graphs n in {8..20} (SWAP networks), chi=32 "
                        "kappa=4, c64 contractions with FP64 Grams/eigensolvers",
            "seconds_per_batch": t, "instances_per_s": 384 / t, "gates_per_s": r["gates"] / t,
            "timed_batches": len(r["seconds"]),
            "mean_cut_fraction": float(np.mean(cuts)),
            "ghz_fidelity_point0": r["instances"][0]["ghz_fidelity"]}


def gemm_tiles_leg():
    """The GEMM kernel on full tiles (mpdo_test_gemm_rate: device operands,
    HIP events around 10 launches): one 2048^3 complex product and 16
    batched 512 x 1024 x 512 products (the size of the chi = 128 contractions),
    in both MFMA precisions, as context for the workloads' ragged mixes."""
    from paper_2508_07610_amd import mpdo as M
    out = {}
    for prec, name, peak in ((0, "fp64", PEAK["f64_mfma"]), (1, "fp32", PEAK["f32_mfma"])):
        for (m, n, k, items) in ((2048, 2048, 2048, 1), (512, 512, 1024, 16)):
            ms = M.test_gemm_rate(prec, m, n, k, items, 10)
            tf = 8.0 * m * n * k * items / (ms * 1e-3) / 1e12
            out[f"{name}_{items}x{m}x{n}x{k}"] = {"ms": ms, "tflops": tf, "frac": tf / peak}
    return out


def sampling_leg(shots=4096):
    """Computational-basis sampling of the benchmark state (parameter point 0
    of the noisy RY/CZ ansatz, n=16, depth 10, chi=64, kappa=8, c128): shots
    per second of mpdo_sample, the right environments included."""
    import numpy as np
    import torch
    from paper_2508_07610_amd import mpdo as M
    from paper_2508_07610_amd import workloads as W
    prog = W.ghz_ansatz(N_QUBITS, DEPTH, W.ansatz_params(N_QUBITS, DEPTH, 0))
    st = M.MPDO(N_QUBITS, chi_max=CHI, kappa_max=KAPPA, max_kraus=16, svd_cutoff=SVD_CUT, kappa_cutoff=1e-14)
    M.run_program(prog, st, [M.Channel(c, 1 if c.shape[0] == 4 else 2) for c in prog.chis])
    u = np.random.default_rng(7616).random((shots, N_QUBITS))
    st.sample(u[:64])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bits, pz = st.sample(u)
    dt = time.perf_counter() - t0
    distinct = len({b.tobytes() for b in bits})
    st.close()
    return {"workload": f"mpdo_sample of the benchmark state (parameter point 0, n={N_QUBITS} depth={DEPTH} "
                        f"chi={CHI} kappa={KAPPA}, c128), caller uniforms, one call",
            "shots": shots, "seconds": dt, "shots_per_s": shots / dt, "distinct_strings": distinct,
            "max_p_drawn": float(pz.max())}


def noise_models_leg(shots=4096):
    """Bitstring distributions of the noisy RY/CZ ansatz (n=8, depth 4,
    parameter point 0) under the QPT-style channels and the two standard
    models (Fig. fig_unifiedNoise: thermal relaxation T1 = 30 us, T2 = 20 us
    over 30 / 300 ns gates, depolarizing 1e-3 / 1e-2 on the target only or on
    both qubits, read-out flips 2 %); the Jensen-Shannon divergence (Eq. (18))
    of each from the QPT-style one, and of a sampled histogram from its exact
    distribution."""
    import numpy as np
    from paper_2508_07610_amd import distributions as D
    from paper_2508_07610_amd import mpdo as M
    from paper_2508_07610_amd import workloads as W
    n, depth = 8, 4
    base = W.ghz_ansatz(n, depth, W.ansatz_params(n, depth, 0))
    c1 = W.chi_standard_1q(1e-3, 0.03, 30.0, 20.0)
    models = {"qpt": base,
              "unified": W.with_channels(base, c1, W.chi_unified_2q(1e-2, 0.3, 30.0, 20.0)),
              "ideal_noisy": W.with_channels(base, c1, W.chi_ideal_noisy_2q(1e-2, 0.3, 30.0, 20.0))}
    probs, hist = {}, None
    for name, prog in models.items():
        st = M.MPDO(n, chi_max=32, kappa_max=8, max_kraus=64, svd_cutoff=SVD_CUT, kappa_cutoff=KAP_CUT)
        M.run_program(prog, st, [M.Channel(c, 1 if c.shape[0] == 4 else 2) for c in prog.chis])
        probs[name] = st.probabilities(D.all_bitstrings(n))
        if name == "qpt":
            bits, _ = st.sample(np.random.default_rng(7617).random((shots, n)))
            idx = bits.astype(np.int64) @ (1 << np.arange(n - 1, -1, -1))
            hist = np.bincount(idx, minlength=1 << n) / shots
        st.close()
    q = probs["qpt"]
    return {"workload": f"noisy RY/CZ ansatz n={n} depth={depth}, chi=32 kappa=8, c128, full distributions "
                        "from mpdo_probabilities",
            "jsd_vs_qpt": {k: D.jsd(q, v) for k, v in probs.items() if k != "qpt"},
            "jsd_vs_qpt_with_readout_flips": {k: D.jsd(q, D.measurement_flip(v, n, 0.02))
                                              for k, v in probs.items() if k != "qpt"},
            "jsd_sampled_vs_exact": {"shots": shots, "jsd": D.jsd(q, hist)}}


def truncation_study_leg(ncirc=16):
    """Sec. IV.C: mean Uhlmann fidelity between lossless and truncated states
    of random circuits with RZ crosstalk (Q = 3 and 6, depth 4) over a grid
    of (chi, kappa), ncirc circuits each, per-gate calls, FP64."""
    from paper_2508_07610_amd import truncation_study as TS
    limits = [(2, 2), (4, 4), (8, 8), (16, 4), (16, 16)]
    out = {}
    for q in (3, 6):
        t0 = time.perf_counter()
        r = TS.run(q, 4, limits, ncirc=ncirc)
        out[f"Q={q},depth=4"] = {"fidelity": r, "seconds": time.perf_counter() - t0}
    return {"workload": f"{ncirc} random RX/RY/RZ + CNOT circuits per Q, RZ(alpha) crosstalk on the neighbour of "
                        "every CNOT, QPT-style channels, lossless reference at chi=64 kappa=64", "results": out}


def crosstalk_leg():
    """Three-site crosstalk channels with Kraus pruning: the random circuit n=24,
    depth 12, chi=128, kappa=16, mixed precision, once per pruning threshold;
    observables <Z_i>, <Z_i Z_i+1> of every run against the eps = 0 run."""
    from paper_2508_07610_amd import crosstalk as X
    from paper_2508_07610_amd import mpdo as M
    M.profile_enable(True)
    res = X.run(n=24, depth=12, chi_max=128, kappa_max=16, eps_list=(0.0, 1e-4, 1e-3))
    prof = {M.PROF_NAMES[c]: M.profile_read(c) for c in M.PROF_NAMES}
    M.profile_enable(False)
    small = X.run(n=8, depth=12, chi_max=64, kappa_max=16, eps_list=(0.0, 1e-4, 1e-3), dense=True)
    nb = 8
    bat = X.run_batch(nb=nb, n=24, depth=12, chi_max=128, kappa_max=16, eps=1e-4)
    b32 = bat["profile"][M.PROF_NAMES[M.PROF_GEMM_F32]]
    tb32 = b32["flops"] / (b32["ms"] * 1e-3) / 1e12 if b32["ms"] > 0 else 0.0
    g32 = prof[M.PROF_NAMES[M.PROF_GEMM_F32]]
    tf32 = g32["flops"] / (g32["ms"] * 1e-3) / 1e12 if g32["ms"] > 0 else 0.0
    return {"workload": "random RX/RY/RZ + CZ-brick circuit n=24 depth=12, 2q channel after every CZ and a random "
                        "CPTP 3-site channel on the neighbouring triple, chi=128 kappa=16 svd_cutoff=1e-10, "
                        "c64 contractions with FP64 Grams/eigensolvers, per-gate C-ABI calls",
            "runs": [{"eps": r["eps"], "kraus_counts": r["kraus"], "seconds": r["seconds"],
                      "discarded_weight": r["discarded"], "trace": r["trace"], "max_bond": r["max_bond"],
                      "max_obs_dev_vs_eps0": r["max_dev_vs_eps0"]} for r in res],
            "kernel_time_ms": {k: {"ms": v["ms"], "launches": v["launches"],
                                   "tflops": v["flops"] / (v["ms"] * 1e-3) / 1e12 if v["ms"] > 0 else 0.0}
                               for k, v in prof.items()},
            "fp32_contractions": {"achieved": tf32, "peak": PEAK["f32_mfma"], "unit": "TFLOP/s", "frac": tf32 / PEAK["f32_mfma"],
                                  "launches": g32["launches"], "avg_launch_ms": g32["ms"] / max(1, g32["launches"]),
                                  "note": "the chi=128 FP32 MFMA contractions of the three runs, algorithmic flops "
                                          "over HIP-event time per launch (per-gate calls: one item per launch)"},
            "batched": {"workload": f"{nb} seeded instances of the same construction (own 3-site channels each), "
                                    "eps=1e-4, one mpdo_batch_run (launch by launch, after one sizing run)",
                        "seconds": bat["seconds"], "seconds_per_instance": bat["seconds"] / nb,
                        "kernel_time_ms": {k: {"ms": v["ms"], "launches": v["launches"],
                                               "tflops": v["flops"] / (v["ms"] * 1e-3) / 1e12 if v["ms"] > 0 else 0.0}
                                           for k, v in bat["profile"].items()},
                        "fp32_contractions": {"achieved": tb32, "peak": PEAK["f32_mfma"], "unit": "TFLOP/s",
                                              "frac": tb32 / PEAK["f32_mfma"], "launches": b32["launches"]}},
            "slice_n8": {"note": "same construction at n=8, chi=64 (dense states from mpdo_to_dense); Uhlmann fidelity "
                                 "F(rho_eps0, rho_eps) computed on the host from the two dense matrices",
                         "fidelity_vs_eps0": {str(r["eps"]): r["fidelity_vs_eps0"] for r in small},
                         "jsd_vs_eps0": {str(r["eps"]): r["jsd_vs_eps0"] for r in small},
                         "seconds": {str(r["eps"]): r["seconds"] for r in small}}}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only (the MPDO path is not sharded); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    if a.copy_calibration:
        x = torch.ones(2 ** 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print("copied 1 GiB x 3", flush=True)
        return
    from paper_2508_07610_amd import mpdo as M
    from paper_2508_07610_amd import workloads as W
    torch.cuda.set_device(0)
    prec = M.C128 if a.prec == "c128" else M.C64_MIXED
    prog = W.ghz_ansatz(N_QUBITS, a.depth, W.ansatz_params(N_QUBITS, DEPTH, 0))
    chans = [M.Channel(prog.chis[0], 1), M.Channel(prog.chis[1], 2)]
    if a.mode == "plain":
        ninst = 1

        def step(graph=False):
            return gpu_step(M, W, prog, chans, prec)
    else:
        ninst = a.batch
        P = np.stack([W.ansatz_params(N_QUBITS, DEPTH, t) for t in range(ninst)])
        progs = [W.ghz_ansatz(N_QUBITS, a.depth, P[b]) for b in range(ninst)]
        pdev = torch.tensor(P, dtype=torch.float64, device="cuda")
        obs = observables(N_QUBITS)
        nobs = obs.shape[0]
        # the circuits' host-side form is built once; each step evaluates
        # every parameter point on the device
        plan = M.BatchPlan(progs, [obs] * ninst, use_params=True)

        def step(graph=a.graph):
            r = M.batch_run(plan, pdev, chans, None, chi_max=CHI, kappa_max=KAPPA, max_kraus=16,
                            svd_cutoff=SVD_CUT, kappa_cutoff=KAP_CUT, prec=prec, use_graph=graph)
            r = r.view(ninst, nobs)
            f = 0.5 * (r[0, -3] + r[0, -2] + 2 * r[0, -1]).real.item()
            return f, r[0, : N_QUBITS - 1].real.cpu().tolist()
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    profiled_timed = not (a.mode == "batched" and a.graph)
    if profiled_timed:
        M.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(a.steps):
        f, zz = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if not profiled_timed:
        M.profile_enable(True)
        step(graph=False)
        torch.cuda.synchronize()
    roof, share = roofline(M, prec == M.C128, a.steps if profiled_timed else 1)
    M.profile_enable(False)
    ms = 1e3 * dt / a.steps
    value = ninst * a.depth * a.steps / dt
    if a.mode == "plain":
        wl = (f"plain MPDO, noisy RY/CZ ansatz n={N_QUBITS} depth={a.depth} chi={CHI} kappa={KAPPA} "
              f"svd_cutoff={SVD_CUT}, per-gate C-ABI calls, one instance")
    else:
        wl = (f"batched MPDO, {ninst} parameter points of the noisy RY/CZ ansatz n={N_QUBITS} depth={a.depth} "
              f"chi={CHI} kappa={KAPPA} svd_cutoff={SVD_CUT}, one mpdo_batch_run per step"
              + (" captured in one HIP graph" if a.graph else ""))
    out = {
        "metric": "MPDO gate-layers/s (n=16,chi=64,kappa=8) plain vs batched; surrogate time-to-fidelity",
        "value": value, "unit": "gate-layers/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c128" if prec == M.C128 else "c64+f64", "data": "synthetic",
        "config": {"workload": wl, "instances": ninst, "mode": a.mode, "ghz_fidelity_instance0": f,
                   "zz01_instance0": zz[0], "roofline_from": "timed steps" if profiled_timed
                   else "one extra profiled step (graph launches are not profiled)"},
        "roofline": roof,
        "kernel_time_ms": share,
        "cpu_baseline": None if a.no_cpu else cpu_baseline(W, a.cpu_layers),
        "time_to_fidelity": None if a.no_ttf else ttf_leg(a.ttf_steps),
        "maxcut_batch": None if a.no_maxcut else maxcut_leg(),
        "gemm_full_tiles": None if a.no_gemm_tiles else gemm_tiles_leg(),
        "sampling": None if a.no_sampling else sampling_leg(),
        "noise_models": None if a.no_noise_models else noise_models_leg(),
        "truncation_study": None if a.no_truncation_study else truncation_study_leg(),
        "crosstalk": None if a.no_crosstalk else crosstalk_leg(),
    }
    print(json.dumps(out, default=lambda o: o.item() if hasattr(o, "item") else str(o)))


if __name__ == "__main__":
    main()
