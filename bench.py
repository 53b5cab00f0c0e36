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
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2508_07610_amd.pmc_summary import kernel_sources_hash  # noqa: E402

N_QUBITS, DEPTH, CHI, KAPPA = 16, 10, 64, 8
SVD_CUT, KAP_CUT = 1e-10, 1e-10
# MI355X published peaks
PEAK = {"f64_mfma": 78.6, "f32_mfma": 157.3, "f64_valu": 78.6, "hbm": 8000.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", choices=["c128", "c64"], default="c128")
    ap.add_argument("--depth", type=int, default=DEPTH)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--mode", choices=["batched", "plain"], default="batched")
    ap.add_argument("--batch", type=int, default=64, help="parameter points per step (batched mode)")
    ap.add_argument("--no-ttf", action="store_true", help="skip the time-to-fidelity leg (C5 variational loop)")
    ap.add_argument("--ttf-steps", type=int, default=30)
    ap.add_argument("--no-maxcut", action="store_true",
                    help="skip the mixed GHZ-ansatz / QAOA MaxCut batch leg")
    ap.add_argument("--no-sampling", action="store_true", help="skip the bitstring sampling leg")
    ap.add_argument("--no-gemm-tiles", action="store_true", help="skip the full-tile GEMM throughput leg")
    ap.add_argument("--no-eig-lone", action="store_true",
                    help="skip the lone-eigenproblem leg (shared reduction against one workgroup per matrix)")
    ap.add_argument("--no-noise-models", action="store_true", help="skip the standard noise model comparison")
    ap.add_argument("--no-truncation-study", action="store_true", help="skip the truncation study leg")
    ap.add_argument("--no-mitigation", action="store_true", help="skip the error-mitigation leg")
    ap.add_argument("--no-crosstalk", action="store_true",
                    help="skip the crosstalk leg (three-site channels, Kraus pruning thresholds)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB three times (b.copy_(a), 2^28 float32): the reference run that "
                         "scales the FETCH_SIZE / WRITE_SIZE counters to bytes")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch each batched step kernel by kernel instead of as one captured HIP graph (with "
                         "the graph, the roofline comes from one extra profiled step outside the timed region)")
    ap.add_argument("--cpu-threads1", action="store_true",
                    help="also time the oracle's two-site gate on one BLAS thread (minutes)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the library's built-in GEMM choices (no autotuner settings)")
    ap.add_argument("--retune", action="store_true",
                    help="run the GEMM autotuner even if its cache holds settings for this workload")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the plain-vs-batched sweep (B, precision, noise strength)")
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


def cpu_baseline(W, threads1=True):
    """The oracle MPDO as it stands, timed at the workload's steady state: one
    two-site and one one-site noisy gate (CZ then the 2q channel, RY then the
    1q channel) on a state whose touched sites are at the full limits
    (bonds chi = 64, inner kappa = 8; random right-orthonormal tensors, whose
    values do not change the cost of the dense decompositions).  A layer is
    15 two-site and 32 one-site gates, so gate-layers/s = 1 / (15 t2 + 32 t1).
    Timed with every host core and with one BLAS thread."""
    import numpy as np
    from oracle import channels as OC
    from oracle import mpdo as OM

    rng = np.random.default_rng(7690)

    def site(l, r):
        a = rng.normal(size=(l, 2 * KAPPA * r)) + 1j * rng.normal(size=(l, 2 * KAPPA * r))
        q, _ = np.linalg.qr(a.conj().T)
        return q.conj().T.reshape(l, 2, KAPPA, r)

    edge = 2 * KAPPA

    def fresh():
        # bonds edge, chi, chi, chi, edge: the gate's sites 2, 3 see chi on both sides
        m = OM.MPDO(6, CHI, KAPPA, SVD_CUT, KAP_CUT)
        dims = [1, edge, CHI, CHI, CHI, edge, 1]
        m.T = [site(dims[i], dims[i + 1]) for i in range(6)]
        m.lam = []
        for d in dims[1:-1]:
            lam = np.sort(rng.uniform(size=d))[::-1] ** 4
            m.lam.append(lam / np.linalg.norm(lam))
        return m

    k1 = OC.kraus_from_chi(W.chi_1q_default())[0]
    k2 = OC.kraus_from_chi(W.chi_2q_default())[0]
    G1 = [K @ W.ry(0.7) for K in k1]
    G2 = [K @ W.CZ for K in k2]

    def timed(two=True):
        t2 = None
        if two:
            m = fresh()
            t0 = time.perf_counter()
            m.apply_2q(2, G2)
            t2 = time.perf_counter() - t0
        m = fresh()
        t0 = time.perf_counter()
        m.apply_1q(2, G1)
        t1 = time.perf_counter() - t0
        return t2, t1

    cores = blas_threads()
    t2, t1 = timed()
    rate = 1.0 / (15 * t2 + 32 * t1)
    one = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            u2, u1 = timed(two=threads1)
        if threads1:
            one = {"value": 1.0 / (15 * u2 + 32 * u1), "unit": "gate-layers/s", "cores": 1,
                   "sample": f"one 2q gate {u2:.2f} s, one 1q gate {u1:.2f} s, one BLAS thread"}
        else:
            one = {"one_site_gate_seconds": u1, "cores": 1,
                   "note": "one BLAS thread, one-site gate only (the two-site gate takes minutes on one thread; "
                           "bench.py --cpu-threads1 times it)"}
    except ImportError:
        pass
    host = ""
    try:
        with open("/proc/cpuinfo") as f:
            host = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": rate, "unit": "gate-layers/s", "cores": cores, "kind": "oracle",
            "sample": f"steady state of the same workload: one two-site noisy gate ({t2:.2f} s) and one one-site "
                      f"noisy gate ({t1:.2f} s) on sites at chi={CHI}, kappa={KAPPA} (complex128 NumPy/LAPACK), "
                      f"scaled to a layer of 15 + 32 gates",
            "host_cpu": host, "one_thread": one, "c5_row": c5_row_seconds(W)}


def c5_row_seconds(W):
    """The oracle's truncated MPDO on one parameter row of the variational
    workload (noisy RY/CZ ansatz n=12, depth 6, chi=32, kappa=4, cutoffs
    1e-10, complex128, every host core): the CPU cost of one MPDO evaluation,
    from which the time-to-fidelity leg estimates the oracle's time to the
    same target (its rows to target times this)."""
    import math
    import numpy as np
    from oracle import channels as OC
    from oracle import mpdo as OM
    n, depth = 12, 6
    th = np.random.default_rng(7611).uniform(0, 2 * math.pi, 2 * n * depth)
    prog = W.ghz_ansatz_noise(n, depth, th, None)
    kr = [OC.kraus_from_chi(c)[0] for c in prog.chis]
    t0 = time.perf_counter()
    o = OM.run_program(prog, OM.MPDO(n, 32, 4, 1e-10, 1e-10), kr)
    o.fidelity_ghz()
    return {"seconds": time.perf_counter() - t0, "cores": blas_threads(),
            "sample": "one parameter row of the n=12 depth-6 ansatz (chi=32, kappa=4, complex128), "
                      "circuit and GHZ fidelity"}


def oracle_error(zz, f, noise_scale=1.0):
    """Error of instance 0 (parameter point 0) against the oracle's truncated
    MPDO of the same circuit, stored by tests/golden/make_c2_reference.py
    (complex128, oracle/ only)."""
    path = os.path.join(ROOT, "tests", "golden", "c2_reference.json")
    try:
        with open(path) as fh:
            ref = json.load(fh)
    except (OSError, ValueError):
        return None
    case = next((c for c in ref["cases"] if c["noise_scale"] == noise_scale and c["param_tag"] == 0), None)
    if case is None:
        return None
    ezz = max(abs(a - b) for a, b in zip(zz, case["zz"]))
    return {"max_abs_err_zz": ezz, "abs_err_ghz_fidelity": abs(f - case["ghz_fidelity"]),
            "reference": "oracle truncated MPDO, complex128 (tests/golden/c2_reference.json)"}


def batched_rate(M, W, ninst, prec, noise_scale=1.0, graph=True, steps=2, warmup=1, depth=DEPTH):
    """gate-layers/s of ninst parameter points of the C2 circuit in one
    mpdo_batch_run per step, and instance 0's <Z_i Z_i+1> and GHZ fidelity."""
    import numpy as np
    import torch
    prog0 = W.ghz_ansatz(N_QUBITS, depth, W.ansatz_params(N_QUBITS, DEPTH, 0), noise_scale=noise_scale)
    chans = [M.Channel(prog0.chis[0], 1), M.Channel(prog0.chis[1], 2)]
    P = np.stack([W.ansatz_params(N_QUBITS, DEPTH, t) for t in range(ninst)])
    progs = [W.ghz_ansatz(N_QUBITS, depth, P[b], noise_scale=noise_scale) for b in range(ninst)]
    pdev = torch.tensor(P, dtype=torch.float64, device="cuda")
    obs = observables(N_QUBITS)
    nobs = obs.shape[0]
    plan = M.BatchPlan(progs, [obs] * ninst, use_params=True)

    def step():
        return M.batch_run(plan, pdev, chans, None, chi_max=CHI, kappa_max=KAPPA, max_kraus=16,
                           svd_cutoff=SVD_CUT, kappa_cutoff=KAP_CUT, prec=prec, use_graph=graph).view(ninst, nobs)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    f = 0.5 * (r[0, -3] + r[0, -2] + 2 * r[0, -1]).real.item()
    return ninst * depth * steps / dt, r[0, : N_QUBITS - 1].real.cpu().tolist(), f


def plain_rate(M, W, prec, noise_scale=1.0):
    """gate-layers/s of one instance of the C2 circuit through per-gate calls."""
    import torch
    prog = W.ghz_ansatz(N_QUBITS, DEPTH, W.ansatz_params(N_QUBITS, DEPTH, 0), noise_scale=noise_scale)
    chans = [M.Channel(prog.chis[0], 1), M.Channel(prog.chis[1], 2)]
    gpu_step(M, W, prog, chans, prec)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f, zz = gpu_step(M, W, prog, chans, prec)
    dt = time.perf_counter() - t0
    return DEPTH / dt, zz, f


def sweep_leg(M, W):
    """Plain (per-gate calls, one instance) against batched (B parameter points
    in one graph-captured mpdo_batch_run) on the C2 circuit, in both precisions,
    noise strengths x1 and x3, with each configuration's error against the
    oracle (instance 0)."""
    out = {"plain": {}, "batched": {}}
    for pname, prec in (("c128", M.C128), ("c64+f64", M.C64_MIXED)):
        for ns in (1.0, 3.0):
            v, zz, f = plain_rate(M, W, prec, ns)
            out["plain"][f"{pname},noise_x{ns:g}"] = {"gate_layers_per_s": v,
                                                       "error_vs_oracle": oracle_error(zz, f, ns)}
        for B in (16, 64, 256):
            for ns in ((1.0, 3.0) if B == 64 else (1.0,)):
                v, zz, f = batched_rate(M, W, B, prec, ns, graph=True, steps=1 if B == 256 else 2)
                out["batched"][f"{pname},B={B},noise_x{ns:g}"] = {"gate_layers_per_s": v,
                                                                  "error_vs_oracle": oracle_error(zz, f, ns)}
    return out


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


def ttf_leg(steps, nsamples=65536, pretrain_steps=6000, seeds=tuple(range(8))):
    """Time to fidelity of the variational GHZ loop (C5: n=12, depth 6,
    chi=32, kappa=4, complex128 MPDO as the verifier).  The surrogate is trained first on
    `nsamples` MPDO-generated samples (theta ~ U[0, 2 pi)^144, noise strengths
    ~ U[0.5, 2]^24, complex64 contractions), then plain parameter-shift Adam
    and the surrogate-assisted loop start from the same random angles; the
    target is 0.9 x F_best, F_best the best fidelity of `steps` plain steps
    from a reference start (the 0.9 target itself is out of reach under this
    noise).  Times are from the start of each optimisation; the data
    generation and pre-training are reported apart, with the number of
    optimisations after which they are repaid."""
    import math
    import numpy as np
    import torch
    from paper_2508_07610_amd import mpdo as M
    from paper_2508_07610_amd import surrogate as S
    from paper_2508_07610_amd import variational as V
    n, depth = 12, 6
    P = 2 * n * depth
    ev = V.AnsatzEvaluator(n, depth, chi_max=32, kappa_max=4)
    ev64 = V.AnsatzEvaluator(n, depth, chi_max=32, kappa_max=4, prec=M.C64_MIXED)
    rng = np.random.default_rng(7620)
    ev64(rng.uniform(0, 2 * math.pi, (4, P)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, Y = V.generate_dataset(ev64, nsamples, rng)
    t_gen = time.perf_counter() - t0
    net = S.MLP(list(S.C5_WIDTHS), max_batch=1024, seed=0)
    pre = V.pretrain(net, X, Y, steps=pretrain_steps)
    params = net.get_params()
    net.close()
    ref = V.plain_optimize(ev, np.random.default_rng(7610).uniform(0, 2 * math.pi, P), target=2.0,
                           max_steps=steps, lr=0.05)
    target = 0.9 * ref["best"]
    runs = []
    for sd in seeds:
        th0 = np.random.default_rng(7611 + sd).uniform(0, 2 * math.pi, P)
        plain = V.plain_optimize(ev, th0, target=target, max_steps=3 * steps, lr=0.05)
        net = S.MLP(list(S.C5_WIDTHS), max_batch=1024, seed=sd)
        net.set_params(params)
        sur = V.surrogate_optimize(ev, net, th0, target=target, max_rows=3 * max(plain["evaluations"], 2000))
        net.close()
        runs.append({"seed": sd, "plain_seconds": plain["time"], "plain_mpdo_rows": plain["rows_to_target"],
                     "surrogate_seconds": sur["time"], "surrogate_mpdo_rows": sur["rows_to_target"],
                     "surrogate_gradients": sur["gradients"], "proposal_rounds": sur["proposal_rounds"],
                     "surrogate_steps_accepted": sur["surrogate_accepted"],
                     "surrogate_abs_err_on_verified": sur["surrogate_abs_err"]})
    ok = [r for r in runs if r["plain_seconds"] and r["surrogate_seconds"]]
    tp = float(np.mean([r["plain_seconds"] for r in ok])) if ok else None
    tsur = float(np.mean([r["surrogate_seconds"] for r in ok])) if ok else None
    rp = float(np.mean([r["plain_mpdo_rows"] for r in ok])) if ok else None
    rsur = float(np.mean([r["surrogate_mpdo_rows"] for r in ok])) if ok else None
    overhead = t_gen + pre["train_seconds"]
    return {"workload": "variational GHZ fidelity, noisy RY/CZ ansatz n=12 depth=6 chi=32 kappa=4, c128 MPDO verifier, "
                        "parameter-shift gradients (289 rows per step in one mpdo_batch_run); surrogate 168-256-256-"
                        "256-12 GELU, bf16 operands, FP32 accumulation, trained by the library's kernels",
            "f_best_plain": ref["best"], "target": target, "runs": runs,
            "mean_plain_seconds": tp, "mean_surrogate_seconds": tsur,
            "mean_plain_mpdo_rows": rp, "mean_surrogate_mpdo_rows": rsur,
            "mean_surrogate_seconds_with_data": (tsur + t_gen + pre["train_seconds"]) if tsur else None,
            "data_generation": {"samples": nsamples, "seconds": t_gen, "precision": "c64 contractions + FP64 truncation"},
            "pretraining": pre,
            "break_even_optimisations": (overhead / (tp - tsur)) if tp and tsur and tp > tsur else None}


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


def eig_lone_leg():
    """Lone Hermitian eigenproblems of the crosstalk workload's sizes (the
    three-site update's N / E3 Grams n = 256 with all vectors, its bond Grams
    n = 512 with chi = 128 vectors, its Gamma n = 1024 with kappa = 16), one
    per launch as the per-gate path issues them: the library's eigensolver
    window (HIP events of the in-library profiler) with the reduction shared
    by several workgroups per matrix (the default for launches of at most 32
    matrices) and with one workgroup per matrix."""
    import numpy as np
    from paper_2508_07610_amd import mpdo as M
    rng = np.random.default_rng(7617)
    out = {}
    for n, kvec in ((256, 256), (512, 128), (1024, 16)):
        X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        A = X @ X.conj().T
        rec = {}
        for coop in (True, False):
            prev = M.eig_coop(coop)
            try:
                for _ in range(2):  # the second call is timed
                    M.profile_enable(True)
                    M.test_eigh(A, kvec)
                    r = M.profile_read(M.PROF_EIG_GLOBAL)
                    M.profile_enable(False)
            finally:
                M.eig_coop(prev)
            rec["shared_ms" if coop else "one_workgroup_ms"] = r["ms"]
        rec["speedup"] = rec["one_workgroup_ms"] / rec["shared_ms"]
        out[f"n={n},vectors={kvec}"] = rec
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
    st = M.MPDO(N_QUBITS, chi_max=CHI, kappa_max=KAPPA, max_kraus=16, svd_cutoff=SVD_CUT, kappa_cutoff=KAP_CUT)
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


def truncation_study_leg(ncirc=1000):
    """Sec. IV.C at the paper's scale: mean Uhlmann fidelity between reference
    and truncated states of random circuits with RZ crosstalk (Q = 3 and 6,
    depth 4), 1,000 circuits per point, over a grid of (chi, kappa); every
    circuit of a point and limit in one mpdo_batch_run_dense, FP64."""
    from paper_2508_07610_amd import truncation_study as TS
    limits = [(2, 2), (4, 4), (8, 8), (16, 4), (16, 16)]
    out = {}
    for q in (3, 6):
        t0 = time.perf_counter()
        r = TS.run_batched(q, 4, limits, ncirc=ncirc)
        out[f"Q={q},depth=4"] = {"fidelity": r["fidelity"], "device_seconds": r["device_seconds"],
                                 "seconds": time.perf_counter() - t0}
    return {"workload": f"{ncirc} random RX/RY/RZ + CNOT circuits per Q, RZ(alpha) crosstalk on the neighbour of "
                        "every CNOT, QPT-style channels, reference at chi=64 kappa=64 (lossless to its own discarded weight), one batched dense "
                        "run per limit", "results": out}


def mitigation_leg(n=16, scale=3.0):
    """Sec. V: the output of a noisy GHZ preparation (H and compiled CNOTs on
    a chain of n qubits, QPT-style channels x`scale` after every gate) mapped
    by the inverse of the noisy process on an MPO of rho, with the circuit's
    own channels as the model (exact: fidelity 1 in closed form) and with a
    standard noise model (thermal relaxation + depolarizing, unified 2q form)
    in their place; GHZ fidelity before and after, and the device time."""
    import torch
    from paper_2508_07610_amd import mitigation as GM
    from paper_2508_07610_amd import mpdo as M
    from paper_2508_07610_amd import workloads as W
    chis = [W.chi_1q_default(scale), W.chi_2q_default(scale)]
    ops = [W.Op((0,), W.H, 0, "h")]
    for q in range(n - 1):
        for name, loc, U in W.cnot_compiled():
            ops.append(W.Op(tuple(q + s for s in loc), U, 0 if len(loc) == 1 else 1, name))
    prog = W.Program(n, ops, chis, 0)
    chans = [M.Channel(chis[0], 1), M.Channel(chis[1], 2)]
    std = [M.Channel(W.chi_standard_1q(3e-3, 0.03, 30.0, 20.0), 1),
           M.Channel(W.chi_unified_2q(3e-2, 0.3, 30.0, 20.0), 2)]
    st = M.MPDO(n, chi_max=64, kappa_max=64, max_kraus=16, svd_cutoff=1e-14, kappa_cutoff=1e-14)
    M.run_program(prog, st, chans)
    f_noisy = st.fidelity_ghz()
    res = {}
    for name, model in (("exact_model", chans), ("standard_model", std)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m = GM.mitigate(prog, st, model, d_max=256, cutoff=1e-12)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        bonds, disc = m.dims()
        res[name] = {"ghz_fidelity": GM.ghz_fidelity(m), "seconds": dt, "max_bond": max(bonds),
                     "discarded": disc}
        m.close()
    nmaps = sum(1 for o in ops if o.chan >= 0) + 2 * (len(ops) - 1)   # inverse channels, U^-1 and U replays
    for r in res.values():
        r["maps"] = nmaps
        r["ms_per_map"] = 1e3 * r["seconds"] / nmaps
    st.close()
    for c in chans + std:
        c.close()
    return {"workload": f"noisy GHZ preparation n={n} (H + {n - 1} compiled CNOTs), QPT-style channels x{scale:g}, "
                        "MPO of rho from the lossless MPDO, d_max=256 cutoff=1e-12, FP64",
            "ghz_fidelity_noisy": f_noisy, "mitigated": res}


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
    # the GEMM sites' settings tuned on this batch (autotune.tune, cached), if
    # the cache holds them; the previous settings are restored afterwards
    from paper_2508_07610_amd import autotune as AT
    key = AT.cache_key(M.C64_MIXED, 128, 16, 16, f"crosstalk n=24 depth=12 nb={nb} eps=1e-4")
    tuned = AT.load(os.path.join(ROOT, "paper_2508_07610_amd", "autotune_cache.json"), key)
    with AT.applied(tuned):
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
                        "autotune": {"cache_key": key, "settings": tuned},
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

        def step(graph=not a.no_graph):
            r = M.batch_run(plan, pdev, chans, None, chi_max=CHI, kappa_max=KAPPA, max_kraus=16,
                            svd_cutoff=SVD_CUT, kappa_cutoff=KAP_CUT, prec=prec, use_graph=graph)
            r = r.view(ninst, nobs)
            f = 0.5 * (r[0, -3] + r[0, -2] + 2 * r[0, -1]).real.item()
            return f, r[0, : N_QUBITS - 1].real.cpu().tolist()
    tune_info = None
    if a.mode == "batched" and not a.no_tune:
        from paper_2508_07610_amd import autotune as AT
        path = os.path.join(ROOT, "paper_2508_07610_amd", "autotune_cache.json")
        key = AT.cache_key(prec, CHI, KAPPA, 16, f"ansatz n={N_QUBITS} depth={a.depth} B={ninst}")
        if a.retune:
            AT.save(path, key, None)
        t_tune = time.perf_counter()
        tune_info = AT.tuned(lambda: step(graph=False), path, key, top=12)
        tune_info["seconds"] = time.perf_counter() - t_tune
        tune_info["cache_key"] = key
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    profiled_timed = not (a.mode == "batched" and not a.no_graph)
    if profiled_timed:
        M.profile_enable(True)
    t0 = time.perf_counter()
    step_s = []
    for _ in range(a.steps):
        ts = time.perf_counter()
        f, zz = step()  # returns host values: each step ends synchronised
        step_s.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if not profiled_timed:
        M.profile_enable(True)
        step(graph=False)
        torch.cuda.synchronize()
    roof, share = roofline(M, prec == M.C128, a.steps if profiled_timed else 1)
    gcls = M.PROF_GEMM_F64 if prec == M.C128 else M.PROF_GEMM_F32
    g = M.profile_read(gcls)
    gemm_tf = g["flops"] / (g["ms"] * 1e-3) / 1e12 if g["ms"] > 0 else 0.0
    gpeak = PEAK["f64_mfma"] if prec == M.C128 else PEAK["f32_mfma"]
    gemm_roof = {"kernel": M.PROF_NAMES[gcls], "bound": "mfma", "achieved": gemm_tf, "peak": gpeak,
                 "unit": "TFLOP/s", "frac": gemm_tf / gpeak, "launches": g["launches"],
                 "avg_launch_ms": g["ms"] / max(1, g["launches"]),
                 "note": "the contraction class, reported beside the dominant class"}
    sites = M.profile_sites()
    M.profile_enable(False)
    ms = 1e3 * dt / a.steps
    value = ninst * a.depth * a.steps / dt
    if a.mode == "plain":
        wl = (f"plain MPDO, noisy RY/CZ ansatz n={N_QUBITS} depth={a.depth} chi={CHI} kappa={KAPPA} "
              f"svd_cutoff={SVD_CUT}, per-gate C-ABI calls, one instance")
    else:
        wl = (f"batched MPDO, {ninst} parameter points of the noisy RY/CZ ansatz n={N_QUBITS} depth={a.depth} "
              f"chi={CHI} kappa={KAPPA} svd_cutoff={SVD_CUT}, one mpdo_batch_run per step"
              + ("" if a.no_graph else " captured in one HIP graph"))
    cpu = None if a.no_cpu else cpu_baseline(W, threads1=a.cpu_threads1)
    ttf = None if a.no_ttf else ttf_leg(a.ttf_steps)
    if cpu and ttf and ttf.get("mean_plain_mpdo_rows"):
        row = cpu["c5_row"]
        ttf["cpu_oracle_estimate"] = {
            "seconds": row["seconds"] * ttf["mean_plain_mpdo_rows"], "cores": row["cores"],
            "note": "the plain optimizer's mean MPDO rows to the target times the oracle's seconds per row "
                    "(cpu_baseline.c5_row): an estimate from one timed row, not a run"}
    out = {
        "metric": "MPDO gate-layers/s (n=16,chi=64,kappa=8) plain vs batched; surrogate time-to-fidelity",
        "value": value, "unit": "gate-layers/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms, "ms_per_step_median": 1e3 * float(np.median(step_s)), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c128" if prec == M.C128 else "c64+f64", "data": "synthetic",
        "config": {"workload": wl, "instances": ninst, "mode": a.mode, "ghz_fidelity_instance0": f,
                   "zz01_instance0": zz[0], "roofline_from": "timed steps" if profiled_timed
                   else "one extra profiled step (graph launches are not profiled)"},
        "error_vs_oracle_instance0": oracle_error(zz, f) if a.depth == DEPTH else None,
        "roofline": roof,
        "gemm_roofline": gemm_roof,
        "kernel_time_ms": share,
        "gemm_sites": {k: {"ms": v["ms"], "launches": v["launches"], "tflops": v["tflops"]} for k, v in sites.items()},
        "autotune": tune_info,
        "sweep": None if a.no_sweep else sweep_leg(M, W),
        "cpu_baseline": cpu,
        "time_to_fidelity": ttf,
        "maxcut_batch": None if a.no_maxcut else maxcut_leg(),
        "gemm_full_tiles": None if a.no_gemm_tiles else gemm_tiles_leg(),
        "eig_lone": None if a.no_eig_lone else eig_lone_leg(),
        "sampling": None if a.no_sampling else sampling_leg(),
        "noise_models": None if a.no_noise_models else noise_models_leg(),
        "truncation_study": None if a.no_truncation_study else truncation_study_leg(),
        "crosstalk": None if a.no_crosstalk else crosstalk_leg(),
        "mitigation": None if a.no_mitigation else mitigation_leg(),
    }
    print(json.dumps(out, default=lambda o: o.item() if hasattr(o, "item") else str(o)))


if __name__ == "__main__":
    main()
