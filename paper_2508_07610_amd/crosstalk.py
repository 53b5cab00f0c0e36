"""Crosstalk workload: random circuits with three-site crosstalk channels and
Kraus pruning by weight (Sec. III, Fig. randomCirc_fig(b)).

A 1D random circuit (random RX/RY/RZ layers and a CNOT brick compiled to
RY . CZ . RY) with the two-site channel after every CZ and a random CPTP
three-site channel on the neighbouring triple.  The same circuit runs once
for every pruning threshold eps; the Kraus sets of the three-site channels
keep the operators above weight eps (Eq. (16) and the weight rule), and the
results are compared with the eps = 0 run.  Everything runs through the C ABI
(argument marshalling only).
"""
from __future__ import annotations

import dataclasses
import time
from typing import Dict, List, Sequence

import numpy as np

from . import mpdo as M
from .distributions import all_bitstrings, jsd  # noqa: F401 (re-exported)
from . import workloads as W


def circuit(n: int, depth: int, seed_tag: int = 0):
    """The random circuit with two distinct three-site channels (seeded)."""
    rng = W.rng_for(7000 + seed_tag)
    chi3 = [W.random_cptp_near_identity_3q(rng) for _ in range(2)]
    return W.random_circuit(n, depth, rng, chi2=W.chi_2q_default(), chi3=chi3)


def z_products(n: int) -> np.ndarray:
    """<Z_i> (n entries) then <Z_i Z_i+1> (n - 1 entries) as product operators."""
    I, Z = np.eye(2, dtype=np.complex128), np.diag([1.0, -1.0]).astype(np.complex128)
    ops = []
    for i in range(n):
        o = np.stack([I] * n)
        o[i] = Z
        ops.append(o)
    for i in range(n - 1):
        o = np.stack([I] * n)
        o[i] = o[i + 1] = Z
        ops.append(o)
    return np.stack(ops)


def uhlmann_fidelity(rho: np.ndarray, sigma: np.ndarray) -> float:
    """F(rho, sigma) = (Tr sqrt(sqrt(rho) sigma sqrt(rho)))^2 (the fidelity the
    paper uses to compare truncated and untruncated states), for two dense
    density matrices of unit trace; a host-side measurement of results."""
    w, v = np.linalg.eigh((rho + rho.conj().T) / 2)
    w = np.where(w > 1e-12 * w.max(), w, 0.0)          # rounding-level eigenvalues are zero
    sq = (v * np.sqrt(w)) @ v.conj().T
    mid = sq @ ((sigma + sigma.conj().T) / 2) @ sq
    ev = np.linalg.eigvalsh((mid + mid.conj().T) / 2)
    ev = np.where(ev > 1e-12 * ev.max(), ev, 0.0)
    return float(np.sum(np.sqrt(ev)) ** 2)


def run(n: int = 24, depth: int = 12, chi_max: int = 128, kappa_max: int = 16,
        eps_list: Sequence[float] = (0.0, 1e-4, 1e-3), prec: int = M.C64_MIXED,
        seed_tag: int = 0, dense: bool = False) -> List[Dict]:
    """One run per eps; returns per eps the Kraus counts of the channels, the
    wall time, the summed discarded weight, the observables and their largest
    deviation from the eps = 0 run (the first entry of eps_list).  With
    `dense` (n <= 12) also the dense state of each run (trace-normalised), its
    fidelity with the first run's, the bitstring distribution
    (mpdo_probabilities) and its Jensen-Shannon divergence from the first
    run's."""
    import torch
    prog = circuit(n, depth, seed_tag)
    qs = [int(round(np.log(c.shape[0]) / np.log(4))) for c in prog.chis]
    obs = z_products(n)
    out: List[Dict] = []
    ref = None
    for eps in eps_list:
        chans = [M.Channel(c, q, eps=eps if q == 3 else 0.0) for c, q in zip(prog.chis, qs)]
        mk = max(ch.nkraus for ch in chans)
        st = M.MPDO(n, chi_max=chi_max, kappa_max=kappa_max, max_kraus=mk, svd_cutoff=1e-10,
                    kappa_cutoff=1e-10, prec=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        M.run_program(prog, st, chans)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        vals = st.expect_products(obs).real
        bonds, inner, disc = st.dims()
        rec = {"eps": eps, "kraus": [ch.nkraus for ch in chans], "seconds": dt, "discarded": disc,
               "max_bond": max(bonds), "max_inner": max(inner), "trace": st.trace(), "obs": vals,
               "min_gap": st.stats()["min_gap"]}
        if dense:
            rho = st.to_dense()
            rec["rho"] = rho / np.trace(rho).real
            rec["probs"] = st.probabilities(all_bitstrings(n))
        if ref is None:
            ref = vals
            rho0 = rec.get("rho")
            p0 = rec.get("probs")
        rec["max_dev_vs_eps0"] = float(np.abs(vals - ref).max())
        if dense:
            rec["fidelity_vs_eps0"] = uhlmann_fidelity(rho0, rec["rho"])
            rec["jsd_vs_eps0"] = jsd(p0, rec["probs"])
        out.append(rec)
        st.close()
        for ch in chans:
            ch.close()
    return out


def run_batch(nb: int = 16, n: int = 24, depth: int = 12, chi_max: int = 128, kappa_max: int = 16,
              eps: float = 1e-4, prec: int = M.C64_MIXED) -> Dict:
    """nb seeded instances of the crosstalk circuit (seed tags 0 .. nb-1, each
    with its own pair of three-site channels) in one mpdo_batch_run: the
    two-site channel is shared, the three-site channels of instance b are
    channels 1 + 2b and 2 + 2b.  Returns the wall time, the observables
    (<Z_i>, <Z_i Z_i+1> per instance) and the library's per-class kernel
    profile of the run."""
    import torch
    circs = [circuit(n, depth, t) for t in range(nb)]
    chis = [circs[0].chis[0]]
    progs = []
    for b, pr in enumerate(circs):
        assert np.array_equal(pr.chis[0], chis[0])
        chis.extend(pr.chis[1:])
        ops = [dataclasses.replace(o, chan=-1 if o.chan < 0 else (0 if o.chan == 0 else o.chan + 2 * b))
               for o in pr.ops]
        progs.append(W.Program(pr.n, ops, [], pr.layers))
    qs = [int(round(np.log(c.shape[0]) / np.log(4))) for c in chis]
    chans = [M.Channel(c, q, eps=eps if q == 3 else 0.0) for c, q in zip(chis, qs)]
    mk = max(ch.nkraus for ch in chans)
    obs = [z_products(n)] * nb
    kw = dict(chi_max=chi_max, kappa_max=kappa_max, max_kraus=mk, svd_cutoff=1e-10, kappa_cutoff=1e-10, prec=prec)
    M.batch_run(progs, None, chans, obs, use_graph=False, **kw)  # warm-up (workspace sizing)
    torch.cuda.synchronize()
    M.profile_enable(True)
    t0 = time.perf_counter()
    out = M.batch_run(progs, None, chans, obs, use_graph=False, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = {M.PROF_NAMES[c]: M.profile_read(c) for c in M.PROF_NAMES}
    M.profile_enable(False)
    vals = out.cpu().numpy().real.reshape(nb, -1)
    kraus = [ch.nkraus for ch in chans[:3]]
    for ch in chans:
        ch.close()
    return {"seconds": dt, "obs": vals, "profile": prof, "kraus": kraus}
