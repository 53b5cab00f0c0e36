"""Seeded synthetic inputs shared by the GPU path, the benchmarks and the tests.

This module only *builds inputs*: gate matrices, Kraus sets of textbook
noise channels, the Pauli-basis process matrix chi of such a channel (the
quantity quantum process tomography reports, Sec. III, Eq. (12)), circuit
programs and random graphs.  It holds none of the simulator's arithmetic:
turning chi into Kraus operators (Eqs. (13)-(16)), applying channels to a
matrix product density operator and truncating it live in the library (GPU)
and, independently, in the oracle (CPU).

Conventions
-----------
* Qubit 0 is the leftmost site and the most significant bit of a dense index.
* Pauli order I, X, Y, Z.  A q-qubit Pauli index is m = sum_t m_t 4**(q-1-t)
  with t = 0 the lowest site.
* R_P(theta) = exp(-i theta P / 2); CZ = diag(1, 1, 1, -1).
* Two-qubit matrices act on (s1 s2) with s1 the lower site.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
PAULI = (I2, X, Y, Z)
PAULI_CHARS = "IXYZ"
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)
CZ = np.diag([1, 1, 1, -1]).astype(np.complex128)
SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]],
                dtype=np.complex128)

SEED_BASE = 7610


def rng_for(tag: int) -> np.random.Generator:
    """Seeded generator; `tag` distinguishes instances of one workload."""
    return np.random.default_rng(SEED_BASE + int(tag))


# ----------------------------------------------------------------------------
# gates
# ----------------------------------------------------------------------------

def rot(P: np.ndarray, theta: float) -> np.ndarray:
    """exp(-i theta P / 2) for an involutory P (P @ P = I)."""
    d = P.shape[0]
    return math.cos(theta / 2) * np.eye(d, dtype=np.complex128) - 1j * math.sin(theta / 2) * P


def rx(t: float) -> np.ndarray:
    return rot(X, t)


def ry(t: float) -> np.ndarray:
    return rot(Y, t)


def rz(t: float) -> np.ndarray:
    return rot(Z, t)


def zz_rot(phi: float) -> np.ndarray:
    """exp(-i phi Z(x)Z / 2): the coherent ZZ crosstalk unitary."""
    return rot(np.kron(Z, Z), phi)


def qaoa_cost(gamma: float) -> np.ndarray:
    """exp(-i gamma (1 - Z Z) / 2), the per-edge cost unitary of Eq. (21)."""
    zz = np.array([1.0, -1.0, -1.0, 1.0])
    return np.diag(np.exp(-1j * gamma * (1.0 - zz) / 2.0)).astype(np.complex128)


def qaoa_mixer(beta: float) -> np.ndarray:
    """exp(-i beta X), the per-qubit mixer of Eq. (21)."""
    return rot(X, 2.0 * beta)


def cnot_compiled() -> List[Tuple[str, Tuple[int, ...], np.ndarray]]:
    """CNOT(control = first site) as RY(-pi/2) on the target, CZ, RY(pi/2) on
    the target (Fig. fig_compileCX).  Returned as a gate list on local sites
    (0 = control, 1 = target), applied in order."""
    return [("u1", (1,), ry(-math.pi / 2)), ("u2", (0, 1), CZ.copy()), ("u1", (1,), ry(math.pi / 2))]


# ----------------------------------------------------------------------------
# textbook channels (Kraus sets) and their Pauli process matrices
# ----------------------------------------------------------------------------

def kraus_depolarizing(p: float) -> List[np.ndarray]:
    """(1-p) rho + p I/2, Eq. (3): sqrt(1-3p/4) I and sqrt(p/4) X, Y, Z."""
    return [math.sqrt(1 - 3 * p / 4) * I2, math.sqrt(p / 4) * X, math.sqrt(p / 4) * Y,
            math.sqrt(p / 4) * Z]


def kraus_depolarizing2(p: float) -> List[np.ndarray]:
    """(1-p) rho + p I/4 on two qubits: sqrt(1-15p/16) I(x)I and sqrt(p/16) on
    each of the 15 non-identity Pauli pairs."""
    ks = []
    for a in range(4):
        for b in range(4):
            w = 1 - 15 * p / 16 if (a == 0 and b == 0) else p / 16
            ks.append(math.sqrt(w) * np.kron(PAULI[a], PAULI[b]))
    return ks


def kraus_amplitude_damping(gamma: float) -> List[np.ndarray]:
    k0 = np.array([[1, 0], [0, math.sqrt(1 - gamma)]], dtype=np.complex128)
    k1 = np.array([[0, math.sqrt(gamma)], [0, 0]], dtype=np.complex128)
    return [k0, k1]


def kraus_unitary(U: np.ndarray) -> List[np.ndarray]:
    return [np.asarray(U, dtype=np.complex128)]


def compose(first: Sequence[np.ndarray], then: Sequence[np.ndarray]) -> List[np.ndarray]:
    """Kraus set of the channel `then` o `first`."""
    return [b @ a for a in first for b in then]


def pauli_basis(q: int) -> List[np.ndarray]:
    """Unnormalised q-qubit Pauli operators in index order m = sum m_t 4**(q-1-t)."""
    basis = [np.ones((1, 1), dtype=np.complex128)]
    for _ in range(q):
        basis = [np.kron(b, p) for b in basis for p in PAULI]
    return basis


def chi_from_kraus(kraus: Sequence[np.ndarray]) -> np.ndarray:
    """Process matrix in the unnormalised Pauli basis:
    eps(rho) = sum_mn chi_mn sigma_m rho sigma_n^dagger  (Eq. (12)).
    Expanding K_i = sum_m c_im sigma_m with c_im = Tr(sigma_m^dag K_i) / d gives
    chi_mn = sum_i c_im conj(c_in)."""
    d = kraus[0].shape[0]
    q = int(round(math.log2(d)))
    basis = pauli_basis(q)
    c = np.array([[np.trace(s.conj().T @ K) / d for s in basis] for K in kraus])
    return c.T @ c.conj()


def chi_1q_default(scale: float = 1.0) -> np.ndarray:
    """Synthetic 1q QPT channel: depolarizing p=1e-3, then amplitude damping
    gamma=2e-3, then a Z over-rotation of 0.01 rad; strengths times `scale`."""
    ks = compose(kraus_depolarizing(1e-3 * scale), kraus_amplitude_damping(2e-3 * scale))
    ks = compose(ks, kraus_unitary(rz(0.01 * scale)))
    return chi_from_kraus(ks)


def chi_2q_default(scale: float = 1.0) -> np.ndarray:
    """Synthetic 2q QPT channel: ZZ crosstalk rotation of 0.02 rad, then 2q
    depolarizing p=1e-2; strengths times `scale`."""
    ks = compose(kraus_unitary(zz_rot(0.02 * scale)), kraus_depolarizing2(1e-2 * scale))
    return chi_from_kraus(ks)


# ----------------------------------------------------------------------------
# standard (non-QPT) noise models of the circuit model (Sec. II.B, Fig.
# `fig_unifiedNoise`): thermal relaxation over a gate duration, depolarizing
# after the gate, state-preparation and measurement flips; emitted as the same
# Pauli chi-matrices the QPT channels use, so either kind drives the simulator.
# ----------------------------------------------------------------------------

def kraus_phase_damping(lam: float) -> List[np.ndarray]:
    """Pure dephasing: diag(1, sqrt(1-lam)) and diag(0, sqrt(lam)); the
    coherence rho_01 shrinks by sqrt(1-lam)."""
    return [np.diag([1.0, math.sqrt(1 - lam)]).astype(np.complex128),
            np.diag([0.0, math.sqrt(lam)]).astype(np.complex128)]


def kraus_bit_flip(p: float) -> List[np.ndarray]:
    """X with probability p (the SPAM preparation error of the unified model)."""
    return [math.sqrt(1 - p) * I2, math.sqrt(p) * X]


def kraus_thermal_relaxation(t: float, T1: float, T2: float) -> List[np.ndarray]:
    """Thermal relaxation over a duration t (T2 <= 2 T1): amplitude damping
    gamma = 1 - exp(-t/T1), then pure dephasing with exp(-t/T_phi),
    1/T_phi = 1/T2 - 1/(2 T1), so that P(1) decays as exp(-t/T1) and the
    coherence as exp(-t/T2)."""
    if T2 > 2 * T1:
        raise ValueError("thermal relaxation needs T2 <= 2 T1")
    gamma = 1 - math.exp(-t / T1)
    rphi = 1 / T2 - 1 / (2 * T1)
    lam = 1 - math.exp(-2 * t * rphi)
    return compose(kraus_amplitude_damping(gamma), kraus_phase_damping(lam))


def kron_kraus(a: Sequence[np.ndarray], b: Sequence[np.ndarray]) -> List[np.ndarray]:
    """Kraus set of the product channel a (x) b (a on the first qubit)."""
    return [np.kron(x, y) for x in a for y in b]


def chi_standard_1q(p_dep: float, t: float, T1: float, T2: float) -> np.ndarray:
    """One-qubit gate noise of the standard models: thermal relaxation over
    the gate time t, then depolarizing p_dep after the gate."""
    return chi_from_kraus(compose(kraus_thermal_relaxation(t, T1, T2), kraus_depolarizing(p_dep)))


def chi_unified_2q(p_dep: float, t: float, T1: float, T2: float, target: int = 1) -> np.ndarray:
    """Two-qubit gate noise of the unified model (Fig. `fig_unifiedNoise`(b)):
    thermal relaxation on both qubits over the gate time t, then depolarizing
    p_dep on the target qubit only (target 0 or 1 of the pair)."""
    trc = kraus_thermal_relaxation(t, T1, T2)
    dep = kraus_depolarizing(p_dep)
    idk = [I2.copy()]
    dep2 = kron_kraus(idk, dep) if target == 1 else kron_kraus(dep, idk)
    return chi_from_kraus(compose(kron_kraus(trc, trc), dep2))


def chi_ideal_noisy_2q(p_dep: float, t: float, T1: float, T2: float) -> np.ndarray:
    """Two-qubit gate noise of the general model (Fig. `fig_unifiedNoise`(c)):
    thermal relaxation over t, then depolarizing p_dep, on both qubits."""
    one = compose(kraus_thermal_relaxation(t, T1, T2), kraus_depolarizing(p_dep))
    return chi_from_kraus(kron_kraus(one, one))


def with_channels(prog: "Program", chi1: np.ndarray, chi2: np.ndarray) -> "Program":
    """The same gates with every one-qubit gate followed by chi1 and every
    two-qubit gate by chi2 (channels 0 and 1 of the returned program)."""
    ops = [dataclasses.replace(o, chan=-1 if o.chan < 0 else (0 if len(o.sites) == 1 else 1)) for o in prog.ops]
    return Program(prog.n, ops, [chi1, chi2], prog.layers)


def random_cptp_near_identity_3q(rng: np.random.Generator, spread: float = 1e-2) -> np.ndarray:
    """3-qubit CPTP map close to the identity, as a Pauli chi-matrix (64x64).
    A0 = exp(-i eps H) with H a GUE matrix of scale 1e-2; A_1..A_63 Ginibre
    matrices of Frobenius norm sqrt(w_i) with weights w_i proportional to
    10**(-4u), u ~ U[0,1], summing to `spread`; the set is made trace
    preserving by K_i = A_i S^(-1/2), S = sum A_i^dag A_i."""
    d = 8
    g = (rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))) / math.sqrt(2)
    herm = (g + g.conj().T) / 2
    w, v = np.linalg.eigh(herm)
    a0 = (v * np.exp(-1j * 1e-2 * w)) @ v.conj().T
    u = rng.uniform(size=63)
    wts = 10.0 ** (-4 * u)
    wts *= spread / wts.sum()
    As = [a0]
    for wi in wts:
        gi = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
        As.append(math.sqrt(wi) * gi / np.linalg.norm(gi))
    S = sum(A.conj().T @ A for A in As)
    ev, evec = np.linalg.eigh(S)
    s_inv_half = (evec * (1.0 / np.sqrt(ev))) @ evec.conj().T
    return chi_from_kraus([A @ s_inv_half for A in As])


# ----------------------------------------------------------------------------
# circuit programs
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Op:
    """One noisy gate: an ideal unitary U on `sites` (ascending, adjacent)
    followed by the channel `chan` (an index into Program.chis, or -1)."""
    sites: Tuple[int, ...]
    U: np.ndarray
    chan: int = -1
    kind: str = ""          # gate name, informational
    param: int = -1         # index into the parameter vector, or -1
    pscale: float = 1.0     # angle = pscale * params[param] (informational)


@dataclasses.dataclass
class Program:
    n: int
    ops: List[Op]
    chis: List[np.ndarray]
    layers: int = 0

    def sublayers(self) -> List[List[Op]]:
        """Greedy split into groups of ops on pairwise disjoint sites,
        preserving the order of ops that share a site."""
        groups: List[List[Op]] = []
        busy: List[set] = []
        last_group_of_site = {}
        for op in self.ops:
            g = 1 + max((last_group_of_site.get(s, -1) for s in op.sites), default=-1)
            while g < len(groups) and any(s in busy[g] for s in op.sites):
                g += 1
            if g == len(groups):
                groups.append([])
                busy.append(set())
            groups[g].append(op)
            busy[g].update(op.sites)
            for s in op.sites:
                last_group_of_site[s] = g
        return groups


def ansatz_params(n: int, depth: int, tag: int = 0) -> np.ndarray:
    """theta ~ U[0, 2pi): 2 n angles per layer (two RY sublayers)."""
    return rng_for(tag).uniform(0.0, 2 * math.pi, size=2 * n * depth)


def ghz_ansatz(n: int, depth: int, theta: np.ndarray, noise_scale: float = 1.0,
               noisy: bool = True) -> Program:
    """Layer = RY(all) -> CZ(0,1),(2,3),... -> RY(all) -> CZ(1,2),(3,4),...,
    each gate followed by the synthetic QPT channel of its arity."""
    chis = [chi_1q_default(noise_scale), chi_2q_default(noise_scale)] if noisy else []
    c1, c2 = (0, 1) if noisy else (-1, -1)
    ops: List[Op] = []
    k = 0
    for _ in range(depth):
        for parity in (0, 1):
            for q in range(n):
                ops.append(Op((q,), ry(float(theta[k])), c1, "ry", k))
                k += 1
            for q in range(parity, n - 1, 2):
                ops.append(Op((q, q + 1), CZ.copy(), c2, "cz"))
    return Program(n, ops, chis, depth)


def random_3_regular(n: int, rng: np.random.Generator, max_tries: int = 1000) -> List[Tuple[int, int]]:
    """Random simple 3-regular graph on n (even) vertices by the pairing model
    with rejection of loops and multi-edges."""
    if n % 2 or n < 4:
        raise ValueError("3-regular graphs need an even n >= 4")
    for _ in range(max_tries):
        stubs = np.repeat(np.arange(n), 3)
        rng.shuffle(stubs)
        pairs = stubs.reshape(-1, 2)
        edges = set()
        ok = True
        for a, b in pairs:
            a, b = int(a), int(b)
            if a == b or (min(a, b), max(a, b)) in edges:
                ok = False
                break
            edges.add((min(a, b), max(a, b)))
        if ok:
            return sorted(edges)
    raise RuntimeError("pairing model failed")


def qaoa_swap_network(n: int, edges: Sequence[Tuple[int, int]], gammas: Sequence[float],
                      betas: Sequence[float], noise_scale: float = 1.0,
                      noisy: bool = True) -> Tuple[Program, List[int]]:
    """QAOA (Eqs. (21)-(22)) on a line via an odd-even transposition SWAP network.

    H on every qubit; per level l: the network of n rounds of adjacent SWAPs,
    each fused with the edge's cost phase when the two logical qubits it
    exchanges share an edge (an edge is applied once, when first adjacent),
    then the mixer exp(-i beta X) on every site.  Every two-site gate is
    followed by the 2q channel, every 1q gate by the 1q channel.  Levels
    alternate the direction of the network so the logical order returns.
    Gate angles refer to the parameter row (gamma_1, beta_1, gamma_2, ...):
    cost gates read index 2 l, mixers index 2 l + 1 (angle 2 beta).
    Returns the program and the final map position -> logical qubit."""
    chis = [chi_1q_default(noise_scale), chi_2q_default(noise_scale)] if noisy else []
    c1, c2 = (0, 1) if noisy else (-1, -1)
    eset = {(min(a, b), max(a, b)) for a, b in edges}
    ops: List[Op] = [Op((q,), H.copy(), c1, "h") for q in range(n)]
    pos = list(range(n))  # pos[site] = logical qubit
    for lvl, (g, b) in enumerate(zip(gammas, betas)):
        done = set()
        for rnd in range(n):
            start = rnd % 2
            for s in range(start, n - 1, 2):
                a, c = pos[s], pos[s + 1]
                key = (min(a, c), max(a, c))
                if key in eset and key not in done:
                    ops.append(Op((s, s + 1), SWAP @ qaoa_cost(g), c2, "swapzz", 2 * lvl, 1.0))
                    done.add(key)
                else:
                    ops.append(Op((s, s + 1), SWAP.copy(), c2, "swap"))
                pos[s], pos[s + 1] = c, a
        missing = eset - done
        if missing:
            raise RuntimeError(f"swap network missed edges {missing}")
        for q in range(n):
            ops.append(Op((q,), qaoa_mixer(b), c1, "mix", 2 * lvl + 1, 2.0))
    return Program(n, ops, chis, len(gammas)), pos


def random_circuit(n: int, depth: int, rng: np.random.Generator,
                   chi2: Optional[np.ndarray] = None,
                   chi3: Optional[Sequence[np.ndarray]] = None) -> Program:
    """Random 1D circuit: random RX/RY/RZ with angle U(0, 2pi] on every qubit,
    then a CNOT brick (even pairs on even layers, odd pairs on odd layers)
    compiled to RY(-pi/2) . CZ . RY(pi/2); repeated `depth` times, then a
    final 1q layer.  After each CZ: the 2q channel `chi2` (if given), then
    the 3q channel chi3[k] on the neighbouring triple (i, i+1, i+2), or
    (i-1, i, i+1) at the right edge (if given)."""
    chis: List[np.ndarray] = []
    c2 = -1
    if chi2 is not None:
        chis.append(chi2)
        c2 = 0
    c3base = len(chis)
    if chi3 is not None:
        chis.extend(chi3)
    gates = (rx, ry, rz)
    ops: List[Op] = []
    k3 = 0

    def one_q_layer():
        for q in range(n):
            g = gates[int(rng.integers(0, 3))]
            ops.append(Op((q,), g(float(2 * math.pi - rng.uniform(0, 2 * math.pi))), -1, "r"))

    for d in range(depth):
        one_q_layer()
        for q in range(d % 2, n - 1, 2):
            ops.append(Op((q + 1,), ry(-math.pi / 2), -1, "ry-"))
            ops.append(Op((q, q + 1), CZ.copy(), c2, "cz"))
            ops.append(Op((q + 1,), ry(math.pi / 2), -1, "ry+"))
            if chi3 is not None and n >= 3:
                trip = (q, q + 1, q + 2) if q + 2 < n else (q - 1, q, q + 1)
                ops.append(Op(trip, np.eye(8, dtype=np.complex128), c3base + (k3 % len(chi3)), "xtalk"))
                k3 += 1
    one_q_layer()
    return Program(n, ops, chis, depth)


def pauli_string(n: int, terms: dict) -> str:
    s = ["I"] * n
    for q, c in terms.items():
        s[q] = c
    return "".join(s)


def pauli_ops(s: str) -> np.ndarray:
    """The product operator of a Pauli string as per-site 2x2 factors,
    shape (n, 2, 2) (an observable row of a batch run)."""
    return np.stack([PAULI[PAULI_CHARS.index(c)] for c in s]).astype(np.complex128)


def zz_strings(n: int) -> List[str]:
    return [pauli_string(n, {i: "Z", i + 1: "Z"}) for i in range(n - 1)]


# ----------------------------------------------------------------------------
# per-gate noise strengths (surrogate inputs)
# ----------------------------------------------------------------------------
NOISE_LEVELS = 33
_LOG_LO, _LOG_HI = math.log(0.25), math.log(4.0)


def noise_level_scale(i: int) -> float:
    """Channel strength multiplier of level i: a log grid on [1/4, 4]; level 16 is exactly 1."""
    return math.exp(_LOG_LO + (_LOG_HI - _LOG_LO) * i / (NOISE_LEVELS - 1))


def noise_levels(s: np.ndarray) -> np.ndarray:
    """Nearest level of each strength multiplier (clipped to [1/4, 4])."""
    x = (np.log(np.clip(s, 0.25, 4.0)) - _LOG_LO) / (_LOG_HI - _LOG_LO) * (NOISE_LEVELS - 1)
    return np.clip(np.rint(x), 0, NOISE_LEVELS - 1).astype(np.int32)


def gate_noise_levels(n: int, noise: Optional[np.ndarray]) -> Tuple[np.ndarray, np.ndarray]:
    """The 2n noise inputs -- n per-qubit scales of the 1q channel, n - 1
    per-bond scales of the 2q channel, one global scale -- as channel levels
    of every qubit's 1q gates and every bond's CZ."""
    if noise is None:
        noise = np.ones(2 * n)
    noise = np.asarray(noise, dtype=np.float64)
    return noise_levels(noise[:n] * noise[-1]), noise_levels(noise[n:2 * n - 1] * noise[-1])


def ghz_ansatz_noise(n: int, depth: int, theta: np.ndarray, noise: Optional[np.ndarray]) -> Program:
    """ghz_ansatz with per-gate channel strengths: chis holds the 1q channels of
    all levels, then the 2q channels of all levels; op.chan selects them."""
    l1, l2 = gate_noise_levels(n, noise)
    chis = ([chi_1q_default(noise_level_scale(i)) for i in range(NOISE_LEVELS)]
            + [chi_2q_default(noise_level_scale(i)) for i in range(NOISE_LEVELS)])
    ops: List[Op] = []
    k = 0
    for _ in range(depth):
        for parity in (0, 1):
            for q in range(n):
                ops.append(Op((q,), ry(float(theta[k])), int(l1[q]), "ry", k))
                k += 1
            for q in range(parity, n - 1, 2):
                ops.append(Op((q, q + 1), CZ.copy(), NOISE_LEVELS + int(l2[q]), "cz"))
    return Program(n, ops, chis, depth)


def z_pair_products(n: int, pairs) -> np.ndarray:
    """(len(pairs), n, 2, 2): the product operators Z_a Z_b of `pairs`."""
    I2_, Z_ = np.eye(2, dtype=np.complex128), np.diag([1.0, -1.0]).astype(np.complex128)
    ops = np.zeros((len(pairs), n, 2, 2), dtype=np.complex128)
    for k, (a, b) in enumerate(pairs):
        for s in range(n):
            ops[k, s] = Z_ if s in (a, b) else I2_
    return ops


def ghz_terms(n: int) -> np.ndarray:
    """The three product operators of the GHZ fidelity: |0><0|^n, |1><1|^n
    and |0><1|^n (F = (t0 + t1) / 2 + Re t2)."""
    p0, p1 = np.diag([1.0, 0.0]), np.diag([0.0, 1.0])
    up = np.array([[0, 1], [0, 0]], dtype=np.complex128)
    return np.stack([np.stack([m.astype(np.complex128)] * n) for m in (p0, p1, up)])


def maxcut_batch_instances(n_ghz: int = 256, n_qaoa: int = 128, depth: int = 6, seed_tag: int = 0):
    """The mixed batch of variational GHZ points and QAOA MaxCut instances:
    `n_ghz` parameter points of the noisy RY/CZ ansatz (n = 12, `depth`
    layers) and `n_qaoa` QAOA p = 2 instances on random 3-regular graphs with
    n drawn from {8, 10, ..., 20}, edges routed through the odd-even SWAP
    network.  Returns the programs, the parameter matrix (rows padded with
    zeros), the observables (<Z_i Z_i+1> and the GHZ fidelity terms of the
    ansatz points, <Z_a Z_b> of every graph edge) and per-instance info."""
    progs, params, obs, info = [], [], [], []
    for t in range(n_ghz):
        th = ansatz_params(12, depth, 100000 * (seed_tag + 1) + t)
        progs.append(ghz_ansatz(12, depth, th))
        params.append(th)
        obs.append(np.concatenate([z_pair_products(12, [(i, i + 1) for i in range(11)]), ghz_terms(12)]))
        info.append({"kind": "ghz", "n": 12})
    rng = rng_for(9000 + seed_tag)
    for t in range(n_qaoa):
        n = int(rng.choice(np.arange(8, 21, 2)))
        edges = random_3_regular(n, rng)
        gb = rng.uniform(0, math.pi, size=4)
        prog, pos = qaoa_swap_network(n, edges, gb[0::2], gb[1::2])
        where = {lq: s for s, lq in enumerate(pos)}
        progs.append(prog)
        params.append(gb)
        obs.append(z_pair_products(n, [(where[u], where[v]) for u, v in edges]))
        info.append({"kind": "qaoa", "n": n, "edges": len(edges)})
    width = max(len(p) for p in params)
    P = np.zeros((len(params), width))
    for b, p in enumerate(params):
        P[b, : len(p)] = p
    return progs, P, obs, info
