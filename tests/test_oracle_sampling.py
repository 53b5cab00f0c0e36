"""Pins of the measurement oracle (oracle/sampling.py): bitstring
probabilities against a closed form, and the sequential-conditional sampler
against identities it must satisfy and against frequencies."""
import numpy as np
import pytest

from oracle import channels, dense
from oracle import sampling as S
from paper_2508_07610_amd import workloads as W


@pytest.mark.parametrize("n,p", [(3, 0.05), (5, 0.2)])
def test_depolarized_ghz_probabilities_closed_form(n, p):
    """GHZ_n then local depolarizing p (Eq. (3)): each qubit flips with
    probability p/2, so P(z) = [prod_i a(z_i) + prod_i a(1 - z_i)] / 2 with
    a(0) = 1 - p/2, a(1) = p/2."""
    dep = channels.kraus_from_chi(W.chi_from_kraus(W.kraus_depolarizing(p)))[0]
    sim = dense.DenseSim(n)
    g = dense.ghz_state(n)
    sim.rho = np.outer(g, g.conj())
    for q in range(n):
        sim.apply_kraus((q,), dep)
    P = S.basis_probabilities(sim.rho)
    a = {0: 1 - p / 2, 1: p / 2}
    for z in range(1 << n):
        b = S.bits_of(z, n)
        ref = 0.5 * (np.prod([a[x] for x in b]) + np.prod([a[1 - x] for x in b]))
        assert abs(P[z] - ref) < 1e-15
    assert abs(P.sum() - 1) < 1e-14


def test_conditionals_multiply_to_the_joint_probability():
    """The probability returned with a draw is the joint P(z) of the drawn
    string (a wrong marginal axis or normalisation breaks this)."""
    rng = np.random.default_rng(3)
    n = 4
    P = rng.random(1 << n) ** 3
    P /= P.sum()
    for _ in range(200):
        u = rng.random(n)
        bits, pz, _ = S.conditional_sample(P, n, u)
        z = int("".join(map(str, bits)), 2)
        assert abs(pz - P[z]) < 1e-15


def test_product_distribution_conditionals_are_the_marginals():
    """For a product distribution the conditional of qubit i is its own
    marginal, whatever the prefix: the order of the qubits (qubit 0 = MSB)."""
    n = 4
    c = [0.9, 0.3, 0.55, 0.05]  # P(z_i = 0)
    P = np.array([np.prod([c[i] if b == 0 else 1 - c[i] for i, b in enumerate(S.bits_of(z, n))])
                  for z in range(1 << n)])
    rng = np.random.default_rng(4)
    for _ in range(20):
        _, _, q0 = S.conditional_sample(P, n, rng.random(n))
        assert np.allclose(q0, c, atol=1e-15)
    # u below / above the first conditional decides qubit 0
    assert S.conditional_sample(P, n, [0.899, 0, 0, 0])[0][0] == 0
    assert S.conditional_sample(P, n, [0.901, 0, 0, 0])[0][0] == 1


def test_frequencies_follow_the_distribution():
    """40000 seeded draws: every frequency within 5 standard deviations."""
    rng = np.random.default_rng(5)
    n = 3
    P = np.array([0.4, 0.0, 0.1, 0.05, 0.2, 0.15, 0.0, 0.1])
    cnt = np.zeros(1 << n)
    shots = 40000
    for _ in range(shots):
        bits, _, _ = S.conditional_sample(P, n, rng.random(n))
        cnt[int("".join(map(str, bits)), 2)] += 1
    f = cnt / shots
    sd = np.sqrt(P * (1 - P) / shots)
    assert np.all(np.abs(f - P) <= 5 * sd + 1e-12)
    assert cnt[1] == 0 and cnt[6] == 0  # zero-probability strings are never drawn
