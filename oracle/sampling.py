"""Oracle: computational-basis measurement of a density matrix (test
infrastructure: only tests/, __graft_entry__.smoke() and bench.py's CPU
baseline use oracle/).

Written from the paper's comparison of bitstring distributions (Sec. IV.A,
Fig. `fig_exp2`): the probability of a bitstring z is the diagonal entry <z|rho|z>,
and two distributions are compared by the Jensen-Shannon divergence of
Eq. (18) (`oracle.dense.jsd`).  Sampling draws
qubit after qubit from its conditional distribution given the bits already
drawn; the uniform numbers are inputs, so a draw can be replayed exactly.
Qubit 0 is the most significant bit of a dense index.
"""
import numpy as np


def basis_probabilities(rho):
    """P(z) = <z|rho|z> / Tr rho for every z (index = bitstring, qubit 0 the MSB)."""
    d = np.real(np.diag(np.asarray(rho)))
    return d / d.sum()


def bits_of(index, n):
    """The bitstring of a dense index, qubit 0 first."""
    return [(index >> (n - 1 - i)) & 1 for i in range(n)]


def conditional_sample(prob, n, u):
    """Sequential conditionals: with p = P(z_0 .. z_{i-1}, z_i = 0) and
    q = P(z_0 .. z_{i-1}, z_i = 1) (marginals of the full distribution over
    the remaining qubits), bit i is 0 when u[i] < p / (p + q), else 1.
    Returns the bits and the probability of the drawn string, which is the
    product of the chosen conditionals.  Also returns, per qubit, the
    conditional P(z_i = 0 | prefix) used in the decision."""
    P = np.asarray(prob, dtype=np.float64).reshape((2,) * n)
    bits, q0s = [], []
    pz = 1.0
    marg = P
    for i in range(n):
        # sum out the qubits after i
        m = marg.reshape(2, -1).sum(axis=1)
        tot = m[0] + m[1]
        c0 = m[0] / tot
        b = 0 if u[i] < c0 else 1
        bits.append(b)
        q0s.append(c0)
        pz *= (m[b] / tot)
        marg = marg[b]
    return bits, pz, q0s
