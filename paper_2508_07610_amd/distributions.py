"""Host-side analysis of bitstring distributions (results of
mpdo_probabilities / mpdo_sample): the Jensen-Shannon divergence the paper
uses to compare distributions (Sec. IV.A, Eq. (18)), the bit order of dense
indices, and read-out flips (the measurement error of the standard noise
models, Sec. II.B)."""
from __future__ import annotations

import numpy as np


def jsd(p: np.ndarray, q: np.ndarray) -> float:
    """Jensen-Shannon divergence of two bitstring distributions, Eq. (18):
    half the summed Kullback-Leibler divergences (natural logarithm) of P and
    Q from their midpoint M = (P + Q) / 2, empty bins contributing nothing."""
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    mid = 0.5 * (p + q)
    out = 0.0
    for a in (p, q):
        keep = a > 0
        out += 0.5 * float(np.dot(a[keep], np.log(a[keep] / mid[keep])))
    return out


def all_bitstrings(n: int) -> np.ndarray:
    """(2^n, n) uint8, row z = the bits of z with qubit 0 the most significant."""
    z = np.arange(1 << n)
    return ((z[:, None] >> (n - 1 - np.arange(n))[None, :]) & 1).astype(np.uint8)


def measurement_flip(probs: np.ndarray, n: int, p_m: float) -> np.ndarray:
    """Bitstring distribution after independent read-out flips of probability
    p_m on every qubit (the measurement SPAM error); qubit 0 is the most
    significant bit of the index."""
    P = np.asarray(probs, dtype=np.float64).reshape((2,) * n)
    flip = np.array([[1 - p_m, p_m], [p_m, 1 - p_m]])
    for ax in range(n):
        P = np.moveaxis(np.tensordot(flip, P, axes=([1], [ax])), 0, ax)
    return P.reshape(-1)
