"""Pins of the float64 MLP oracle: GELU special values and its derivative,
bfloat16 rounding of exactly representable and tie values, the gradient of a
one-layer linear network in closed form, and central finite differences of
the full network (parameters and input)."""
import math

import numpy as np

from oracle import mlp as OM


def _params(widths, rng, scale=0.3):
    n = sum(widths[l] * widths[l - 1] + widths[l] for l in range(1, len(widths)))
    return rng.normal(scale=scale, size=n)


def test_gelu_values():
    z = np.array([0.0, 1.0, -1.0, 3.0])
    g = OM.gelu(z)
    assert g[0] == 0.0
    assert abs(g[1] - 0.5 * (1 + math.erf(1 / math.sqrt(2)))) < 1e-15
    assert abs(g[1] - g[2] - 1.0) < 1e-15       # GELU(z) - GELU(-z) = z
    assert abs(OM.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-15
    h = 1e-6
    for x in (-2.0, -0.3, 0.7, 2.5):
        fd = (OM.gelu(np.array([x + h])) - OM.gelu(np.array([x - h])))[0] / (2 * h)
        assert abs(fd - OM.gelu_grad(np.array([x]))[0]) < 1e-8


def test_bf16_rounding():
    exact = np.array([1.0, -2.0, 0.5, 3.0, 1.0 + 2 ** -7])
    assert np.array_equal(OM.bf16_round(exact), exact)
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even -> 1
    assert OM.bf16_round(np.array([1.0 + 2 ** -8]))[0] == 1.0
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: ties to even -> 1 + 2^-6
    assert OM.bf16_round(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6
    x = np.random.default_rng(0).normal(size=1000)
    assert np.max(np.abs(OM.bf16_round(x) - x) / np.abs(x)) <= 2 ** -8


def test_linear_layer_closed_form():
    rng = np.random.default_rng(1)
    W, b = rng.normal(size=(3, 4)), rng.normal(size=3)
    net = OM.MLP([4, 3], np.concatenate([W.ravel(), b]))
    x, t = rng.normal(size=(5, 4)), rng.normal(size=(5, 3))
    loss, grad, dx = net.loss_and_grad(x, t)
    r = x @ W.T + b - t
    assert abs(loss - np.mean(r ** 2)) < 1e-14
    gW = 2.0 / r.size * r.T @ x
    gb = 2.0 / r.size * r.sum(axis=0)
    assert np.abs(grad - np.concatenate([gW.ravel(), gb])).max() < 1e-14
    assert np.abs(dx - 2.0 / r.size * r @ W).max() < 1e-14


def test_finite_differences():
    rng = np.random.default_rng(2)
    widths = [6, 9, 7, 4]
    p = _params(widths, rng)
    x, t = rng.normal(size=(5, 6)), rng.normal(size=(5, 4))
    loss, grad, dx = OM.MLP(widths, p).loss_and_grad(x, t)
    h = 1e-6
    for i in rng.choice(p.size, size=40, replace=False):
        e = np.zeros_like(p)
        e[i] = h
        fd = (OM.MLP(widths, p + e).loss_and_grad(x, t)[0] - OM.MLP(widths, p - e).loss_and_grad(x, t)[0]) / (2 * h)
        assert abs(fd - grad[i]) < 1e-7 * max(1.0, abs(fd)), i
    for (a, c) in [(0, 0), (3, 5), (4, 2)]:
        e = np.zeros_like(x)
        e[a, c] = h
        fd = (OM.MLP(widths, p).loss_and_grad(x + e, t)[0] - OM.MLP(widths, p).loss_and_grad(x - e, t)[0]) / (2 * h)
        assert abs(fd - dx[a, c]) < 1e-7


def test_bf16_mode_stays_close_to_exact():
    rng = np.random.default_rng(3)
    widths = [10, 16, 16, 3]
    p = _params(widths, rng)
    x = rng.normal(size=(8, 10))
    y64, _ = OM.MLP(widths, p).forward(x)
    y16, _ = OM.MLP(widths, p, bf16=True).forward(x)
    assert 0 < np.abs(y64 - y16).max() < 5e-2
