"""Surrogate network kernels (bf16 MFMA, FP32 accumulation) against the float64
oracle MLP evaluated at the same bfloat16 rounding points.

Tolerance.  Both sides round the same operands to bfloat16; they differ in
the accumulation (FP32 on the GPU, float64 here) and in erf.  Those
differences (~1e-6 relative) flip a bfloat16 rounding only for values within
~1e-6 of a rounding boundary; a flipped hidden activation moves by one
bfloat16 step (2^-8 relative), which changes an output by at most
2^-8 * |w| * |h| for that one term.  The bounds below (3e-3 relative to the
largest output / gradient entry) leave room for a few such flips."""
import numpy as np
import pytest

from oracle import mlp as OM
from paper_2508_07610_amd import surrogate as S
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


@pytest.mark.parametrize("widths,batch", [([20, 40, 33, 5], 70), ([16, 64, 16], 64), ([3, 1, 2], 1),
                                          (list(S.C5_WIDTHS), 256)])
def test_forward_matches_oracle(widths, batch):
    require_gpu()
    rng = np.random.default_rng(sum(widths) + batch)
    p = S.init_params(widths, rng)
    p[-widths[-1]:] = rng.normal(size=widths[-1])  # nonzero output bias
    net = S.MLP(widths, max_batch=max(batch, 8), params=p)
    x = rng.normal(size=(batch, widths[0])).astype(np.float32)
    y = net.forward(_t(x)).cpu().numpy()
    ref, _ = OM.MLP(widths, p.astype(np.float64), bf16=True).forward(x.astype(np.float64))
    err = float(np.abs(y - ref).max())
    assert err <= 3e-3 * max(1.0, float(np.abs(ref).max())), err
    net.close()


@pytest.mark.parametrize("widths,batch", [([20, 40, 33, 5], 70), (list(S.C5_WIDTHS), 128)])
def test_gradients_match_oracle(widths, batch):
    require_gpu()
    rng = np.random.default_rng(7 + batch)
    p = S.init_params(widths, rng)
    net = S.MLP(widths, max_batch=batch, params=p)
    x = rng.normal(size=(batch, widths[0])).astype(np.float32)
    t = rng.normal(size=(batch, widths[-1])).astype(np.float32)
    y, g, dx, loss = net.backward(_t(x), t=_t(t), want_grad=True, want_dx=True)
    o = OM.MLP(widths, p.astype(np.float64), bf16=True)
    lo, go, dxo = o.loss_and_grad(x.astype(np.float64), t.astype(np.float64))
    assert abs(loss - lo) <= 3e-3 * max(1.0, lo)
    g = g.cpu().numpy()
    off = 0
    for l in range(1, len(widths)):
        n = widths[l] * widths[l - 1] + widths[l]
        a, b = g[off: off + n], go[off: off + n]
        assert np.abs(a - b).max() <= 3e-3 * np.abs(b).max(), (l, float(np.abs(a - b).max()), float(np.abs(b).max()))
        off += n
    dx = dx.cpu().numpy()
    assert np.abs(dx - dxo).max() <= 3e-3 * np.abs(dxo).max()


def test_output_cotangent_gives_input_gradient():
    require_gpu()
    widths = [12, 32, 4]
    rng = np.random.default_rng(3)
    p = S.init_params(widths, rng)
    net = S.MLP(widths, max_batch=16, params=p)
    x = rng.normal(size=(9, 12)).astype(np.float32)
    gy = rng.normal(size=(9, 4)).astype(np.float32)
    _, _, dx, _ = net.backward(_t(x), gy=_t(gy), want_dx=True, want_loss=False)
    o = OM.MLP(widths, p.astype(np.float64), bf16=True)
    _, cache = o.forward(x.astype(np.float64))
    _, dxo = o.backward_from(cache, gy.astype(np.float64))
    assert np.abs(dx.cpu().numpy() - dxo).max() <= 3e-3 * np.abs(dxo).max()


def test_training_reduces_the_loss():
    require_gpu()
    widths = [8, 64, 64, 2]
    rng = np.random.default_rng(5)
    net = S.MLP(widths, max_batch=256, seed=1)
    x = rng.uniform(-1, 1, size=(256, 8)).astype(np.float32)
    t = np.stack([np.sin(x[:, 0] + x[:, 1]), x[:, 2] * x[:, 3]], axis=1).astype(np.float32)
    xd, td = _t(x), _t(t)
    first = net.train_step(xd, td, 3e-3)
    for _ in range(300):
        last = net.train_step(xd, td, 3e-3)
    assert last < 0.1 * first, (first, last)


def test_adam_step_matches_reference():
    require_gpu()
    widths = [4, 3]
    rng = np.random.default_rng(9)
    p = S.init_params(widths, rng)
    net = S.MLP(widths, max_batch=8, params=p)
    x = rng.normal(size=(8, 4)).astype(np.float32)
    t = rng.normal(size=(8, 3)).astype(np.float32)
    _, g, _, _ = net.backward(_t(x), t=_t(t), want_grad=True)
    net.adam(0.01)
    g = g.cpu().numpy().astype(np.float64)
    m = 0.1 * g
    v = 0.001 * g * g
    ref = p - 0.01 * (m / 0.1) / (np.sqrt(v / 0.001) + 1e-8)
    assert np.abs(net.get_params() - ref).max() < 1e-6
