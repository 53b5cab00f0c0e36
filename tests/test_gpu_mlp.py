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


@pytest.mark.parametrize("widths,batch", [([20, 40, 33, 5], 70), (list(S.C5_WIDTHS), 128),
                                          (list(S.C5_WIDTHS), 512), ([20, 40, 33, 5], 1), ([7, 65, 3], 37)])
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


M64 = (1 << 64) - 1


def splitmix64(seed: int, k: int) -> int:
    """The k-th output of SplitMix64 seeded with `seed` (Steele, Lea and
    Flood, 2014): the finalizer applied to seed + k * 0x9E3779B97F4A7C15."""
    z = (seed + k * 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def test_splitmix64_reference_values():
    # first outputs of SplitMix64 seeded with 1234567, as published with the
    # generator's reference implementation
    assert [splitmix64(1234567, k) for k in (1, 2, 3)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423]


@pytest.mark.parametrize("batch,steps,nrows", [(64, 6, 300), (512, 3, 2312), (1, 4, 5)])
def test_fit_equals_train_steps_on_the_same_rows(batch, steps, nrows):
    """mpdo_mlp_fit = the per-step path on the minibatches its generator
    names: same kernels, same rounding points, so the parameters agree
    bit for bit."""
    require_gpu()
    widths = list(S.C5_WIDTHS)
    rng = np.random.default_rng(11 + batch)
    p = S.init_params(widths, rng)
    x = rng.normal(size=(nrows, widths[0])).astype(np.float32)
    t = rng.normal(size=(nrows, widths[-1])).astype(np.float32)
    seed = 987654321 + batch
    a = S.MLP(widths, max_batch=max(batch, 8), params=p)
    a.fit(_t(x), _t(t), steps, batch, 2e-3, seed=seed)
    b = S.MLP(widths, max_batch=max(batch, 8), params=p)
    for s in range(steps):
        idx = [splitmix64(seed, s * batch + j + 1) % nrows for j in range(batch)]
        b.train_step(_t(x[idx]), _t(t[idx]), 2e-3, want_loss=False)
    pa, pb = a.get_params(), b.get_params()
    assert np.array_equal(pa, pb), float(np.abs(pa - pb).max())
    assert not np.array_equal(pa, p)
    a.close()
    b.close()


def test_fit_reduces_the_loss_with_cosine_schedule():
    require_gpu()
    widths = [8, 64, 64, 2]
    rng = np.random.default_rng(5)
    net = S.MLP(widths, max_batch=256, seed=1)
    x = rng.uniform(-1, 1, size=(1000, 8)).astype(np.float32)
    t = np.stack([np.sin(x[:, 0] + x[:, 1]), x[:, 2] * x[:, 3]], axis=1).astype(np.float32)
    first = net.fit(_t(x), _t(t), 1, 256, 3e-3, want_loss=True)
    last = net.fit(_t(x), _t(t), 600, 256, 3e-3, cosine=True, seed=3, want_loss=True)
    assert last < 0.1 * first, (first, last)


def _host_ascent(net, x0, nfree, steps, lr, eps, m=None, v=None, t0=0):
    """The same Adam ascent driven from the host: one backward per step with a
    one-hot output cotangent, the update in float64 on the host."""
    import torch
    x = x0.astype(np.float64).copy()
    m = np.zeros(nfree) if m is None else m
    v = np.zeros(nfree) if v is None else v
    gy = np.zeros((1, net.widths[-1]), np.float32)
    gy[0, 0] = 1.0
    rows = []
    for s in range(1, steps + 1):
        _, _, dx, _ = net.backward(_t(x[None, :]), gy=_t(gy), want_dx=True, want_loss=False)
        g = dx.cpu().numpy()[0, :nfree].astype(np.float64)
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        k = t0 + s
        x[:nfree] += lr * (m / (1 - 0.9 ** k)) / (np.sqrt(v / (1 - 0.999 ** k)) + eps)
        rows.append(x.copy())
    return np.array(rows), m, v


def test_ascend_matches_host_loop_and_continues():
    require_gpu()
    widths = list(S.C5_WIDTHS)
    rng = np.random.default_rng(21)
    net = S.MLP(widths, max_batch=16, params=S.init_params(widths, rng))
    x0 = np.concatenate([rng.uniform(-0.2, 0.2, 144), np.ones(24)]).astype(np.float32)
    xs = net.ascend(_t(x0), 144, 12, 0.01, eps=1e-7).cpu().numpy()
    ref, m, v = _host_ascent(net, x0, 144, 12, 0.01, 1e-7)
    # float32 state on the device, float64 here: the paths agree to rounding
    assert np.abs(xs - ref).max() <= 1e-5, float(np.abs(xs - ref).max())
    assert np.array_equal(xs[:, 144:], np.tile(x0[144:], (12, 1)))
    # continuing (moments kept) from the sixth row = the host loop continued
    more = net.ascend(_t(xs[5]), 144, 4, 0.01, eps=1e-7, reset=False).cpu().numpy()
    ref2, _, _ = _host_ascent(net, xs[5], 144, 4, 0.01, 1e-7, m=m, v=v, t0=12)
    assert np.abs(more - ref2).max() <= 1e-5, float(np.abs(more - ref2).max())
    # a reset restarts the moments: the first step is lr * sign(g) up to eps
    again = net.ascend(_t(x0), 144, 1, 0.01, eps=1e-7).cpu().numpy()
    assert np.abs(again[0] - xs[0]).max() == 0.0
    net.close()
