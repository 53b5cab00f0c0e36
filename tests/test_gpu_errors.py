"""Failure handling and metrics of the C ABI on the GPU, every failure forced
from the host (the kernels run to their normal end):

* an error after device work has started makes the handle unusable
  (sticky), while mpdo_dims and mpdo_stats still report its state;
* an eigenpair failing its residual bound (forced by a negative bound)
  surfaces as ENOTCONV at the next synchronising call, and from
  mpdo_batch_run after its results are written;
* mpdo_stats agrees with mpdo_dims / mpdo_trace and the oracle's discarded
  weight;
* device memory from torch's caching allocator (the mpdo_config hooks)
  gives the same state as the library's own cache."""
import math

import numpy as np
import pytest

from oracle import channels as OC
from oracle import mpdo as OM
from paper_2508_07610_amd import mpdo as M
from paper_2508_07610_amd import workloads as W
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _state(n=5, depth=2, tag=3, chi=16, kap=4, **kw):
    prog = W.ghz_ansatz(n, depth, W.ansatz_params(n, depth, tag))
    chans = [M.Channel(c, int(round(math.log(c.shape[0], 4)))) for c in prog.chis]
    st = M.MPDO(n, chi_max=chi, kappa_max=kap, max_kraus=16, svd_cutoff=1e-10, kappa_cutoff=1e-10, **kw)
    M.run_program(prog, st, chans)
    return prog, chans, st


@pytest.mark.parametrize("status", [M.ENOMEM, M.EDEVICE])
def test_error_after_device_work_is_sticky(status):
    require_gpu()
    _, chans, st = _state()
    before = st.dims()
    st.apply_channel([1], chans[0], W.ry(0.3))
    M.test_fail_next_update(status)
    with pytest.raises(M.MPDOError) as e:
        st.flush()
    assert e.value.status == status
    for call in (lambda: st.expect("Z" * 5), lambda: st.fidelity_ghz(), lambda: st.trace(),
                 lambda: st.apply_gate([0], W.H), lambda: st.truncate(4, 2, 0.0), lambda: st.flush(),
                 lambda: st.bond_weights(0), lambda: st.sample(np.full((1, 5), 0.5))):
        with pytest.raises(M.MPDOError) as e2:
            call()
        assert e2.value.status == M.EDEVICE
    assert st.dims() == before          # the state as it was: the failed sublayer never launched
    assert math.isnan(st.stats()["trace"])
    M.test_fail_next_update(0)


def test_rejected_arguments_leave_the_handle_usable():
    require_gpu()
    _, _, st = _state()
    before = st.trace()
    with pytest.raises(M.MPDOError) as e:
        st.apply_gate([1, 3], W.CZ)
    assert e.value.status == M.EINVAL
    assert st.trace() == before
    st.apply_gate([1, 2], W.CZ)
    assert st.stats()["failures"] == 0


def test_eigensolver_residual_failure_is_reported():
    require_gpu()
    _, chans, st = _state()
    try:
        M.test_eig_residual_bound(-1.0)
        st.apply_channel([2], chans[0], W.ry(0.7))
        with pytest.raises(M.MPDOError) as e:
            st.expect("IIZII")
        assert e.value.status == M.ENOTCONV
    finally:
        M.test_eig_residual_bound(0.0)
    s = st.stats()
    assert s["failures"] > 0
    with pytest.raises(M.MPDOError) as e:
        st.trace()
    assert e.value.status == M.EDEVICE
    # a fresh handle after restoring the bound runs clean
    _, _, st2 = _state()
    assert st2.stats()["failures"] == 0


@pytest.mark.parametrize("graph", [True, False])
def test_batch_run_reports_eigensolver_failure(graph):
    require_gpu()
    import torch
    progs = [W.ghz_ansatz(4, 1, W.ansatz_params(4, 1, t)) for t in range(3)]
    obs = [np.stack([W.pauli_ops("ZZII")]) for _ in progs]
    chans = [M.Channel(c, int(round(math.log(c.shape[0], 4)))) for c in progs[0].chis]
    kw = dict(chi_max=8, kappa_max=4, max_kraus=16, svd_cutoff=1e-10, kappa_cutoff=1e-10, use_graph=graph)
    good = M.batch_run(progs, None, chans, obs, **kw).cpu().numpy()
    try:
        M.test_eig_residual_bound(-1.0)
        with pytest.raises(M.MPDOError) as e:
            M.batch_run(progs, None, chans, obs, **kw)
        assert e.value.status == M.ENOTCONV
    finally:
        M.test_eig_residual_bound(0.0)
    again = M.batch_run(progs, None, chans, obs, **kw).cpu().numpy()
    assert np.array_equal(good, again)
    torch.cuda.synchronize()


def test_stats_match_dims_trace_and_oracle():
    require_gpu()
    n, depth, chi, kap, tag = 8, 3, 16, 4, 5
    prog, _, st = _state(n, depth, tag, chi, kap)
    kr = [OC.kraus_from_chi(c)[0] for c in prog.chis]
    o = OM.run_program(prog, OM.MPDO(n, chi, kap, 1e-10, 1e-10), kr)
    s = st.stats()
    bonds, inner, disc = st.dims()
    assert s["failures"] == 0
    assert s["truncations"] > 0
    assert abs(s["discarded"] - disc) < 1e-15
    assert abs(s["discarded"] - o.discarded) < 1e-7
    assert 0 < s["max_discarded"] <= s["discarded"] + 1e-15
    assert s["min_gap"] > 0
    assert abs(s["trace"] - st.trace()) < 1e-12
    assert abs(s["trace"] - o.trace()) < 1e-10
    assert s["max_bond"] == max(bonds) and s["max_inner"] == max(inner)


def test_torch_allocator_hooks_give_the_same_state():
    require_gpu()
    import torch
    alloc = M.TorchAllocator()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    prog, chans, ref = _state(6, 2, 7, 16, 4)
    st = M.MPDO(6, chi_max=16, kappa_max=4, max_kraus=16, svd_cutoff=1e-10, kappa_cutoff=1e-10, allocator=alloc)
    M.run_program(prog, st, chans)
    assert torch.cuda.memory_allocated() > base          # the handle's tensors live in torch's pool
    for s in W.zz_strings(6) + ["XXXXXX"]:
        assert st.expect(s) == ref.expect(s)
    assert st.dims() == ref.dims()
    st.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base
    obs = [np.stack([W.pauli_ops("ZZIIII")])]
    a = M.batch_run([prog], None, chans, obs, chi_max=16, kappa_max=4, max_kraus=16, svd_cutoff=1e-10,
                    kappa_cutoff=1e-10, allocator=alloc).cpu().numpy()
    b = M.batch_run([prog], None, chans, obs, chi_max=16, kappa_max=4, max_kraus=16, svd_cutoff=1e-10,
                    kappa_cutoff=1e-10).cpu().numpy()
    assert np.array_equal(a, b)


def test_library_cache_holds_released_blocks():
    require_gpu()
    _, _, st = _state()
    st.close()
    assert M.release_cached_memory() > 0
    assert M.release_cached_memory() == 0
