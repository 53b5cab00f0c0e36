"""mpdo_kraus_from_chi_noalloc (include/mpdo_noalloc.h) against the entry
point it varies, mpdo_channel_from_chi: the same Kraus operators, counts and
completeness, on two calls in a row (a three-qubit channel, then a smaller
two-qubit one, which reuses the same scratch), with pruning."""
import ctypes

import numpy as np
import pytest

from paper_2508_07610_amd import mpdo as M
from paper_2508_07610_amd import workloads as W
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _fn():
    L = M.lib()
    f = L.mpdo_kraus_from_chi_noalloc
    f.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_void_p]
    f.restype = ctypes.c_int
    return f


def _noalloc(chi, q, eps, kraus, info, stream):
    import torch
    x = torch.tensor(np.ascontiguousarray(chi, dtype=np.complex128).view(np.float64).reshape(-1),
                     dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    st = _fn()(x.data_ptr(), q, eps, kraus.data_ptr(), info.data_ptr(), stream.cuda_stream)
    M.check(st)
    stream.synchronize()
    inf = info.cpu().numpy()
    m, d = int(inf[0]), 2 ** q
    ks = kraus.cpu().numpy()[: 2 * m * d * d].view(np.complex128).reshape(m, d, d)
    return ks, inf


@pytest.mark.parametrize("eps", [0.0, 1e-4])
def test_noalloc_matches_channel_from_chi_twice(eps):
    require_gpu()
    import torch
    rng = W.rng_for(4242)
    cases = [(W.random_cptp_near_identity_3q(rng), 3), (W.chi_2q_default(3.0), 2)]
    stream = torch.cuda.Stream()
    kraus = torch.zeros(2 * 64 * 64, dtype=torch.float64, device="cuda")
    info = torch.zeros(4, dtype=torch.float64, device="cuda")
    for chi, q in cases:                       # the second call is the smaller one
        ks, inf = _noalloc(chi, q, eps, kraus, info, stream)
        ref = M.Channel(chi, q, eps=eps)
        kr = ref.info()
        assert ks.shape == kr.shape
        assert np.abs(ks - kr).max() < 1e-12
        assert inf[1] < 1e-8 and inf[3] >= len(kr)


def test_noalloc_rejects_bad_arguments():
    require_gpu()
    import torch
    k = torch.zeros(8, dtype=torch.float64, device="cuda")
    f = _fn()
    assert f(k.data_ptr(), 4, 0.0, k.data_ptr(), k.data_ptr(), None) == M.EINVAL
    assert f(k.data_ptr(), 0, 0.0, k.data_ptr(), k.data_ptr(), None) == M.EINVAL
    assert f(None, 1, 0.0, k.data_ptr(), k.data_ptr(), None) == M.EINVAL
    assert f(k.data_ptr(), 1, 1.5, k.data_ptr(), k.data_ptr(), None) == M.EINVAL
