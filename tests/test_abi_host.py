"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point its headers declare, and rejects invalid arguments before
touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2508_07610_amd import mpdo as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in sorted(f for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h")):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(mpdo_[a-z_0-9]+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    L = M.lib()
    declared = _declared()
    assert {"mpdo_create", "mpdo_apply_gate", "mpdo_apply_channel", "mpdo_truncate", "mpdo_expect",
            "mpdo_batch_run"} <= declared
    for name in declared:
        assert hasattr(L, name), name
    assert set(M.EXPORTED) <= declared


def test_version_string():
    assert b"gfx950" in M.lib().mpdo_version()


@pytest.mark.parametrize("field,value", [("n", 0), ("n", 65), ("chi_max", 0), ("chi_max", 129), ("kappa_max", 0),
                                         ("max_kraus", 0), ("max_kraus", 257), ("svd_cutoff", -1.0), ("prec", 7)])
def test_create_rejects_bad_config(field, value):
    cfg = M.mpdo_config(6, 16, 4, 16, 1e-10, 1e-10, 0)
    setattr(cfg, field, value)
    h = ctypes.c_void_p()
    st = M.lib().mpdo_create(ctypes.byref(cfg), None, ctypes.byref(h))
    assert st == M.EINVAL
    assert not h.value
    assert len(M.lib().mpdo_last_error()) > 0


def test_create_rejects_a_single_allocator_hook():
    cfg = M.mpdo_config(6, 16, 4, 16, 1e-10, 1e-10, 0)
    cfg.alloc = M.ALLOC_FN(lambda n, ctx: None)
    h = ctypes.c_void_p()
    assert M.lib().mpdo_create(ctypes.byref(cfg), None, ctypes.byref(h)) == M.EINVAL
    assert b"hooks" in M.lib().mpdo_last_error()
    assert not h.value


def test_handle_calls_reject_null_handles():
    L = M.lib()
    st = M.mpdo_stats_t()
    assert L.mpdo_stats(None, ctypes.byref(st)) == M.EINVAL
    assert L.mpdo_flush(None) == M.EINVAL
    assert L.mpdo_dims(None, None, None, None) == M.EINVAL


def test_channel_rejects_bad_chi():
    h = ctypes.c_void_p()
    chi = np.zeros((4, 4), complex)
    chi[0, 1] = 1.0                                   # not Hermitian
    buf = chi.view(np.float64).copy()
    assert M.lib().mpdo_channel_from_chi(M._dptr(buf), 1, 0.0, None, ctypes.byref(h)) == M.EINVAL
    assert M.lib().mpdo_channel_from_chi(M._dptr(buf), 4, 0.0, None, ctypes.byref(h)) == M.EINVAL
    chi = np.full((4, 4), np.nan, complex)
    buf = chi.view(np.float64).copy()
    assert M.lib().mpdo_channel_from_chi(M._dptr(buf), 1, 0.0, None, ctypes.byref(h)) == M.EINVAL


def test_null_handles_are_rejected():
    L = M.lib()
    re_, im_ = ctypes.c_double(), ctypes.c_double()
    assert L.mpdo_expect(None, b"Z", ctypes.byref(re_), ctypes.byref(im_)) == M.EINVAL
    assert L.mpdo_flush(None) == M.EINVAL
    assert L.mpdo_destroy(None) == M.OK
    assert L.mpdo_channel_info(None, None, None, None) == M.EINVAL


def test_mpo_calls_reject_null_handles():
    """The error-mitigation entry points check their handles and output
    pointers before any device work."""
    L = M.lib()
    h = ctypes.c_void_p(1234)
    assert L.mpdo_mpo_from_state(None, 8, 0.0, ctypes.byref(h)) == M.EINVAL
    assert not h.value                                  # cleared on failure
    assert L.mpdo_mpo_from_state(None, 8, 0.0, None) == M.EINVAL
    u = np.eye(2, dtype=np.complex128).view(np.float64).copy()
    assert L.mpdo_mpo_apply_gate(None, 0, 1, M._dptr(u), 0) == M.EINVAL
    assert L.mpdo_mpo_apply_channel(None, 0, None, 1) == M.EINVAL
    out = np.zeros(2)
    assert L.mpdo_mpo_expect(None, M._dptr(u), 1, M._dptr(out)) == M.EINVAL
    assert L.mpdo_mpo_dims(None, None, None) == M.EINVAL
    assert L.mpdo_mpo_to_dense(None, M._dptr(out)) == M.EINVAL
    assert L.mpdo_mpo_destroy(None) == M.OK


def test_mlp_loops_reject_null_handles():
    """The training and ascent loops check the handle before any device work."""
    L = M.lib()
    loss = ctypes.c_float()
    assert L.mpdo_mlp_fit(None, None, None, 10, 4, 1, 1e-3, 0, 1, ctypes.byref(loss)) == M.EINVAL
    assert L.mpdo_mlp_ascend(None, None, 1, 0, 1, 1e-2, 0.9, 0.999, 1e-8, 1, None) == M.EINVAL
    assert L.mpdo_mlp_adam(None, 1e-3, 0.9, 0.999, 1e-8) == M.EINVAL


def test_test_entry_points_validate_sizes():
    L = M.lib()
    a = np.zeros(8)
    M._testing_lib()
    assert L.mpdo_test_eigh(0, 1, M._dptr(a), M._dptr(a), M._dptr(a), None) == M.EINVAL
    L.mpdo_test_gemm.argtypes = [ctypes.c_int32] * 6 + [ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                                        ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                                        ctypes.c_int32, ctypes.c_int32,
                                                        ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                                        ctypes.c_int32, ctypes.c_double,
                                                        ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                                        ctypes.c_int32]
    # A too small for op(A) = N with M = 4 rows
    assert L.mpdo_test_gemm(0, 0, 0, 4, 2, 2, M._dptr(a), 2, 2, M._dptr(a), 2, 2, None, 1, 1, 1.0,
                            M._dptr(a), 64, 0) == M.EINVAL
    assert L.mpdo_test_gemm(0, 0, 0, 2, 2, 2, M._dptr(a), 2, 2, M._dptr(a), 2, 2, None, 1, 1, 1.0,
                            M._dptr(a), 48, 0) == M.EINVAL
    # a Hermitian C must be square; herm is 0 or 1
    assert L.mpdo_test_gemm(0, 0, 0, 2, 1, 2, M._dptr(a), 2, 2, M._dptr(a), 2, 2, None, 1, 1, 1.0,
                            M._dptr(a), 64, 1) == M.EINVAL
    assert L.mpdo_test_gemm(0, 0, 0, 2, 2, 2, M._dptr(a), 2, 2, M._dptr(a), 2, 2, None, 1, 1, 1.0,
                            M._dptr(a), 64, 2) == M.EINVAL


def test_eigensolver_switches_validate_and_restore():
    """The eigensolver routing switches take 0 or 1, report the previous
    setting and touch no device."""
    L = M._testing_lib()
    prev = ctypes.c_int32(-1)
    assert L.mpdo_test_eig_coop(2, ctypes.byref(prev)) == M.EINVAL
    assert L.mpdo_test_eig_coop(0, ctypes.byref(prev)) == M.OK and prev.value == 1  # on by default
    assert L.mpdo_test_eig_coop(1, ctypes.byref(prev)) == M.OK and prev.value == 0
    assert M.eig_coop(True) is True
    assert L.mpdo_test_eig_band(-1, None) == M.EINVAL
    assert L.mpdo_test_gram_vector(3, None) == M.EINVAL
    assert M.gram_vector(True) is True  # on by default


def test_profile_read_rejects_unknown_class():
    L = M.lib()
    assert L.mpdo_profile_read(-1, None, None, None, None) == M.EINVAL
    assert L.mpdo_profile_read(6, None, None, None, None) == M.EINVAL


@pytest.mark.parametrize("q,kind,fixed,chi,status", [(3, 0, 0, 16, M.EINVAL), (3, 1, -1, 16, M.EINVAL),
                                                     (4, 0, -1, 16, M.EINVAL), (2, 0, -2, 16, M.EINVAL)])
def test_batch_run_validates_op_arity(q, kind, fixed, chi, status):
    """Three-site ops in batch runs are channels without a gate matrix; the
    call fails before touching the device."""
    cfg = M.mpdo_config(6, chi, 4, 16, 1e-10, 1e-10, 0)
    ops = (M.mpdo_op * 1)()
    ops[0].q, ops[0].site, ops[0].kind, ops[0].param, ops[0].scale, ops[0].chan, ops[0].fixed = (
        q, 0, kind, -1, 1.0, -1, fixed)
    prog = (M.mpdo_program * 1)()
    prog[0].n, prog[0].nops, prog[0].ops, prog[0].nobs = 6, 1, ops, 0
    u = np.eye(4, dtype=complex).view(np.float64).copy()
    st = M.lib().mpdo_batch_run(ctypes.byref(cfg), prog, 1, None, 0, M._dptr(u), 1, None, 0, None, 0, None)
    assert st == status, M.lib().mpdo_last_error()
