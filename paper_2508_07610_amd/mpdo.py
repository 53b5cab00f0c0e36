"""Python binding of libmpdo (ctypes).  Argument marshalling only: every step
of the simulation runs in the library's HIP kernels.

The names follow the C ABI in ``include/mpdo.h``.  The binding fails loudly
when ``libmpdo.so`` has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpdo.so")

OK, EINVAL, ENOTCPTP, ENOMEM, EDEVICE, ENOTCONV, EUNSUPPORTED = range(7)
C128, C64_MIXED = 0, 1
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOTCPTP", 3: "ENOMEM", 4: "EDEVICE", 5: "ENOTCONV", 6: "EUNSUPPORTED"}

EXPORTED = (
    "mpdo_last_error", "mpdo_version", "mpdo_create", "mpdo_destroy", "mpdo_channel_from_chi",
    "mpdo_channel_info", "mpdo_channel_destroy", "mpdo_apply_gate", "mpdo_apply_channel", "mpdo_flush",
    "mpdo_truncate", "mpdo_expect", "mpdo_expect_products", "mpdo_fidelity_ghz", "mpdo_trace", "mpdo_dims",
    "mpdo_bond_weights", "mpdo_to_dense", "mpdo_probabilities", "mpdo_sample", "mpdo_batch_run",
    "mpdo_stats", "mpdo_release_cached_memory", "mpdo_batch_run_dense", "mpdo_tune_set", "mpdo_tune_get",
    "mpdo_mpo_from_state", "mpdo_mpo_destroy", "mpdo_mpo_apply_gate", "mpdo_mpo_apply_channel", "mpdo_mpo_expect",
    "mpdo_mpo_dims", "mpdo_mpo_to_dense",
)


class MPDOError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class mpdo_config(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("chi_max", ctypes.c_int32), ("kappa_max", ctypes.c_int32),
                ("max_kraus", ctypes.c_int32), ("svd_cutoff", ctypes.c_double),
                ("kappa_cutoff", ctypes.c_double), ("prec", ctypes.c_int32),
                ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_ctx", ctypes.c_void_p)]


class mpdo_stats_t(ctypes.Structure):
    _fields_ = [("truncations", ctypes.c_int64), ("failures", ctypes.c_int64), ("discarded", ctypes.c_double),
                ("max_discarded", ctypes.c_double), ("min_gap", ctypes.c_double), ("trace", ctypes.c_double),
                ("max_bond", ctypes.c_int32), ("max_inner", ctypes.c_int32)]


class TorchAllocator:
    """Device memory for the library from torch's caching allocator, through
    the allocator hooks of mpdo_config: handles and batch runs then draw from
    (and return to) the same pool as the caller's tensors.  Keep the object
    alive while any handle made with it exists."""

    def __init__(self, stream=None):
        import torch
        self._torch = torch
        self._stream = stream
        dev = torch.cuda.current_device()

        def _alloc(nbytes, _ctx):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), dev, self._stream))
            except Exception:
                return None

        def _free(ptr, _ctx):
            if ptr:
                torch.cuda.caching_allocator_delete(int(ptr))

        self.alloc = ALLOC_FN(_alloc)
        self.free = FREE_FN(_free)

    def apply(self, cfg: "mpdo_config") -> None:
        cfg.alloc = self.alloc
        cfg.free = self.free
        cfg.alloc_ctx = None


def release_cached_memory() -> int:
    """Return the library's cache of released device blocks to the driver;
    returns the bytes it held."""
    n = ctypes.c_size_t()
    check(lib().mpdo_release_cached_memory(ctypes.byref(n)))
    return n.value


class mpdo_op(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int32), ("site", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("param", ctypes.c_int32), ("scale", ctypes.c_double), ("chan", ctypes.c_int32),
                ("fixed", ctypes.c_int32)]


class mpdo_program(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nops", ctypes.c_int32), ("ops", ctypes.POINTER(mpdo_op)),
                ("nobs", ctypes.c_int32), ("obs", ctypes.POINTER(ctypes.c_double))]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2508_07610_amd.build`")
    # torch ships its own HIP runtime under the same soname as the system one
    # the library links against; importing torch first makes the process load
    # exactly one runtime (torch's), so device buffers are shared between them.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    pd, pi = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
    L.mpdo_last_error.restype = ctypes.c_char_p
    L.mpdo_version.restype = ctypes.c_char_p
    sig = {
        "mpdo_create": [ctypes.POINTER(mpdo_config), vp, ctypes.POINTER(vp)],
        "mpdo_destroy": [vp],
        "mpdo_channel_from_chi": [pd, i32, dbl, vp, ctypes.POINTER(vp)],
        "mpdo_channel_info": [vp, pi, pi, pd],
        "mpdo_channel_destroy": [vp],
        "mpdo_apply_gate": [vp, pi, i32, pd],
        "mpdo_apply_channel": [vp, pi, i32, pd, vp],
        "mpdo_flush": [vp],
        "mpdo_truncate": [vp, i32, i32, dbl, pd],
        "mpdo_expect": [vp, ctypes.c_char_p, pd, pd],
        "mpdo_expect_products": [vp, pd, i32, pd],
        "mpdo_fidelity_ghz": [vp, pd],
        "mpdo_trace": [vp, pd],
        "mpdo_dims": [vp, pi, pi, pd],
        "mpdo_bond_weights": [vp, i32, pd, i32, pi],
        "mpdo_stats": [vp, ctypes.POINTER(mpdo_stats_t)],
        "mpdo_release_cached_memory": [ctypes.POINTER(ctypes.c_size_t)],
        "mpdo_to_dense": [vp, pd],
        "mpdo_probabilities": [vp, ctypes.POINTER(ctypes.c_uint8), i32, pd],
        "mpdo_sample": [vp, pd, i32, ctypes.POINTER(ctypes.c_uint8), pd],
        "mpdo_batch_run": [ctypes.POINTER(mpdo_config), ctypes.POINTER(mpdo_program), i32, vp, i32, pd, i32,
                           ctypes.POINTER(vp), i32, vp, i32, vp],
        "mpdo_batch_run_dense": [ctypes.POINTER(mpdo_config), ctypes.POINTER(mpdo_program), i32, vp, i32, pd, i32,
                                 ctypes.POINTER(vp), i32, vp, vp],
        "mpdo_tune_set": [i32, i32, i32, dbl],
        "mpdo_mpo_from_state": [vp, i32, dbl, ctypes.POINTER(vp)],
        "mpdo_mpo_destroy": [vp],
        "mpdo_mpo_apply_gate": [vp, i32, i32, pd, i32],
        "mpdo_mpo_apply_channel": [vp, i32, vp, i32],
        "mpdo_mpo_expect": [vp, pd, i32, pd],
        "mpdo_mpo_dims": [vp, pi, pd],
        "mpdo_mpo_to_dense": [vp, pd],
        "mpdo_tune_get": [i32, pi, pi, pd],
        "mpdo_profile_enable": [i32],
        "mpdo_profile_read": [i32, pi, pd, pd, pd],
        "mpdo_mlp_create": [pi, i32, i32, vp, ctypes.POINTER(vp)],
        "mpdo_mlp_destroy": [vp],
        "mpdo_mlp_info": [vp, ctypes.POINTER(ctypes.c_int64)],
        "mpdo_mlp_set_params": [vp, ctypes.POINTER(ctypes.c_float)],
        "mpdo_mlp_get_params": [vp, ctypes.POINTER(ctypes.c_float)],
        "mpdo_mlp_forward": [vp, vp, i32, vp],
        "mpdo_mlp_backward": [vp, vp, vp, vp, i32, vp, vp, vp, ctypes.POINTER(ctypes.c_float)],
        "mpdo_mlp_adam": [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float],
        "mpdo_mlp_fit": [vp, vp, vp, ctypes.c_int64, i32, i32, ctypes.c_float, i32, ctypes.c_uint64,
                         ctypes.POINTER(ctypes.c_float)],
        "mpdo_mlp_ascend": [vp, vp, i32, i32, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                            i32, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    _lib = L
    return L


def check(status: int) -> None:
    if status != OK:
        raise MPDOError(status, lib().mpdo_last_error().decode())


def _cplx(a: np.ndarray) -> np.ndarray:
    """Interleaved (re, im) float64 copy of a complex array."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    return a.view(np.float64).copy()


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def stream_handle(stream=None) -> Optional[int]:
    """hipStream_t of a torch stream (or an int handle, or None = default)."""
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class Channel:
    """Process-tomography channel: chi (4^q x 4^q, Pauli basis) -> Kraus on the GPU."""

    def __init__(self, chi: np.ndarray, q: int, eps: float = 0.0, stream=None):
        chi = np.asarray(chi, dtype=np.complex128)
        if chi.shape != (4 ** q, 4 ** q):
            raise ValueError("chi must be 4^q x 4^q")
        buf = _cplx(chi)
        h = ctypes.c_void_p()
        check(lib().mpdo_channel_from_chi(_dptr(buf), q, float(eps), stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self.q = q

    @property
    def handle(self):
        return self._h

    def info(self):
        q, m = ctypes.c_int32(), ctypes.c_int32()
        check(lib().mpdo_channel_info(self._h, ctypes.byref(q), ctypes.byref(m), None))
        d = 2 ** q.value
        out = np.zeros(2 * m.value * d * d)
        check(lib().mpdo_channel_info(self._h, None, None, _dptr(out)))
        return out.view(np.complex128).reshape(m.value, d, d)

    @property
    def nkraus(self) -> int:
        m = ctypes.c_int32()
        check(lib().mpdo_channel_info(self._h, None, ctypes.byref(m), None))
        return m.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().mpdo_channel_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MPDO:
    """One MPDO state on the GPU (see include/mpdo.h)."""

    def __init__(self, n: int, chi_max: int, kappa_max: int, max_kraus: int = 16,
                 svd_cutoff: float = 1e-14, kappa_cutoff: float = 1e-14, prec: int = C128, stream=None,
                 allocator: Optional[TorchAllocator] = None):
        self.n = n
        self.cfg = mpdo_config(n, chi_max, kappa_max, max_kraus, svd_cutoff, kappa_cutoff, prec)
        self._allocator = allocator
        if allocator is not None:
            allocator.apply(self.cfg)
        h = ctypes.c_void_p()
        check(lib().mpdo_create(ctypes.byref(self.cfg), stream_handle(stream), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().mpdo_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @staticmethod
    def _sites(sites: Sequence[int]):
        arr = (ctypes.c_int32 * len(sites))(*sites)
        return arr

    def apply_gate(self, sites: Sequence[int], U: np.ndarray) -> None:
        u = _cplx(U)
        check(lib().mpdo_apply_gate(self._h, self._sites(sites), len(sites), _dptr(u)))

    def apply_channel(self, sites: Sequence[int], ch: Channel, U: Optional[np.ndarray] = None) -> None:
        u = None if U is None else _cplx(U)
        check(lib().mpdo_apply_channel(self._h, self._sites(sites), len(sites), _dptr(u), ch.handle))

    def flush(self) -> None:
        check(lib().mpdo_flush(self._h))

    def truncate(self, chi_max: int, kappa_max: int, cutoff: float) -> float:
        d = ctypes.c_double()
        check(lib().mpdo_truncate(self._h, chi_max, kappa_max, cutoff, ctypes.byref(d)))
        return d.value

    def expect(self, pauli: str) -> complex:
        re, im = ctypes.c_double(), ctypes.c_double()
        check(lib().mpdo_expect(self._h, pauli.encode(), ctypes.byref(re), ctypes.byref(im)))
        return complex(re.value, im.value)

    def expect_products(self, ops: np.ndarray) -> np.ndarray:
        """ops: (nops, n, 2, 2) complex -> Tr(O rho)/Tr(rho) for each."""
        ops = np.asarray(ops, dtype=np.complex128)
        buf = _cplx(ops)
        out = np.zeros(2 * ops.shape[0])
        check(lib().mpdo_expect_products(self._h, _dptr(buf), ops.shape[0], _dptr(out)))
        return out.view(np.complex128)

    def fidelity_ghz(self) -> float:
        f = ctypes.c_double()
        check(lib().mpdo_fidelity_ghz(self._h, ctypes.byref(f)))
        return f.value

    def trace(self) -> float:
        t = ctypes.c_double()
        check(lib().mpdo_trace(self._h, ctypes.byref(t)))
        return t.value

    def dims(self):
        b = (ctypes.c_int32 * max(1, self.n - 1))()
        k = (ctypes.c_int32 * self.n)()
        d = ctypes.c_double()
        check(lib().mpdo_dims(self._h, b, k, ctypes.byref(d)))
        return list(b)[: self.n - 1], list(k), d.value

    def to_dense(self) -> np.ndarray:
        """rho as a (2^n, 2^n) complex array (n <= 12)."""
        d = 1 << self.n
        out = np.zeros(2 * d * d)
        check(lib().mpdo_to_dense(self._h, _dptr(out)))
        return out.view(np.complex128).reshape(d, d)

    def to_mpo(self, d_max: int = 256, cutoff: float = 0.0) -> "MPO":
        """rho as an MPO of local density tensors (see MPO)."""
        return MPO(self, d_max, cutoff)

    def probabilities(self, bits: np.ndarray) -> np.ndarray:
        """bits: (nz, n) of 0/1 -> <z|rho|z> / Tr(rho) for each row."""
        b = np.ascontiguousarray(np.asarray(bits, dtype=np.uint8).reshape(-1, self.n))
        out = np.zeros(b.shape[0])
        check(lib().mpdo_probabilities(self._h, b.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), b.shape[0],
                                       _dptr(out)))
        return out

    def sample(self, u: np.ndarray):
        """u: (nshots, n) uniforms in [0, 1) -> (bits (nshots, n) uint8, P(z) of each draw)."""
        uu = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(-1, self.n))
        bits = np.zeros(uu.shape, dtype=np.uint8)
        pz = np.zeros(uu.shape[0])
        check(lib().mpdo_sample(self._h, _dptr(uu), uu.shape[0], bits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                _dptr(pz)))
        return bits, pz

    def stats(self) -> dict:
        """Truncation statistics (mpdo_stats): truncations, failures, summed
        and largest discarded weight, smallest gap at a cut, Tr(rho), largest
        bond and inner dimension."""
        st = mpdo_stats_t()
        check(lib().mpdo_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in mpdo_stats_t._fields_}

    def bond_weights(self, bond: int) -> np.ndarray:
        cap = self.cfg.chi_max
        out = np.zeros(cap)
        ln = ctypes.c_int32()
        check(lib().mpdo_bond_weights(self._h, bond, _dptr(out), cap, ctypes.byref(ln)))
        return out[: ln.value].copy()


G_FIXED, G_RX, G_RY, G_RZ, G_ZZPHASE, G_SWAPZZ = range(6)
_PARAM_KINDS = {"ry": (G_RY, 1), "rx": (G_RX, 1), "rz": (G_RZ, 1), "swapzz": (G_SWAPZZ, 2), "mix": (G_RX, 1)}


def program_ops(prog, fixed: List[np.ndarray], fixed_index: dict, use_params: bool = True):
    """mpdo_op array of a workloads.Program.  Parametrised gates (kind ry, rx,
    rz, mix, swapzz with a parameter index) read their angle from the
    instance's parameter row on the device; every other gate is a fixed
    matrix appended to `fixed` (deduplicated through `fixed_index`)."""
    ops = (mpdo_op * max(1, len(prog.ops)))()
    for j, op in enumerate(prog.ops):
        q = len(op.sites)
        o = ops[j]
        o.q, o.site, o.chan, o.param, o.scale, o.fixed = q, op.sites[0], op.chan, -1, 1.0, 0
        if use_params and op.param >= 0 and op.kind in _PARAM_KINDS:
            o.kind = _PARAM_KINDS[op.kind][0]
            o.param = op.param
            o.scale = float(op.pscale)
        elif q == 3:  # three-site ops in batch runs: the channel alone
            if not np.allclose(op.U, np.eye(8)):
                raise ValueError("batch runs take 3-site ops without a gate matrix")
            o.kind, o.fixed = G_FIXED, -1
        else:
            o.kind = G_FIXED
            U = np.asarray(op.U, dtype=np.complex128)
            slot = np.zeros((4, 4), dtype=np.complex128)
            slot[: U.shape[0], : U.shape[1]] = U
            key = slot.tobytes()
            if key not in fixed_index:
                fixed_index[key] = len(fixed)
                fixed.append(slot)
            o.fixed = fixed_index[key]
    return ops


class BatchPlan:
    """The host-side form of a batch of programs and their observables
    (mpdo_program records, operation arrays, fixed gate matrices), built once
    and reusable across batch_run calls that vary only the device parameters."""

    def __init__(self, programs, observables, use_params: bool):
        ninst = len(programs)
        fixed: List[np.ndarray] = []
        fidx: dict = {}
        self.keep = []
        self.progs = (mpdo_program * ninst)()
        for b, pr in enumerate(programs):
            ops = program_ops(pr, fixed, fidx, use_params=use_params)
            obs = np.ascontiguousarray(np.asarray(observables[b], dtype=np.complex128))
            obuf = obs.view(np.float64).reshape(-1).copy() if obs.size else np.zeros(8)
            self.keep += [ops, obuf]
            self.progs[b].n = pr.n
            self.progs[b].nops = len(pr.ops)
            self.progs[b].ops = ops
            self.progs[b].nobs = obs.shape[0] if obs.size else 0
            self.progs[b].obs = _dptr(obuf)
        self.ninst = ninst
        self.use_params = use_params
        self.total = sum(self.progs[b].nobs for b in range(ninst))
        self.nfixed = len(fixed)
        self.fbuf = _cplx(np.array(fixed)) if fixed else np.zeros(32)


def batch_run(programs, params, channels: Sequence[Channel], observables, chi_max: int, kappa_max: int,
              max_kraus: int = 16, svd_cutoff: float = 1e-14, kappa_cutoff: float = 1e-14, prec: int = C128,
              use_graph: bool = True, stream=None, out=None, allocator: Optional[TorchAllocator] = None):
    """Run many programs through mpdo_batch_run.

    programs: workloads.Program list, or a BatchPlan built from them (then
    observables is ignored); params: torch float64 CUDA tensor (ninst, P) of
    per-instance parameters (or None); observables: per program a
    (nobs, n, 2, 2) complex array.  Returns a torch complex128 CUDA tensor
    of all expectation values (instance-major)."""
    import torch
    plan = programs if isinstance(programs, BatchPlan) else BatchPlan(programs, observables, params is not None)
    if plan.use_params != (params is not None):
        raise ValueError("the plan was built for a different parameter mode")
    ninst, progs, total = plan.ninst, plan.progs, plan.total
    if out is None:
        out = torch.zeros(max(1, total), dtype=torch.complex128, device="cuda")
    chans = (ctypes.c_void_p * max(1, len(channels)))(*[c.handle.value for c in channels])
    if out.dtype != torch.complex128 or not out.is_cuda or not out.is_contiguous() or out.numel() < total:
        raise ValueError("out must be a contiguous complex128 CUDA tensor of at least %d entries" % total)
    cfg = mpdo_config(0, chi_max, kappa_max, max_kraus, svd_cutoff, kappa_cutoff, prec)
    if allocator is not None:
        allocator.apply(cfg)
    pptr, pstride = None, 0
    if params is not None:
        if not (params.is_cuda and params.dtype == torch.float64 and params.is_contiguous()):
            raise ValueError("params must be a contiguous float64 CUDA tensor")
        if params.ndim != 2 or params.shape[0] < ninst:
            raise ValueError("params must have shape (>= %d instances, P)" % ninst)
        pptr, pstride = params.data_ptr(), params.shape[1]
    check(lib().mpdo_batch_run(ctypes.byref(cfg), progs, ninst, pptr, pstride, _dptr(plan.fbuf), plan.nfixed, chans,
                               len(channels), out.data_ptr(), 1 if use_graph else 0, stream_handle(stream)))
    return out[:total]


def batch_run_dense(programs, params, channels: Sequence[Channel], chi_max: int, kappa_max: int,
                    max_kraus: int = 16, svd_cutoff: float = 1e-14, kappa_cutoff: float = 1e-14, prec: int = C128,
                    stream=None):
    """Run many programs (n <= 12) through mpdo_batch_run_dense and return the
    list of their dense density matrices (unnormalised) as torch complex128
    CUDA tensors (2^n, 2^n) viewing one device buffer."""
    import torch
    plan = programs if isinstance(programs, BatchPlan) else BatchPlan(programs, [np.zeros((0,))] * len(programs),
                                                                     params is not None)
    ns = [plan.progs[b].n for b in range(plan.ninst)]
    sizes = [4 ** n for n in ns]
    buf = torch.zeros(sum(sizes), dtype=torch.complex128, device="cuda")
    chans = (ctypes.c_void_p * max(1, len(channels)))(*[c.handle.value for c in channels])
    cfg = mpdo_config(0, chi_max, kappa_max, max_kraus, svd_cutoff, kappa_cutoff, prec)
    pptr, pstride = None, 0
    if params is not None:
        if params.ndim != 2 or params.shape[0] < plan.ninst or params.dtype != torch.float64 or not params.is_cuda:
            raise ValueError("params must be a float64 CUDA tensor of shape (>= ninst, P)")
        params = params.contiguous()
        pptr, pstride = params.data_ptr(), params.shape[1]
    check(lib().mpdo_batch_run_dense(ctypes.byref(cfg), plan.progs, plan.ninst, pptr, pstride, _dptr(plan.fbuf),
                                     plan.nfixed, chans, len(channels), buf.data_ptr(), stream_handle(stream)))
    out, off = [], 0
    for n, sz in zip(ns, sizes):
        out.append(buf[off: off + sz].view(2 ** n, 2 ** n))
        off += sz
    return out


def tune_set(site: int, tile: int = 0, form: int = 0, split_scale: float = 0.0) -> None:
    """GEMM settings of one call site (see mpdo_tune_set); zeros restore the built-in choice."""
    check(lib().mpdo_tune_set(site, tile, form, float(split_scale)))


def tune_get(site: int):
    t, f, s = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    check(lib().mpdo_tune_get(site, ctypes.byref(t), ctypes.byref(f), ctypes.byref(s)))
    return t.value, f.value, s.value


PROF_GEMM_F64, PROF_GEMM_F32, PROF_EIG_REG, PROF_EIG_GLOBAL, PROF_EIG_BAND, PROF_CHOL = range(6)
PROF_NAMES = {PROF_GEMM_F64: "k_gemm (FP64 MFMA)", PROF_GEMM_F32: "k_gemm (FP32 MFMA)",
              PROF_EIG_REG: "k_heev_reg", PROF_EIG_GLOBAL: "k_heev_global", PROF_EIG_BAND: "k_heev_band",
              PROF_CHOL: "k_q2_chol_e"}


def profile_enable(on: bool = True) -> None:
    """Reset the kernel profile counters and switch profiling on or off."""
    check(lib().mpdo_profile_enable(1 if on else 0))


def profile_read(cls: int) -> dict:
    """Launches, summed HIP-event time (ms), algorithmic flops and bytes of one class."""
    n = ctypes.c_int32()
    ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    check(lib().mpdo_profile_read(cls, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(by)))
    return {"launches": n.value, "ms": ms.value, "flops": fl.value, "bytes": by.value}


def run_program(prog, state: MPDO, channels: Sequence[Channel]) -> MPDO:
    """Apply a workloads.Program gate by gate through the C ABI."""
    for op in prog.ops:
        if op.chan >= 0:
            state.apply_channel(op.sites, channels[op.chan], op.U)
        else:
            state.apply_gate(op.sites, op.U)
    state.flush()
    return state


# ---------------------------------------------------------------------------
# kernel-level test entry points (include/mpdo_testing.h)
# ---------------------------------------------------------------------------
def _testing_lib():
    L = lib()
    if not getattr(L, "_testing_sig", False):
        pd = ctypes.POINTER(ctypes.c_double)
        i32 = ctypes.c_int32
        L.mpdo_test_gemm.argtypes = [i32] * 6 + [pd, i32, i32, pd, i32, i32, pd, i32, i32, ctypes.c_double, pd, i32,
                                                 i32]
        L.mpdo_test_gemm.restype = ctypes.c_int
        L.mpdo_test_eigh.argtypes = [i32, i32, pd, pd, pd, pd]
        L.mpdo_test_gemm_rate.argtypes = [i32] * 6 + [pd]
        L.mpdo_test_gemm_rate.restype = ctypes.c_int
        L.mpdo_test_eigh.restype = ctypes.c_int
        L.mpdo_test_eig_residual_bound.argtypes = [ctypes.c_double]
        L.mpdo_test_eig_residual_bound.restype = ctypes.c_int
        L.mpdo_test_fail_next_update.argtypes = [i32]
        L.mpdo_test_fail_next_update.restype = ctypes.c_int
        L.mpdo_test_profile_site.argtypes = [i32, ctypes.POINTER(i32), pd, pd]
        L.mpdo_test_profile_site.restype = ctypes.c_int
        L.mpdo_test_gemm_form.argtypes = [i32, i32, i32, ctypes.POINTER(i32)]
        L.mpdo_test_gemm_form.restype = ctypes.c_int
        L.mpdo_test_eig_band.argtypes = [i32, ctypes.POINTER(i32)]
        L.mpdo_test_eig_band.restype = ctypes.c_int
        L.mpdo_test_eig_coop.argtypes = [i32, ctypes.POINTER(i32)]
        L.mpdo_test_eig_coop.restype = ctypes.c_int
        L.mpdo_test_gram_vector.argtypes = [i32, ctypes.POINTER(i32)]
        L.mpdo_test_gram_vector.restype = ctypes.c_int
        L._testing_sig = True
    return L


def test_eig_residual_bound(rtol: float) -> None:
    """Residual bound of the eigensolver (0: the default 1e-9; negative:
    every eigenpair fails its check)."""
    check(_testing_lib().mpdo_test_eig_residual_bound(float(rtol)))


GEMM_SITES = ("other", "q1_gram", "q1_proj", "q2_gram_E", "q2_theta", "q2_gram_H", "q2_theta2", "q2_gram_C",
              "q2_X", "q2_out", "transfer_R", "transfer_L", "q3_gram_NE", "q3_Xt", "q3_Psi", "q3_gram_H", "q3_Psi2",
              "q3_gram_C1", "q3_Y1", "q3_W1", "q3_gram_C2", "q3_Y3", "q3_out", "sweep_gram", "sweep_out")


def profile_sites() -> dict:
    """Per call site of the GEMM: launches, summed event ms, algorithmic
    flops and TFLOP/s (sites with launches only)."""
    L = _testing_lib()
    out = {}
    for i, name in enumerate(GEMM_SITES):
        n = ctypes.c_int32()
        ms, fl = ctypes.c_double(), ctypes.c_double()
        check(L.mpdo_test_profile_site(i, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl)))
        if n.value:
            out[name] = {"launches": n.value, "ms": ms.value, "flops": fl.value,
                         "tflops": fl.value / (ms.value * 1e-3) / 1e12 if ms.value > 0 else 0.0}
    return out


def gemm_form(prec: int, tile: int, form: int) -> int:
    """Set the complex-product form (3 or 4 real products) of the GEMM
    launches of one MFMA precision (0: FP64, 1: FP32) and tile edge; returns
    the previous form."""
    prev = ctypes.c_int32()
    check(_testing_lib().mpdo_test_gemm_form(prec, tile, form, ctypes.byref(prev)))
    return prev.value


def eig_band(on: bool) -> bool:
    """Route 128 < n <= 256 eigenproblems through the two-stage band
    reduction (True) or the one-stage panel reduction (False, the default);
    returns the previous setting."""
    prev = ctypes.c_int32()
    check(_testing_lib().mpdo_test_eig_band(1 if on else 0, ctypes.byref(prev)))
    return bool(prev.value)


def eig_coop(on: bool) -> bool:
    """Share each matrix of launches with at most 32 eigenproblems of n > 128
    among several workgroups during the reduction to tridiagonal form (True,
    the default) or keep one workgroup per matrix (False); returns the
    previous setting."""
    prev = ctypes.c_int32()
    check(_testing_lib().mpdo_test_eig_coop(1 if on else 0, ctypes.byref(prev)))
    return bool(prev.value)


def gram_vector(on: bool) -> bool:
    """Run the one- and two-site inner Grams on the vector units when their
    size (2 kappa_max, 4 kappa_max) is at most 16 (True, the default) or on
    the MFMA GEMM kernel (False); returns the previous setting."""
    prev = ctypes.c_int32()
    check(_testing_lib().mpdo_test_gram_vector(1 if on else 0, ctypes.byref(prev)))
    return bool(prev.value)


def e_cholesky(on: bool) -> bool:
    """Build the two-site update's right-factor basis from a pivoted Cholesky
    factorisation of E (True, the default) or from its eigendecomposition
    (False); returns the previous setting."""
    prev = ctypes.c_int32()
    check(_testing_lib().mpdo_test_e_cholesky(1 if on else 0, ctypes.byref(prev)))
    return bool(prev.value)


def test_fail_next_update(status: int) -> None:
    """The next sublayer of gates fails with `status` before launching."""
    check(_testing_lib().mpdo_test_fail_next_update(int(status)))


def test_gemm(prec: int, opA: int, opB: int, M: int, N: int, K: int, A: np.ndarray, B: np.ndarray,
              w: Optional[np.ndarray] = None, wdiv: int = 1, splits: int = 1, alpha: float = 1.0,
              tile: int = 64, herm: bool = False) -> np.ndarray:
    """Run the library GEMM kernel once: alpha op(A) op(B), A and B 2-D complex.
    herm: C is Hermitian; only its tiles on and above the diagonal are
    computed (those below are returned as 0)."""
    A = np.ascontiguousarray(A, dtype=np.complex128)
    B = np.ascontiguousarray(B, dtype=np.complex128)
    a, b = _cplx(A), _cplx(B)
    ww = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    out = np.zeros(2 * M * N)
    check(_testing_lib().mpdo_test_gemm(prec, opA, opB, M, N, K, _dptr(a), A.shape[0], A.shape[1], _dptr(b),
                                        B.shape[0], B.shape[1], _dptr(ww), wdiv, splits, alpha, _dptr(out), tile,
                                        int(herm)))
    return out.view(np.complex128).reshape(M, N)


def test_eigh(A: np.ndarray, kvec: Optional[int] = None):
    """Library eigensolver on host data: (leading eigenvalues, eigenvectors, trace)."""
    A = np.ascontiguousarray(A, dtype=np.complex128)
    n = A.shape[0]
    kvec = n if kvec is None else kvec
    a = _cplx(A)
    ev = np.zeros(n)
    vec = np.zeros(2 * n * n)
    tr = ctypes.c_double()
    check(_testing_lib().mpdo_test_eigh(n, kvec, _dptr(a), _dptr(ev), _dptr(vec), ctypes.byref(tr)))
    return ev, vec.view(np.complex128).reshape(n, n), tr.value


def test_gemm_rate(prec: int, M: int, N: int, K: int, items: int = 1, reps: int = 10) -> float:
    """Average milliseconds per launch of `items` complex M x K by K x N
    products on full tiles (prec 0: FP64 MFMA, 1: FP32 MFMA)."""
    ms = ctypes.c_double()
    check(_testing_lib().mpdo_test_gemm_rate(prec, M, N, K, items, reps, ctypes.byref(ms)))
    return ms.value


class MPO:
    """rho of a state as the chain of local density tensors (Eq. (6)), on the
    GPU, for error mitigation by inverse maps (Sec. V; include/mpdo.h,
    mpdo_mpo_*).  Runs on the stream of the state it was made from."""

    def __init__(self, state: "MPDO", d_max: int = 256, cutoff: float = 0.0):
        self.n = state.n
        h = ctypes.c_void_p()
        check(lib().mpdo_mpo_from_state(state._h, d_max, cutoff, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().mpdo_mpo_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def apply_gate(self, site: int, U: np.ndarray, inverse: bool = False) -> None:
        U = np.asarray(U, dtype=np.complex128)
        q = int(round(np.log2(U.shape[0])))
        u = _cplx(U)
        check(lib().mpdo_mpo_apply_gate(self._h, site, q, _dptr(u), 1 if inverse else 0))

    def apply_channel(self, site: int, ch: Channel, inverse: bool = False) -> None:
        check(lib().mpdo_mpo_apply_channel(self._h, site, ch.handle, 1 if inverse else 0))

    def expect_products(self, ops: np.ndarray) -> np.ndarray:
        """ops: (nops, n, 2, 2) complex -> Tr(O rho) (unnormalised) for each."""
        ops = np.asarray(ops, dtype=np.complex128)
        buf = _cplx(ops)
        out = np.zeros(2 * ops.shape[0])
        check(lib().mpdo_mpo_expect(self._h, _dptr(buf), ops.shape[0], _dptr(out)))
        return out.view(np.complex128)

    def dims(self):
        b = (ctypes.c_int32 * max(1, self.n - 1))()
        d = ctypes.c_double()
        check(lib().mpdo_mpo_dims(self._h, b, ctypes.byref(d)))
        return list(b)[: self.n - 1], d.value

    def to_dense(self) -> np.ndarray:
        d = 1 << self.n
        out = np.zeros(2 * d * d)
        check(lib().mpdo_mpo_to_dense(self._h, _dptr(out)))
        return out.view(np.complex128).reshape(d, d)
