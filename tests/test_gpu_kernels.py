"""Kernel unit tests on the GPU: the MFMA complex GEMM (every operand mode,
ragged shapes, split-K, weights, all precisions) and the Hermitian
eigensolver (register-resident and global-memory variants), each against
NumPy; and the profiler's launch and work accounting."""
import numpy as np
import pytest

from paper_2508_07610_amd import mpdo as M
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _op(X, mode):
    return {0: X, 1: X.T, 2: X.conj(), 3: X.conj().T}[mode]


def _rand(shape, rng):
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


@pytest.mark.parametrize("M_,N_,K_", [(1, 1, 1), (16, 16, 4), (64, 64, 16), (65, 70, 33), (130, 37, 257),
                                      (5, 300, 9)])
@pytest.mark.parametrize("opA,opB", [(0, 0), (1, 0), (2, 1), (3, 3), (0, 3), (3, 0)])
@pytest.mark.parametrize("tile", [64, 32])
def test_gemm_fp64(M_, N_, K_, opA, opB, tile):
    require_gpu()
    rng = np.random.default_rng(M_ * 1000 + N_ * 10 + K_)
    A = _rand((K_, M_) if opA in (1, 3) else (M_, K_), rng)
    B = _rand((N_, K_) if opB in (1, 3) else (K_, N_), rng)
    C = M.test_gemm(0, opA, opB, M_, N_, K_, A, B, alpha=0.75, tile=tile)
    ref = 0.75 * _op(A, opA) @ _op(B, opB)
    err = float(np.abs(C - ref).max())
    bad = np.argwhere(np.abs(C - ref) > 1e-9)[:8].tolist()
    assert err <= 1e-12 * max(1.0, float(np.abs(ref).max())) * np.sqrt(K_), (err, bad)


@pytest.mark.parametrize("M_,N_,K_", [(1, 1, 1), (65, 70, 33), (130, 37, 257), (5, 300, 9)])
@pytest.mark.parametrize("opA,opB", [(0, 0), (2, 1), (3, 0)])
@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("tile", [64, 32])
def test_gemm_three_product_form(M_, N_, K_, opA, opB, prec, tile):
    """Gauss's three-product form of the complex product against NumPy, in
    every precision (FP64 MFMA for prec 0 and 2, FP32 for prec 1)."""
    require_gpu()
    fp64 = 0 if prec != 1 else 1
    prev = M.gemm_form(fp64, tile, 3)
    try:
        rng = np.random.default_rng(M_ * 100 + N_ + K_ + prec)
        A = _rand((K_, M_) if opA in (1, 3) else (M_, K_), rng)
        B = _rand((N_, K_) if opB in (1, 3) else (K_, N_), rng)
        C = M.test_gemm(prec, opA, opB, M_, N_, K_, A, B, alpha=0.5, tile=tile)
    finally:
        M.gemm_form(fp64, tile, prev)
    if prec:
        A, B = A.astype(np.complex64).astype(np.complex128), B.astype(np.complex64).astype(np.complex128)
    ref = 0.5 * _op(A, opA) @ _op(B, opB)
    tol = (3e-6 if prec == 1 else 3e-12) * max(1.0, float(np.abs(ref).max())) * np.sqrt(K_)
    err = float(np.abs(C - ref).max())
    assert err <= tol, (err, tol)


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("tile", [64, 32])
def test_gemm_fp32_paths(prec, tile):
    require_gpu()
    rng = np.random.default_rng(3)
    A = _rand((200, 96), rng)
    B = _rand((96, 150), rng)
    C = M.test_gemm(prec, 0, 0, 200, 150, 96, A, B, tile=tile)
    A32, B32 = A.astype(np.complex64), B.astype(np.complex64)
    ref = A32.astype(np.complex128) @ B32.astype(np.complex128)
    tol = 1e-5 if prec == 1 else 1e-12
    err = float(np.abs(C - ref).max() / np.abs(ref).max())
    bad = np.argwhere(np.abs(C - ref) > 1e-3)[:8].tolist()
    assert err < tol, (err, bad)


@pytest.mark.parametrize("tile", [64, 32])
def test_gemm_split_k_and_weights(tile):
    """Weighted Gram with split-K: C = A^H diag(w[k / wdiv]) A."""
    require_gpu()
    rng = np.random.default_rng(4)
    K_, N_ = 4100, 48
    A = _rand((K_, N_), rng)
    w = rng.uniform(0.1, 2.0, size=(K_ + 3) // 4)
    C = M.test_gemm(0, 3, 0, N_, N_, K_, A, A, w=w, wdiv=4, splits=7, tile=tile)
    wk = np.repeat(w, 4)[:K_]
    ref = A.conj().T @ (wk[:, None] * A)
    err = float(np.abs(C - ref).max() / np.abs(ref).max())
    assert err < 1e-13, err


@pytest.mark.parametrize("N_,K_,splits", [(1, 3, 1), (48, 70, 1), (64, 33, 2), (100, 257, 3), (130, 40, 1),
                                           (257, 96, 5), (300, 128, 1)])
@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("tile", [64, 32])
def test_gemm_hermitian_tiles(N_, K_, splits, prec, tile):
    """Hermitian C = A^H diag(w) A with only the tiles on and above the
    diagonal launched (numbered along the upper triangle): every entry of
    those tiles equals the full product, every tile below the diagonal is
    left untouched (0)."""
    require_gpu()
    rng = np.random.default_rng(N_ * 7 + K_ + splits)
    A = _rand((K_, N_), rng)
    w = rng.uniform(0.5, 1.5, size=K_)
    C = M.test_gemm(prec, 3, 0, N_, N_, K_, A, A, w=w, splits=splits, tile=tile, herm=True)
    Ar = A.astype(np.complex64).astype(np.complex128) if prec else A
    ref = Ar.conj().T @ (w[:, None] * Ar)
    tm = np.arange(N_)[:, None] // tile
    tn = np.arange(N_)[None, :] // tile
    upper = tm <= tn
    tol = (1e-4 if prec == 1 else 1e-12) * float(np.abs(ref).max())
    err = float(np.abs(np.where(upper, C - ref, 0)).max())
    assert err < tol, (err, np.argwhere(upper & (np.abs(C - ref) > tol))[:8].tolist())
    assert not np.any(C[~upper]), "a tile below the diagonal was written"


@pytest.mark.parametrize("n", [1, 2, 3, 8, 17, 32, 64, 65, 100, 128, 129, 255, 256, 257, 512, 513, 1024])
def test_eigh_against_numpy(n):
    require_gpu()
    rng = np.random.default_rng(n)
    X = _rand((n, n + 3), rng)
    A = X @ X.conj().T                      # Gram-like PSD
    ev, V, tr = M.test_eigh(A)
    ref = np.sort(np.linalg.eigvalsh(A))[::-1]
    scale = float(np.abs(ref).max())
    e1 = float(np.abs(ev - ref).max()) / scale
    e2 = float(np.abs(V.conj().T @ V - np.eye(n)).max())
    e3 = float(np.abs(A @ V - V * ev).max()) / scale
    # inverse iteration: orthogonality ~ eps ||A|| / gap for the dense
    # Wishart spectrum near zero (the gaps there shrink as n grows), residuals
    # at eps
    assert e1 <= 1e-13 and e2 < 2e-14 * max(n, 500) and e3 < 1e-12, (e1, e2, e3)
    assert abs(tr - np.trace(A).real) < 1e-12 * scale * n
    assert bool(np.all(np.diff(ev) <= 0))


@pytest.mark.parametrize("n,kvec", [(20, 3), (32, 8), (32, 15), (33, 8), (40, 5), (64, 9), (100, 8), (128, 8), (128, 9),
                                    (128, 16), (129, 64), (200, 40), (256, 1), (256, 64), (256, 65), (300, 100),
                                    (700, 17), (1024, 16)])
def test_eigh_leading_subset(n, kvec):
    """Only the leading kvec eigenpairs (and kvec + 1 eigenvalues) are produced."""
    require_gpu()
    rng = np.random.default_rng(n + kvec)
    X = _rand((n, n // 2), rng)              # rank-deficient
    A = X @ X.conj().T
    ev, V, tr = M.test_eigh(A, kvec)
    ref = np.sort(np.linalg.eigvalsh(A))[::-1]
    scale = float(ref[0])
    kb = min(n, kvec + 1)
    assert float(np.abs(ev[:kb] - ref[:kb]).max()) <= 1e-13 * scale
    assert bool(np.all(ev[kb:] == 0))
    Vk = V[:, :kvec]
    e2 = float(np.abs(Vk.conj().T @ Vk - np.eye(kvec)).max())
    e3 = float(np.abs(A @ Vk - Vk * ev[:kvec]).max()) / scale
    assert e2 < 1e-12 and e3 < 1e-12, (e2, e3)


@pytest.mark.parametrize("n", [24, 40, 200])
def test_eigh_rank_deficient_and_degenerate(n):
    """One case per eigensolver variant (n <= 32, n <= 128, n <= 256)."""
    require_gpu()
    rng = np.random.default_rng(9 + n)
    Q, _ = np.linalg.qr(_rand((n, n), rng))
    d = np.array([5.0, 5.0, 2.0] + [1e-9] * 5 + [0.0] * (n - 8))
    A = (Q * d) @ Q.conj().T
    ev, V, _ = M.test_eigh(A)
    e1 = float(np.abs(ev - np.sort(d)[::-1]).max())
    assert e1 < 1e-13 * 5, e1
    # the leading eigenspace (degenerate pair) is recovered exactly
    P = V[:, :2] @ V[:, :2].conj().T
    Pref = Q[:, :2] @ Q[:, :2].conj().T
    e2 = float(np.abs(P - Pref).max())
    assert e2 < 1e-12, e2
    # the 1e-9 multiplet: an orthonormal basis of its eigenspace
    P = V[:, 3:8] @ V[:, 3:8].conj().T
    Pref = Q[:, 3:8] @ Q[:, 3:8].conj().T
    assert float(np.abs(P - Pref).max()) < 1e-6
    # null space (below 1e-13 of the largest eigenvalue): zero vectors
    assert float(np.abs(V[:, 8:]).max()) == 0.0


def test_eigh_diagonal_and_tiny():
    """Already-diagonal input (every reflector trivial) and a 1 x 1 matrix."""
    require_gpu()
    d = np.array([3.0, -1.0, 2.0, 0.5])
    ev, V, tr = M.test_eigh(np.diag(d).astype(complex))
    assert np.allclose(ev, [3.0, 2.0, 0.5, -1.0], atol=1e-15)
    assert abs(tr - d.sum()) < 1e-15
    ev, V, tr = M.test_eigh(np.array([[2.5 + 0j]]))
    assert abs(ev[0] - 2.5) < 1e-15 and abs(abs(V[0, 0]) - 1) < 1e-15


def test_profiler_counts_gemm_and_eig_work():
    require_gpu()
    rng = np.random.default_rng(5)
    A, B = _rand((70, 33), rng), _rand((33, 90), rng)
    M.profile_enable(True)
    M.test_gemm(0, 0, 0, 70, 90, 33, A, B)
    g = M.profile_read(M.PROF_GEMM_F64)
    X = _rand((100, 100), rng)
    M.test_eigh(X @ X.conj().T, 10)
    e = M.profile_read(M.PROF_EIG_REG)
    Y = _rand((200, 200), rng)
    prev = M.eig_band(True)
    try:
        M.test_eigh(Y @ Y.conj().T, 20)
    finally:
        M.eig_band(prev)
    e2 = M.profile_read(M.PROF_EIG_BAND)
    Z = _rand((300, 300), rng)
    M.test_eigh(Z @ Z.conj().T, 30)
    e3 = M.profile_read(M.PROF_EIG_GLOBAL)
    M.profile_enable(False)
    assert g["launches"] == 1 and g["ms"] > 0
    assert g["flops"] == 8.0 * 70 * 90 * 33
    assert g["bytes"] == 16.0 * (70 * 33 + 33 * 90 + 70 * 90)
    assert e["launches"] == 1 and abs(e["flops"] - (16.0 / 3.0 * 100 ** 3 + 8.0 * 100 ** 2 * 10)) < 1.0
    assert e2["launches"] == 1 and abs(e2["flops"] - (16.0 / 3.0 * 200 ** 3 + 8.0 * 200 ** 2 * 20)) < 1.0
    assert e3["launches"] == 1 and abs(e3["flops"] - (16.0 / 3.0 * 300 ** 3 + 8.0 * 300 ** 2 * 30)) < 1.0


@pytest.mark.parametrize("band", [True, False])
@pytest.mark.parametrize("n,kvec", [(129, 129), (144, 20), (200, 64), (256, 65), (256, 256)])
def test_eigh_band_and_panel_paths(band, n, kvec):
    """128 < n <= 256 through the two-stage reduction (dense -> band of
    half-width 16 by blocked Householder, bulge chasing to tridiagonal,
    back-transformation through both) and through the one-stage panel
    reduction: eigenvalues to 1e-13, orthonormal vectors and residuals to
    1e-12 of the largest eigenvalue, on a spectrum with a degenerate pair, a
    tight cluster and a null space (as in a bond Gram)."""
    require_gpu()
    rng = np.random.default_rng(n + kvec)
    Q, _ = np.linalg.qr(_rand((n, n), rng))
    d = np.concatenate([[3.0, 3.0], np.sort(rng.uniform(0.0, 1.0, n // 2))[::-1],
                        1e-3 * (1 + 1e-9 * np.arange(6)), np.zeros(n - n // 2 - 8)])
    A = (Q * d) @ Q.conj().T
    prev = M.eig_band(band)
    prev_coop = M.eig_coop(False)  # one workgroup per matrix: the panel kernel itself
    try:
        ev, V, tr = M.test_eigh(A, kvec)
    finally:
        M.eig_band(prev)
        M.eig_coop(prev_coop)
    ref = np.sort(np.linalg.eigvalsh(A))[::-1]
    kb = min(n, kvec + 1)
    assert float(np.abs(ev[:kb] - ref[:kb]).max()) <= 1e-13 * 3
    assert abs(tr - np.trace(A).real) < 1e-12 * n
    kz = int(np.sum(ref[:kvec] > 1e-13 * ref[0]))
    Vk = V[:, :kz]
    assert float(np.abs(Vk.conj().T @ Vk - np.eye(kz)).max()) < 1e-12
    assert float(np.abs(A @ Vk - Vk * ev[:kz]).max()) < 1e-12 * 3
    assert float(np.abs(V[:, kz:kvec]).max(initial=0.0)) == 0.0


def test_gemm_rate_entry_point():
    """mpdo_test_gemm_rate times launches on device operands; bad sizes are
    rejected before any allocation."""
    require_gpu()
    ms = M.test_gemm_rate(0, 256, 256, 256, 2, 3)
    assert 0 < ms < 1000
    assert 0 < M.test_gemm_rate(1, 128, 64, 32, 1, 1) < 1000
    for bad in ((2, 64, 64, 64, 1, 1), (0, 0, 64, 64, 1, 1), (0, 64, 64, 64, 1, 0), (0, 65536, 65536, 4096, 1, 1)):
        with pytest.raises(M.MPDOError) as e:
            M.test_gemm_rate(*bad)
        assert e.value.status == M.EINVAL


@pytest.mark.parametrize("n,kvec", [(129, 129), (130, 8), (200, 64), (257, 257), (258, 65), (300, 100), (513, 64),
                                    (700, 17), (1024, 16), (1024, 1024)])
def test_eigh_shared_reduction(n, kvec):
    """Lone eigenproblems with n > 128 go through the reduction shared by
    several workgroups (one launch per Householder step while the trailing
    block is wider than 128, one workgroup for the rest): eigenvalues to
    1e-13, residuals to 1e-12 of the largest eigenvalue, orthonormal vectors
    to 2e-14 max(n, 500) (inverse iteration: eps ||A|| / gap, and n / 2
    eigenvalues in [0, 1] leave gaps of about 2 / n), with the degenerate
    pair, the cluster and the null space of a bond Gram; the one-workgroup
    kernels give the same to rounding."""
    require_gpu()
    rng = np.random.default_rng(3 * n + kvec)
    Q, _ = np.linalg.qr(_rand((n, n), rng))
    d = np.concatenate([[3.0, 3.0], np.sort(rng.uniform(0.0, 1.0, n // 2))[::-1],
                        1e-3 * (1 + 1e-9 * np.arange(6)), np.zeros(n - n // 2 - 8)])
    A = (Q * d) @ Q.conj().T
    ref = np.sort(np.linalg.eigvalsh(A))[::-1]
    kb = min(n, kvec + 1)
    kz = int(np.sum(ref[:kvec] > 1e-13 * ref[0]))
    out = {}
    for coop in (True, False):
        prev = M.eig_coop(coop)
        try:
            out[coop] = M.test_eigh(A, kvec)
        finally:
            M.eig_coop(prev)
        ev, V, tr = out[coop]
        assert float(np.abs(ev[:kb] - ref[:kb]).max()) <= 1e-13 * 3, coop
        assert abs(tr - np.trace(A).real) < 1e-12 * n
        Vk = V[:, :kz]
        assert float(np.abs(Vk.conj().T @ Vk - np.eye(kz)).max()) < 2e-14 * max(n, 500), coop
        assert float(np.abs(A @ Vk - Vk * ev[:kz]).max()) < 1e-12 * 3, coop
        assert float(np.abs(V[:, kz:kvec]).max(initial=0.0)) == 0.0
    assert float(np.abs(out[True][0] - out[False][0]).max()) <= 1e-13 * 3
