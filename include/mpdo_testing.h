/*
 * libmpdo kernel-level entry points for unit tests (C ABI).
 *
 * These run one of the library's internal kernels on host data so that a
 * test can compare it with a reference on the CPU.  All buffers are host
 * memory owned by the caller; complex values are interleaved (re, im)
 * doubles; matrices are row-major.  Each call allocates, copies, runs on the
 * default stream, copies back and synchronises.  Errors: MPDO_EINVAL for bad
 * sizes or modes, MPDO_EDEVICE / MPDO_ENOMEM for HIP failures.
 */
#ifndef MPDO_TESTING_H
#define MPDO_TESTING_H

#include "mpdo.h"

#ifdef __cplusplus
extern "C" {
#endif

/* C = alpha * op(A) op(B) with the batched MFMA GEMM.
 *   prec: 0 = complex128 on FP64 MFMA, 1 = complex64 on FP32 MFMA,
 *         2 = complex64 inputs with FP64 MFMA and complex128 output.
 *   opA, opB: 0 = N, 1 = T, 2 = conj, 3 = conj-transpose (element (i, k) of
 *   op(A) is A[i*lda+k], A[k*lda+i], conj(A[i*lda+k]), conj(A[k*lda+i])).
 *   A holds rowsA x lda values, B rowsB x ldb; C is M x N (leading dim N).
 *   w (may be NULL): real weights, op(A)(i, k) is multiplied by w[k / wdiv].
 *   splits: split-K count (1..64).
 *   tile: output tile edge of the kernel variant, 64 or 32.
 *   herm: 1 = C is Hermitian (M == N, e.g. a Gram matrix A^H A): only the
 *   tiles on and above the diagonal are computed, the entries of the tiles
 *   below it are returned as 0; 0 = the full product.  EINVAL for herm = 1
 *   with M != N or any other value. */
mpdo_status mpdo_test_gemm(int32_t prec, int32_t opA, int32_t opB, int32_t M, int32_t N, int32_t K,
                           const double* A, int32_t rowsA, int32_t lda, const double* B, int32_t rowsB,
                           int32_t ldb, const double* w, int32_t wdiv, int32_t splits, double alpha, double* C,
                           int32_t tile, int32_t herm);

/* Throughput of the batched MFMA GEMM on full tiles: items independent
 * products C = A B (op N, N; M x K times K x N, complex128 on FP64 MFMA for
 * prec 0, complex64 on FP32 MFMA for prec 1) on device operands the call
 * allocates and fills; one warm-up launch, then reps launches (1..1000)
 * between HIP events; *ms = average milliseconds per launch.  EINVAL when
 * the operands would exceed 32 GiB. */
mpdo_status mpdo_test_gemm_rate(int32_t prec, int32_t M, int32_t N, int32_t K, int32_t items, int32_t reps,
                                double* ms);

/* Hermitian eigendecomposition of A (n x n, 1 <= n <= 1024) with the
 * library's eigensolver: the leading min(n, kvec + 1) eigenvalues in
 * descending order in evals (the rest of the n entries zero), the
 * eigenvectors of the leading kvec eigenvalues as the first kvec columns of
 * evecs (n x n complex, row-major; eigenvectors of eigenvalues at or below
 * 1e-13 times the largest are zero), and Tr(A) in *trace (may be NULL). */
mpdo_status mpdo_test_eigh(int32_t n, int32_t kvec, const double* A, double* evals, double* evecs,
                           double* trace);

/* Failure injection for the tests of error handling (forced from the host;
 * every kernel still runs to its normal end):
 *   mpdo_test_eig_residual_bound: residual bound of the eigensolver on the
 *     current device, relative to ||T|| (0 restores 1e-9; a negative bound
 *     makes every eigenpair fail its check, which the library reports as
 *     ENOTCONV);
 *   mpdo_test_fail_next_update: the next sublayer of gates of any handle
 *     fails with `status` before launching anything (0 cancels). */
mpdo_status mpdo_test_eig_residual_bound(double rtol);

/* Complex-product form of the GEMM launches of one MFMA precision (prec 0:
 * FP64, 1: FP32) and tile edge (32 or 64), process-wide: form 4 = four real
 * MFMA products per complex product, form 3 = Gauss's three (P1 = Ar Br,
 * P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi); Re = P1 - P2, Im = P3 - P1 - P2).
 * *previous (may be NULL) receives the form in force before the call.  The
 * defaults: 3 for FP32, 4 for FP64. */
mpdo_status mpdo_test_gemm_form(int32_t prec, int32_t tile, int32_t form, int32_t* previous);

/* Profile of one GEMM call site of the MPDO update (while profiling is on,
 * see mpdo_profile_enable): launches, summed HIP-event milliseconds and
 * algorithmic flops of the contractions labelled `site` (0: other; 1-2 the
 * one-site update's Gram and projection; 3-9 the two-site update's E Gram,
 * theta, H Gram, theta'', C Gram, X and output products; 10-11 right and left
 * transfer steps; 12-22 the three-site update; 23-24 the truncation sweep).
 * EINVAL outside 0..24. */
mpdo_status mpdo_test_profile_site(int32_t site, int32_t* launches, double* ms, double* flops);
mpdo_status mpdo_test_fail_next_update(int32_t status);

/* Eigenproblems with 128 < n <= 256 through the two-stage reduction via a
 * band of half-width 16 (on = 1) or the one-stage panel reduction (on = 0,
 * the default); process-wide.  *previous (may be NULL) receives the
 * setting before the call.  EINVAL unless on is 0 or 1. */
mpdo_status mpdo_test_eig_band(int32_t on, int32_t* previous);

/* Eigenproblems with n > 128 in launches of at most 32 matrices: several
 * workgroups share each matrix during the Householder reduction to
 * tridiagonal form, one launch per step while the trailing block is wider
 * than 128, then one workgroup per matrix finishes (on = 1, the default); or
 * one workgroup per matrix throughout (on = 0).  Same results up to rounding
 * order.  Process-wide; *previous (may be NULL) receives the setting before
 * the call.  EINVAL unless on is 0 or 1. */
mpdo_status mpdo_test_eig_coop(int32_t on, int32_t* previous);

/* The inner-index Grams of the one- and two-site updates (Eq. (9): the
 * lambda^2-weighted Gram of the site tensor, or of the two-site block in the
 * right factor's basis, over its bond indices) on the vector units when
 * their size 2 kappa_max, 4 kappa_max is at most 16 (on = 1, the default),
 * or on the MFMA GEMM kernel (on = 0).  Same results up to rounding order.
 * Process-wide; *previous (may be NULL) receives the setting before the
 * call.  EINVAL unless on is 0 or 1. */
mpdo_status mpdo_test_gram_vector(int32_t on, int32_t* previous);

/* The basis of the two-site update's right factor (E = F F^H, n = 2 chi <=
 * 128): a pivoted Cholesky factorisation of E (on = 1, the default) or its
 * eigendecomposition (on = 0); both give F = L_F Q with orthonormal rows Q
 * (Sec. II.D splits are unchanged).  Process-wide; *previous (may be NULL)
 * receives the setting before the call.  EINVAL unless on is 0 or 1. */
mpdo_status mpdo_test_e_cholesky(int32_t on, int32_t* previous);

#ifdef __cplusplus
}
#endif
#endif /* MPDO_TESTING_H */
