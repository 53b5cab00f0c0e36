// Shared device/host definitions of libmpdo (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpdo {

// Interleaved complex number of real type R.
template <typename R> struct cpx { R re, im; };

template <typename R> __host__ __device__ inline cpx<R> mk(R a, R b) { cpx<R> z; z.re = a; z.im = b; return z; }
template <typename R> __host__ __device__ inline cpx<R> operator+(cpx<R> a, cpx<R> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename R> __host__ __device__ inline cpx<R> operator-(cpx<R> a, cpx<R> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename R> __host__ __device__ inline cpx<R> operator*(cpx<R> a, cpx<R> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename R> __host__ __device__ inline cpx<R> operator*(R s, cpx<R> a) { return mk(s * a.re, s * a.im); }
template <typename R> __host__ __device__ inline cpx<R> cconj(cpx<R> a) { return mk(a.re, -a.im); }
template <typename R> __host__ __device__ inline R cabs2(cpx<R> a) { return a.re * a.re + a.im * a.im; }

// Operand modes of the batched GEMM: element (i, k) of op(A) is
//   N: A[i*ld + k]   T: A[k*ld + i]   C: conj(A[i*ld + k])   H: conj(A[k*ld + i])
enum Op : int { OP_N = 0, OP_T = 1, OP_C = 2, OP_H = 3 };

// One product C[s] (+)= alpha * op(A) op(B) of a batch.  All sizes are read
// on the device, so a launch sized for the largest shape serves ragged items
// whose dimensions were produced by earlier kernels.
//
// The K index may be two-level: the memory offset of k is
//   (k / kinner) * kstride + (k % kinner)
// which lets one product run over a sum of blocks (a weighted Gram matrix
// over an outer index).  Optional real weights w[k / wdiv] multiply op(A).
// An inner batch of nbatch products uses strides sA, sB, sC.  With
// splits > 1 the K range is cut into `splits` parts and part s is written to
// C + s * sSplit (summed later by reduce_splits).
struct GemmDesc {
  const void* A;
  const void* B;
  void* C;
  const double* w;
  long long kstride;
  long long sA, sB, sC, sSplit;
  int M, N, K;
  int lda, ldb, ldc;
  int kinner, wdiv;
  int nbatch, splits;
  int opA, opB;
  int beta;        // 0: overwrite, 1: accumulate
  int active;      // 0: item skipped
  int herm;        // 1: C is Hermitian (a Gram matrix): only its upper
                   // triangle of tiles is computed (and reduced)
  int hpad;
  double alpha;
};

// A Hermitian eigenproblem of size n (1 <= n <= EIG_NMAX).  The matrix at `a`
// (n x n, row-major, leading dimension lda, complex double) is read only.
// The leading kb = min(n, kvec + 1) eigenvalues are written in descending
// order to evals[0..kb) (the rest of evals[0..n) is set to zero), *trace
// receives Tr(A), and the eigenvectors of the leading kvec eigenvalues are
// written as the columns of `evecs` (n x kvec used of an n x n array with
// leading dimension n).  Eigenvectors of eigenvalues at or below
// vfloor * evals[0] (EIG_FLOOR when vfloor is 0) are returned as zero
// (numerical null space).
// `work` must hold eig_work_doubles(n) doubles.
struct EigDesc {
  double* a;
  double* evals;
  double* evecs;
  double* work;
  double* trace;
  double vfloor;  // relative floor of the returned vectors; 0: EIG_FLOOR
  int n, lda;
  int kvec;
  int active;
  int upper;      // 1: only the upper triangle of `a` is valid (lower = conj)
  int upad;
};

// Per-site record of the truncations applied to a site (device, doubles):
// summed discarded weight, largest single discarded weight, number of
// truncations, smallest relative gap eta_{r-1}/eta_r - 1 at a cut that
// dropped weight, numerical failures (non-finite weights, an eigensolver
// residual above its bound, a non-positive or non-finite trace).
enum StatField : int { ST_DISC = 0, ST_MAXD = 1, ST_CUTS = 2, ST_GAP = 3, ST_FAIL = 4, ST_W = 5 };

// Relative floor of the Gram eigenvalues the library keeps (its FP64 Gram
// matrices resolve eigenvalues to about 1e-15 of the largest; below this
// floor an eigenvector is noise).  A truncation with cutoff >= N * 1e-13
// (N the Gram size, <= 1024) cannot be changed by the floor.
constexpr double EIG_FLOOR = 1e-13;
constexpr int EIG_NMAX = 1024;
constexpr int EIG_THREADS = 512;

// matrix (2 n^2) + two n x np solve vectors + five n x np factor arrays
// and, for 128 < n <= 256 (the band path), the panels' T (16 of 16 x 16)
// and the bulge-chasing reflectors (at most n^2 / 32 + n records of 18)
__host__ __device__ inline long long eig_work_doubles(int n) {
  const long long np = (n + 63) / 64 * 64;
  const long long band = (n > 128 && n <= 256) ? 2LL * 16 * 256 + 36LL * ((long long)n * n / 32 + n) : 0;
  return 2LL * n * n + 7LL * n * np + 64 + band;
}

}  // namespace mpdo
