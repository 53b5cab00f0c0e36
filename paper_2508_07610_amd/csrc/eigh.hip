// Hermitian eigensolver: two-sided cyclic Jacobi in FP64, one workgroup per
// matrix, parallel (round-robin) ordering so that every round rotates n/2
// disjoint index pairs at once.  Eigenvalues descending, eigenvectors as
// columns.  Used for the Gram matrices of the inner (Eqs. (9)-(11)) and bond
// (Sec. II.D) truncations and for the Choi matrix of a channel (Eq. (15)).
//
// Rotation of the pair (p, q) with a = A_pp, d = A_qq, b = A_pq = |b| u:
//   tau = (d - a) / (2|b|),  t = sgn(tau) / (|tau| + sqrt(1 + tau^2)),
//   c = 1 / sqrt(1 + t^2),  s = t c,
//   J = [[c, s u], [-s conj(u), c]]  (columns p, q),   A <- J^H A J,  V <- V J,
// which zeroes A_pq and leaves A_pp = a - t|b|, A_qq = d + t|b|.
#include "common.h"
#include "kernels.h"

namespace mpdo {

namespace {
constexpr int EIG_THREADS = 256;
constexpr int EIG_LDS_N = 64;
constexpr int MAXPAIRS = 256;  // n <= 512

struct Pair {
  int p, q;
  double c, s, ure, uim;
};

__device__ inline double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;
}

// A: n x n (leading dimension n), V: n x n, both generic pointers (LDS or global).
__device__ int jacobi_core(cpx<double>* __restrict__ A, cpx<double>* __restrict__ V, int n, int max_sweeps,
                           double tol, Pair* pairs, double* red) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int np = (n + 1) & ~1;  // even number of players
  const int half = np / 2;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    // convergence test on the whole matrix
    double off = 0, tot = 0;
    for (int e = tid; e < n * n; e += nt) {
      const double v = cabs2(A[e]);
      tot += v;
      if (e / n != e % n) off += v;
    }
    off = block_sum(off, red);
    tot = block_sum(tot, red);
    if (off <= tol * tol * tot || tot == 0.0) break;
    const double skip = 1e-40 * tot;
    for (int r = 0; r < np - 1; ++r) {
      for (int k = tid; k < half; k += nt) {
        const int pa = k, pb = np - 1 - k;
        int p = (pa == 0) ? 0 : ((pa - 1 + r) % (np - 1)) + 1;
        int q = (pb == 0) ? 0 : ((pb - 1 + r) % (np - 1)) + 1;
        if (p > q) { const int t = p; p = q; q = t; }
        Pair pr;
        pr.p = p; pr.q = q; pr.c = 1; pr.s = 0; pr.ure = 1; pr.uim = 0;
        if (q < n) {
          const cpx<double> b = A[p * n + q];
          const double ab2 = cabs2(b);
          if (ab2 > skip) {
            const double ab = sqrt(ab2);
            const double a = A[p * n + p].re, dd = A[q * n + q].re;
            const double tau = (dd - a) / (2 * ab);
            const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1 + tau * tau));
            const double c = 1 / sqrt(1 + t * t);
            pr.c = c; pr.s = t * c; pr.ure = b.re / ab; pr.uim = b.im / ab;
          }
        }
        pairs[k] = pr;
      }
      __syncthreads();
      // A <- J^H A J on 2 x 2 quads (row pair kr, column pair kc)
      for (int e = tid; e < half * half; e += nt) {
        const int kr = e / half, kc = e % half;
        const Pair R = pairs[kr], Cc = pairs[kc];
        if (R.s == 0 && Cc.s == 0) continue;
        const bool rq = R.q < n, cq = Cc.q < n;
        cpx<double> x00 = A[R.p * n + Cc.p];
        cpx<double> x01 = cq ? A[R.p * n + Cc.q] : mk(0.0, 0.0);
        cpx<double> x10 = rq ? A[R.q * n + Cc.p] : mk(0.0, 0.0);
        cpx<double> x11 = (rq && cq) ? A[R.q * n + Cc.q] : mk(0.0, 0.0);
        // right: Y = X J_c
        const cpx<double> uc = mk(Cc.ure, Cc.uim);
        const cpx<double> su_c = Cc.s * uc, suc_c = Cc.s * cconj(uc);
        cpx<double> y00 = Cc.c * x00 - x01 * suc_c;
        cpx<double> y01 = x00 * su_c + Cc.c * x01;
        cpx<double> y10 = Cc.c * x10 - x11 * suc_c;
        cpx<double> y11 = x10 * su_c + Cc.c * x11;
        // left: Z = J_r^H Y
        const cpx<double> ur = mk(R.ure, R.uim);
        const cpx<double> su_r = R.s * ur, suc_r = R.s * cconj(ur);
        cpx<double> z00 = R.c * y00 - su_r * y10;
        cpx<double> z01 = R.c * y01 - su_r * y11;
        cpx<double> z10 = suc_r * y00 + R.c * y10;
        cpx<double> z11 = suc_r * y01 + R.c * y11;
        if (kr == kc) {
          z01 = mk(0.0, 0.0);
          z10 = mk(0.0, 0.0);
          z00.im = 0;
          z11.im = 0;
        }
        A[R.p * n + Cc.p] = z00;
        if (cq) A[R.p * n + Cc.q] = z01;
        if (rq) A[R.q * n + Cc.p] = z10;
        if (rq && cq) A[R.q * n + Cc.q] = z11;
      }
      // V <- V J
      for (int e = tid; e < n * half; e += nt) {
        const int row = e / half, k = e % half;
        const Pair P = pairs[k];
        if (P.s == 0 || P.q >= n) continue;
        const cpx<double> u = mk(P.ure, P.uim);
        const cpx<double> vp = V[row * n + P.p], vq = V[row * n + P.q];
        V[row * n + P.p] = P.c * vp - vq * (P.s * cconj(u));
        V[row * n + P.q] = vp * (P.s * u) + P.c * vq;
      }
      __syncthreads();
    }
  }
  return sweep;
}

__device__ void finish(const EigDesc& d, const cpx<double>* A, const cpx<double>* V, int n) {
  // rank of eigenvalue i in descending order (ties by index)
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double ei = A[i * n + i].re;
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double ej = A[j * n + j].re;
      rank += (ej > ei) || (ej == ei && j < i);
    }
    d.evals[rank] = ei;
    for (int row = 0; row < n; ++row) {
      const cpx<double> v = V[row * n + i];
      d.evecs[2 * (row * n + rank)] = v.re;
      d.evecs[2 * (row * n + rank) + 1] = v.im;
    }
  }
}
}  // namespace

// Small matrices (n <= 64): A and V live in LDS.
__global__ __launch_bounds__(EIG_THREADS) void k_jacobi_lds(const EigDesc* __restrict__ descs,
                                                            int* __restrict__ sweeps_out, int max_sweeps,
                                                            double tol) {
  __shared__ cpx<double> sA[EIG_LDS_N * EIG_LDS_N];
  __shared__ cpx<double> sV[EIG_LDS_N * EIG_LDS_N];
  __shared__ Pair pairs[EIG_LDS_N / 2];
  __shared__ double red[EIG_THREADS / 64];
  const EigDesc& d = descs[blockIdx.x];
  const int n = d.n;
  if (!d.active || n <= 0 || n > EIG_LDS_N) return;  // larger problems: k_jacobi_global
  const cpx<double>* a = reinterpret_cast<const cpx<double>*>(d.a);
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    const cpx<double> x = a[(long long)i * d.lda + j], y = a[(long long)j * d.lda + i];
    sA[e] = mk(0.5 * (x.re + y.re), 0.5 * (x.im - y.im));
    sV[e] = mk(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const int sw = jacobi_core(sA, sV, n, max_sweeps, tol, pairs, red);
  __syncthreads();
  finish(d, sA, sV, n);
  if (threadIdx.x == 0 && sweeps_out) sweeps_out[blockIdx.x] = (sw >= max_sweeps) ? -sw : sw;
}

// Larger matrices (n <= 512): A in `work`, V in the input buffer, both global.
__global__ __launch_bounds__(EIG_THREADS) void k_jacobi_global(const EigDesc* __restrict__ descs,
                                                               int* __restrict__ sweeps_out, int max_sweeps,
                                                               double tol) {
  __shared__ Pair pairs[MAXPAIRS];
  __shared__ double red[EIG_THREADS / 64];
  const EigDesc& d = descs[blockIdx.x];
  const int n = d.n;
  if (!d.active || n <= EIG_LDS_N || n > 2 * MAXPAIRS) return;  // small problems: k_jacobi_lds
  cpx<double>* a = reinterpret_cast<cpx<double>*>(d.a);
  cpx<double>* W = reinterpret_cast<cpx<double>*>(d.work);
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    const cpx<double> x = a[(long long)i * d.lda + j], y = a[(long long)j * d.lda + i];
    W[e] = mk(0.5 * (x.re + y.re), 0.5 * (x.im - y.im));
  }
  __syncthreads();
  // the input is consumed; reuse it as V with leading dimension n
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) a[e] = mk((e / n == e % n) ? 1.0 : 0.0, 0.0);
  __syncthreads();
  const int sw = jacobi_core(W, a, n, max_sweeps, tol, pairs, red);
  __syncthreads();
  finish(d, W, a, n);
  if (threadIdx.x == 0 && sweeps_out) sweeps_out[blockIdx.x] = (sw >= max_sweeps) ? -sw : sw;
}

void launch_eigh(const EigDesc* d_descs, int nitems, int maxn, int* d_sweeps, hipStream_t s) {
  if (nitems <= 0) return;
  const int max_sweeps = 60;
  const double tol = 1e-14;
  hipLaunchKernelGGL(k_jacobi_lds, dim3(nitems), dim3(EIG_THREADS), 0, s, d_descs, d_sweeps, max_sweeps, tol);
  if (maxn > EIG_LDS_N)
    hipLaunchKernelGGL(k_jacobi_global, dim3(nitems), dim3(EIG_THREADS), 0, s, d_descs, d_sweeps, max_sweeps,
                       tol);
}

}  // namespace mpdo
