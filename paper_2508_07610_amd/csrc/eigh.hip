// Hermitian eigensolver for the truncations (FP64), one workgroup of 1024
// threads per matrix:
//
//  1. Householder reduction to real symmetric tridiagonal form
//     T = Q^H A Q,  Q = H_0 H_1 ... H_{n-2},  H_k = I - tau_k v_k v_k^H,
//     with the reflector chosen so that H_k^H x = beta e_1, beta real.  The
//     trailing update A <- A - v w^H - w v^H (w = tau p - |tau|^2 (v^H p)/2 v,
//     p = A v) of step k is fused with the matrix-vector product of step k+1
//     into one pass over the trailing block, column-parallel (Hermitian
//     symmetry turns the row products into coalesced column reads) with
//     eight independent loads in flight per thread.  The matrix lives in LDS
//     for n <= 64 and in global memory (L2-resident) otherwise.
//  2. The leading kvec + 1 eigenvalues of T by bisection on Sturm counts, one
//     thread per eigenvalue.
//  3. Their eigenvectors by inverse iteration on T (tridiagonal LU with
//     partial pivoting, three solves from a fixed pseudo-random start), one
//     thread per vector, the solves streaming batches of eight entries
//     between two buffers; then Gram-Schmidt (twice) inside clusters of
//     eigenvalues closer than 1e-6 (degenerate multiplets).
//  4. Back-transformation z <- H_0 ... H_{n-2} z, columns in parallel with the
//     rows of each reflector split over the remaining threads.
//
// Only the eigenpairs a truncation can keep are computed; the discarded
// weight comes from Tr(A) minus the kept eigenvalues.
#include "common.h"
#include "kernels.h"

namespace mpdo {

namespace {
constexpr int NT = EIG_THREADS;
constexpr int NW = NT / 64;
constexpr int LDS_N = 64;
constexpr int UB = 8;  // loads in flight per thread

// Block-wide sum with one barrier: consecutive calls alternate between the
// two halves of red[2 NW], so a half is rewritten only after the barrier of
// the call in between.
__device__ inline double block_sum(double v, double* red, int& parity) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* r = red + parity * NW;
  parity ^= 1;
  if (lane == 0) r[wave] = v;
  __syncthreads();
  double s = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) s += r[i];
  return s;
}

// number of eigenvalues of T (diag d, squared off-diagonal e2) below x
__device__ int sturm_count(const double* d, const double* e2, int n, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0;
  for (int i = 1; i < n; ++i) {
    q = (d[i] - x) - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0;
  }
  return cnt;
}

// deterministic start vector entries in [-1, 1]
__device__ inline double start_entry(int j, int i) {
  unsigned h = (unsigned)(j * 2654435761u) ^ (unsigned)(i * 2246822519u + 0x9E3779B9u);
  h ^= h >> 15;
  h *= 2246822519u;
  h ^= h >> 13;
  h *= 3266489917u;
  h ^= h >> 16;
  return (double)(h & 0xFFFFFF) / (double)0x800000 - 1.0;
}

struct Shared {
  double d[512], e[512], e2[512];
  cpx<double> tau[512];
  cpx<double> v[512];              // reflector of the current step
  cpx<double> vp[512], wp[512];    // pending rank-2 update of the previous step
  cpx<double> pp[NT];              // partial products (row chunk, column)
  double ev[513];
  double red[2 * NW];
  double scal[4];
  int flag[4];
  int clus[513];
};

// Pending update (vp, wp; index 0 = row `base`) on rows/cols [c0, n) and,
// if `act`, p = A22 v (v indexed from c0) into S.pp[0..m).
__device__ void fused_pass(cpx<double>* __restrict__ A, int n, int c0, int base, bool pend, bool act,
                           Shared& S) {
  const int m = n - c0;
  if (m <= 0) return;
  int nq = NT / m;
  if (nq < 1) nq = 1;
  if (nq > 16) nq = 16;
  const int tid = threadIdx.x;
  const int rows_per = (m + nq - 1) / nq;
  for (int t = tid; t < m * nq; t += NT) {
    const int cl = t % m, q = t / m;
    const int c = c0 + cl;
    const cpx<double> wpc = pend ? cconj(S.wp[c - base]) : mk(0.0, 0.0);
    const cpx<double> vpc = pend ? cconj(S.vp[c - base]) : mk(0.0, 0.0);
    double ar = 0, ai = 0;
    const int i0 = c0 + q * rows_per, i1 = min(n, i0 + rows_per);
    int i = i0;
    for (; i + UB <= i1; i += UB) {
      cpx<double> a[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) a[u] = A[(long long)(i + u) * n + c];
      if (pend) {
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          a[u] = a[u] - S.vp[i + u - base] * wpc - S.wp[i + u - base] * vpc;
          A[(long long)(i + u) * n + c] = a[u];
        }
      }
      if (act) {
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          const cpx<double> v = S.v[i + u - c0];
          ar += a[u].re * v.re + a[u].im * v.im;  // conj(a) v
          ai += a[u].re * v.im - a[u].im * v.re;
        }
      }
    }
    for (; i < i1; ++i) {
      cpx<double> a = A[(long long)i * n + c];
      if (pend) {
        a = a - S.vp[i - base] * wpc - S.wp[i - base] * vpc;
        A[(long long)i * n + c] = a;
      }
      if (act) {
        const cpx<double> v = S.v[i - c0];
        ar += a.re * v.re + a.im * v.im;
        ai += a.re * v.im - a.im * v.re;
      }
    }
    S.pp[q * m + cl] = mk(ar, ai);
  }
  __syncthreads();
  if (act && nq > 1) {
    cpx<double> s[1];
    for (int cl = tid; cl < m; cl += NT) {  // m <= 512 < NT: one column per thread
      cpx<double> a = S.pp[cl];
      for (int q = 1; q < nq; ++q) a = a + S.pp[q * m + cl];
      s[0] = a;
    }
    __syncthreads();
    if (tid < m) S.pp[tid] = s[0];
    __syncthreads();
  }
}

__device__ void heev_core(const EigDesc& dsc, cpx<double>* __restrict__ A, Shared& S) {
  const int n = dsc.n, tid = threadIdx.x;
  double* work = dsc.work;
  int par = 0;  // block_sum buffer parity
  // ---- 1. load (symmetrised) ----
  const cpx<double>* a = reinterpret_cast<const cpx<double>*>(dsc.a);
  for (int e = tid; e < n * n; e += NT) {
    const int i = e / n, j = e % n;
    const cpx<double> x = a[(long long)i * dsc.lda + j], y = a[(long long)j * dsc.lda + i];
    A[e] = mk(0.5 * (x.re + y.re), 0.5 * (x.im - y.im));
  }
  __syncthreads();
  double tr = 0;
  for (int i = tid; i < n; i += NT) tr += A[i * n + i].re;
  tr = block_sum(tr, S.red, par);
  // ---- 2. tridiagonalisation ----
  bool pend = false;  // a rank-2 update (vp, wp; index 0 = row k) is pending
  for (int k = 0; k + 1 < n; ++k) {
    const int m = n - k - 1;
    const int c0 = k + 1;
    if (pend) {  // bring column k (rows k..n-1) up to date first
      const cpx<double> wk = cconj(S.wp[0]), vk = cconj(S.vp[0]);
      for (int i = k + tid; i < n; i += NT) {
        cpx<double> x = A[(long long)i * n + k];
        x = x - S.vp[i - k] * wk - S.wp[i - k] * vk;
        A[(long long)i * n + k] = x;
      }
      __syncthreads();
    }
    if (tid == 0) S.d[k] = A[(long long)k * n + k].re;
    double xn = 0;
    for (int i = 1 + tid; i < m; i += NT) xn += cabs2(A[(long long)(c0 + i) * n + k]);
    xn = block_sum(xn, S.red, par);
    if (tid == 0) {
      const cpx<double> alpha = A[(long long)c0 * n + k];
      if (xn == 0.0 && alpha.im == 0.0) {
        S.tau[k] = mk(0.0, 0.0);
        S.e[k] = alpha.re;
        S.flag[0] = 0;
      } else {
        const double nrm = sqrt(cabs2(alpha) + xn);
        const double beta = alpha.re >= 0 ? -nrm : nrm;
        S.tau[k] = mk((beta - alpha.re) / beta, -alpha.im / beta);
        const cpx<double> den = mk(alpha.re - beta, alpha.im);  // scal = 1 / (alpha - beta)
        const double dd = cabs2(den);
        S.scal[0] = den.re / dd;
        S.scal[1] = -den.im / dd;
        S.e[k] = beta;
        S.flag[0] = 1;
      }
    }
    __syncthreads();
    const bool act = S.flag[0] != 0;
    const cpx<double> tau = S.tau[k];
    if (act) {
      const cpx<double> sc = mk(S.scal[0], S.scal[1]);
      for (int i = tid; i < m; i += NT) {
        const cpx<double> v = (i == 0) ? mk(1.0, 0.0) : A[(long long)(c0 + i) * n + k] * sc;
        S.v[i] = v;
        A[(long long)(c0 + i) * n + k] = v;  // kept for the back-transformation
      }
    }
    __syncthreads();
    fused_pass(A, n, c0, k, pend, act, S);
    if (act) {
      double g = 0;  // gamma = v^H p
      for (int i = tid; i < m; i += NT) g += S.v[i].re * S.pp[i].re + S.v[i].im * S.pp[i].im;
      g = block_sum(g, S.red, par);
      const double cc = 0.5 * cabs2(tau) * g;
      for (int i = tid; i < m; i += NT) {
        S.wp[i] = tau * S.pp[i] - cc * S.v[i];
        S.vp[i] = S.v[i];
      }
      __syncthreads();
    }
    pend = act;
  }
  if (pend) {  // the last pending update touches only A[n-1][n-1]
    if (tid == 0) {
      cpx<double> x = A[(long long)(n - 1) * n + n - 1];
      x = x - S.vp[0] * cconj(S.wp[0]) - S.wp[0] * cconj(S.vp[0]);
      A[(long long)(n - 1) * n + n - 1] = x;
    }
    __syncthreads();
  }
  if (tid == 0) S.d[n - 1] = A[(long long)(n - 1) * n + n - 1].re;
  for (int i = tid; i + 1 < n; i += NT) S.e2[i] = S.e[i] * S.e[i];
  __syncthreads();
  // ---- 3. bisection for the leading kb eigenvalues ----
  const int kvec = dsc.kvec < n ? dsc.kvec : n;
  const int kb = (kvec + 1 < n) ? kvec + 1 : n;
  double lo = 1e300, hi = -1e300, emax2 = 0;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? fabs(S.e[i - 1]) : 0.0) + (i + 1 < n ? fabs(S.e[i]) : 0.0);
    lo = fmin(lo, S.d[i] - r);
    hi = fmax(hi, S.d[i] + r);
    if (i + 1 < n) emax2 = fmax(emax2, S.e2[i]);
  }
  const double tnorm = fmax(fabs(lo), fabs(hi));
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
  for (int j = tid; j < kb; j += NT) {
    const int target = n - 1 - j;  // eigenvalues strictly below lambda_j (no ties)
    double l = lo, h = hi;
    for (int it = 0; it < 120; ++it) {
      const double mid = 0.5 * (l + h);
      if (h - l <= fmax(2.5e-16 * fmax(fabs(l), fabs(h)), 4e-17 * tnorm) || mid == l || mid == h) break;
      if (sturm_count(S.d, S.e2, n, mid, pivmin) > target) h = mid;
      else l = mid;
    }
    S.ev[j] = 0.5 * (l + h);
  }
  __syncthreads();
  for (int j = tid; j < n; j += NT) dsc.evals[j] = j < kb ? S.ev[j] : 0.0;
  if (tid == 0 && dsc.trace) *dsc.trace = tr;
  if (kvec <= 0) return;
  const double floorv = EIG_FLOOR * S.ev[0];
  int kz = 0;  // vectors above the numerical-zero floor (a leading block)
  while (kz < kvec && S.ev[kz] > floorv && S.ev[0] > 0) ++kz;
  cpx<double>* __restrict__ Z = reinterpret_cast<cpx<double>*>(dsc.evecs);
  // ---- 4. inverse iteration on T, one thread per vector ----
  {
    const long long ks = (kz + 63) / 64 * 64;  // interleave stride of the solve arrays
    double* __restrict__ X = work + 2LL * n * n;
    double* __restrict__ Y = X + (long long)n * ks;
    double* __restrict__ U0 = Y + (long long)n * ks;
    double* __restrict__ U1 = U0 + (long long)n * ks;
    double* __restrict__ U2 = U1 + (long long)n * ks;
    double* __restrict__ LL = U2 + (long long)n * ks;
    const double pivtol = 2.2204460492503131e-16 * fmax(tnorm, 1e-300);
    for (int j = tid; j < kvec; j += NT) {
      if (j >= kz) {
        for (int i = 0; i < n; ++i) Z[(long long)i * n + j] = mk(0.0, 0.0);
        continue;
      }
      const double lam = S.ev[j];
      unsigned long long pivbits[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      double u0 = S.d[0] - lam, u1 = n > 1 ? S.e[0] : 0.0, u2 = 0.0;
      for (int k = 0; k + 1 < n; ++k) {
        const double l = S.e[k], ak1 = S.d[k + 1] - lam, ek1 = (k + 2 < n) ? S.e[k + 1] : 0.0;
        const long long o = (long long)k * ks + j;
        if (fabs(u0) >= fabs(l) || fabs(l) < pivtol) {
          double piv = u0;
          if (fabs(piv) < pivtol) piv = piv >= 0 ? pivtol : -pivtol;
          const double mult = l / piv;
          U0[o] = piv; U1[o] = u1; U2[o] = u2; LL[o] = mult;
          const double nu0 = ak1 - mult * u1, nu1 = ek1 - mult * u2;
          u0 = nu0; u1 = nu1; u2 = 0.0;
        } else {
          const double mult = u0 / l;
          U0[o] = l; U1[o] = ak1; U2[o] = ek1; LL[o] = mult;
          pivbits[k >> 6] |= 1ULL << (k & 63);
          const double nu0 = u1 - mult * ak1, nu1 = u2 - mult * ek1;
          u0 = nu0; u1 = nu1; u2 = 0.0;
        }
      }
      if (fabs(u0) < pivtol) u0 = u0 >= 0 ? pivtol : -pivtol;
      {
        const long long o = (long long)(n - 1) * ks + j;
        U0[o] = u0; U1[o] = 0; U2[o] = 0; LL[o] = 0;
      }
      for (int i = 0; i < n; ++i) X[(long long)i * ks + j] = start_entry(j, i);
      double scale = 1.0;
      for (int iter = 0; iter < 3; ++iter) {
        // forward (row swaps, L): X -> Y, the running entry carried in a register
        double carry = X[j] * scale;
        int k = 0;
        for (; k + UB < n; k += UB) {
          double nx[UB], lm[UB];
#pragma unroll
          for (int u = 0; u < UB; ++u) {
            nx[u] = X[(long long)(k + 1 + u) * ks + j];
            lm[u] = LL[(long long)(k + u) * ks + j];
          }
#pragma unroll
          for (int u = 0; u < UB; ++u) {
            double bk = carry, b1 = nx[u] * scale;
            if ((pivbits[(k + u) >> 6] >> ((k + u) & 63)) & 1ULL) { const double t = bk; bk = b1; b1 = t; }
            b1 -= lm[u] * bk;
            Y[(long long)(k + u) * ks + j] = bk;
            carry = b1;
          }
        }
        for (; k + 1 < n; ++k) {
          double bk = carry, b1 = X[(long long)(k + 1) * ks + j] * scale;
          if ((pivbits[k >> 6] >> (k & 63)) & 1ULL) { const double t = bk; bk = b1; b1 = t; }
          b1 -= LL[(long long)k * ks + j] * bk;
          Y[(long long)k * ks + j] = bk;
          carry = b1;
        }
        Y[(long long)(n - 1) * ks + j] = carry;
        // backward (U): Y -> X
        double xn1 = 0, xn2 = 0, mx = 0;
        k = n - 1;
        for (; k - UB + 1 >= 0; k -= UB) {
          double y[UB], a0[UB], a1[UB], a2[UB];
#pragma unroll
          for (int u = 0; u < UB; ++u) {
            const long long o = (long long)(k - u) * ks + j;
            y[u] = Y[o]; a0[u] = U0[o]; a1[u] = U1[o]; a2[u] = U2[o];
          }
#pragma unroll
          for (int u = 0; u < UB; ++u) {
            const double x = (y[u] - a1[u] * xn1 - a2[u] * xn2) / a0[u];
            X[(long long)(k - u) * ks + j] = x;
            xn2 = xn1;
            xn1 = x;
            mx = fmax(mx, fabs(x));
          }
        }
        for (; k >= 0; --k) {
          const long long o = (long long)k * ks + j;
          const double x = (Y[o] - U1[o] * xn1 - U2[o] * xn2) / U0[o];
          X[o] = x;
          xn2 = xn1;
          xn1 = x;
          mx = fmax(mx, fabs(x));
        }
        scale = mx > 0 ? 1.0 / mx : 1.0;
      }
      double nn = 0;
      for (int i = 0; i < n; ++i) {
        const double x = X[(long long)i * ks + j] * scale;
        nn += x * x;
      }
      const double s = scale / sqrt(nn);
      for (int i = 0; i < n; ++i) Z[(long long)i * n + j] = mk(X[(long long)i * ks + j] * s, 0.0);
    }
  }
  __syncthreads();
  // ---- 5. Gram-Schmidt (twice) inside clusters of close eigenvalues ----
  if (tid == 0) {
    int c = 0;
    for (int j = 0; j < kz; ++j) {
      if (j > 0 && S.ev[j - 1] - S.ev[j] > 1e-6 * fabs(S.ev[j - 1])) ++c;
      S.clus[j] = c;
    }
  }
  __syncthreads();
  for (int j = 1; j < kz; ++j) {
    if (S.clus[j] != S.clus[j - 1]) continue;  // uniform across the block
    int i0 = j - 1;
    while (i0 > 0 && S.clus[i0 - 1] == S.clus[j]) --i0;
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = i0; i < j; ++i) {
        double s = 0;
        for (int r = tid; r < n; r += NT) s += Z[(long long)r * n + i].re * Z[(long long)r * n + j].re;
        s = block_sum(s, S.red, par);
        for (int r = tid; r < n; r += NT) Z[(long long)r * n + j].re -= s * Z[(long long)r * n + i].re;
        __syncthreads();
      }
      double nn = 0;
      for (int r = tid; r < n; r += NT) nn += Z[(long long)r * n + j].re * Z[(long long)r * n + j].re;
      nn = block_sum(nn, S.red, par);
      const double sc = 1.0 / sqrt(nn);
      for (int r = tid; r < n; r += NT) Z[(long long)r * n + j].re *= sc;
      __syncthreads();
    }
  }
  // ---- 6. back-transformation z <- H_0 ... H_{n-2} z ----
  if (kz > 0) {
    int nq = NT / kz;
    if (nq < 1) nq = 1;
    if (nq > 16) nq = 16;
    for (int k = n - 2; k >= 0; --k) {
      const cpx<double> t = S.tau[k];
      if (t.re == 0.0 && t.im == 0.0) continue;
      const int m = n - k - 1, r0 = k + 1;
      for (int i = tid; i < m; i += NT) S.v[i] = (i == 0) ? mk(1.0, 0.0) : A[(long long)(r0 + i) * n + k];
      __syncthreads();
      const int rows_per = (m + nq - 1) / nq;
      for (int u = tid; u < kz * nq; u += NT) {
        const int c = u % kz, q = u / kz;
        const int i0 = q * rows_per, i1 = min(m, i0 + rows_per);
        double yr = 0, yi = 0;
        for (int i = i0; i < i1; ++i) {
          const cpx<double> v = S.v[i];
          const cpx<double> z = Z[(long long)(r0 + i) * n + c];
          yr += v.re * z.re + v.im * z.im;  // conj(v) z
          yi += v.re * z.im - v.im * z.re;
        }
        S.pp[q * kz + c] = mk(yr, yi);
      }
      __syncthreads();
      for (int u = tid; u < kz * nq; u += NT) {
        const int c = u % kz, q = u / kz;
        cpx<double> y = S.pp[c];
        for (int qq = 1; qq < nq; ++qq) y = y + S.pp[qq * kz + c];
        const cpx<double> ty = t * y;
        const int i0 = q * rows_per, i1 = min(m, i0 + rows_per);
        for (int i = i0; i < i1; ++i) {
          cpx<double> z = Z[(long long)(r0 + i) * n + c];
          z = z - S.v[i] * ty;
          Z[(long long)(r0 + i) * n + c] = z;
        }
      }
      __syncthreads();
    }
  }
}
}  // namespace

__global__ __launch_bounds__(NT) void k_heev_lds(const EigDesc* __restrict__ descs, int* __restrict__ status) {
  __shared__ cpx<double> sA[LDS_N * LDS_N];
  __shared__ Shared S;
  const EigDesc& d = descs[blockIdx.x];
  if (!d.active || d.n <= 0 || d.n > LDS_N) return;
  heev_core(d, sA, S);
  if (threadIdx.x == 0 && status) status[blockIdx.x] = 1;
}

__global__ __launch_bounds__(NT) void k_heev_global(const EigDesc* __restrict__ descs, int* __restrict__ status) {
  __shared__ Shared S;
  const EigDesc& d = descs[blockIdx.x];
  if (!d.active || d.n <= LDS_N || d.n > 512) return;
  heev_core(d, reinterpret_cast<cpx<double>*>(d.work), S);
  if (threadIdx.x == 0 && status) status[blockIdx.x] = 1;
}

void launch_eigh(const EigDesc* d_descs, int nitems, int maxn, int* d_status, hipStream_t s) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(k_heev_lds, dim3(nitems), dim3(NT), 0, s, d_descs, d_status);
  if (maxn > LDS_N) hipLaunchKernelGGL(k_heev_global, dim3(nitems), dim3(NT), 0, s, d_descs, d_status);
}

}  // namespace mpdo
