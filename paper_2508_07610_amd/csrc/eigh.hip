// Hermitian eigensolver for the truncations (FP64), one workgroup per matrix:
//
//  1. Householder reduction to real symmetric tridiagonal form
//     T = Q^H A Q,  Q = H_0 H_1 ... H_{n-2},  H_k = I - tau_k v_k v_k^H,
//     with the reflector chosen so that H_k^H x = beta e_1, beta real
//     (trailing update A <- A - v w^H - w v^H, w = tau p - |tau|^2 (v^H p)/2 v,
//     p = A v).  The matrix lives in LDS for n <= 64, in global memory
//     (L2-resident) otherwise; matrix-vector products run one wavefront per
//     row with a shuffle reduction.
//  2. The leading kvec + 1 eigenvalues of T by bisection on Sturm counts, one
//     thread per eigenvalue.
//  3. Their eigenvectors by inverse iteration on T (tridiagonal LU with
//     partial pivoting, three solves from a fixed pseudo-random start), one
//     thread per vector, then classical Gram-Schmidt applied twice in
//     descending eigenvalue order (fixes degenerate and clustered pairs).
//  4. Back-transformation z <- H_0 ... H_{n-2} z, a group of lanes per vector.
//
// Only the eigenpairs a truncation can keep are computed; the discarded
// weight comes from Tr(A) minus the kept eigenvalues.
#include "common.h"
#include "kernels.h"

namespace mpdo {

namespace {
constexpr int NT = EIG_THREADS;
constexpr int LDS_N = 64;

__device__ inline double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0;
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  __syncthreads();
  return s;
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// number of eigenvalues of T (diag d, off-diagonal e) strictly below x
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
  cpx<double> v[512], p[512], w[512];
  double ev[513];
  double red[NT / 64];
  double scal[4];
  int flag[4];
};

__device__ void heev_core(const EigDesc& dsc, cpx<double>* A, Shared& S) {
  const int n = dsc.n, tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  double* work = dsc.work;
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
  tr = block_sum(tr, S.red);
  // ---- 2. tridiagonalisation ----
  for (int k = 0; k + 1 < n; ++k) {
    const int m = n - k - 1;
    const int c0 = k + 1;  // first row/col of the trailing block
    double xn = 0;
    for (int i = 1 + tid; i < m; i += NT) xn += cabs2(A[(c0 + i) * n + k]);
    xn = block_sum(xn, S.red);
    if (tid == 0) {
      const cpx<double> alpha = A[c0 * n + k];
      if (xn == 0.0 && alpha.im == 0.0) {
        S.tau[k] = mk(0.0, 0.0);
        S.e[k] = alpha.re;
        S.flag[0] = 0;
      } else {
        const double nrm = sqrt(cabs2(alpha) + xn);
        const double beta = alpha.re >= 0 ? -nrm : nrm;
        S.tau[k] = mk((beta - alpha.re) / beta, -alpha.im / beta);
        // scal = 1 / (alpha - beta)
        const cpx<double> den = mk(alpha.re - beta, alpha.im);
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
        const cpx<double> v = (i == 0) ? mk(1.0, 0.0) : A[(c0 + i) * n + k] * sc;
        S.v[i] = v;
        A[(c0 + i) * n + k] = v;  // keep v_k for the back-transformation
      }
    } else {
      for (int i = tid; i < m; i += NT) S.v[i] = mk(i == 0 ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    if (!act) continue;
    // p = A22 v, one wavefront per row
    for (int r = wave; r < m; r += NT / 64) {
      const cpx<double>* row = A + (long long)(c0 + r) * n + c0;
      double sre = 0, sim = 0;
      for (int j = lane; j < m; j += 64) {
        const cpx<double> x = row[j], v = S.v[j];
        sre += x.re * v.re - x.im * v.im;
        sim += x.re * v.im + x.im * v.re;
      }
      sre = wave_sum(sre);
      sim = wave_sum(sim);
      if (lane == 0) S.p[r] = mk(sre, sim);
    }
    __syncthreads();
    double g = 0;  // gamma = v^H p (real)
    for (int i = tid; i < m; i += NT) g += S.v[i].re * S.p[i].re + S.v[i].im * S.p[i].im;
    g = block_sum(g, S.red);
    const double cc = 0.5 * cabs2(tau) * g;
    for (int i = tid; i < m; i += NT) S.w[i] = tau * S.p[i] - cc * S.v[i];
    __syncthreads();
    for (int e = tid; e < m * m; e += NT) {
      const int i = e / m, j = e % m;
      cpx<double>& x = A[(long long)(c0 + i) * n + c0 + j];
      x = x - S.v[i] * cconj(S.w[j]) - S.w[i] * cconj(S.v[j]);
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += NT) S.d[i] = A[i * n + i].re;
  __syncthreads();
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
  // ---- 4. inverse iteration, one thread per vector ----
  // scratch (interleaved by thread): U0, U1, U2, L, x  [n][NT] each
  double* U0 = work + 2LL * n * n;
  double* U1 = U0 + (long long)n * NT;
  double* U2 = U1 + (long long)n * NT;
  double* LL = U2 + (long long)n * NT;
  double* X = LL + (long long)n * NT;
  cpx<double>* Z = reinterpret_cast<cpx<double>*>(dsc.evecs);
  const double floorv = EIG_FLOOR * S.ev[0];
  const double pivtol = 2.2204460492503131e-16 * fmax(tnorm, 1e-300);
  for (int j0 = 0; j0 < kvec; j0 += NT) {
    const int j = j0 + tid;
    if (j < kvec) {
      const double lam = S.ev[j];
      if (!(lam > floorv) || S.ev[0] <= 0) {
        for (int i = 0; i < n; ++i) Z[(long long)i * n + j] = mk(0.0, 0.0);
      } else {
        // LU of T - lam I with partial pivoting; U has up to two superdiagonals
        unsigned long long pivbits[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        double u0 = S.d[0] - lam, u1 = n > 1 ? S.e[0] : 0.0, u2 = 0.0;
        for (int k = 0; k + 1 < n; ++k) {
          const double l = S.e[k], ak1 = S.d[k + 1] - lam, ek1 = (k + 2 < n) ? S.e[k + 1] : 0.0;
          if (fabs(u0) >= fabs(l) || fabs(l) < pivtol) {
            double piv = u0;
            if (fabs(piv) < pivtol) piv = piv >= 0 ? pivtol : -pivtol;
            const double mult = l / piv;
            U0[(long long)k * NT + tid] = piv; U1[(long long)k * NT + tid] = u1; U2[(long long)k * NT + tid] = u2;
            LL[(long long)k * NT + tid] = mult;
            const double nu0 = ak1 - mult * u1, nu1 = ek1 - mult * u2;
            u0 = nu0; u1 = nu1; u2 = 0.0;
          } else {
            const double mult = u0 / l;
            U0[(long long)k * NT + tid] = l; U1[(long long)k * NT + tid] = ak1; U2[(long long)k * NT + tid] = ek1;
            LL[(long long)k * NT + tid] = mult;
            pivbits[k >> 6] |= 1ULL << (k & 63);
            const double nu0 = u1 - mult * ak1, nu1 = u2 - mult * ek1;
            u0 = nu0; u1 = nu1; u2 = 0.0;
          }
        }
        if (fabs(u0) < pivtol) u0 = u0 >= 0 ? pivtol : -pivtol;
        U0[(long long)(n - 1) * NT + tid] = u0;
        U1[(long long)(n - 1) * NT + tid] = 0;
        U2[(long long)(n - 1) * NT + tid] = 0;
        for (int i = 0; i < n; ++i) X[(long long)i * NT + tid] = start_entry(j, i);
        for (int iter = 0; iter < 3; ++iter) {
          // forward: P and L
          for (int k = 0; k + 1 < n; ++k) {
            double bk = X[(long long)k * NT + tid], bk1 = X[(long long)(k + 1) * NT + tid];
            if ((pivbits[k >> 6] >> (k & 63)) & 1ULL) { const double t = bk; bk = bk1; bk1 = t; }
            bk1 -= LL[(long long)k * NT + tid] * bk;
            X[(long long)k * NT + tid] = bk;
            X[(long long)(k + 1) * NT + tid] = bk1;
          }
          // backward: U
          double xn1 = 0, xn2 = 0, mx = 0;
          for (int k = n - 1; k >= 0; --k) {
            const double x = (X[(long long)k * NT + tid] - U1[(long long)k * NT + tid] * xn1 -
                              U2[(long long)k * NT + tid] * xn2) / U0[(long long)k * NT + tid];
            X[(long long)k * NT + tid] = x;
            xn2 = xn1;
            xn1 = x;
            mx = fmax(mx, fabs(x));
          }
          const double s = mx > 0 ? 1.0 / mx : 1.0;
          for (int i = 0; i < n; ++i) X[(long long)i * NT + tid] *= s;
        }
        double nn = 0;
        for (int i = 0; i < n; ++i) nn += X[(long long)i * NT + tid] * X[(long long)i * NT + tid];
        const double s = 1.0 / sqrt(nn);
        for (int i = 0; i < n; ++i) Z[(long long)i * n + j] = mk(X[(long long)i * NT + tid] * s, 0.0);
      }
    }
    __syncthreads();
  }
  __syncthreads();
  // ---- 5. classical Gram-Schmidt, twice, in descending order ----
  int kz = 0;  // number of nonzero vectors (leading block)
  while (kz < kvec && S.ev[kz] > floorv && S.ev[0] > 0) ++kz;
  double* cbuf = S.red;  // unused here; dot products go to S.p (real parts)
  (void)cbuf;
  for (int j = 1; j < kz; ++j) {
    for (int pass = 0; pass < 2; ++pass) {
      // dots c_i = z_i . z_j for i < j, a wavefront per dot
      for (int i = wave; i < j; i += NT / 64) {
        double s = 0;
        for (int r = lane; r < n; r += 64) s += Z[(long long)r * n + i].re * Z[(long long)r * n + j].re;
        s = wave_sum(s);
        if (lane == 0) S.p[i].re = s;
      }
      __syncthreads();
      for (int r = tid; r < n; r += NT) {
        double x = Z[(long long)r * n + j].re;
        for (int i = 0; i < j; ++i) x -= S.p[i].re * Z[(long long)r * n + i].re;
        Z[(long long)r * n + j].re = x;
      }
      __syncthreads();
    }
    double nn = 0;
    for (int r = tid; r < n; r += NT) nn += Z[(long long)r * n + j].re * Z[(long long)r * n + j].re;
    nn = block_sum(nn, S.red);
    const double s = 1.0 / sqrt(nn);
    for (int r = tid; r < n; r += NT) Z[(long long)r * n + j].re *= s;
    __syncthreads();
  }
  // ---- 6. back-transformation z <- H_0 ... H_{n-2} z ----
  if (kz > 0) {
    int g = 1;  // lanes per vector
    while (g < 64 && g * 2 * kz <= NT) g *= 2;
    const int gid = tid / g, gl = tid % g;
    const int ngroups = NT / g;
    for (int c0 = 0; c0 < kz; c0 += ngroups) {
      const int c = c0 + gid;
      const bool mine = c < kz;
      for (int k = n - 2; k >= 0; --k) {
        const cpx<double> t = S.tau[k];
        if (t.re == 0.0 && t.im == 0.0) continue;
        const int m = n - k - 1, r0 = k + 1;
        double yr = 0, yi = 0;
        if (mine) {
          for (int i = gl; i < m; i += g) {
            const cpx<double> v = (i == 0) ? mk(1.0, 0.0) : A[(long long)(r0 + i) * n + k];
            const cpx<double> z = Z[(long long)(r0 + i) * n + c];
            yr += v.re * z.re + v.im * z.im;  // conj(v) z
            yi += v.re * z.im - v.im * z.re;
          }
        }
        for (int off = g / 2; off > 0; off >>= 1) {
          yr += __shfl_xor(yr, off, 64);
          yi += __shfl_xor(yi, off, 64);
        }
        if (mine) {
          const cpx<double> ty = t * mk(yr, yi);
          for (int i = gl; i < m; i += g) {
            const cpx<double> v = (i == 0) ? mk(1.0, 0.0) : A[(long long)(r0 + i) * n + k];
            cpx<double>& z = Z[(long long)(r0 + i) * n + c];
            z = z - v * ty;
          }
        }
      }
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
