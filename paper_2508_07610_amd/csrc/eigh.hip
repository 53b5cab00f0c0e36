// Hermitian eigensolver for the truncations (FP64), one workgroup per matrix
// (512 threads; 64 for n <= 32), except in launches of at most 32 matrices
// with n > 128, which share each matrix among several workgroups (the k_coop_*
// kernels further down):
//
//  1. Householder reduction to real symmetric tridiagonal form
//     T = Q^H A Q,  Q = H_0 H_1 ... H_{n-2},  H_k = I - tau_k v_k v_k^H,
//     with the reflector chosen so that H_k^H x = beta e_1, beta real, and
//     w = tau p - |tau|^2 (v^H p)/2 v, p = A v, for the rank-2 update
//     A <- A - v w^H - w v^H.  Three forms:
//     - n <= 128: the matrix is held in registers (k_heev_reg; n <= 32 with
//       one wave per matrix);
//     - n <= 512: panels of eight columns (k_heev_global): each step reads
//       the trailing block once and corrects p for the panel's pending
//       updates; the block is written once per panel, in 4 x 4 register
//       blocks with the panel factors staged in LDS;
//     - n <= 1024: one column per step, the update of step k fused with the
//       matrix-vector pass of step k+1 (k_heev_big; lowest latency for a
//       lone matrix).
//  2. The leading kvec + 1 eigenvalues of T by multisection on Sturm counts
//     (a group of lanes per eigenvalue, SP counts per lane and round).
//  3. Their eigenvectors by inverse iteration on T (tridiagonal LU with
//     partial pivoting, three solves from a fixed pseudo-random start), one
//     thread per vector; then Gram-Schmidt (twice) inside clusters of
//     eigenvalues closer than 1e-6 of their size or 1e-10 of the largest
//     (degenerate multiplets).
//  4. Back-transformation z <- H_0 ... H_{n-2} z: with the vector block in
//     registers for n <= 128 and, in the panel form, for n <= 256 with at
//     most 64 vectors; otherwise in blocks of eight reflectors (compact WY).
//
// Only the eigenpairs a truncation can keep are computed; the discarded
// weight comes from Tr(A) minus the kept eigenvalues.
#include <algorithm>

#include "common.h"
#include "kernels.h"
#include "profile.h"

namespace mpdo {

// Residual bound of an eigenpair relative to ||T||, and a host-set
// override (0: the default; tests force a failure with a negative bound).
constexpr double EIG_RESIDUAL_BOUND = 1e-9;
__device__ double g_eig_rtol = 0.0;

namespace {
constexpr int NT = EIG_THREADS;
constexpr int NW = NT / 64;
constexpr int UB = 8;  // loads in flight per thread

// Complex multiply-adds written as real FMAs (a complex product followed by
// a subtraction would round the product first and take half again as many
// instructions).
// a - x y - u w
__device__ inline cpx<double> sub2prod(cpx<double> a, cpx<double> x, cpx<double> y, cpx<double> u,
                                       cpx<double> w) {
  double re = fma(-x.re, y.re, a.re);
  re = fma(x.im, y.im, re);
  re = fma(-u.re, w.re, re);
  re = fma(u.im, w.im, re);
  double im = fma(-x.re, y.im, a.im);
  im = fma(-x.im, y.re, im);
  im = fma(-u.re, w.im, im);
  im = fma(-u.im, w.re, im);
  return mk(re, im);
}
// a - x y
__device__ inline cpx<double> subprod(cpx<double> a, cpx<double> x, cpx<double> y) {
  double re = fma(-x.re, y.re, a.re);
  re = fma(x.im, y.im, re);
  double im = fma(-x.re, y.im, a.im);
  im = fma(-x.im, y.re, im);
  return mk(re, im);
}
// (re, im) += conj(x) y
__device__ inline void dotacc(double& re, double& im, cpx<double> x, cpx<double> y) {
  re = fma(x.re, y.re, re);
  re = fma(x.im, y.im, re);
  im = fma(x.re, y.im, im);
  im = fma(-x.im, y.re, im);
}

// Block-wide sum with one barrier: consecutive calls alternate between the
// two halves of red[2 NW], so a half is rewritten only after the barrier of
// the call in between.
template <int NTH = NT>
__device__ inline double block_sum(double v, double* red, int& parity) {
  constexpr int NWH = NTH / 64;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* r = red + parity * NWH;
  parity ^= 1;
  if (lane == 0) r[wave] = v;
  __syncthreads();
  double s = 0;
#pragma unroll
  for (int i = 0; i < NWH; ++i) s += r[i];
  return s;
}

// cnt[p]: number of eigenvalues of T (diag d, squared off-diagonal e2)
// below x[p], for SP points at once (independent chains interleaved).  SP = 1:
// with eight waves per CU the other waves' chains already hide the latency of
// the reciprocal, and four points per lane made the C2 step's eigensolvers 8 %
// slower for 1.6 times fewer rounds.
// e2 / q is formed as e2 times the hardware reciprocal estimate of q refined
// by two Newton steps (relative error at the rounding level; the IEEE divide
// sequence is several times longer on this dependent chain).  |q| >= pivmin
// keeps the reciprocal finite, and the count stays backward stable.
constexpr int SP = 1;
__device__ void sturm_counts(const double* d, const double* e2, int n, const double* x, double pivmin, int* cnt) {
  double q[SP];
#pragma unroll
  for (int p = 0; p < SP; ++p) {
    q[p] = d[0] - x[p];
    if (fabs(q[p]) < pivmin) q[p] = -pivmin;
    cnt[p] = q[p] < 0;
  }
  // the entries of T are read eight steps at a time, ahead of the dependent
  // chain (the chain itself is unchanged)
  constexpr int SB = 8;
  int i = 1;
  for (; i + SB <= n; i += SB) {
    double dd[SB], ee[SB];
#pragma unroll
    for (int u = 0; u < SB; ++u) {
      dd[u] = d[i + u];
      ee[u] = e2[i + u - 1];
    }
#pragma unroll
    for (int u = 0; u < SB; ++u)
#pragma unroll
      for (int p = 0; p < SP; ++p) {
        double r = __builtin_amdgcn_rcp(q[p]);
        r = r * (2.0 - q[p] * r);
        r = r * (2.0 - q[p] * r);
        q[p] = (dd[u] - x[p]) - ee[u] * r;
        if (fabs(q[p]) < pivmin) q[p] = -pivmin;
        cnt[p] += q[p] < 0;
      }
  }
  for (; i < n; ++i) {
    const double di = d[i], ei = e2[i - 1];
#pragma unroll
    for (int p = 0; p < SP; ++p) {
      double r = __builtin_amdgcn_rcp(q[p]);
      r = r * (2.0 - q[p] * r);
      r = r * (2.0 - q[p] * r);
      q[p] = (di - x[p]) - ei * r;
      if (fabs(q[p]) < pivmin) q[p] = -pivmin;
      cnt[p] += q[p] < 0;
    }
  }
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

// Workgroup state of the global-memory solver for n <= NMAX.
template <int NMAX> struct alignas(16) SharedG {
  alignas(16) cpx<double> tau[NMAX];
  alignas(16) cpx<double> v[NMAX];             // reflector of the current step
  alignas(16) cpx<double> vp[NMAX];            // pending rank-2 update of the previous step
  alignas(16) cpx<double> wp[NMAX];
  alignas(16) cpx<double> pp[NMAX > NT ? NMAX : NT];  // partial products (row chunk, column)
  double d[NMAX], e[NMAX], e2[NMAX];
  double ev[NMAX + 1];
  double red[2 * NW];
  double scal[4];
  int flag[4];
  int clus[NMAX + 1];
  // panel form, n <= 256: conj(V), conj(W) of the panel, transposed (t, column)
  // (conj(W) follows at offset 8 * 256; the back-transformation reuses the
  // whole array for its block of reflectors, n <= 512 rows of 8)
  alignas(16) cpx<double> pf[NMAX <= 512 ? 2 * 8 * 256 : 1];
  static constexpr int SOLVE_CAP = 0;  // no LDS room for the inverse-iteration arrays
  __device__ double* solve() { return nullptr; }
};

// Pending update (vp, wp; index 0 = row `base`) on rows/cols [c0, n) and,
// if `act`, p = A22 v (v indexed from c0) into S.pp[0..m).
template <class SH>
__device__ void fused_pass(cpx<double>* __restrict__ A, int n, int c0, int base, bool pend, bool act, SH& S) {
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
          a[u] = sub2prod(a[u], S.vp[i + u - base], wpc, S.wp[i + u - base], vpc);
          A[(long long)(i + u) * n + c] = a[u];
        }
      }
      if (act) {
#pragma unroll
        for (int u = 0; u < UB; ++u) dotacc(ar, ai, a[u], S.v[i + u - c0]);  // conj(a) v
      }
    }
    for (; i < i1; ++i) {
      cpx<double> a = A[(long long)i * n + c];
      if (pend) {
        a = sub2prod(a, S.vp[i - base], wpc, S.wp[i - base], vpc);
        A[(long long)i * n + c] = a;
      }
      if (act) dotacc(ar, ai, a, S.v[i - c0]);
    }
    S.pp[q * m + cl] = mk(ar, ai);
  }
  __syncthreads();
  if (act && nq > 1) {
    cpx<double> s[1];
    for (int cl = tid; cl < m; cl += NT) {  // nq > 1 means m <= NT / 2: one column per thread
      cpx<double> a = S.pp[cl];
      for (int q = 1; q < nq; ++q) a = a + S.pp[q * m + cl];
      s[0] = a;
    }
    __syncthreads();
    if (tid < m) S.pp[tid] = s[0];
    __syncthreads();
  }
}

// Steps 2, 3 and the cluster re-orthogonalisation on the tridiagonal matrix
// (S.d, S.e, S.e2); eigenvalues to dsc.evals, real eigenvectors of T to
// dsc.evecs.  Returns the number of vectors above the numerical-zero floor.
template <int NTH, class SH>
__device__ int eig_tail(const EigDesc& dsc, int n, double tr, SH& S, int& par) {
  const int tid = threadIdx.x;
  __shared__ int s_resbad;  // an eigenpair failed its residual bound
  if (tid == 0) s_resbad = 0;
  // ---- multisection for the leading kb = kvec + 1 eigenvalues ----
  // A group of L lanes (inside one wave) brackets one eigenvalue;
  // each round evaluates L Sturm counts at equally spaced interior points
  // and keeps the sub-interval where the count passes the target, so the
  // bracket shrinks by L + 1 per round (L = 1 is plain bisection).
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
  {
    // groups stay inside a wave: the widest L that still gives every
    // eigenvalue a group (the last 64 mod L lanes of each wave sit out); each
    // lane evaluates SP points, so a round cuts the bracket into L SP + 1
    // pieces
    int L = 64;
    while (L > 1 && (64 / L) * (NTH / 64) < kb) --L;
    const int gpw = 64 / L, groups = gpw * (NTH / 64);
    const int gi = (tid & 63) / L;  // group within the wave
    const int gl = (tid & 63) - gi * L;
    const int first = gi * L;  // first lane of the group in its wave
    const unsigned long long gmask = (L == 64) ? ~0ULL : ((1ULL << L) - 1ULL);
    const int K = L * SP;
    const double inv = 1.0 / (double)(K + 1);
    for (int j = gi < gpw ? (tid >> 6) * gpw + gi : kb; j < kb; j += groups) {
      const int target = n - 1 - j;  // eigenvalues strictly below lambda_j (no ties)
      double l = lo, h = hi;
      for (int it = 0; it < 120; ++it) {
        if (h - l <= fmax(2.5e-16 * fmax(fabs(l), fabs(h)), 4e-17 * tnorm)) break;
        const double w = h - l;
        double x[SP];
        int cnt[SP];
#pragma unroll
        for (int p = 0; p < SP; ++p) x[p] = l + w * ((double)(gl * SP + p + 1) * inv);
        sturm_counts(S.d, S.e2, n, x, pivmin, cnt);
        // this lane's first point at or above the eigenvalue (SP if none);
        // the counts grow with x, so the points above form a suffix
        int fp = SP;
#pragma unroll
        for (int p = SP - 1; p >= 0; --p)
          if (cnt[p] > target) fp = p;
        const unsigned long long m = (__ballot(fp < SP) >> first) & gmask;
        // first point of the group at or above the eigenvalue (K if none)
        const int j0 = m ? __builtin_ctzll(m) : L;
        const int fpj = __shfl(fp, first + (j0 < L ? j0 : 0), 64);
        const int k0 = j0 < L ? j0 * SP + fpj : K;
        const double nl = (k0 == 0) ? l : l + w * ((double)k0 * inv);
        const double nh = (k0 == K) ? h : l + w * ((double)(k0 + 1) * inv);
        if (nl == l && nh == h) break;
        l = nl;
        h = nh;
      }
      if (gl == 0) S.ev[j] = 0.5 * (l + h);
    }
  }
  __syncthreads();
  for (int j = tid; j < n; j += NTH) dsc.evals[j] = j < kb ? S.ev[j] : 0.0;
  if (tid == 0 && dsc.trace) *dsc.trace = tr;
  if (kvec <= 0) return 0;
  const double floorv = (dsc.vfloor > 0 ? dsc.vfloor : EIG_FLOOR) * S.ev[0];
  int kz = 0;  // vectors above the numerical-zero floor (a leading block)
  while (kz < kvec && S.ev[kz] > floorv && S.ev[0] > 0) ++kz;
  cpx<double>* __restrict__ Z = reinterpret_cast<cpx<double>*>(dsc.evecs);
  double* work = dsc.work;
  // ---- 4. inverse iteration on T, one thread per vector ----
  // T - lambda = P L U with partial pivoting; per step k the factor arrays
  // hold 1/u_kk, u_k,k+1, u_k,k+2, the multiplier and the swap flag.  The
  // arrays live in LDS when the workgroup has room for them (the sweeps are
  // latency-bound), else in the work array.
  {
    const bool lds = SH::SOLVE_CAP > 0 && 7LL * n * kz <= SH::SOLVE_CAP;
    const long long ks = lds ? kz : (kz + 63) / 64 * 64;  // interleave stride of the solve arrays
    double* __restrict__ X = lds ? S.solve() : work + 2LL * n * n;
    double* __restrict__ Y = X + (long long)n * ks;
    double* __restrict__ U0 = Y + (long long)n * ks;
    double* __restrict__ U1 = U0 + (long long)n * ks;
    double* __restrict__ U2 = U1 + (long long)n * ks;
    double* __restrict__ LL = U2 + (long long)n * ks;
    double* __restrict__ PV = LL + (long long)n * ks;
    const double pivtol = 2.2204460492503131e-16 * fmax(tnorm, 1e-300);
  const double rtol = g_eig_rtol != 0.0 ? g_eig_rtol : EIG_RESIDUAL_BOUND;
    for (int j = tid; j < kvec; j += NTH) {
      if (j >= kz) {
        for (int i = 0; i < n; ++i) Z[(long long)i * n + j] = mk(0.0, 0.0);
        continue;
      }
      const double lam = S.ev[j];
      double u0 = S.d[0] - lam, u1 = n > 1 ? S.e[0] : 0.0, u2 = 0.0;
      for (int k = 0; k + 1 < n; ++k) {
        const double l = S.e[k], ak1 = S.d[k + 1] - lam, ek1 = (k + 2 < n) ? S.e[k + 1] : 0.0;
        const long long o = (long long)k * ks + j;
        if (fabs(u0) >= fabs(l) || fabs(l) < pivtol) {
          double piv = u0;
          if (fabs(piv) < pivtol) piv = piv >= 0 ? pivtol : -pivtol;
          const double rp = 1.0 / piv;
          const double mult = l * rp;
          U0[o] = rp; U1[o] = u1; U2[o] = u2; LL[o] = mult; PV[o] = 0.0;
          const double nu0 = ak1 - mult * u1, nu1 = ek1 - mult * u2;
          u0 = nu0; u1 = nu1; u2 = 0.0;
        } else {
          const double rl = 1.0 / l;
          const double mult = u0 * rl;
          U0[o] = rl; U1[o] = ak1; U2[o] = ek1; LL[o] = mult; PV[o] = 1.0;
          const double nu0 = u1 - mult * ak1, nu1 = u2 - mult * ek1;
          u0 = nu0; u1 = nu1; u2 = 0.0;
        }
      }
      if (fabs(u0) < pivtol) u0 = u0 >= 0 ? pivtol : -pivtol;
      {
        const long long o = (long long)(n - 1) * ks + j;
        U0[o] = 1.0 / u0; U1[o] = 0; U2[o] = 0; LL[o] = 0; PV[o] = 0.0;
      }
      for (int i = 0; i < n; ++i) X[(long long)i * ks + j] = start_entry(j, i);
      double scale = 1.0;
      for (int iter = 0; iter < 3; ++iter) {
        // forward (row swaps, L): X -> Y, the running entry carried in a register
        double carry = X[j] * scale;
        int k = 0;
        for (; k + UB < n; k += UB) {
          double nx[UB], lm[UB], pv[UB];
#pragma unroll
          for (int u = 0; u < UB; ++u) {
            nx[u] = X[(long long)(k + 1 + u) * ks + j];
            lm[u] = LL[(long long)(k + u) * ks + j];
            pv[u] = PV[(long long)(k + u) * ks + j];
          }
#pragma unroll
          for (int u = 0; u < UB; ++u) {
            const double b1r = nx[u] * scale;
            const bool sw = pv[u] != 0.0;
            const double bk = sw ? b1r : carry, b1 = sw ? carry : b1r;
            Y[(long long)(k + u) * ks + j] = bk;
            carry = b1 - lm[u] * bk;
          }
        }
        for (; k + 1 < n; ++k) {
          const double b1r = X[(long long)(k + 1) * ks + j] * scale;
          const bool sw = PV[(long long)k * ks + j] != 0.0;
          const double bk = sw ? b1r : carry, b1 = sw ? carry : b1r;
          Y[(long long)k * ks + j] = bk;
          carry = b1 - LL[(long long)k * ks + j] * bk;
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
            const double x = (y[u] - a1[u] * xn1 - a2[u] * xn2) * a0[u];
            X[(long long)(k - u) * ks + j] = x;
            xn2 = xn1;
            xn1 = x;
            mx = fmax(mx, fabs(x));
          }
        }
        for (; k >= 0; --k) {
          const long long o = (long long)k * ks + j;
          const double x = (Y[o] - U1[o] * xn1 - U2[o] * xn2) * U0[o];
          X[o] = x;
          xn2 = xn1;
          xn1 = x;
          mx = fmax(mx, fabs(x));
        }
        scale = mx > 0 ? 1.0 / mx : 1.0;
      }
      // norm, store and residual read X in blocks of UB loads issued ahead
      // (the arithmetic and its order are those of one element at a time)
      double nn = 0;
      {
        int i = 0;
        for (; i + UB <= n; i += UB) {
          double xv[UB];
#pragma unroll
          for (int u = 0; u < UB; ++u) xv[u] = X[(long long)(i + u) * ks + j];
#pragma unroll
          for (int u = 0; u < UB; ++u) {
            const double x = xv[u] * scale;
            nn += x * x;
          }
        }
        for (; i < n; ++i) {
          const double x = X[(long long)i * ks + j] * scale;
          nn += x * x;
        }
      }
      const double s = scale / sqrt(nn);
      // z = X s to Z, and the residual of the tridiagonal eigenpair
      // ||(T - lambda) z|| <= rtol ||T|| (inverse iteration from a bisected
      // eigenvalue reaches about eps ||T||) from the same values
      double rr = 0, zp = 0, zc = X[j] * s;
      {
        int i = 0;
        for (; i + UB < n; i += UB) {
          double zb[UB + 1];
#pragma unroll
          for (int u = 1; u <= UB; ++u) zb[u] = X[(long long)(i + u) * ks + j] * s;
          zb[0] = zc;
#pragma unroll
          for (int u = 0; u < UB; ++u) {
            Z[(long long)(i + u) * n + j] = mk(zb[u], 0.0);
            const double zn = zb[u + 1];
            double t = (S.d[i + u] - lam) * zb[u];
            if (i + u > 0) t += S.e[i + u - 1] * zp;
            t += S.e[i + u] * zn;
            rr += t * t;
            zp = zb[u];
          }
          zc = zb[UB];
        }
        for (; i < n; ++i) {
          Z[(long long)i * n + j] = mk(zc, 0.0);
          const double zn = i + 1 < n ? X[(long long)(i + 1) * ks + j] * s : 0.0;
          double t = (S.d[i] - lam) * zc;
          if (i > 0) t += S.e[i - 1] * zp;
          if (i + 1 < n) t += S.e[i] * zn;
          rr += t * t;
          zp = zc;
          zc = zn;
        }
      }
      if (!(sqrt(rr) <= rtol * tnorm)) s_resbad = 1;
    }
  }
  __syncthreads();
  // a failed bound or a non-finite spectrum marks the result by a NaN trace,
  // which the consumers of the eigenvalues count as a numerical failure
  if (tid == 0 && dsc.trace && (s_resbad || !(tnorm < 1e300))) *dsc.trace = __builtin_nan("");
  // ---- 5. Gram-Schmidt (twice) inside clusters of close eigenvalues ----
  // Inverse iteration leaves vectors of eigenvalues closer than about
  // eps ||T|| / gap non-orthogonal, so a cluster joins eigenvalues whose gap
  // is below 1e-6 of their size or below 1e-10 of the largest.  Each vector
  // is orthogonalised against the earlier members of its cluster in two
  // blocked passes (one dot product per wave, then one update per row).
  if (tid == 0) {
    int c = 0;
    const double agap = 1e-10 * fabs(S.ev[0]);
    for (int j = 0; j < kz; ++j) {
      if (j > 0 && S.ev[j - 1] - S.ev[j] > fmax(1e-6 * fabs(S.ev[j - 1]), agap)) ++c;
      S.clus[j] = c;
    }
  }
  __syncthreads();
  {
    double* dots = reinterpret_cast<double*>(&S.pp);  // free after the tridiagonalisation
    constexpr int NWV = NTH / 64;
    const int lane = tid & 63, wave = tid >> 6;
    for (int j = 1; j < kz; ++j) {
      if (S.clus[j] != S.clus[j - 1]) continue;  // uniform across the block
      int i0 = j - 1;
      while (i0 > 0 && S.clus[i0 - 1] == S.clus[j]) --i0;
      const int cnt = j - i0;
      for (int pass = 0; pass < 2; ++pass) {
        for (int ib = wave; ib < cnt; ib += NWV) {
          double s = 0;
          for (int r = lane; r < n; r += 64) s += Z[(long long)r * n + i0 + ib].re * Z[(long long)r * n + j].re;
          for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
          if (lane == 0) dots[ib] = s;
        }
        __syncthreads();
        for (int r = tid; r < n; r += NTH) {
          double a = Z[(long long)r * n + j].re;
          for (int i = 0; i < cnt; ++i) a -= dots[i] * Z[(long long)r * n + i0 + i].re;
          Z[(long long)r * n + j].re = a;
        }
        __syncthreads();
      }
      double nn = 0;
      for (int r = tid; r < n; r += NTH) nn += Z[(long long)r * n + j].re * Z[(long long)r * n + j].re;
      nn = block_sum<NTH>(nn, S.red, par);
      const double sc = 1.0 / sqrt(nn);
      for (int r = tid; r < n; r += NTH) Z[(long long)r * n + j].re *= sc;
      __syncthreads();
    }
  }
  return kz;
}

// Z <- H_0 H_1 ... H_{n-2} Z for the kz leading columns of Z (ld n), the
// reflectors H_k = I - tau_k v_k v_k^H stored below the diagonal in column k
// of A (v_k(k+1) = 1).  Blocks of BTB reflectors, from the last, are applied
// in compact form Q = H_k0 ... H_k1-1 = I - V T V^H (T upper triangular,
// T_jj = tau_j, T(0:j, j) = -tau_j T(0:j, 0:j) V(:, 0:j)^H v_j):
// W = V^H Z, W <- T W, Z <- Z - V W, so Z is read twice and written once per
// block instead of once per reflector.
constexpr int BTB = 8;
constexpr int BT_NQ = 64;  // most row chunks per column in the back-transformation
constexpr int TRB = 8;  // tridiagonalisation panel width
template <class SH>
__device__ void back_transform(const EigDesc& dsc, const cpx<double>* __restrict__ A, int n, int kz, SH& S,
                               int cz0 = 0, cpx<double>* scratch = nullptr) {
  // columns cz0 .. cz0 + kz - 1 of the eigenvector block
  cpx<double>* __restrict__ Z = reinterpret_cast<cpx<double>*>(dsc.evecs) + cz0;
  // scratch (default: after the matrix, free once the inverse iteration is done)
  cpx<double>* const Vg = scratch ? scratch : reinterpret_cast<cpx<double>*>(dsc.work + 2LL * n * n);  // n x BTB
  cpx<double>* __restrict__ part = Vg + (long long)n * BTB;                        // nq x BTB x kz
  // the block of reflectors in LDS when the panel factors' array holds it
  constexpr int LV = sizeof(S.pf) / sizeof(S.pf[0]);
  cpx<double>* __restrict__ Vb = n * BTB <= LV ? S.pf : Vg;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // row chunks per column (at most BT_NQ: their partial sums are added up
  // by one thread per reflector and column)
  const int nq = kz < NT ? (NT / kz < BT_NQ ? NT / kz : BT_NQ) : 1;
  cpx<double>* __restrict__ Wt = part + (long long)nq * BTB * kz;                       // BTB x kz
  cpx<double>* G = S.v;                          // BTB x BTB (LDS, free here)
  cpx<double>* T = S.vp;
  for (int kend = n - 1; kend > 0; kend -= BTB) {
    const int k0 = kend > BTB ? kend - BTB : 0, nb = kend - k0;
    const int r0 = k0 + 1, m = n - r0;
    // V block, row r0 + i: v_{k0+j}(row) for j < nb (zero above v's first row
    // and for tau = 0)
    for (int e = tid; e < m * BTB; e += NT) {
      const int i = e / BTB, j = e % BTB, r = r0 + i, k = k0 + j;
      cpx<double> v = mk(0.0, 0.0);
      if (j < nb && r >= k + 1 && (S.tau[k].re != 0.0 || S.tau[k].im != 0.0))
        v = (r == k + 1) ? mk(1.0, 0.0) : A[(long long)r * n + k];
      Vb[e] = v;
    }
    __syncthreads();
    // G(i, j) = v_i^H v_j for i < j, one wave per pair
    for (int pr = wave; pr < BTB * BTB; pr += NT / 64) {
      const int i = pr / BTB, j = pr % BTB;
      if (i >= j || j >= nb) continue;  // uniform per wave
      double gr = 0, gi = 0;
      for (int r = lane; r < m; r += 64) {
        const cpx<double> a = Vb[(long long)r * BTB + i], b = Vb[(long long)r * BTB + j];
        gr += a.re * b.re + a.im * b.im;
        gi += a.re * b.im - a.im * b.re;
      }
      for (int off = 32; off > 0; off >>= 1) {
        gr += __shfl_xor(gr, off, 64);
        gi += __shfl_xor(gi, off, 64);
      }
      if (lane == 0) G[i * BTB + j] = mk(gr, gi);
    }
    __syncthreads();
    // T, one lane per row (row i of T depends only on its own earlier
    // entries, which the same lane wrote)
    if (wave == 0 && lane < BTB) {
      const int i = lane;
      for (int j = 0; j < BTB; ++j) {
        cpx<double> x = mk(0.0, 0.0);
        if (j < nb) {
          const cpx<double> t = S.tau[k0 + j];
          if (i == j) {
            x = t;
          } else if (i < j) {
            cpx<double> acc = mk(0.0, 0.0);
            for (int q = i; q < j; ++q) acc = acc + T[i * BTB + q] * G[q * BTB + j];
            x = mk(0.0, 0.0) - t * acc;
          }
        }
        T[i * BTB + j] = x;
      }
    }
    // partial W = V^H Z over row chunks: thread (column c, chunk q)
    const int rows_per = (m + nq - 1) / nq;
    for (int u = tid; u < kz * nq; u += NT) {
      const int c = u % kz, q = u / kz;
      cpx<double> acc[BTB];
#pragma unroll
      for (int j = 0; j < BTB; ++j) acc[j] = mk(0.0, 0.0);
      const int i1 = min(m, (q + 1) * rows_per);
      int i = q * rows_per;
      for (; i + UB <= i1; i += UB) {  // the rows' loads issued together
        cpx<double> zb[UB];
#pragma unroll
        for (int x = 0; x < UB; ++x) zb[x] = Z[(long long)(r0 + i + x) * n + c];
#pragma unroll
        for (int x = 0; x < UB; ++x) {
#pragma unroll
          for (int j = 0; j < BTB; ++j) {
            const cpx<double> v = Vb[(long long)(i + x) * BTB + j], z = zb[x];
            acc[j] = acc[j] + mk(v.re * z.re + v.im * z.im, v.re * z.im - v.im * z.re);  // conj(v) z
          }
        }
      }
      for (; i < i1; ++i) {
        const cpx<double> z = Z[(long long)(r0 + i) * n + c];
#pragma unroll
        for (int j = 0; j < BTB; ++j) {
          const cpx<double> v = Vb[(long long)i * BTB + j];
          acc[j] = acc[j] + mk(v.re * z.re + v.im * z.im, v.re * z.im - v.im * z.re);  // conj(v) z
        }
      }
#pragma unroll
      for (int j = 0; j < BTB; ++j) part[((long long)q * BTB + j) * kz + c] = acc[j];
    }
    __syncthreads();
    // W = V^H Z: the partials added up (in chunk order), one thread per
    // reflector and column, loads issued eight chunks ahead; into Wt
    for (int u = tid; u < BTB * kz; u += NT) {
      const int j = u / kz, c = u % kz;
      cpx<double> x = mk(0.0, 0.0);
      int q = 0;
      for (; q + 8 <= nq; q += 8) {
        cpx<double> p8[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) p8[r] = part[((long long)(q + r) * BTB + j) * kz + c];
#pragma unroll
        for (int r = 0; r < 8; ++r) x = x + p8[r];
      }
      for (; q < nq; ++q) x = x + part[((long long)q * BTB + j) * kz + c];
      Wt[(long long)j * kz + c] = x;
    }
    __syncthreads();
    // Wt = T W, one thread per column (in place: the column is read first)
    for (int c = tid; c < kz; c += NT) {
      cpx<double> w[BTB];
#pragma unroll
      for (int j = 0; j < BTB; ++j) w[j] = Wt[(long long)j * kz + c];
#pragma unroll
      for (int i = 0; i < BTB; ++i) {
        cpx<double> x = mk(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < BTB; ++j)
          if (j >= i) x = x + T[i * BTB + j] * w[j];
        Wt[(long long)i * kz + c] = x;
      }
    }
    __syncthreads();
    // Z <- Z - V Wt
    for (int u = tid; u < kz * nq; u += NT) {
      const int c = u % kz, q = u / kz;
      cpx<double> w[BTB];
#pragma unroll
      for (int j = 0; j < BTB; ++j) w[j] = Wt[(long long)j * kz + c];
      const int i1 = min(m, (q + 1) * rows_per);
      int i = q * rows_per;
      for (; i + UB <= i1; i += UB) {
        cpx<double> zb[UB];
#pragma unroll
        for (int x = 0; x < UB; ++x) zb[x] = Z[(long long)(r0 + i + x) * n + c];
#pragma unroll
        for (int x = 0; x < UB; ++x) {
          cpx<double> z = zb[x];
#pragma unroll
          for (int j = 0; j < BTB; ++j) z = z - Vb[(long long)(i + x) * BTB + j] * w[j];
          Z[(long long)(r0 + i + x) * n + c] = z;
        }
      }
      for (; i < i1; ++i) {
        cpx<double> z = Z[(long long)(r0 + i) * n + c];
#pragma unroll
        for (int j = 0; j < BTB; ++j) z = z - Vb[(long long)i * BTB + j] * w[j];
        Z[(long long)(r0 + i) * n + c] = z;
      }
    }
    __syncthreads();
  }
}

// Z <- H_0 ... H_{n-2} Z with the vector block in registers, for n <= 256
// and kz <= 64 (the panel form's LDS holds the reflectors): thread t owns
// columns t % 32 and t % 32 + 32 over rows 16 (t / 32) .. 16 (t / 32) + 15
// of Z.  Per reflector, from the last: partial y = v^H z over each thread's
// rows, summed over the wave's two row blocks by a lane exchange and then
// over the eight waves by every thread of a column, then z -= tau v y;
// one barrier per reflector (reflector buffers rotate over three slots and
// the partial sums over two, so a slot is rewritten only after every thread
// has passed the barrier that follows its last read).
template <class SH>
__device__ void back_transform_reg(const EigDesc& dsc, const cpx<double>* __restrict__ A, int n, int kz, SH& S) {
  // Thread t holds vectors c and c + 32 (c = t mod 32) over 16 rows, so each
  // reflector entry read from LDS serves two vectors; the two row blocks of a
  // wave are summed with one lane exchange before the partial sums go to LDS.
  constexpr int RB = 16;  // rows per thread
  cpx<double>* __restrict__ Z = reinterpret_cast<cpx<double>*>(dsc.evecs);
  const int tid = threadIdx.x, c = tid & 31, q = tid >> 5, r0 = q * RB, wave = tid >> 6;
  cpx<double>* vb[3] = {S.pf, S.pf + 256, S.pf + 512};  // reflector k in vb[k % 3]
  cpx<double>* pw[2] = {S.pf + 1024, S.pf + 1536};      // 8 waves x 64 vectors
  cpx<double> z[2][RB];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int u = 0; u < RB; ++u) {
      const int r = r0 + u, cj = c + 32 * j;
      z[j][u] = (cj < kz && r < n) ? Z[(long long)r * n + cj] : mk(0.0, 0.0);
    }
  static_assert(NT >= 256, "one reflector entry per thread");
  static_assert(NT / 32 * RB == 256, "16 row blocks of 16 rows");
  // entry i of v_k over all 256 rows (zero outside k+1 .. n-1); the entries
  // of reflector k - 1 are read during step k + 1, a step before they are
  // stored for use
  auto vent = [&](int k, int i) {
    return (i == k + 1) ? mk(1.0, 0.0) : (i > k + 1 && i < n) ? A[(long long)i * n + k] : mk(0.0, 0.0);
  };
  if (n >= 2 && tid < 256) vb[(n - 2) % 3][tid] = vent(n - 2, tid);
  cpx<double> vq = (n >= 3 && tid < 256) ? vent(n - 3, tid) : mk(0.0, 0.0);
  __syncthreads();
  for (int k = n - 2; k >= 0; --k) {
    const cpx<double>* v = vb[k % 3];
    const cpx<double> vq2 = (k >= 2 && tid < 256) ? vent(k - 2, tid) : mk(0.0, 0.0);
    const cpx<double> t = S.tau[k];
    const bool act = !(t.re == 0.0 && t.im == 0.0);  // uniform across the block
    const bool rows = r0 + RB > k + 1;
    if (act) {
      double yr[2][2] = {{0, 0}, {0, 0}}, yi[2][2] = {{0, 0}, {0, 0}};
      if (rows) {
#pragma unroll
        for (int u = 0; u < RB; ++u) {
          const cpx<double> vv = v[r0 + u];
#pragma unroll
          for (int j = 0; j < 2; ++j) dotacc(yr[j][u & 1], yi[j][u & 1], vv, z[j][u]);  // conj(v) z
        }
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        double sr = yr[j][0] + yr[j][1], si = yi[j][0] + yi[j][1];
        sr += __shfl_xor(sr, 32, 64);  // the other row block of this wave
        si += __shfl_xor(si, 32, 64);
        if ((tid & 32) == 0) pw[k & 1][wave * 64 + c + 32 * j] = mk(sr, si);
      }
    }
    if (k >= 1 && tid < 256) vb[(k - 1) % 3][tid] = vq;
    vq = vq2;
    __syncthreads();
    if (act && rows) {
      cpx<double> ty[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        cpx<double> y = mk(0.0, 0.0);
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) y = y + pw[k & 1][w * 64 + c + 32 * j];
        ty[j] = t * y;
      }
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const cpx<double> vv = v[r0 + u];
#pragma unroll
        for (int j = 0; j < 2; ++j) z[j][u] = subprod(z[j][u], vv, ty[j]);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j)
    if (c + 32 * j < kz) {
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int r = r0 + u;
        if (r < n) Z[(long long)r * n + c + 32 * j] = z[j][u];
      }
    }
}

// Step 2 in the panel form (see heev_core); LV: the panel's V and W live in
// LDS (n <= 256), else in the work array after the matrix.
template <bool LV, class SH>
__device__ void panel_tridiag(const EigDesc& dsc, cpx<double>* __restrict__ A, int n, SH& S, int& par) {
  const int tid = threadIdx.x;
  // ---- 2. tridiagonalisation, in panels of TRB columns ----
  // Within a panel the trailing block is not updated: after j steps it is
  // A - V W^H - W V^H with the panel's reflectors v_q and w_q = tau p -
  // (|tau|^2 / 2)(v^H p) v (zero above their first row), so a step reads the
  // trailing block once (p = A v - V (W^H v) - W (V^H v)) and the block is
  // written once per panel.
  cpx<double>* __restrict__ Vp = reinterpret_cast<cpx<double>*>(dsc.work + 2LL * n * n);  // n x TRB
  cpx<double>* __restrict__ Wp = Vp + (long long)n * TRB;
  // n <= 256: V and W of the panel live in LDS, transposed (t, row)
  constexpr bool lv = LV;
  auto vp = [&](int row, int t) -> cpx<double>& { return lv ? S.pf[t * 256 + row] : Vp[(long long)row * TRB + t]; };
  auto wp = [&](int row, int t) -> cpx<double>& {
    return lv ? S.pf[2048 + t * 256 + row] : Wp[(long long)row * TRB + t];
  };
  cpx<double>* xk = S.wp;     // current column k (rows k..n-1)
  cpx<double>* y12 = S.vp;    // W^H v (0..TRB) and V^H v (TRB..2 TRB)
  const int lane = tid & 63, wave = tid >> 6;
  for (int p0 = 0; p0 + 1 < n; p0 += TRB) {
    const int np = min(TRB, n - 1 - p0);
    for (int j = 0; j < np; ++j) {
      const int k = p0 + j, m = n - k - 1, c0 = k + 1;
      // current column k from row k of the stored matrix and the panel so far
      for (int i = k + tid; i < n; i += NT) {
        cpx<double> x = cconj(A[(long long)k * n + i]);
        for (int q = 0; q < j; ++q)
          x = sub2prod(x, vp(i, q), cconj(wp(k, q)), wp(i, q), cconj(vp(k, q)));
        xk[i - k] = x;
      }
      __syncthreads();
      if (tid == 0) S.d[k] = xk[0].re;
      double xn = 0;
      for (int i = 2 + tid; i <= m; i += NT) xn += cabs2(xk[i]);
      xn = block_sum(xn, S.red, par);
      // every thread forms the reflector from the same values (no extra
      // phase for one thread to publish it)
      const cpx<double> alpha = xk[1];
      const bool act = !(xn == 0.0 && alpha.im == 0.0);
      cpx<double> tau = mk(0.0, 0.0), sc = mk(0.0, 0.0);
      if (act) {
        const double nrm = sqrt(cabs2(alpha) + xn);
        const double beta = alpha.re >= 0 ? -nrm : nrm;
        tau = mk((beta - alpha.re) / beta, -alpha.im / beta);
        const cpx<double> den = mk(alpha.re - beta, alpha.im);  // sc = 1 / (alpha - beta)
        const double dd = cabs2(den);
        sc = mk(den.re / dd, -den.im / dd);
        if (tid == 0) S.e[k] = beta;
      } else if (tid == 0) {
        S.e[k] = alpha.re;
      }
      if (tid == 0) S.tau[k] = tau;
      for (int i = tid; i < m; i += NT) {
        const cpx<double> v = !act ? mk(0.0, 0.0) : (i == 0) ? mk(1.0, 0.0) : xk[1 + i] * sc;
        S.v[i] = v;
        if (act) A[(long long)(c0 + i) * n + k] = v;  // kept for the back-transformation
        vp(c0 + i, j) = v;
      }
      __syncthreads();
      if (!act) {
        for (int i = tid; i < m; i += NT) wp(c0 + i, j) = mk(0.0, 0.0);
        __syncthreads();
        continue;
      }
      // y1 = W^H v, y2 = V^H v over rows c0..n-1, one wave per dot product
      // (in the phase of the matrix-vector pass, which ends with a barrier;
      // y12 lives in S.vp, which the pass does not touch without a pending
      // update)
      for (int d = wave; d < 2 * j; d += NT / 64) {
        const bool isw = d < j;
        const int q = isw ? d : d - j;
        double yr = 0, yi = 0;
        for (int i = lane; i < m; i += 64) {
          dotacc(yr, yi, isw ? wp(c0 + i, q) : vp(c0 + i, q), S.v[i]);  // conj(a) v
        }
        for (int off = 32; off > 0; off >>= 1) {
          yr += __shfl_xor(yr, off, 64);
          yi += __shfl_xor(yi, off, 64);
        }
        if (lane == 0) y12[(d < j ? 0 : TRB) + q] = mk(yr, yi);
      }
      fused_pass(A, n, c0, k, false, true, S);  // S.pp = A22 v (stored block)
      double g = 0;  // gamma = v^H p with p corrected for the panel
      for (int i = tid; i < m; i += NT) {
        cpx<double> pv = S.pp[i];
        for (int q = 0; q < j; ++q)
          pv = sub2prod(pv, vp(c0 + i, q), y12[q], wp(c0 + i, q), y12[TRB + q]);
        S.pp[i] = pv;
        g += S.v[i].re * pv.re + S.v[i].im * pv.im;
      }
      g = block_sum(g, S.red, par);
      const double cc = 0.5 * cabs2(tau) * g;
      for (int i = tid; i < m; i += NT) wp(c0 + i, j) = tau * S.pp[i] - cc * S.v[i];
      __syncthreads();
    }
    // trailing block [p1, n)^2 <- A - V W^H - W V^H
    const int p1 = p0 + np;
    const int mt = n - p1;
    if (mt > 0) {
      // 4 x 4 blocks per thread, all loads of a block independent.  For
      // n <= 256 the factors are read where they live (LDS); otherwise the
      // column factors conj(V), conj(W) are staged in LDS, transposed (t,
      // column), in windows of 256 columns, and the row factors come from
      // LDS too when one window holds the whole block (mt <= 256), else from
      // the panel in global memory (one row block per wave: a broadcast).
      static_assert(TRB == 8, "LDS panel factors hold eight columns");
      const bool one = mt <= 256;
      for (int cw = 0; cw < mt; cw += 256) {
        const int wn = min(256, mt - cw);
        if (!lv) {
          for (int e = tid; e < np * wn; e += NT) {
            const int t = e / wn, c = e % wn;
            S.pf[t * 256 + c] = cconj(Vp[(long long)(p1 + cw + c) * TRB + t]);
            S.pf[2048 + t * 256 + c] = cconj(Wp[(long long)(p1 + cw + c) * TRB + t]);
          }
          __syncthreads();
        }
        const int nbr = (mt + 3) >> 2, nbc = (wn + 3) >> 2;
        for (int u = tid; u < nbr * nbc; u += NT) {
          const int r0 = 4 * (u / nbc), q0 = 4 * (u % nbc);  // rows from p1, columns from p1 + cw
          cpx<double> x[4][4];
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
              x[i][j] = (r0 + i < mt && q0 + j < wn) ? A[(long long)(p1 + r0 + i) * n + p1 + cw + q0 + j]
                                                      : mk(0.0, 0.0);
#pragma unroll
          for (int t = 0; t < TRB; ++t) {
            if (t >= np) break;
            cpx<double> vr[4], wr[4], vc[4], wc[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {  // indices below 256; entries past mt, wn are not stored back
              if (lv) {
                const int rr = min(p1 + r0 + i, 255), cc = min(p1 + q0 + i, 255);
                vr[i] = S.pf[t * 256 + rr];
                wr[i] = S.pf[2048 + t * 256 + rr];
                vc[i] = cconj(S.pf[t * 256 + cc]);
                wc[i] = cconj(S.pf[2048 + t * 256 + cc]);
                continue;
              }
              if (one) {
                vr[i] = cconj(S.pf[t * 256 + r0 + i]);
                wr[i] = cconj(S.pf[2048 + t * 256 + r0 + i]);
              } else {
                const bool ok = r0 + i < mt;
                vr[i] = ok ? Vp[(long long)(p1 + r0 + i) * TRB + t] : mk(0.0, 0.0);
                wr[i] = ok ? Wp[(long long)(p1 + r0 + i) * TRB + t] : mk(0.0, 0.0);
              }
              vc[i] = S.pf[t * 256 + q0 + i];
              wc[i] = S.pf[2048 + t * 256 + q0 + i];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
              for (int j = 0; j < 4; ++j) x[i][j] = sub2prod(x[i][j], vr[i], wc[j], wr[i], vc[j]);
          }
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
              if (r0 + i < mt && q0 + j < wn) A[(long long)(p1 + r0 + i) * n + p1 + cw + q0 + j] = x[i][j];
        }
        __syncthreads();
      }
    }
  }
}

// Steps k0 .. n-2 of the reduction with one column per step (the previous
// step's rank-2 update fused with this step's matrix-vector pass) on A in
// global memory; `pend`: the update of step k0 - 1 (S.vp, S.wp; index 0 = row
// k0) is still to be applied to the block [k0, n)^2.  Writes S.d, S.e, S.tau
// from k0 on (S.d[n - 1] excepted: A[n-1][n-1] holds it at the end).
template <class SH>
__device__ void onecol_steps(cpx<double>* __restrict__ A, int n, int k0, bool pend, SH& S, int& par) {
  const int tid = threadIdx.x;
  for (int k = k0; k + 1 < n; ++k) {
    const int m = n - k - 1;
    const int c0 = k + 1;
    if (pend) {  // bring column k (rows k..n-1) up to date first
      const cpx<double> wk = cconj(S.wp[0]), vk = cconj(S.vp[0]);
      for (int i = k + tid; i < n; i += NT) {
        cpx<double> x = A[(long long)i * n + k];
        x = sub2prod(x, S.vp[i - k], wk, S.wp[i - k], vk);
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
}

// PANEL: the panel-blocked reduction (less memory traffic per step, more
// work per step: faster when many matrices share the memory system);
// otherwise one fused pass per step (lower latency for a lone matrix).
template <bool PANEL, class SH>
__device__ void heev_core(const EigDesc& dsc, cpx<double>* __restrict__ A, SH& S) {
  const int n = dsc.n, tid = threadIdx.x;
  int par = 0;  // block_sum buffer parity
  // ---- 1. load (symmetrised) ----
  const cpx<double>* a = reinterpret_cast<const cpx<double>*>(dsc.a);
  for (int e = tid; e < n * n; e += NT) {
    const int i = e / n, j = e % n;
    if (dsc.upper) {  // only the upper triangle is valid
      const cpx<double> x = i <= j ? a[(long long)i * dsc.lda + j] : a[(long long)j * dsc.lda + i];
      A[e] = i < j ? x : i > j ? cconj(x) : mk(x.re, 0.0);
    } else {
      const cpx<double> x = a[(long long)i * dsc.lda + j], y = a[(long long)j * dsc.lda + i];
      A[e] = mk(0.5 * (x.re + y.re), 0.5 * (x.im - y.im));
    }
  }
  __syncthreads();
  double tr = 0;
  for (int i = tid; i < n; i += NT) tr += A[i * n + i].re;
  tr = block_sum(tr, S.red, par);
  if constexpr (PANEL) {
    if (n <= 256) panel_tridiag<true>(dsc, A, n, S, par);
    else panel_tridiag<false>(dsc, A, n, S, par);
  } else {
    // ---- 2. tridiagonalisation, one column per step ----
    onecol_steps(A, n, 0, false, S, par);
  }
  if (tid == 0) S.d[n - 1] = A[(long long)(n - 1) * n + n - 1].re;
  for (int i = tid; i + 1 < n; i += NT) S.e2[i] = S.e[i] * S.e[i];
  __syncthreads();
  const int kz = eig_tail<NT>(dsc, n, tr, S, par);
  // ---- 6. back-transformation z <- H_0 ... H_{n-2} z, in blocks ----
  if constexpr (PANEL) {
    if (kz > 0 && n <= 256 && kz <= 64) back_transform_reg(dsc, A, n, kz, S);
    else if (kz > 0) back_transform(dsc, A, n, kz, S);
  } else if (kz > 0) {
    back_transform(dsc, A, n, kz, S);
  }
}

// ---------------------------------------------------------------------------
// Two-stage reduction for 128 < n <= 256 (the new-bond Grams of the two-site
// update, n = 2 r_F):
//
//  1. dense -> band of half-width BW: Householder QR of each BW-column panel
//     below the band (in LDS), Q = I - V T V^H (T upper triangular), and the
//     two-sided update A22 <- Q^H A22 Q = A22 - W V^H - V W^H with
//     X = A22 V T, W = X - V (T^H V^H X) / 2: the trailing block is read twice
//     and written once per BW columns (the one-stage form reads it once per
//     column);
//  2. band -> real symmetric tridiagonal by bulge chasing in LDS (lower band
//     with room for the bulge, 2 BW + 1 entries per column): sweep j reduces
//     column j with a reflector on rows j+1..j+BW, then chases the bulge it
//     creates down the band block by block (right application to the block
//     below, a reflector on that block's first column, its left application
//     to the rest, two-sided application to the next diagonal block).  The
//     eight waves run consecutive sweeps concurrently: step t of sweep j
//     waits until sweep j - 1 has finished step t + 2 (the steps touch rows
//     [j + 1 + (t - 1) BW, j + 1 + (t + 1) BW)), through progress stamps in
//     LDS;
//  3. eigenvalues and eigenvectors of the tridiagonal matrix (eig_tail);
//  4. back-transformation z <- Q1 Q2 z: the chase reflectors in reverse
//     order, one 16-lane group per eigenvector column (no barriers: a column
//     is one group's sequential work), then the panels' Q in reverse.
// ---------------------------------------------------------------------------
constexpr int BW = 16;
constexpr int BS_NMAX = 256;
constexpr int BS_LD = 2 * BW + 1;
constexpr int BS_ROWS = BS_NMAX - BW;
constexpr int BS_ZC = 32;  // eigenvector columns per back-transformation pass
constexpr int BS_RC = 16;  // chase reflectors staged in LDS per chunk
constexpr int BS_REC = 18; // complex entries per chase reflector record: v[BW], tau, (row0, len)
constexpr int BS_PANELS = BS_NMAX / BW; // panel T matrices kept for the back-transformation
constexpr int BS_BIG_S1 = 2 * BS_ROWS * BW + 3 * BW * BW;
constexpr int BS_BIG_S2 = BS_NMAX * BS_LD;
constexpr int BS_BIG_S4 = BS_NMAX * BS_ZC + (BS_RC * BS_REC > BW * BS_ZC ? BS_RC * BS_REC : BW * BS_ZC);
constexpr int BS_BIG = BS_BIG_S1 > BS_BIG_S2 ? (BS_BIG_S1 > BS_BIG_S4 ? BS_BIG_S1 : BS_BIG_S4)
                                             : (BS_BIG_S2 > BS_BIG_S4 ? BS_BIG_S2 : BS_BIG_S4);

// number of chase reflectors of an n x n band reduction (sweep j has
// ceil((n - 1 - j) / BW) steps)
__host__ __device__ inline int band_reflectors(int n) {
  int c = 0;
  for (int k = 1; k < n; ++k) c += (k + BW - 1) / BW;
  return c;
}

struct alignas(16) SharedBand {
  alignas(16) cpx<double> big[BS_BIG];
  alignas(16) cpx<double> pp[BS_NMAX];  // eig_tail's dot products
  cpx<double> tau[BW];
  double d[BS_NMAX], e[BS_NMAX], e2[BS_NMAX];
  double ev[BS_NMAX + 1];
  double red[2 * NW];
  double scal[4];
  int flag[4];
  int clus[BS_NMAX + 1];
  int stamp[NW];  // per wave: sweep * 65536 + steps done (65535: sweep finished)
  int fail;
  static constexpr int SOLVE_CAP = 0;
  __device__ double* solve() { return nullptr; }
};

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Householder reflector of x (length len <= BW, lanes 4 i + q hold x_i when
// q == 0; other lanes pass zero): (I - tau v v^H)^H x = beta e_1, beta real,
// v_0 = 1.  Every lane returns tau, beta and its v_i (lanes 4 i + q, any q).
__device__ inline void wave_house(cpx<double> x, int len, cpx<double>& v, cpx<double>& tau, double& beta) {
  const int lane = threadIdx.x & 63, i = lane >> 2;
  const cpx<double> alpha = mk(__shfl(x.re, 0, 64), __shfl(x.im, 0, 64));
  double xn = ((lane & 3) == 0 && i >= 1 && i < len) ? cabs2(x) : 0.0;
  for (int off = 32; off > 0; off >>= 1) xn += __shfl_xor(xn, off, 64);
  const cpx<double> xi = mk(__shfl(x.re, 4 * i, 64), __shfl(x.im, 4 * i, 64));
  if (xn == 0.0 && alpha.im == 0.0) {
    tau = mk(0.0, 0.0);
    beta = alpha.re;
    v = i == 0 ? mk(1.0, 0.0) : mk(0.0, 0.0);
    return;
  }
  const double nrm = sqrt(cabs2(alpha) + xn);
  beta = alpha.re >= 0 ? -nrm : nrm;
  tau = mk((beta - alpha.re) / beta, -alpha.im / beta);
  const cpx<double> den = mk(alpha.re - beta, alpha.im);
  const double dd = cabs2(den);
  const cpx<double> sc = mk(den.re / dd, -den.im / dd);
  v = i == 0 ? mk(1.0, 0.0) : (i < len ? xi * sc : mk(0.0, 0.0));
}

// Stage 1: A (n x n, both triangles) -> lower band of half-width BW in place;
// the panels' V stay below the band, their T go to Tg (BW x BW each).
template <class SH>
__device__ void band_stage1(cpx<double>* __restrict__ A, int n, cpx<double>* __restrict__ Tg, SH& S, int& par) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  cpx<double>* Pl = S.big;                  // panel, m x BW: R on top, V below the diagonal
  cpx<double>* Xl = S.big + BS_ROWS * BW;   // Y = V T, then X = A22 Y, then W
  cpx<double>* Gs = Xl + BS_ROWS * BW;      // BW x BW scratch
  cpx<double>* Ts = Gs + BW * BW;
  cpx<double>* Ms = Ts + BW * BW;
  for (int kb = 0, p = 0; kb + BW < n; kb += BW, ++p) {
    const int r0 = kb + BW, m = n - r0, nc = m < BW ? m : BW;
    for (int e = tid; e < m * BW; e += NT) Pl[e] = A[(long long)(r0 + e / BW) * n + kb + e % BW];
    __syncthreads();
    // Householder QR of the panel
    for (int c = 0; c < nc; ++c) {
      double xn = 0;
      for (int i = c + 1 + tid; i < m; i += NT) xn += cabs2(Pl[i * BW + c]);
      xn = block_sum(xn, S.red, par);
      if (tid == 0) {
        const cpx<double> alpha = Pl[c * BW + c];
        if (xn == 0.0 && alpha.im == 0.0) {
          S.tau[c] = mk(0.0, 0.0);
          S.flag[0] = 0;
        } else {
          const double nrm = sqrt(cabs2(alpha) + xn);
          const double beta = alpha.re >= 0 ? -nrm : nrm;
          S.tau[c] = mk((beta - alpha.re) / beta, -alpha.im / beta);
          const cpx<double> den = mk(alpha.re - beta, alpha.im);
          const double dd = cabs2(den);
          S.scal[0] = den.re / dd;
          S.scal[1] = -den.im / dd;
          S.scal[2] = beta;
          S.flag[0] = 1;
        }
      }
      __syncthreads();
      if (S.flag[0] == 0) continue;  // uniform: the reflector is the identity
      const cpx<double> sc = mk(S.scal[0], S.scal[1]);
      for (int i = c + 1 + tid; i < m; i += NT) Pl[i * BW + c] = Pl[i * BW + c] * sc;
      __syncthreads();
      if (tid == 0) Pl[c * BW + c] = mk(S.scal[2], 0.0);
      // H^H on the panel's later columns: s = v^H P[c:, cc], P[c:, cc] -= conj(tau) v s
      for (int cc = c + 1 + wave; cc < BW; cc += NW) {
        double sr = 0, si = 0;
        for (int i = c + lane; i < m; i += 64) {
          const cpx<double> v = i == c ? mk(1.0, 0.0) : Pl[i * BW + c];
          dotacc(sr, si, v, Pl[i * BW + cc]);
        }
        for (int off = 32; off > 0; off >>= 1) {
          sr += __shfl_xor(sr, off, 64);
          si += __shfl_xor(si, off, 64);
        }
        if (lane == 0) Gs[cc] = mk(sr, si);
      }
      __syncthreads();
      const cpx<double> ct = cconj(S.tau[c]);
      const int w = BW - c - 1;
      for (int e = tid; e < (m - c) * w; e += NT) {
        const int i = c + e / w, cc = c + 1 + e % w;
        const cpx<double> v = i == c ? mk(1.0, 0.0) : Pl[i * BW + c];
        Pl[i * BW + cc] = subprod(Pl[i * BW + cc], ct * v, Gs[cc]);
      }
      __syncthreads();
    }
    auto V = [&](int i, int c) -> cpx<double> {
      return (c >= nc || i < c) ? mk(0.0, 0.0) : (i == c ? mk(1.0, 0.0) : Pl[i * BW + c]);
    };
    // T: T_cc = tau_c, T(0:c, c) = -tau_c T(0:c, 0:c) (V(:, 0:c)^H v_c)
    for (int e = tid; e < BW * BW; e += NT) {
      const int c1 = e / BW, c2 = e % BW;
      double sr = 0, si = 0;
      if (c1 < c2 && c2 < nc)
        for (int i = c2; i < m; ++i) dotacc(sr, si, V(i, c1), V(i, c2));
      Gs[e] = mk(sr, si);
    }
    __syncthreads();
    if (tid == 0) {
      for (int e = 0; e < BW * BW; ++e) Ts[e] = mk(0.0, 0.0);
      for (int c = 0; c < nc; ++c) {
        const cpx<double> t = S.tau[c];
        Ts[c * BW + c] = t;
        for (int r = 0; r < c; ++r) {
          cpx<double> s = mk(0.0, 0.0);
          for (int k = r; k < c; ++k) s = s + Ts[r * BW + k] * Gs[k * BW + c];
          Ts[r * BW + c] = mk(-(t.re * s.re - t.im * s.im), -(t.re * s.im + t.im * s.re));
        }
      }
    }
    __syncthreads();
    for (int e = tid; e < BW * BW; e += NT) Tg[(long long)p * BW * BW + e] = Ts[e];
    // Y = V T
    for (int e = tid; e < m * BW; e += NT) {
      const int i = e / BW, c = e % BW;
      cpx<double> s = mk(0.0, 0.0);
      const int kmax = min(c, min(i, nc - 1));
      for (int k = 0; k <= kmax; ++k) s = s + V(i, k) * Ts[k * BW + c];
      Xl[e] = s;
    }
    __syncthreads();
    // X = A22 Y: thread (i, h) sums its row's eight columns 8 h .. 8 h + 7
    {
      cpx<double> acc[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] = mk(0.0, 0.0);
      const bool own = tid < 2 * m;
      const int i = tid % (m > 0 ? m : 1), h = tid / (m > 0 ? m : 1);
      if (own) {
        for (int j = 0; j < m; ++j) {
          const cpx<double> a = cconj(A[(long long)(r0 + j) * n + r0 + i]);  // A22[i][j]
          const cpx<double>* y = Xl + j * BW + 8 * h;
#pragma unroll
          for (int u = 0; u < 8; ++u) acc[u] = acc[u] + a * y[u];
        }
      }
      __syncthreads();
      if (own)
#pragma unroll
        for (int u = 0; u < 8; ++u) Xl[i * BW + 8 * h + u] = acc[u];
      __syncthreads();
    }
    // G = V^H X, M = T^H G, W = X - V M / 2
    for (int e = tid; e < BW * BW; e += NT) {
      const int c1 = e / BW, c2 = e % BW;
      double sr = 0, si = 0;
      if (c1 < nc)
        for (int i = c1; i < m; ++i) dotacc(sr, si, V(i, c1), Xl[i * BW + c2]);
      Gs[e] = mk(sr, si);
    }
    __syncthreads();
    for (int e = tid; e < BW * BW; e += NT) {
      const int c1 = e / BW, c2 = e % BW;
      double sr = 0, si = 0;
      for (int k = 0; k <= c1; ++k) dotacc(sr, si, Ts[k * BW + c1], Gs[k * BW + c2]);
      Ms[e] = mk(sr, si);
    }
    __syncthreads();
    for (int e = tid; e < m * BW; e += NT) {
      const int i = e / BW, c = e % BW;
      cpx<double> s = mk(0.0, 0.0);
      const int kmax = min(i, nc - 1);
      for (int k = 0; k <= kmax; ++k) s = s + V(i, k) * Ms[k * BW + c];
      Xl[e] = Xl[e] - 0.5 * s;
    }
    // the panel back: R on and above the diagonal, V below
    for (int e = tid; e < m * BW; e += NT) A[(long long)(r0 + e / BW) * n + kb + e % BW] = Pl[e];
    __syncthreads();
    // A22 -= W V^H + V W^H, 4 x 4 blocks per thread
    const int nb = (m + 3) >> 2;
    for (int u = tid; u < nb * nb; u += NT) {
      const int i0 = 4 * (u / nb), j0 = 4 * (u % nb);
      cpx<double> x[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          x[a][b] = (i0 + a < m && j0 + b < m) ? A[(long long)(r0 + i0 + a) * n + r0 + j0 + b] : mk(0.0, 0.0);
      for (int c = 0; c < nc; ++c) {
        cpx<double> vr[4], wr[4], vc[4], wc[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int ir = min(i0 + a, m - 1), jc = min(j0 + a, m - 1);
          vr[a] = V(ir, c);
          wr[a] = Xl[ir * BW + c];
          vc[a] = cconj(V(jc, c));
          wc[a] = cconj(Xl[jc * BW + c]);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) x[a][b] = sub2prod(x[a][b], wr[a], vc[b], vr[a], wc[b]);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if (i0 + a < m && j0 + b < m) A[(long long)(r0 + i0 + a) * n + r0 + j0 + b] = x[a][b];
    }
    __syncthreads();
  }
}


// Stage 2: the lower band (half-width BW) of A -> real symmetric tridiagonal
// (S.d, S.e); the chase reflectors go to R2 in application order, BS_REC
// complex each: v[0..BW) (v_0 = 1, zero past len), tau, (row0, len).
// Returns false if a wave waited past its spin limit (the result is then
// marked failed by the caller).
template <class SH>
__device__ bool band_stage2(const cpx<double>* __restrict__ A, int n, cpx<double>* __restrict__ R2, SH& S) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  cpx<double>* L = S.big;  // L[c * BS_LD + d] = A[c + d][c], d <= 2 BW
  for (int e = tid; e < n * BS_LD; e += NT) {
    const int c = e / BS_LD, d = e % BS_LD;
    cpx<double> x = (d <= BW && c + d < n) ? A[(long long)(c + d) * n + c] : mk(0.0, 0.0);
    if (d == 0) x.im = 0.0;
    L[e] = x;
  }
  if (tid < NW) S.stamp[tid] = -1;
  if (tid == 0) S.fail = 0;
  __syncthreads();
  // lane = 4 bi + bq owns row bi of a BW x BW block and its columns 4 bq .. 4 bq + 3
  const int bi = lane >> 2, bq = lane & 3;
  auto at = [&](int i, int j) -> cpx<double>& { return L[j * BS_LD + (i - j)]; };  // i >= j
  auto bcast = [&](cpx<double> x, int k) -> cpx<double> {  // row k's value from lane 4 k
    return mk(__shfl(x.re, 4 * k, 64), __shfl(x.im, 4 * k, 64));
  };
  // D <- H^H D H on the diagonal block [r, r + len): p = D v, w = tau p -
  // (|tau|^2 / 2)(v^H p) v, D -= w v^H + v w^H (lower triangle written)
  auto two_sided = [&](int r, int len, cpx<double> v, cpx<double> tau) {
    cpx<double> dl[4];
    double pr = 0, pim = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = 4 * bq + u;
      const cpx<double> vk = bcast(v, k);
      dl[u] = mk(0.0, 0.0);
      if (bi < len && k < len) dl[u] = bi >= k ? at(r + bi, r + k) : cconj(at(r + k, r + bi));
      const cpx<double> t = dl[u] * vk;
      pr += t.re;
      pim += t.im;
    }
    pr += __shfl_xor(pr, 1, 64);
    pim += __shfl_xor(pim, 1, 64);
    pr += __shfl_xor(pr, 2, 64);
    pim += __shfl_xor(pim, 2, 64);
    const cpx<double> p = mk(pr, pim);
    double g = bq == 0 ? v.re * p.re + v.im * p.im : 0.0;
    for (int off = 32; off > 0; off >>= 1) g += __shfl_xor(g, off, 64);
    const double cc = 0.5 * cabs2(tau) * g;
    const cpx<double> w = tau * p - cc * v;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = 4 * bq + u;
      const cpx<double> vk = bcast(v, k), wk = bcast(w, k);
      if (bi < len && k <= bi) {
        cpx<double> x = sub2prod(dl[u], w, cconj(vk), v, cconj(wk));
        if (k == bi) x.im = 0.0;
        at(r + bi, r + k) = x;
      }
    }
  };
  auto record = [&](int idx, int r, int len, cpx<double> v, cpx<double> tau) {
    cpx<double>* rec = R2 + (long long)idx * BS_REC;
    if (bq == 0) rec[bi] = v;
    if (lane == 0) {
      rec[BW] = tau;
      rec[BW + 1] = mk((double)r, (double)len);
    }
  };
  bool ok = true;
  for (int j = wave; j + 1 < n; j += NW) {
    int idx = 0;  // first reflector of sweep j
    for (int jj = 0; jj < j; ++jj) idx += (n - 1 - jj + BW - 1) / BW;
    cpx<double> pv = mk(0.0, 0.0), ptau = mk(0.0, 0.0);  // the previous step's reflector
    for (int t = 0;; ++t) {
      const int r = j + 1 + t * BW;  // this step's diagonal block [r, r + len)
      if (r > n - 1) break;
      const int len = min(BW, n - r);
      if (j > 0 && ok) {  // sweep j - 1 must have finished its step t + 2
        // (a step takes microseconds: a wait past the spin limit means a
        // fault of this code; the wave then stops waiting and the result is
        // reported as failed, so the kernel always ends)
        const int target = (j - 1) * 65536 + t + 3;
        int spins = 0;
        while (__hip_atomic_load(&S.stamp[(j - 1) % NW], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < target) {
          if (++spins > (1 << 20)) {
            ok = false;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      cpx<double> v, tau;
      double beta;
      if (t == 0) {
        // column j, rows [r, r + len)
        const cpx<double> x = (bq == 0 && bi < len) ? at(r + bi, j) : mk(0.0, 0.0);
        wave_house(x, len, v, tau, beta);
        if (bq == 0 && bi < len) at(r + bi, j) = bi == 0 ? mk(beta, 0.0) : mk(0.0, 0.0);
        if (lane == 0) S.e[j] = beta;
      } else {
        // the block B below the previous diagonal block: rows [r, r + len),
        // columns [pr, pr + BW): B <- B H_prev, then the reflector of B's
        // first column and its left application to the other columns
        const int pr = r - BW;
        cpx<double> b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) b[u] = bi < len ? at(r + bi, pr + 4 * bq + u) : mk(0.0, 0.0);
        double sr = 0, si = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const cpx<double> t2 = b[u] * bcast(pv, 4 * bq + u);
          sr += t2.re;
          si += t2.im;
        }
        sr += __shfl_xor(sr, 1, 64);
        si += __shfl_xor(si, 1, 64);
        sr += __shfl_xor(sr, 2, 64);
        si += __shfl_xor(si, 2, 64);
        const cpx<double> ts = ptau * mk(sr, si);
#pragma unroll
        for (int u = 0; u < 4; ++u) b[u] = subprod(b[u], ts, cconj(bcast(pv, 4 * bq + u)));
        const cpx<double> x = (bq == 0 && bi < len) ? b[0] : mk(0.0, 0.0);
        wave_house(x, len, v, tau, beta);
        const cpx<double> ctv = cconj(tau) * v;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          double qr = 0, qi = 0;
          dotacc(qr, qi, v, b[u]);  // conj(v_bi) B[bi][k]
          for (int off = 4; off < 64; off <<= 1) {
            qr += __shfl_xor(qr, off, 64);
            qi += __shfl_xor(qi, off, 64);
          }
          if (4 * bq + u >= 1) b[u] = subprod(b[u], ctv, mk(qr, qi));
        }
        if (bq == 0) b[0] = bi == 0 ? mk(beta, 0.0) : mk(0.0, 0.0);
        if (bi < len)
#pragma unroll
          for (int u = 0; u < 4; ++u) at(r + bi, pr + 4 * bq + u) = b[u];
      }
      record(idx + t, r, len, v, tau);
      two_sided(r, len, v, tau);
      pv = v;
      ptau = tau;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __hip_atomic_store(&S.stamp[wave], j * 65536 + t + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __hip_atomic_store(&S.stamp[wave], j * 65536 + 65535, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  if (!ok) S.fail = 1;
  __syncthreads();
  for (int c = tid; c < n; c += NT) S.d[c] = L[c * BS_LD].re;
  __syncthreads();
  return S.fail == 0;
}

// Stage 4: Z <- Q1 Q2 Z for the kz leading columns of dsc.evecs (ld n).
template <class SH>
__device__ void band_back(const EigDesc& dsc, const cpx<double>* __restrict__ A, int n, int kz,
                          const cpx<double>* __restrict__ Tg, const cpx<double>* __restrict__ R2, SH& S) {
  cpx<double>* __restrict__ Z = reinterpret_cast<cpx<double>*>(dsc.evecs);
  cpx<double>* Zl = S.big;                       // n x BS_ZC
  cpx<double>* Xl = S.big + BS_NMAX * BS_ZC;     // staged reflectors, then BW x BS_ZC products
  const int tid = threadIdx.x, g = tid >> 4, li = tid & 15;
  const int nrefl = band_reflectors(n);
  int npan = 0;
  while (npan * BW + BW < n) ++npan;
  for (int z0 = 0; z0 < kz; z0 += BS_ZC) {
    const int zc = min(BS_ZC, kz - z0);
    for (int e = tid; e < n * BS_ZC; e += NT) {
      const int r = e / BS_ZC, c = e % BS_ZC;
      Zl[e] = c < zc ? Z[(long long)r * n + z0 + c] : mk(0.0, 0.0);
    }
    __syncthreads();
    // chase reflectors, the last first; group g (16 lanes) owns column g
    for (int top = nrefl; top > 0; top -= BS_RC) {
      const int lo = top > BS_RC ? top - BS_RC : 0, cnt = top - lo;
      for (int e = tid; e < cnt * BS_REC; e += NT) Xl[e] = R2[(long long)lo * BS_REC + e];
      __syncthreads();
      if (g < zc) {
        for (int k = cnt - 1; k >= 0; --k) {
          const cpx<double>* rec = Xl + k * BS_REC;
          const cpx<double> meta = rec[BW + 1];
          const int r = (int)meta.re, len = (int)meta.im;
          const cpx<double> tau = rec[BW];
          const cpx<double> v = rec[li];
          cpx<double> z = li < len ? Zl[(r + li) * BS_ZC + g] : mk(0.0, 0.0);
          double sr = 0, si = 0;
          dotacc(sr, si, v, z);
          for (int off = 1; off < 16; off <<= 1) {
            sr += __shfl_xor(sr, off, 16);
            si += __shfl_xor(si, off, 16);
          }
          z = subprod(z, tau * v, mk(sr, si));
          if (li < len) Zl[(r + li) * BS_ZC + g] = z;
        }
      }
      __syncthreads();
    }
    // panels, the last first: Z[r0:] -= V (T (V^H Z[r0:]))
    for (int p = npan - 1; p >= 0; --p) {
      const int kb = p * BW, r0 = kb + BW, m = n - r0, nc = m < BW ? m : BW;
      auto V = [&](int i, int c) -> cpx<double> {
        return (c >= nc || i < c) ? mk(0.0, 0.0) : (i == c ? mk(1.0, 0.0) : A[(long long)(r0 + i) * n + kb + c]);
      };
      for (int e = tid; e < BW * BS_ZC; e += NT) {
        const int c1 = e / BS_ZC, c = e % BS_ZC;
        double sr = 0, si = 0;
        if (c1 < nc && c < zc)
          for (int i = c1; i < m; ++i) dotacc(sr, si, V(i, c1), Zl[(r0 + i) * BS_ZC + c]);
        Xl[e] = mk(sr, si);
      }
      __syncthreads();
      // Xl <- T Xl in place (T upper triangular: row c1 needs rows >= c1)
      if (tid < zc) {
        const cpx<double>* T = Tg + (long long)p * BW * BW;
        for (int c1 = 0; c1 < nc; ++c1) {
          cpx<double> s = mk(0.0, 0.0);
          for (int k = c1; k < nc; ++k) s = s + T[c1 * BW + k] * Xl[k * BS_ZC + tid];
          Xl[c1 * BS_ZC + tid] = s;
        }
      }
      __syncthreads();
      for (int e = tid; e < m * BS_ZC; e += NT) {
        const int i = e / BS_ZC, c = e % BS_ZC;
        if (c >= zc) continue;
        cpx<double> s = mk(0.0, 0.0);
        const int kmax = min(i, nc - 1);
        for (int k = 0; k <= kmax; ++k) s = s + V(i, k) * Xl[k * BS_ZC + c];
        Zl[(r0 + i) * BS_ZC + c] = Zl[(r0 + i) * BS_ZC + c] - s;
      }
      __syncthreads();
    }
    for (int e = tid; e < n * BS_ZC; e += NT) {
      const int r = e / BS_ZC, c = e % BS_ZC;
      if (c < zc) Z[(long long)r * n + z0 + c] = Zl[e];
    }
    __syncthreads();
  }
}

// The whole solver for 128 < n <= BS_NMAX (see the section comment).
template <class SH>
__device__ void heev_band(const EigDesc& dsc, cpx<double>* __restrict__ A, SH& S) {
  const int n = dsc.n, tid = threadIdx.x;
  int par = 0;
  const cpx<double>* a = reinterpret_cast<const cpx<double>*>(dsc.a);
  for (int e = tid; e < n * n; e += NT) {
    const int i = e / n, j = e % n;
    if (dsc.upper) {
      const cpx<double> x = i <= j ? a[(long long)i * dsc.lda + j] : a[(long long)j * dsc.lda + i];
      A[e] = i < j ? x : i > j ? cconj(x) : mk(x.re, 0.0);
    } else {
      const cpx<double> x = a[(long long)i * dsc.lda + j], y = a[(long long)j * dsc.lda + i];
      A[e] = mk(0.5 * (x.re + y.re), 0.5 * (x.im - y.im));
    }
  }
  __syncthreads();
  double tr = 0;
  for (int i = tid; i < n; i += NT) tr += A[i * n + i].re;
  tr = block_sum(tr, S.red, par);
  const long long np = (n + 63) / 64 * 64;
  cpx<double>* Tg = reinterpret_cast<cpx<double>*>(dsc.work + 2LL * n * n + 7LL * n * np + 64);
  cpx<double>* R2 = Tg + BS_PANELS * BW * BW;
  band_stage1(A, n, Tg, S, par);
  const bool ok = band_stage2(A, n, R2, S);
  for (int i = tid; i + 1 < n; i += NT) S.e2[i] = S.e[i] * S.e[i];
  __syncthreads();
  const int kz = eig_tail<NT>(dsc, n, tr, S, par);
  if (!ok && tid == 0 && dsc.trace) *dsc.trace = __builtin_nan("");
  if (kz > 0) band_back(dsc, A, n, kz, Tg, R2, S);
}
}  // namespace

// ---------------------------------------------------------------------------
// n <= 128: the matrix lives in registers.  Thread t owns columns
// c + (RN / CPT) j, j < CPT, c = t mod (RN / CPT), over one block of rows
// (the variants below).  Each tridiagonalisation step is four
// phases between barriers: (a) the previous step's rank-2 update on the
// owned entries and publication of column k, (b) the reflector (one wave),
// (c) partial products of A v over the owned rows, (d) their sums and
// w (one wave).  The reflectors go to dsc.work for the back-transformation,
// which keeps the eigenvector block in registers (at most two vectors per
// thread).
// ---------------------------------------------------------------------------
// Two variants share the code below (RN: largest n, NTR: threads, NLO:
// smaller n are left to the other variant, CPT: columns per thread):
//   <128, 512, 32, 4>: 32 < n <= 128, two waves per SIMD (256 VGPRs each);
//   each thread holds 8 rows of four columns, so a row value read from LDS
//   serves four columns (the rank-2 updates are bound by these broadcast
//   reads: 1.79 -> 1.70 ms for 512 matrices of n = 128 against two columns);
//   <32, 64, 0, 1>: n <= 32, one wave per matrix, so its barriers cost little
//   and many matrices share a CU.
constexpr int REG_NMAX = 128, SMALL_NMAX = 32;

// 16-byte alignment lets the compiler use 128-bit LDS accesses with
// immediate offsets for the complex vectors.
template <int RN, int NTR, int CPT, int SCAP> struct alignas(16) SharedR {
  static constexpr int RQ = NTR / (RN / CPT);
  alignas(16) cpx<double> tau[RN];
  alignas(16) cpx<double> x[RN];
  alignas(16) cpx<double> v[3][RN];
  alignas(16) cpx<double> vp[RN];
  alignas(16) cpx<double> wp[RN];
  alignas(16) cpx<double> pp[2][RQ][RN];
  double d[RN], e[RN], e2[RN];
  double ev[RN + 1];
  int clus[RN + 1];
  double red[2 * (NTR / 64)];
  int flag[4];
  // the seven inverse-iteration arrays (n x kz each) when 7 n kz <= SCAP
  static constexpr int SOLVE_CAP = SCAP;
  double sv[SOLVE_CAP];
  __device__ double* solve() { return sv; }
};

__device__ inline double wave_allsum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int RN, int NTR, int NLO, int CPT>
__global__ __launch_bounds__(NTR) void k_heev_reg(const EigDesc* __restrict__ descs, int* __restrict__ status) {
  constexpr int CW = RN / CPT;  // thread c holds columns c + CW j, j < CPT
  constexpr int RQ = NTR / CW;  // row blocks
  constexpr int RR = RN / RQ;   // rows per thread
  constexpr int NH = (RN + 63) / 64;  // vector entries per lane of wave 0
  static_assert(RR % 8 == 0, "rows are updated in groups of eight");
  __shared__ SharedR<RN, NTR, CPT, RN == REG_NMAX ? 7 * 1024 : 7 * 256> S;
  const EigDesc& dsc = descs[blockIdx.x];
  if (!dsc.active || dsc.n <= NLO || dsc.n > RN) return;
  const int n = dsc.n, tid = threadIdx.x, lane = tid & 63;
  const int c = tid % CW, q = tid / CW, r0 = q * RR;
  int par = 0;
  cpx<double>* __restrict__ Vg = reinterpret_cast<cpx<double>*>(dsc.work);  // row k: v_k, absolute index
  // ---- load (symmetrised) ----
  cpx<double> a[CPT][RR];
  {
    const cpx<double>* __restrict__ Ain = reinterpret_cast<const cpx<double>*>(dsc.a);
    double trp = 0;
#pragma unroll
    for (int j = 0; j < CPT; ++j)
#pragma unroll
      for (int u = 0; u < RR; ++u) {
        const int r = r0 + u, cj = c + CW * j;
        a[j][u] = mk(0.0, 0.0);
        if (r < n && cj < n) {
          if (dsc.upper) {  // only the upper triangle is valid
            const cpx<double> x = r <= cj ? Ain[(long long)r * dsc.lda + cj] : Ain[(long long)cj * dsc.lda + r];
            a[j][u] = r < cj ? x : r > cj ? cconj(x) : mk(x.re, 0.0);
          } else {
            const cpx<double> x = Ain[(long long)r * dsc.lda + cj], y = Ain[(long long)cj * dsc.lda + r];
            a[j][u] = mk(0.5 * (x.re + y.re), 0.5 * (x.im - y.im));
          }
          if (r == cj) trp += a[j][u].re;
        }
      }
    const double tr = block_sum<NTR>(trp, S.red, par);
    if (tid == 0) S.ev[RN] = tr;  // parked until the tail
  }
  // ---- tridiagonalisation ----
  // The shared vectors v, vp, wp are exactly zero outside the active range
  // of their step, so the register updates and products run over every
  // owned entry without predicates: out-of-range terms are exact zeros.
  for (int i = tid; i < RN; i += NTR) {
    S.vp[i] = mk(0.0, 0.0);
    S.wp[i] = mk(0.0, 0.0);
    S.v[0][i] = mk(0.0, 0.0);
    S.v[1][i] = mk(0.0, 0.0);
  }
  __syncthreads();
  bool pend = false;
  for (int k = 0; k + 1 < n; ++k) {
    const int c0 = k + 1;
    // (a) rank-2 update of step k-1 on [k, n) x [k, n); publish column k
    // (the update is zero outside rows and columns [k, n): finished rows and
    // rows beyond n are skipped per group of eight, uniformly across the
    // wave, finished columns and columns beyond n per thread)
    bool on[CPT], any = false;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      on[j] = c + CW * j >= k && c + CW * j < n;
      any = any || on[j];
    }
    if (pend && r0 + RR > k && r0 < n && any) {
      cpx<double> wc[CPT], vc[CPT];
#pragma unroll
      for (int j = 0; j < CPT; ++j) {
        wc[j] = cconj(S.wp[c + CW * j]);
        vc[j] = cconj(S.vp[c + CW * j]);
      }
#pragma unroll
      for (int u0 = 0; u0 < RR; u0 += 8) {
        if (r0 + u0 + 8 <= k || r0 + u0 >= n) continue;
        cpx<double> vr[8], wr[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          vr[u] = S.vp[r0 + u0 + u];
          wr[u] = S.wp[r0 + u0 + u];
        }
#pragma unroll
        for (int j = 0; j < CPT; ++j)
          if (on[j]) {
#pragma unroll
            for (int u = 0; u < 8; ++u) a[j][u0 + u] = sub2prod(a[j][u0 + u], vr[u], wc[j], wr[u], vc[j]);
          }
      }
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j)
      if (c + CW * j == k) {
#pragma unroll
        for (int u = 0; u < RR; ++u) S.x[r0 + u] = a[j][u];
      }
    __syncthreads();
    // (b) reflector with H^H x = beta e_1, v[c0] = 1 (wave 0, every lane
    // computes the same scalars)
    if (tid < 64) {
      double xn = 0;
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        const int i = lane + 64 * h;
        if (i < RN) {
          const cpx<double> x = S.x[i];
          xn += (i > c0 && i < n) ? cabs2(x) : 0.0;
        }
      }
      xn = wave_allsum(xn);
      const cpx<double> alpha = S.x[c0];
      if (lane == 0) S.d[k] = S.x[k].re;
      if (xn == 0.0 && alpha.im == 0.0) {
        if (lane == 0) {
          S.tau[k] = mk(0.0, 0.0);
          S.e[k] = alpha.re;
          S.flag[0] = 0;
        }
      } else {
        const double nrm = sqrt(cabs2(alpha) + xn);
        const double beta = alpha.re >= 0 ? -nrm : nrm;
        const cpx<double> den = mk(alpha.re - beta, alpha.im);
        const double rdd = 1.0 / cabs2(den);
        const cpx<double> sc = mk(den.re * rdd, -den.im * rdd);
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          const int i = lane + 64 * h;
          if (i < RN) {
            const cpx<double> v = S.x[i] * sc;
            S.v[0][i] = (i == c0) ? mk(1.0, 0.0) : ((i > c0 && i < n) ? v : mk(0.0, 0.0));
          }
        }
        if (lane == 0) {
          const double rb = 1.0 / beta;
          S.tau[k] = mk((beta - alpha.re) * rb, -alpha.im * rb);
          S.e[k] = beta;
          S.flag[0] = 1;
        }
      }
    }
    __syncthreads();
    const bool act = S.flag[0] != 0;
    if (act) {
      // (c) partial p[c] = sum_r conj(A[r][c]) v[r] over the owned rows; the
      // owner of column k keeps v_k in its finished entries
      const bool rows = r0 + RR > c0 && r0 < n;
#pragma unroll
      for (int j = 0; j < CPT; ++j)
        if (c + CW * j == k) {
#pragma unroll
          for (int u = 0; u < RR; ++u) a[j][u] = S.v[0][r0 + u];
        }
      bool in[CPT], anyin = false;
#pragma unroll
      for (int j = 0; j < CPT; ++j) {
        in[j] = c + CW * j >= c0 && c + CW * j < n;
        anyin = anyin || in[j];
      }
      if (anyin) {
        constexpr int NC = CPT == 1 ? 4 : 2;  // independent chains per column
        double pr[CPT][NC], pi[CPT][NC];
#pragma unroll
        for (int j = 0; j < CPT; ++j)
#pragma unroll
          for (int h = 0; h < NC; ++h) pr[j][h] = pi[j][h] = 0.0;
        if (rows) {
#pragma unroll
          for (int u0 = 0; u0 < RR; u0 += 8) {
            if (r0 + u0 + 8 <= c0 || r0 + u0 >= n) continue;  // v is zero there
            cpx<double> vv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) vv[u] = S.v[0][r0 + u0 + u];
#pragma unroll
            for (int j = 0; j < CPT; ++j)
#pragma unroll
              for (int u = 0; u < 8; ++u) dotacc(pr[j][u % NC], pi[j][u % NC], a[j][u0 + u], vv[u]);
          }
        }
#pragma unroll
        for (int j = 0; j < CPT; ++j)
          if (in[j]) {
            double sr = 0, si = 0;
#pragma unroll
            for (int h = 0; h < NC; ++h) {
              sr += pr[j][h];
              si += pi[j][h];
            }
            S.pp[0][q][c + CW * j] = mk(sr, si);
          }
      }
      __syncthreads();
      // (d) p, gamma = v^H p, w = tau p - |tau|^2 gamma / 2 v (wave 0)
      if (tid < 64) {
        const cpx<double> tau = S.tau[k];
        cpx<double> ph[NH], vh[NH];
        double g = 0;
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          const int i = lane + 64 * h;
          const bool in = i >= c0 && i < n;
          cpx<double> p = mk(0.0, 0.0), v = mk(0.0, 0.0);
          if (i < RN) {
#pragma unroll
            for (int qq = 0; qq < RQ; ++qq) p = p + S.pp[0][qq][i];
            v = S.v[0][i];
          }
          p = in ? p : mk(0.0, 0.0);
          g += v.re * p.re + v.im * p.im;
          ph[h] = p;
          vh[h] = v;
        }
        g = wave_allsum(g);
        const double cc = 0.5 * cabs2(tau) * g;
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          const int i = lane + 64 * h;
          if (i < RN) {
            S.wp[i] = tau * ph[h] - cc * vh[h];
            S.vp[i] = vh[h];
          }
        }
      }
      __syncthreads();
    }
    pend = act;
  }
#pragma unroll
  for (int j = 0; j < CPT; ++j)
    if (c + CW * j == n - 1) {
#pragma unroll
      for (int u = 0; u < RR; ++u) {
        if (r0 + u == n - 1) {
          cpx<double> x = a[j][u];
          if (pend) x = x - S.vp[n - 1] * cconj(S.wp[n - 1]) - S.wp[n - 1] * cconj(S.vp[n - 1]);
          S.d[n - 1] = x.re;
        }
      }
    }
  // reflectors to global memory for the back-transformation (column cj of
  // the register block holds v_cj below the diagonal)
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int cj = c + CW * j;
    if (cj + 1 < n) {
#pragma unroll
      for (int u = 0; u < RR; ++u) {
        const int r = r0 + u;
        if (r > cj && r < n) Vg[(long long)cj * n + r] = a[j][u];
      }
    }
  }
  __syncthreads();
  for (int i = tid; i + 1 < n; i += NTR) S.e2[i] = S.e[i] * S.e[i];
  const double tr = S.ev[RN];
  __syncthreads();
  const int kz = eig_tail<NTR>(dsc, n, tr, S, par);
  // ---- back-transformation z <- H_0 ... H_{n-2} z, z in registers ----
  // (its own layout: two vectors per thread at most; with more, each thread
  // would sum more partial products than the shared reads save)
  constexpr int CPTB = CPT < 2 ? CPT : 2, CWB = RN / CPTB, RQB = NTR / CWB, RRB = RN / RQB;
  static_assert(RQB <= RQ, "partial sums fit the tridiagonalisation's array");
  const int cb = tid % CWB, qb = tid / CWB, rb0 = qb * RRB;
  if (kz > 0) {
    cpx<double>* __restrict__ Z = reinterpret_cast<cpx<double>*>(dsc.evecs);
    cpx<double> z[CPTB][RRB];  // vectors cb + CWB j
#pragma unroll
    for (int j = 0; j < CPTB; ++j)
#pragma unroll
      for (int u = 0; u < RRB; ++u) {
        const int r = rb0 + u, cj = cb + CWB * j;
        z[j][u] = (cj < kz && r < n) ? Z[(long long)r * n + cj] : mk(0.0, 0.0);
      }
    // reflector k in S.v[k % 3] (zero outside rows k+1 .. n-1), partial sums
    // in S.pp[k & 1]: one barrier per reflector, since a slot is rewritten
    // only after every thread has passed the barrier that follows its last read
    // The entries of reflector k - 1 are read from global memory during step
    // k + 1, so the load has a whole step to arrive before they are stored.
    for (int i = tid; i < 3 * RN; i += NTR) S.v[i / RN][i % RN] = mk(0.0, 0.0);
    __syncthreads();
    if (n >= 2 && tid == n - 1) S.v[(n - 2) % 3][tid] = Vg[(long long)(n - 2) * n + tid];
    cpx<double> vq = mk(0.0, 0.0);  // reflector k - 1, row tid
    if (n >= 3 && tid >= n - 2 && tid < n) vq = Vg[(long long)(n - 3) * n + tid];
    __syncthreads();
    for (int k = n - 2; k >= 0; --k) {
      const cpx<double>* __restrict__ vk = S.v[k % 3];
      cpx<double> vq2 = mk(0.0, 0.0);  // reflector k - 2, row tid
      if (k >= 2 && tid >= k - 1 && tid < n) vq2 = Vg[(long long)(k - 2) * n + tid];
      const cpx<double> t = S.tau[k];
      const bool active = !(t.re == 0.0 && t.im == 0.0);
      const int r1 = k + 1;
      const bool rows = rb0 + RRB > r1 && rb0 < n;
      if (active && cb < kz) {
        constexpr int NC = CPTB == 1 ? 4 : 2;  // independent chains per vector
        double yr[CPTB][NC], yi[CPTB][NC];
#pragma unroll
        for (int j = 0; j < CPTB; ++j)
#pragma unroll
          for (int h = 0; h < NC; ++h) yr[j][h] = yi[j][h] = 0.0;
        if (rows) {
#pragma unroll
          for (int u = 0; u < RRB; ++u) {
            const cpx<double> vv = vk[rb0 + u];
#pragma unroll
            for (int j = 0; j < CPTB; ++j) dotacc(yr[j][u % NC], yi[j][u % NC], vv, z[j][u]);  // conj(v) z
          }
        }
#pragma unroll
        for (int j = 0; j < CPTB; ++j)
          if (cb + CWB * j < kz) {
            double sr = 0, si = 0;
#pragma unroll
            for (int h = 0; h < NC; ++h) {
              sr += yr[j][h];
              si += yi[j][h];
            }
            S.pp[k & 1][qb][cb + CWB * j] = mk(sr, si);
          }
      }
      if (k >= 1 && tid >= k && tid < n) S.v[(k - 1) % 3][tid] = vq;
      vq = vq2;
      __syncthreads();
      if (active && cb < kz && rows) {
        cpx<double> ty[CPTB];
#pragma unroll
        for (int j = 0; j < CPTB; ++j) {
          cpx<double> y = mk(0.0, 0.0);
          if (cb + CWB * j < kz) {
#pragma unroll
            for (int qq = 0; qq < RQB; ++qq) y = y + S.pp[k & 1][qq][cb + CWB * j];
          }
          ty[j] = t * y;
        }
#pragma unroll
        for (int u = 0; u < RRB; ++u) {
          const cpx<double> vv = vk[rb0 + u];
#pragma unroll
          for (int j = 0; j < CPTB; ++j) z[j][u] = subprod(z[j][u], vv, ty[j]);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < CPTB; ++j)
      if (cb + CWB * j < kz) {
#pragma unroll
        for (int u = 0; u < RRB; ++u) {
          const int r = rb0 + u;
          if (r < n) Z[(long long)r * n + cb + CWB * j] = z[j][u];
        }
      }
  }
  if (threadIdx.x == 0 && status) status[blockIdx.x] = 1;
}

// n in (nlo, 512], nlo >= 128: the matrix in global memory (L2-resident).
__global__ __launch_bounds__(NT) void k_heev_global(const EigDesc* __restrict__ descs, int* __restrict__ status,
                                                    int nlo) {
  __shared__ SharedG<512> S;
  const EigDesc& d = descs[blockIdx.x];
  if (!d.active || d.n <= nlo || d.n > 512) return;
  heev_core<true>(d, reinterpret_cast<cpx<double>*>(d.work), S);
  if (threadIdx.x == 0 && status) status[blockIdx.x] = 1;
}

// n in (128, 256]: the two-stage reduction through a band (heev_band).
__global__ __launch_bounds__(NT) void k_heev_band(const EigDesc* __restrict__ descs, int* __restrict__ status) {
  __shared__ SharedBand S;
  const EigDesc& d = descs[blockIdx.x];
  if (!d.active || d.n <= REG_NMAX || d.n > BS_NMAX) return;
  heev_band(d, reinterpret_cast<cpx<double>*>(d.work), S);
  if (threadIdx.x == 0 && status) status[blockIdx.x] = 1;
}

// n in (512, 1024]: as above with the larger workgroup state.
__global__ __launch_bounds__(NT) void k_heev_big(const EigDesc* __restrict__ descs, int* __restrict__ status) {
  __shared__ SharedG<EIG_NMAX> S;
  const EigDesc& d = descs[blockIdx.x];
  if (!d.active || d.n <= 512 || d.n > EIG_NMAX) return;
  heev_core<false>(d, reinterpret_cast<cpx<double>*>(d.work), S);
  if (threadIdx.x == 0 && status) status[blockIdx.x] = 1;
}

// ---------------------------------------------------------------------------
// Shared reduction for launches of few large matrices.  With one workgroup
// per matrix such a launch leaves most compute units idle, and every
// Householder step waits on one CU's memory latency.  Here G workgroups share
// a matrix during the reduction: workgroup g owns the columns of every G-th
// chunk of CO_CW columns (chunks j = g, g + G, ...), applies the pending
// rank-2 update to its columns of the trailing block and forms their entries
// of p = A v; every workgroup forms the same reflector and the same w from
// the column and the p of the previous step, read back from global memory.
// One kernel launch per step (the launch boundary is the only barrier
// between workgroups), as long as the trailing block is wider than
// CO_TAIL; one workgroup per matrix then finishes the last CO_TAIL steps
// (onecol_steps), the eigenvalues and the eigenvectors of T, and up to
// CO_BMAX workgroups per matrix back-transform the vectors, split by columns.
// Per matrix, after the n x n copy in the work array: v of the last two steps
// (2 n), their p (2 n), tau (n) complex; d and e (n each).
// ---------------------------------------------------------------------------
constexpr int CO_CW = 16;     // columns per ownership chunk
constexpr int CO_TAIL = 128;  // steps left to one workgroup (trailing block <= CO_TAIL)
constexpr int CO_NQ = 32;     // most row groups per column
constexpr int CO_UB = 16;     // rows loaded together per thread in a step

struct CoopBufs {
  cpx<double>* A;
  cpx<double>* x;  // after the matrix: V of even and odd steps, P of even and odd steps, tau
  double* d;
  double* e;
  int n;
  __device__ cpx<double>* V(int k) const { return x + (k & 1) * n; }
  __device__ cpx<double>* P(int k) const { return x + (2 + (k & 1)) * n; }
  __device__ cpx<double>* tau() const { return x + 4 * n; }
};

__device__ inline CoopBufs coop_bufs(const EigDesc& dsc) {
  const int n = dsc.n;
  CoopBufs b;
  b.n = n;
  b.A = reinterpret_cast<cpx<double>*>(dsc.work);
  b.x = b.A + (long long)n * n;
  b.d = reinterpret_cast<double*>(b.x + 5 * n);
  b.e = b.d + n;
  return b;
}

// the matrix takes part in a cooperative step k: a reduction step with a
// trailing block wider than CO_TAIL
__device__ inline bool coop_step_active(const EigDesc& dsc, int nlo, int k) {
  return dsc.active && dsc.n > nlo && dsc.n <= EIG_NMAX && dsc.n - k - 1 > CO_TAIL;
}

struct alignas(16) CoopS {
  alignas(16) cpx<double> v[EIG_NMAX];   // reflector of this step (index 0 = row k + 1)
  alignas(16) cpx<double> vp[EIG_NMAX];  // the previous step's v and w (index 0 = row k)
  alignas(16) cpx<double> wp[EIG_NMAX];
  alignas(16) cpx<double> xk[EIG_NMAX];  // column k, rows k .. n-1, with the previous update
  alignas(16) cpx<double> pp[NT];        // partial products (row group, column)
  double red[2 * NW];
};

// Symmetrised copy of the input into the work array, spread over the G
// workgroups of each matrix.
__global__ __launch_bounds__(NT) void k_coop_load(const EigDesc* __restrict__ descs, int G, int nlo) {
  const EigDesc& dsc = descs[blockIdx.x / G];
  const int g = blockIdx.x % G;
  if (!dsc.active || dsc.n <= nlo || dsc.n > EIG_NMAX) return;
  const int n = dsc.n;
  cpx<double>* __restrict__ A = reinterpret_cast<cpx<double>*>(dsc.work);
  const cpx<double>* a = reinterpret_cast<const cpx<double>*>(dsc.a);
  for (long long e = (long long)g * NT + threadIdx.x; e < (long long)n * n; e += (long long)G * NT) {
    const int i = (int)(e / n), j = (int)(e % n);
    if (dsc.upper) {
      const cpx<double> x = i <= j ? a[(long long)i * dsc.lda + j] : a[(long long)j * dsc.lda + i];
      A[e] = i < j ? x : i > j ? cconj(x) : mk(x.re, 0.0);
    } else {
      const cpx<double> x = a[(long long)i * dsc.lda + j], y = a[(long long)j * dsc.lda + i];
      A[e] = mk(0.5 * (x.re + y.re), 0.5 * (x.im - y.im));
    }
  }
}

// The previous step's w = tau p - (|tau|^2 / 2)(v^H p) v into S.wp, its v
// into S.vp (m1 entries from row k); returns false if that step had no
// reflector (tau = 0).
__device__ bool coop_prev_update(const CoopBufs& b, int k, int m1, CoopS& S, int& par) {
  const int tid = threadIdx.x;
  const cpx<double> tp = b.tau()[k - 1];
  if (tp.re == 0.0 && tp.im == 0.0) return false;
  const cpx<double>* vprev = b.V(k - 1);
  const cpx<double>* pprev = b.P(k - 1);
  double gsum = 0;
  for (int i = tid; i < m1; i += NT) {
    const cpx<double> v = vprev[i], p = pprev[i];
    S.vp[i] = v;
    S.wp[i] = p;
    gsum += v.re * p.re + v.im * p.im;
  }
  gsum = block_sum(gsum, S.red, par);
  const double cc = 0.5 * cabs2(tp) * gsum;
  for (int i = tid; i < m1; i += NT) S.wp[i] = tp * S.wp[i] - cc * S.vp[i];
  __syncthreads();
  return true;
}

// This workgroup's columns of the trailing block [c0, n)^2: the pending
// update (S.vp, S.wp; index 0 = row `base`) applied in place and, if `act`,
// p_c = sum_i conj(A[i][c]) v[i - c0] (= (A v)_c) written to P[c - c0].
__device__ void coop_pass(cpx<double>* __restrict__ A, int n, int c0, int base, bool pend, bool act, CoopS& S,
                          int g, int G, cpx<double>* __restrict__ P) {
  if (!pend && !act) return;
  const int m = n - c0;
  const int jc = c0 / CO_CW;                        // chunk holding column c0
  const int j0 = jc + ((g - jc % G) % G + G) % G;   // this workgroup's first chunk from there
  if (CO_CW * j0 >= n) return;                      // uniform over the workgroup
  const int nch = ((n - 1) / CO_CW - j0) / G + 1;   // its chunks j0, j0 + G, ... below n
  const int off = c0 > CO_CW * j0 ? c0 - CO_CW * j0 : 0;
  const int W = CO_CW * nch - off;                  // its columns from c0 on (some past n)
  int nq = NT / W;
  nq = nq < 1 ? 1 : (nq > CO_NQ ? CO_NQ : nq);
  const int rows_per = (m + nq - 1) / nq;
  const int tid = threadIdx.x;
  for (int t = tid; t < W * nq; t += NT) {
    const int cl = t % W, q = t / W;
    const int u = cl + off;
    const int c = CO_CW * (j0 + (u / CO_CW) * G) + u % CO_CW;
    double ar = 0, ai = 0;
    if (c < n) {
      const cpx<double> wpc = pend ? cconj(S.wp[c - base]) : mk(0.0, 0.0);
      const cpx<double> vpc = pend ? cconj(S.vp[c - base]) : mk(0.0, 0.0);
      const int i0 = c0 + q * rows_per, i1 = min(n, i0 + rows_per);
      int i = i0;
      for (; i + CO_UB <= i1; i += CO_UB) {  // a thread's rows in as few load batches as fit
        cpx<double> a[CO_UB];
#pragma unroll
        for (int x = 0; x < CO_UB; ++x) a[x] = A[(long long)(i + x) * n + c];
        if (pend) {
#pragma unroll
          for (int x = 0; x < CO_UB; ++x) {
            a[x] = sub2prod(a[x], S.vp[i + x - base], wpc, S.wp[i + x - base], vpc);
            A[(long long)(i + x) * n + c] = a[x];
          }
        }
        if (act) {
#pragma unroll
          for (int x = 0; x < CO_UB; ++x) dotacc(ar, ai, a[x], S.v[i + x - c0]);
        }
      }
      for (; i + UB <= i1; i += UB) {
        cpx<double> a[UB];
#pragma unroll
        for (int x = 0; x < UB; ++x) a[x] = A[(long long)(i + x) * n + c];
        if (pend) {
#pragma unroll
          for (int x = 0; x < UB; ++x) {
            a[x] = sub2prod(a[x], S.vp[i + x - base], wpc, S.wp[i + x - base], vpc);
            A[(long long)(i + x) * n + c] = a[x];
          }
        }
        if (act) {
#pragma unroll
          for (int x = 0; x < UB; ++x) dotacc(ar, ai, a[x], S.v[i + x - c0]);
        }
      }
      for (; i < i1; ++i) {
        cpx<double> a = A[(long long)i * n + c];
        if (pend) {
          a = sub2prod(a, S.vp[i - base], wpc, S.wp[i - base], vpc);
          A[(long long)i * n + c] = a;
        }
        if (act) dotacc(ar, ai, a, S.v[i - c0]);
      }
      if (act && nq == 1) P[c - c0] = mk(ar, ai);
    }
    if (nq > 1) S.pp[q * W + cl] = mk(ar, ai);  // nq > 1: W nq <= NT
  }
  if (act && nq > 1) {
    __syncthreads();
    for (int cl = tid; cl < W; cl += NT) {
      const int u = cl + off;
      const int c = CO_CW * (j0 + (u / CO_CW) * G) + u % CO_CW;
      if (c >= n) continue;
      cpx<double> x = S.pp[cl];
      for (int q = 1; q < nq; ++q) x = x + S.pp[q * W + cl];
      P[c - c0] = x;
    }
  }
}

// Step k of the shared reduction for every matrix whose trailing block after
// this step is still wider than CO_TAIL.
__global__ __launch_bounds__(NT) void k_coop_step(const EigDesc* __restrict__ descs, int G, int nlo, int k) {
  __shared__ CoopS S;
  const EigDesc& dsc = descs[blockIdx.x / G];
  const int g = blockIdx.x % G;
  if (!coop_step_active(dsc, nlo, k)) return;
  const int n = dsc.n, tid = threadIdx.x;
  int par = 0;
  const CoopBufs b = coop_bufs(dsc);
  cpx<double>* __restrict__ A = b.A;
  const int m = n - k - 1, c0 = k + 1;
  // 1. the update of step k - 1 (v from row k, w); its reflector goes to
  // column k - 1 for the back-transformation (no workgroup reads that column
  // in this step)
  const bool pend = k > 0 && coop_prev_update(b, k, m + 1, S, par);
  if (pend && g == 0)
    for (int i = tid; i <= m; i += NT) A[(long long)(k + i) * n + (k - 1)] = S.vp[i];
  // 2. column k with that update, and this step's reflector (every workgroup
  // alike; workgroup 0 records d, e, tau and v)
  for (int i = tid; i <= m; i += NT) {
    cpx<double> x = A[(long long)(k + i) * n + k];
    if (pend) x = sub2prod(x, S.vp[i], cconj(S.wp[0]), S.wp[i], cconj(S.vp[0]));
    S.xk[i] = x;
  }
  __syncthreads();
  double xn = 0;
  for (int i = 2 + tid; i <= m; i += NT) xn += cabs2(S.xk[i]);
  xn = block_sum(xn, S.red, par);
  const cpx<double> alpha = S.xk[1];
  const bool act = !(xn == 0.0 && alpha.im == 0.0);
  cpx<double> tau = mk(0.0, 0.0), sc = mk(0.0, 0.0);
  double ek = alpha.re;
  if (act) {
    const double nrm = sqrt(cabs2(alpha) + xn);
    const double beta = alpha.re >= 0 ? -nrm : nrm;
    tau = mk((beta - alpha.re) / beta, -alpha.im / beta);
    const cpx<double> den = mk(alpha.re - beta, alpha.im);  // sc = 1 / (alpha - beta)
    const double dd = cabs2(den);
    sc = mk(den.re / dd, -den.im / dd);
    ek = beta;
  }
  if (g == 0 && tid == 0) {
    b.d[k] = S.xk[0].re;
    b.e[k] = ek;
    b.tau()[k] = tau;
  }
  if (act) {
    cpx<double>* __restrict__ vout = b.V(k);
    for (int i = tid; i < m; i += NT) {
      const cpx<double> v = (i == 0) ? mk(1.0, 0.0) : S.xk[1 + i] * sc;
      S.v[i] = v;
      if (g == 0) vout[i] = v;
    }
  }
  __syncthreads();
  // 3. this workgroup's columns of the trailing block
  coop_pass(A, n, c0, k, pend, act, S, g, G, b.P(k));
}

// One workgroup per matrix: the steps from the first one with a trailing
// block of at most CO_TAIL (onecol_steps), then the tridiagonal eigenpairs
// and the back-transformation, as in heev_core.  Matrices with n in
// (nmin, NMAX].
template <int NMAX>
__global__ __launch_bounds__(NT) void k_coop_tail(const EigDesc* __restrict__ descs, int* __restrict__ status,
                                                  int nlo, int nmin) {
  __shared__ SharedG<NMAX> S;
  const EigDesc& dsc = descs[blockIdx.x];
  const int n = dsc.n;
  if (!dsc.active || n <= nlo || n <= nmin || n > NMAX) return;
  const int tid = threadIdx.x;
  int par = 0;
  const CoopBufs b = coop_bufs(dsc);
  cpx<double>* __restrict__ A = b.A;
  const int ks = n - 1 > CO_TAIL ? n - 1 - CO_TAIL : 0;  // first step left to this workgroup
  for (int i = tid; i < ks; i += NT) {
    S.d[i] = b.d[i];
    S.e[i] = b.e[i];
    S.tau[i] = b.tau()[i];
  }
  // the pending update of step ks - 1 (as coop_prev_update, into S.vp, S.wp)
  bool pend = false;
  if (ks > 0) {
    const cpx<double> tp = b.tau()[ks - 1];
    pend = !(tp.re == 0.0 && tp.im == 0.0);
    if (pend) {
      const int m1 = n - ks;
      const cpx<double>* vprev = b.V(ks - 1);
      const cpx<double>* pprev = b.P(ks - 1);
      double gsum = 0;
      for (int i = tid; i < m1; i += NT) {
        const cpx<double> v = vprev[i], p = pprev[i];
        S.vp[i] = v;
        S.wp[i] = p;
        gsum += v.re * p.re + v.im * p.im;
      }
      gsum = block_sum(gsum, S.red, par);
      const double cc = 0.5 * cabs2(tp) * gsum;
      for (int i = tid; i < m1; i += NT) {
        S.wp[i] = tp * S.wp[i] - cc * S.vp[i];
        A[(long long)(ks + i) * n + (ks - 1)] = S.vp[i];  // reflector ks - 1, for the back-transformation
      }
    }
  }
  double tr = 0;  // trace of the input (its diagonal is real after symmetrisation)
  const cpx<double>* a = reinterpret_cast<const cpx<double>*>(dsc.a);
  for (int i = tid; i < n; i += NT) tr += a[(long long)i * dsc.lda + i].re;
  tr = block_sum(tr, S.red, par);
  __syncthreads();
  onecol_steps(A, n, ks, pend, S, par);
  if (tid == 0) S.d[n - 1] = A[(long long)(n - 1) * n + n - 1].re;
  for (int i = tid; i + 1 < n; i += NT) S.e2[i] = S.e[i] * S.e[i];
  __syncthreads();
  const int kz = eig_tail<NT>(dsc, n, tr, S, par);
  // hand-over to k_coop_back (also for few vectors: split by columns it
  // beats this workgroup's register back-transformation, 3.0 -> 2.8 ms at
  // n = 256 with 64 vectors): tau on the diagonal of A (no longer read), the
  // vector count in its last entry
  for (int i = tid; i + 1 < n; i += NT) A[(long long)i * n + i] = S.tau[i];
  if (tid == 0) A[(long long)(n - 1) * n + n - 1] = mk((double)kz, 0.0);
  if (tid == 0 && status) status[blockIdx.x] = 1;
}

template <int NMAX> struct alignas(16) CoopBackS {
  alignas(16) cpx<double> tau[NMAX];
  alignas(16) cpx<double> v[BTB * BTB];    // G of a reflector block
  alignas(16) cpx<double> vp[BTB * BTB];   // its T
  alignas(16) cpx<double> pf[BTB * NMAX];  // the reflector block (145 KB of LDS in all at NMAX = 1024)
};

// One of Gb workgroups per matrix: the back-transformation z <- H_0 ... H_{n-2} z
// of its share of the eigenvector columns (each column is independent), for
// the matrices whose vectors k_coop_tail left (n in (nmin, NMAX]).  Each
// workgroup's scratch (reflector block, partial sums) lies after the matrix.
template <int NMAX>
__global__ __launch_bounds__(NT) void k_coop_back(const EigDesc* __restrict__ descs, int Gb, int nlo, int nmin) {
  __shared__ CoopBackS<NMAX> S;
  const EigDesc& dsc = descs[blockIdx.x / Gb];
  const int g = blockIdx.x % Gb, n = dsc.n, tid = threadIdx.x;
  if (!dsc.active || n <= nlo || n <= nmin || n > NMAX) return;
  cpx<double>* __restrict__ A = reinterpret_cast<cpx<double>*>(dsc.work);
  const int kz = (int)A[(long long)(n - 1) * n + n - 1].re;
  if (kz <= 0) return;
  // scratch per workgroup (complex): reflector block n BTB, partial sums
  // BTB max(NT, columns), the block product BTB columns; as many workgroups
  // as the work array holds
  const long long np = (n + 63) / 64 * 64;
  const long long per = (long long)BTB * n + (long long)BTB * (NT > kz ? NT : kz) + (long long)BTB * kz;
  const long long room = (7LL * n * np) / 2;  // complex entries after the matrix
  int gb = (int)(room / per);
  gb = gb < Gb ? gb : Gb;
  gb = gb < kz ? gb : kz;
  if (g >= gb) return;
  const int cw = (kz + gb - 1) / gb, c0 = g * cw, c1 = min(kz, c0 + cw);
  if (c0 >= c1) return;
  for (int i = tid; i + 1 < n; i += NT) S.tau[i] = A[(long long)i * n + i];
  __syncthreads();
  cpx<double>* scratch = A + (long long)n * n + (long long)g * per;
  back_transform(dsc, A, n, c1 - c0, S, c0, scratch);
}

namespace {
// n in (128, 256] through the band path.  Off by default: every stage of it
// is a long chain of small dependent steps (about 2,200 chase steps and as
// many reflector applications per n = 256 matrix, each ~1 us), which costs
// more than the one-stage kernel's extra memory traffic on this hardware.
bool g_band = false;
// the shared reduction for launches of at most CO_MAX_ITEMS matrices
bool g_coop = true;
constexpr int CO_MAX_ITEMS = 32;
constexpr int CO_GRID = 256;  // workgroups per step launch (one per CU: 134 VGPRs, 72 KB of LDS)
constexpr int CO_GMAX = 64;   // workgroups per matrix in the reduction
constexpr int CO_BMAX = 16;   // workgroups per matrix in the back-transformation
}  // namespace
void set_eig_band(bool on) { g_band = on; }
bool eig_band() { return g_band; }
void set_eig_coop(bool on) { g_coop = on; }
bool eig_coop() { return g_coop; }

hipError_t set_eig_residual_bound(double rtol) {
  return hipMemcpyToSymbol(HIP_SYMBOL(g_eig_rtol), &rtol, sizeof(double));
}

void launch_eigh(const EigDesc* d_descs, int nitems, int maxn, int* d_status, hipStream_t s) {
  if (nitems <= 0) return;
  // the register variants (n <= 32 and n <= 128) count as one profiled call
  int tok = prof_begin(PC_EIG_REG, s);
  hipLaunchKernelGGL((k_heev_reg<SMALL_NMAX, 64, 0, 1>), dim3(nitems), dim3(64), 0, s, d_descs, d_status);
  if (maxn > SMALL_NMAX)
    hipLaunchKernelGGL((k_heev_reg<REG_NMAX, 512, SMALL_NMAX, 4>), dim3(nitems), dim3(512), 0, s, d_descs, d_status);
  prof_end_eig(tok, PC_EIG_REG, d_descs, nitems, 1, REG_NMAX, s);
  const int nlo = g_band ? BS_NMAX : REG_NMAX;  // largest n left to the band path
  if (maxn > REG_NMAX && g_band) {
    tok = prof_begin(PC_EIG_BAND, s);
    hipLaunchKernelGGL(k_heev_band, dim3(nitems), dim3(NT), 0, s, d_descs, d_status);
    prof_end_eig(tok, PC_EIG_BAND, d_descs, nitems, REG_NMAX + 1, BS_NMAX, s);
  }
  if (maxn > nlo && g_coop && nitems <= CO_MAX_ITEMS) {
    // few matrices: G workgroups share each one during the reduction
    const int chunks = (maxn + CO_CW - 1) / CO_CW;
    int G = CO_GRID / nitems;
    G = std::min(G, std::min(chunks, CO_GMAX));
    G = std::max(G, 1);
    tok = prof_begin(PC_EIG_GLOBAL, s);
    hipLaunchKernelGGL(k_coop_load, dim3(nitems * G), dim3(NT), 0, s, d_descs, G, nlo);
    for (int k = 0; maxn - k - 1 > CO_TAIL; ++k)
      hipLaunchKernelGGL(k_coop_step, dim3(nitems * G), dim3(NT), 0, s, d_descs, G, nlo, k);
    hipLaunchKernelGGL(k_coop_tail<512>, dim3(nitems), dim3(NT), 0, s, d_descs, d_status, nlo, 0);
    if (maxn > 512)
      hipLaunchKernelGGL(k_coop_tail<EIG_NMAX>, dim3(nitems), dim3(NT), 0, s, d_descs, d_status, nlo, 512);
    const int Gb = std::max(1, std::min(CO_BMAX, CO_GRID / nitems));
    hipLaunchKernelGGL(k_coop_back<512>, dim3(nitems * Gb), dim3(NT), 0, s, d_descs, Gb, nlo, 0);
    if (maxn > 512)
      hipLaunchKernelGGL(k_coop_back<EIG_NMAX>, dim3(nitems * Gb), dim3(NT), 0, s, d_descs, Gb, nlo, 512);
    prof_end_eig(tok, PC_EIG_GLOBAL, d_descs, nitems, nlo + 1, EIG_NMAX, s);
    return;
  }
  if (maxn > nlo) {
    tok = prof_begin(PC_EIG_GLOBAL, s);
    hipLaunchKernelGGL(k_heev_global, dim3(nitems), dim3(NT), 0, s, d_descs, d_status, nlo);
    prof_end_eig(tok, PC_EIG_GLOBAL, d_descs, nitems, nlo + 1, 512, s);
  }
  if (maxn > 512) {
    tok = prof_begin(PC_EIG_GLOBAL, s);
    hipLaunchKernelGGL(k_heev_big, dim3(nitems), dim3(NT), 0, s, d_descs, d_status);
    prof_end_eig(tok, PC_EIG_GLOBAL, d_descs, nitems, 513, EIG_NMAX, s);
  }
}

}  // namespace mpdo
