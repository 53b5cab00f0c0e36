// rho as a matrix product operator of local density tensors and the
// error-mitigation maps applied to it (the MPO inverse of a noisy process,
// Sec. V).  Site tensors R_i[(l l'), (p p'), (r r')] = sum_n T_i[l, p, n, r]
// conj(T_i[l', p', n, r']) (Eq. (6)) are built from an MPDO; a q-site
// superoperator S (4^q x 4^q on the pair indices (p_1 p_1' ... p_q p_q')) is
// applied in place for q = 1, and for q = 2 on the contracted pair, which is
// split again by an SVD (Gram matrix and the library's eigensolver) with the
// discarded-weight rule; Tr(O rho) is a chain of vector-matrix products.
// FP64 throughout; one state at a time (a verification and mitigation tool,
// not the batched hot path).
#include <cmath>
#include <algorithm>
#include <cstring>
#include <utility>

#include "common.h"
#include "engine.h"
#include "kernels.h"
#include "mpo.h"

namespace mpdo {

namespace {
constexpr int MT = 256;

template <typename T>
__global__ void k_mpo_from_site(const cpx<T>* __restrict__ B, int l, int k, int r, cpx<double>* __restrict__ R) {
  const long long L2 = (long long)l * l, R2 = (long long)r * r, total = L2 * 4 * R2;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long rr = e % R2, x = (e / R2) % 4, ll = e / (R2 * 4);
    const int a = (int)(ll / l), a2 = (int)(ll % l), b = (int)(rr / r), b2 = (int)(rr % r);
    const int p = (int)(x >> 1), p2 = (int)(x & 1);
    double re = 0, im = 0;
    for (int n = 0; n < k; ++n) {
      const cpx<T> u = B[(((long long)a * 2 + p) * k + n) * r + b];
      const cpx<T> v = B[(((long long)a2 * 2 + p2) * k + n) * r + b2];
      re += (double)u.re * (double)v.re + (double)u.im * (double)v.im;   // u conj(v)
      im += (double)u.im * (double)v.re - (double)u.re * (double)v.im;
    }
    R[e] = mk(re, im);
  }
}

// S = sum_j K_j (x) conj(K_j) in pair order (K_j^dagger instead when adj),
// d = 2^q, S of size 4^q; one thread per entry.
__global__ void k_mpo_superop(const double* __restrict__ K, int m, int q, int adj, cpx<double>* __restrict__ S) {
  const int d = 1 << q, D = d * d;
  for (int e = threadIdx.x; e < D * D; e += blockDim.x) {
    const int row = e / D, col = e % D;
    // pair-ordered indices (p_1 p_1' ... ) -> (p, p') with p = (p_1 .. p_q)
    int p = 0, pp = 0, t = 0, tp = 0;
    for (int s = 0; s < q; ++s) {
      const int rb = (row >> (2 * (q - 1 - s))) & 3, cb = (col >> (2 * (q - 1 - s))) & 3;
      p = 2 * p + (rb >> 1);
      pp = 2 * pp + (rb & 1);
      t = 2 * t + (cb >> 1);
      tp = 2 * tp + (cb & 1);
    }
    double re = 0, im = 0;
    for (int j = 0; j < m; ++j) {
      const double* Kj = K + 2LL * j * d * d;
      // element (x, y) of K or K^dagger
      const int i1 = adj ? t * d + p : p * d + t, i2 = adj ? tp * d + pp : pp * d + tp;
      double ar = Kj[2 * i1], ai = Kj[2 * i1 + 1], br = Kj[2 * i2], bi = Kj[2 * i2 + 1];
      if (adj) {
        ai = -ai;
        bi = -bi;
      }
      re += ar * br + ai * bi;  // a conj(b)
      im += ai * br - ar * bi;
    }
    S[e] = mk(re, im);
  }
}

// In-place inverse of an n x n complex matrix (n <= 16), Gauss-Jordan with
// partial pivoting, one block.  *ok = 0 when a pivot falls below 1e-13 of
// the largest entry of the matrix (numerically singular).
__global__ void k_mpo_invert(cpx<double>* __restrict__ S, int n, int* __restrict__ ok) {
  __shared__ cpx<double> a[16][32];
  __shared__ cpx<double> f[16];
  __shared__ int piv;
  __shared__ double amax;
  const int tid = threadIdx.x;
  for (int e = tid; e < n * 2 * n; e += blockDim.x) {
    const int i = e / (2 * n), j = e % (2 * n);
    a[i][j] = j < n ? S[i * n + j] : mk(j - n == i ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  if (tid == 0) {
    double m = 0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) m = fmax(m, cabs2(a[i][j]));
    amax = m;
  }
  __syncthreads();
  bool good = amax > 0;
  for (int c = 0; c < n; ++c) {
    if (tid == 0) {
      int best = c;
      for (int i = c + 1; i < n; ++i)
        if (cabs2(a[i][c]) > cabs2(a[best][c])) best = i;
      piv = best;
    }
    __syncthreads();
    const int pr = piv;
    if (pr != c)
      for (int j = tid; j < 2 * n; j += blockDim.x) {
        const cpx<double> x = a[c][j];
        a[c][j] = a[pr][j];
        a[pr][j] = x;
      }
    __syncthreads();
    const cpx<double> d = a[c][c];
    const double dd = cabs2(d);
    if (!(dd > 1e-26 * amax)) good = false;
    const cpx<double> inv = dd > 0 ? mk(d.re / dd, -d.im / dd) : mk(0.0, 0.0);
    __syncthreads();
    for (int j = tid; j < 2 * n; j += blockDim.x) a[c][j] = inv * a[c][j];
    for (int i = tid; i < n; i += blockDim.x) f[i] = a[i][c];  // column c before the elimination
    __syncthreads();
    for (int e = tid; e < n * 2 * n; e += blockDim.x) {
      const int i = e / (2 * n), j = e % (2 * n);
      if (i != c) a[i][j] = a[i][j] - f[i] * a[c][j];
    }
    __syncthreads();
  }
  for (int e = tid; e < n * n; e += blockDim.x) S[e] = a[e / n][n + e % n];
  if (tid == 0) *ok = good ? 1 : 0;
}

// out[a, z, c] = sum_w S[z, w] in[a, w, c], w and z < d.
__global__ void k_mpo_op(const cpx<double>* __restrict__ S, int d, const cpx<double>* __restrict__ in,
                         cpx<double>* __restrict__ out, long long A, long long C) {
  const long long total = A * d * C;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long c = e % C, z = (e / C) % d, a = e / (C * d);
    cpx<double> acc = mk(0.0, 0.0);
    for (int w = 0; w < d; ++w) acc = acc + S[z * d + w] * in[(a * d + w) * C + c];
    out[e] = acc;
  }
}

// out[i * r + j] = U[i * n + j] for j < r (the leading r eigenvectors);
// with adj, out[j * n + i] = sqrt(w[j]) conj(U[i * n + j]) (their adjoint,
// r x n, rows scaled by the singular values).
__global__ void k_mpo_take_cols(const cpx<double>* __restrict__ U, int n, int r, int adj,
                                const double* __restrict__ w, cpx<double>* __restrict__ out) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)n * r;
       e += (long long)gridDim.x * blockDim.x) {
    const long long i = e / r, j = e % r;
    if (adj) out[j * n + i] = sqrt(w[j]) * cconj(U[i * n + j]);
    else out[e] = U[i * n + j];
  }
}

// X[i, j] /= sqrt(w[j]) for an m x r matrix (w[j] > 0 for j < r).
__global__ void k_mpo_unscale_cols(cpx<double>* __restrict__ X, long long m, int r, const double* __restrict__ w) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < m * r;
       e += (long long)gridDim.x * blockDim.x)
    X[e] = (1.0 / sqrt(w[e % r])) * X[e];
}

// v'[b] = sum_a v[a] sum_x R[a, x, b] o[x]; one block.
__global__ void k_mpo_chain(const cpx<double>* __restrict__ R, int A, int Bd, const double* __restrict__ o,
                            const cpx<double>* __restrict__ v, cpx<double>* __restrict__ w) {
  cpx<double> oo[4];
  for (int x = 0; x < 4; ++x) oo[x] = mk(o[2 * x], o[2 * x + 1]);
  for (int b = threadIdx.x; b < Bd; b += blockDim.x) {
    cpx<double> acc = mk(0.0, 0.0);
    for (int a = 0; a < A; ++a) {
      cpx<double> t = mk(0.0, 0.0);
      for (int x = 0; x < 4; ++x) t = t + R[((long long)a * 4 + x) * Bd + b] * oo[x];
      acc = acc + v[a] * t;
    }
    w[b] = acc;
  }
}

__global__ void k_mpo_one(cpx<double>* v) { v[0] = mk(1.0, 0.0); }

// rho[(p_1 .. p_n), (p_1' .. p_n')] from the pair-ordered vector
// t[(p_1 p_1' .. p_n p_n')].
__global__ void k_mpo_unpair(const cpx<double>* __restrict__ t, int n, cpx<double>* __restrict__ rho) {
  const long long dim = 1LL << n, total = dim * dim;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long row = e / dim, col = e % dim;
    long long idx = 0;
    for (int s = n - 1; s >= 0; --s) idx = idx * 4 + 2 * ((row >> s) & 1) + ((col >> s) & 1);
    rho[e] = t[idx];
  }
}

void swap_bufs(DevBuf& x, DevBuf& y) {
  std::swap(x.p, y.p);
  std::swap(x.bytes, y.bytes);
  std::swap(x.from, y.from);
  std::swap(x.device, y.device);
}

int grid_for(long long n) { return (int)std::min<long long>(std::max<long long>((n + MT - 1) / MT, 1), 4096); }
}  // namespace

MpoState::MpoState(int n_, int dmax_, double cutoff_, hipStream_t s)
    : n(n_), dmax(dmax_), cutoff(cutoff_), st(s), D(n_ + 1, 1) {
  R.resize(n);
  for (auto& p : R) p.reset(new DevBuf());
}

template <typename T> void MpoState::load_site(int i, const cpx<T>* B, int l, int k, int r) {
  D[i] = l * l;
  D[i + 1] = r * r;
  const long long total = (long long)l * l * 4 * r * r;
  R[i]->alloc(sizeof(cpx<double>) * total);
  hipLaunchKernelGGL(k_mpo_from_site<T>, dim3(grid_for(total)), dim3(MT), 0, st, B, l, k, r, R[i]->as<cpx<double>>());
  hip_check(hipGetLastError(), "launch (mpo from site)");
}
template void MpoState::load_site<double>(int, const cpx<double>*, int, int, int);
template void MpoState::load_site<float>(int, const cpx<float>*, int, int, int);

void MpoState::superop(const double* K, int m, int q, bool adj, bool inverse) {
  const int D4 = 1 << (2 * q);
  sop.alloc(sizeof(cpx<double>) * D4 * D4);
  hipLaunchKernelGGL(k_mpo_superop, dim3(1), dim3(256), 0, st, K, m, q, adj ? 1 : 0, sop.as<cpx<double>>());
  hip_check(hipGetLastError(), "launch (superoperator)");
  if (inverse) {
    okf.alloc(sizeof(int));
    hipLaunchKernelGGL(k_mpo_invert, dim3(1), dim3(256), 0, st, sop.as<cpx<double>>(), D4, okf.as<int>());
    hip_check(hipGetLastError(), "launch (inverse superoperator)");
    int ok = 0;
    hip_check(hipMemcpyAsync(&ok, okf.p, sizeof(int), hipMemcpyDeviceToHost, st), "inverse superoperator");
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    if (!ok) throw Error{5 /*MPDO_ENOTCONV*/, "the channel's superoperator is singular: it has no inverse"};
  }
}

void MpoState::gate_superop(const double* U, int q, bool adj) {
  const size_t bytes = sizeof(double) * (2u << (2 * q));
  ubuf.alloc(bytes);
  hip_check(hipMemcpyAsync(ubuf.p, U, bytes, hipMemcpyHostToDevice, st), "gate upload");
  superop(ubuf.as<double>(), 1, q, adj, false);
}

void MpoState::apply(int site, int q) {
  const cpx<double>* S = sop.as<cpx<double>>();
  if (q == 1) {
    const long long a = D[site], c = D[site + 1];
    tA.alloc(sizeof(cpx<double>) * a * 4 * c);
    hipLaunchKernelGGL(k_mpo_op, dim3(grid_for(a * 4 * c)), dim3(MT), 0, st, S, 4, R[site]->as<cpx<double>>(),
                       tA.as<cpx<double>>(), a, c);
    hip_check(hipGetLastError(), "launch (mpo one-site map)");
    swap_bufs(*R[site], tA);
    return;
  }
  const int a = D[site], b = D[site + 1], c = D[site + 2];
  const int rows = 4 * a, cols = 4 * c;
  const int nn = rows <= EIG_NMAX ? rows : cols;
  if (nn > EIG_NMAX) throw Error{6 /*MPDO_EUNSUPPORTED*/, "MPO split: both outer bonds exceed 256"};
  // theta[(a x), (y c)] = R_i R_{i+1}, then S on (x y)
  tA.alloc(sizeof(cpx<double>) * (size_t)rows * cols);
  tB.alloc(sizeof(cpx<double>) * (size_t)rows * cols);
  gemm_once(desc, R[site]->as<cpx<double>>(), R[site + 1]->as<cpx<double>>(), tA.as<cpx<double>>(), rows, cols, b,
            OP_N, OP_N, b, cols, cols, st, false);
  hipLaunchKernelGGL(k_mpo_op, dim3(grid_for((long long)rows * cols)), dim3(MT), 0, st, S, 16,
                     tA.as<cpx<double>>(), tB.as<cpx<double>>(), (long long)a, (long long)c);
  hip_check(hipGetLastError(), "launch (mpo two-site map)");
  // SVD of theta through the Gram matrix of its smaller side
  const bool left = rows <= EIG_NMAX;  // the right Gram only when the left one is too large
  const cpx<double>* th = tB.as<cpx<double>>();
  tG.alloc(sizeof(cpx<double>) * (size_t)nn * nn);
  if (left) gemm_once(desc, th, th, tG.as<cpx<double>>(), nn, nn, cols, OP_N, OP_H, cols, cols, nn, st, true);
  else gemm_once(desc, th, th, tG.as<cpx<double>>(), nn, nn, rows, OP_H, OP_N, cols, cols, nn, st, true);
  const int kvec = std::min({rows, cols, dmax});  // rank of theta <= min(rows, cols)
  ev.alloc(sizeof(double) * (nn + 1));
  vec.alloc(sizeof(cpx<double>) * (size_t)nn * nn);
  work.alloc(sizeof(double) * eig_work_doubles(nn));
  status.alloc(sizeof(int));
  EigDesc e;
  std::memset(&e, 0, sizeof(e));
  e.a = tG.as<double>(); e.lda = nn; e.n = nn; e.evals = ev.as<double>(); e.evecs = vec.as<double>();
  e.work = work.as<double>(); e.trace = ev.as<double>() + nn; e.kvec = kvec; e.active = 1; e.upper = 1;
  e.vfloor = 1e-300;  // every vector of a positive eigenvalue (rho is linear in R: no floor)
  edesc.alloc(sizeof(EigDesc));
  hip_check(hipMemcpyAsync(edesc.p, &e, sizeof(e), hipMemcpyHostToDevice, st), "descriptor");
  launch_eigh(edesc.as<EigDesc>(), 1, nn, status.as<int>(), st);
  std::vector<double> w(nn + 1);
  hip_check(hipMemcpyAsync(w.data(), ev.p, sizeof(double) * (nn + 1), hipMemcpyDeviceToHost, st), "eigenvalues");
  hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
  const double W = w[nn];
  if (!(W > 0 && W < 1e300))
    throw Error{5 /*MPDO_ENOTCONV*/, "MPO split: non-finite or zero weight, or an eigenpair above its residual bound"};
  // smallest r whose dropped weight is <= cutoff * W, at most kvec; only
  // eigenvectors of positive eigenvalues
  int r = kvec, pos = 0;
  double head = 0;
  for (int cand = 1; cand <= kvec; ++cand) {
    head += std::max(w[cand - 1], 0.0);
    if (W - head <= cutoff * W) {
      r = cand;
      break;
    }
  }
  while (pos < kvec && w[pos] > 0) ++pos;
  r = std::max(1, std::min(r, pos));
  double kept = 0;
  for (int i = 0; i < r; ++i) kept += std::max(w[i], 0.0);
  discarded += std::max(W - kept, 0.0) / W;
  cpx<double>* V = vec.as<cpx<double>>();
  R[site]->alloc(sizeof(cpx<double>) * (size_t)rows * r);
  R[site + 1]->alloc(sizeof(cpx<double>) * (size_t)r * cols);
  // both forms leave R_i = U_r (left-orthonormal) and R_{i+1} = diag(s) V_r^H,
  // so that later splits see the same gauge whichever side was factored
  if (left) {
    hipLaunchKernelGGL(k_mpo_take_cols, dim3(grid_for((long long)rows * r)), dim3(MT), 0, st, V, nn, r, 0,
                       ev.as<double>(), R[site]->as<cpx<double>>());
    gemm_once(desc, V, th, R[site + 1]->as<cpx<double>>(), r, cols, rows, OP_H, OP_N, nn, cols, cols, st, false);
  } else {
    // R_{i+1} = diag(s) V_r^H, R_i = theta V_r diag(1/s)
    hipLaunchKernelGGL(k_mpo_take_cols, dim3(grid_for((long long)cols * r)), dim3(MT), 0, st, V, nn, r, 1,
                       ev.as<double>(), R[site + 1]->as<cpx<double>>());
    gemm_once(desc, th, V, R[site]->as<cpx<double>>(), rows, r, cols, OP_N, OP_N, cols, nn, r, st, false);
    hipLaunchKernelGGL(k_mpo_unscale_cols, dim3(grid_for((long long)rows * r)), dim3(MT), 0, st,
                       R[site]->as<cpx<double>>(), (long long)rows, r, ev.as<double>());
  }
  hip_check(hipGetLastError(), "launch (mpo split)");
  D[site + 1] = r;
}

void MpoState::expect(const double* ops, int nops, double* out) {
  int dmx = 1;
  for (int x : D) dmx = std::max(dmx, x);
  tA.alloc(sizeof(cpx<double>) * (size_t)dmx);
  tB.alloc(sizeof(cpx<double>) * (size_t)dmx);
  res.alloc(sizeof(cpx<double>) * (size_t)std::max(nops, 1));
  // factor of site i: O_i^T at (p p'), i.e. O[p', p]
  std::vector<double> o(8 * (size_t)n * nops);
  const int tr[4] = {0, 2, 1, 3};
  for (size_t f = 0; f < (size_t)n * nops; ++f)
    for (int x = 0; x < 4; ++x) {
      o[8 * f + 2 * x] = ops[8 * f + 2 * tr[x]];
      o[8 * f + 2 * x + 1] = ops[8 * f + 2 * tr[x] + 1];
    }
  obuf.alloc(sizeof(double) * std::max<size_t>(o.size(), 1));
  hip_check(hipMemcpyAsync(obuf.p, o.data(), o.size() * sizeof(double), hipMemcpyHostToDevice, st), "operators");
  for (int k = 0; k < nops; ++k) {
    cpx<double>* v = tA.as<cpx<double>>();
    cpx<double>* w = tB.as<cpx<double>>();
    hipLaunchKernelGGL(k_mpo_one, dim3(1), dim3(1), 0, st, v);
    for (int i = 0; i < n; ++i) {
      hipLaunchKernelGGL(k_mpo_chain, dim3(1), dim3(256), 0, st, R[i]->as<cpx<double>>(), D[i], D[i + 1],
                         obuf.as<double>() + 8 * ((size_t)k * n + i), v, w);
      std::swap(v, w);
    }
    hip_check(hipMemcpyAsync(res.as<cpx<double>>() + k, v, sizeof(cpx<double>), hipMemcpyDeviceToDevice, st),
              "result");
  }
  hip_check(hipGetLastError(), "launch (mpo expectation)");
  hip_check(hipMemcpyAsync(out, res.p, sizeof(cpx<double>) * nops, hipMemcpyDeviceToHost, st), "results");
  hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
}

void MpoState::to_dense(double* out) {
  // t[(P x), b] = sum_a t[P, a] R_i[a, x, b], P the pair indices of sites < i
  long long big = 1LL << (2 * n);
  long long P = 1;
  for (int i = 0; i < n; ++i) {
    P *= 4;
    big = std::max(big, P * D[i + 1]);
  }
  if (big > (1LL << 28)) throw Error{6 /*MPDO_EUNSUPPORTED*/, "dense MPO: intermediate above 2^28 entries"};
  tA.alloc(sizeof(cpx<double>) * big);
  tB.alloc(sizeof(cpx<double>) * big);
  cpx<double>* t = tA.as<cpx<double>>();
  cpx<double>* u = tB.as<cpx<double>>();
  hipLaunchKernelGGL(k_mpo_one, dim3(1), dim3(1), 0, st, t);
  P = 1;
  for (int i = 0; i < n; ++i) {
    gemm_once(desc, t, R[i]->as<cpx<double>>(), u, (int)P, 4 * D[i + 1], D[i], OP_N, OP_N, D[i], 4 * D[i + 1],
              4 * D[i + 1], st, false);
    std::swap(t, u);
    P *= 4;
  }
  hipLaunchKernelGGL(k_mpo_unpair, dim3(grid_for(1LL << (2 * n))), dim3(MT), 0, st, t, n, u);
  hip_check(hipGetLastError(), "launch (dense MPO)");
  hip_check(hipMemcpyAsync(out, u, sizeof(cpx<double>) << (2 * n), hipMemcpyDeviceToHost, st), "dense rho");
  hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
}

}  // namespace mpdo
