// Glue kernels of the MPDO update: fused noisy-gate operators (Eq. (8)), the
// small Gram combinations of the inner truncation (Eqs. (9)-(11)), rank
// selection and renormalisation (Sec. II.D), and the descriptors that size
// the following contractions on the device.  One workgroup per item.
#include "common.h"
#include "ops.h"
#include "profile.h"

namespace mpdo {

namespace {
constexpr int GT = 256;

__device__ inline cpx<double> ld(const double* p, long long i) { return mk(p[2 * i], p[2 * i + 1]); }
__device__ inline void st(double* p, long long i, cpx<double> v) { p[2 * i] = v.re; p[2 * i + 1] = v.im; }

// Ideal unitary of a gate (d = 2^q <= 8) into U (row-major, complex).
__device__ void build_unitary(const GateSrc& g, cpx<double>* U) {
  const int d = 1 << g.q;
  for (int e = 0; e < d * d; ++e) U[e] = mk(0.0, 0.0);
  const double a = g.scale * ((g.pidx >= 0 && g.params) ? g.params[g.pidx] : 1.0);
  const double c = cos(0.5 * a), s = sin(0.5 * a);
  switch (g.kind) {
    case GK_RX: U[0] = mk(c, 0.0); U[1] = mk(0.0, -s); U[2] = mk(0.0, -s); U[3] = mk(c, 0.0); break;
    case GK_RY: U[0] = mk(c, 0.0); U[1] = mk(-s, 0.0); U[2] = mk(s, 0.0); U[3] = mk(c, 0.0); break;
    case GK_RZ: U[0] = mk(c, -s); U[3] = mk(c, s); break;
    case GK_ZZPHASE:
    case GK_SWAPZZ: {
      const cpx<double> e = mk(cos(a), -sin(a));
      U[0] = mk(1.0, 0.0);
      U[15] = mk(1.0, 0.0);
      if (g.kind == GK_ZZPHASE) { U[5] = e; U[10] = e; }
      else { U[6] = e; U[9] = e; }
      break;
    }
    default:
      if (g.ufix) {
        for (int e2 = 0; e2 < d * d; ++e2) U[e2] = ld(g.ufix, e2);
      } else {
        for (int i = 0; i < d; ++i) U[i * d + i] = mk(1.0, 0.0);
      }
  }
}

// G_j = K_j U for j < m (K = identity when kraus == null).
__device__ void build_G(const GateSrc& g, const double* kraus, int m, double* G, cpx<double>* sU) {
  const int d = 1 << g.q;
  if (threadIdx.x == 0) build_unitary(g, sU);
  __syncthreads();
  for (int e = threadIdx.x; e < m * d * d; e += blockDim.x) {
    const int j = e / (d * d), r = (e / d) % d, c = e % d;
    cpx<double> acc = mk(0.0, 0.0);
    if (kraus) {
      for (int t = 0; t < d; ++t) acc = acc + ld(kraus, (long long)j * d * d + r * d + t) * sU[t * d + c];
    } else {
      acc = sU[r * d + c];
    }
    st(G, e, acc);
  }
  __syncthreads();
}

// Smallest r >= 1 with sum_{i >= r} eta_i <= cut * W (W = sum of positive
// eta), capped at maxd; also returns the kept and total weights.
// eta: the leading kb eigenvalues (descending) of a Gram matrix of size n
// and trace W.  Eigenvalues at or below EIG_FLOOR * eta_0 are numerically
// zero and never kept.
__device__ int select_rank(const double* eta, int kb, int n, double W, int maxd, double cut, double* kept,
                           double* total) {
  if (W < 0) W = 0;
  int nz = 0;  // numerical rank among the computed eigenvalues
  while (nz < kb && eta[nz] > EIG_FLOOR * eta[0] && eta[0] > 0) ++nz;
  int r = n;
  double head = 0;
  for (int cand = 1; cand <= kb; ++cand) {
    head += eta[cand - 1] > 0 ? eta[cand - 1] : 0;
    if (W - head <= cut * W) {
      r = cand;
      break;
    }
  }
  if (r > nz) r = nz;
  if (r > maxd) r = maxd;
  if (r < 1) r = 1;
  // a degenerate multiplet straddling the cut is dropped whole, so the kept
  // subspace is unique (multiplets below 1e-11 of the weight are left alone)
  const int r0 = r;
  while (r > 1 && r < kb && eta[r - 1] > 1e-11 * W && eta[r - 1] - eta[r] <= 1e-9 * eta[r - 1]) --r;
  if (r == 1 && kb > 1 && eta[0] - eta[1] <= 1e-9 * eta[0]) r = r0;
  double k = 0;
  for (int i = 0; i < r; ++i) k += eta[i] > 0 ? eta[i] : 0;
  *kept = k;
  *total = W;
  return r;
}

// Records one truncation in a site's statistics (see StatField): the
// discarded fraction, the relative gap at the cut when weight was dropped,
// and a failure when the weights are not finite (a NaN in the state, or an
// eigensolver that marked its result by a non-finite trace).
__device__ void record_cut(double* st, const double* eta, int r, int kb, double tot, double kept) {
  if (!(tot >= 0 && tot < 1e300) || !(kept > 0 && kept < 1e300)) {
    st[ST_FAIL] += 1.0;
    return;
  }
  const double d = tot > 0 ? (tot - kept) / tot : 0.0;
  st[ST_DISC] += d;
  st[ST_MAXD] = fmax(st[ST_MAXD], d);
  st[ST_CUTS] += 1.0;
  if (r < kb && eta[r] > 0) st[ST_GAP] = fmin(st[ST_GAP], eta[r - 1] / eta[r] - 1.0);
}

// A basis eigendecomposition (no truncation): its trace must be finite.
__device__ inline void check_basis(double* st, double trace) {
  if (!(trace >= 0 && trace < 1e300)) st[ST_FAIL] += 1.0;
}

__device__ inline void clear_desc(GemmDesc& d) {
  d.w = nullptr; d.kstride = 0; d.sA = d.sB = d.sC = 0;
  d.M = d.N = d.K = 0; d.lda = d.ldb = d.ldc = 0; d.kinner = 0; d.wdiv = 1;
  d.nbatch = 1; d.splits = 1; d.opA = OP_N; d.opB = OP_N; d.beta = 0; d.active = 1; d.alpha = 1.0;
  d.herm = 0;
}
}  // namespace

// ============================================================================
// one-site noisy gate
// ============================================================================
template <typename T>
__global__ __launch_bounds__(GT) void k_q1_prepare(Ctx1<T>* ctxs, int splitsH) {
  __shared__ cpx<double> sU[64];
  Ctx1<T>& c = ctxs[blockIdx.x];
  build_G(c.g, c.kraus, c.m, c.G, sU);
  if (threadIdx.x != 0) return;
  const int cl = *c.chil, cr = *c.chir, k = *c.kap;
  GemmDesc& d = *c.dH;
  void* C = d.C;
  const long long sSplit = d.sSplit;
  clear_desc(d);
  d.C = C;
  d.sSplit = sSplit;
  if (c.m <= 1 && !c.force) { d.active = 0; return; }
  // H[a][a'] = sum_l lambda_l^2 sum_r conj(B[l][a][r]) B[l][a'][r],  a = (t, k)
  d.A = c.Bold; d.B = c.Bold;
  d.opA = OP_C; d.opB = OP_T;
  d.M = d.N = 2 * k;
  d.K = cl * cr;
  d.lda = d.ldb = cr;
  d.kinner = cr;
  d.kstride = (long long)2 * k * cr;
  d.w = c.laml2;
  d.wdiv = cr;
  d.ldc = 2 * k;
  d.splits = splitsH;
}

template <typename T>
__global__ __launch_bounds__(GT) void k_q1_gamma(Ctx1<T>* ctxs) {
  Ctx1<T>& c = ctxs[blockIdx.x];
  const int m = c.m;
  if (m <= 1 && !c.force) {
    if (threadIdx.x == 0) c.dE->active = 0;
    return;
  }
  const int k = *c.kap, n = k * m;
  // Gamma[(kk j),(kk' j')] = sum_{t,t'} Omega_{jj'}[t,t'] H[(t kk),(t' kk')],
  // Omega_{jj'}[t,t'] = sum_s conj(G_j[s,t]) G_j'[s,t']
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int a = e / n, b = e % n;
    const int kk = a / m, j = a % m, kk2 = b / m, j2 = b % m;
    cpx<double> acc = mk(0.0, 0.0);
    for (int t = 0; t < 2; ++t)
      for (int t2 = 0; t2 < 2; ++t2) {
        cpx<double> om = mk(0.0, 0.0);
        for (int s = 0; s < 2; ++s) om = om + cconj(ld(c.G, j * 4 + s * 2 + t)) * ld(c.G, j2 * 4 + s * 2 + t2);
        acc = acc + om * ld(c.H, (long long)(t * k + kk) * (2 * k) + (t2 * k + kk2));
      }
    st(c.Gam, e, acc);
  }
  if (threadIdx.x == 0) {
    EigDesc& d = *c.dE;
    d.a = c.Gam; d.lda = n; d.n = n; d.evals = c.ev; d.evecs = c.evec; d.trace = c.ev + n; d.active = 1;
  }
}

template <typename T>
__global__ __launch_bounds__(GT) void k_q1_select(Ctx1<T>* ctxs, TruncParams tp) {
  __shared__ int s_kp;
  __shared__ double s_scale;
  __shared__ cpx<double> sU[64];
  Ctx1<T>& c = ctxs[blockIdx.x];
  const int m = c.m;
  const int k = *c.kap, cl = *c.chil, cr = *c.chir;
  const bool trunc = m > 1 || c.force;
  if (threadIdx.x == 0) {
    if (!trunc) {
      s_kp = k;
      s_scale = 1.0;
    } else {
      double kept, tot;
      const int ng = k * m;
      const int kp = select_rank(c.ev, min(ng, tp.kap_max + 1), ng, c.ev[ng], tp.kap_max, tp.kap_cut, &kept, &tot);
      s_kp = kp;
      s_scale = 1.0 / sqrt(kept);
      record_cut(c.disc, c.ev, kp, min(ng, tp.kap_max + 1), tot, kept);
    }
  }
  __syncthreads();
  const int kp = s_kp;
  const double sc = s_scale;
  // W[(s nu),(t kk)] = scale sum_j G_j[s,t] V[(kk j), nu]   (V = identity for m = 1)
  const int nW = (2 * kp) * (2 * k);
  for (int e = threadIdx.x; e < nW; e += blockDim.x) {
    const int row = e / (2 * k), col = e % (2 * k);
    const int s = row / kp, nu = row % kp, t = col / k, kk = col % k;
    cpx<double> acc = mk(0.0, 0.0);
    if (!trunc) {
      if (nu == kk) acc = ld(c.G, s * 2 + t);
    } else {
      for (int j = 0; j < m; ++j)
        acc = acc + ld(c.G, j * 4 + s * 2 + t) * ld(c.evec, (long long)(kk * m + j) * (k * m) + nu);
    }
    c.W[e] = mk<T>((T)(sc * acc.re), (T)(sc * acc.im));
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    GemmDesc& d = *c.dA;
    clear_desc(d);
    d.A = c.W; d.B = c.Bold; d.C = c.Bnew;
    d.M = 2 * kp; d.K = 2 * k; d.N = cr;
    d.lda = 2 * k; d.ldb = cr; d.ldc = cr;
    d.nbatch = cl;
    d.sA = 0; d.sB = (long long)2 * k * cr; d.sC = (long long)2 * kp * cr;
    *c.kap = kp;
  }
  (void)sU;
}

// Weighted Grams with a small output on the vector units: C = op(A)^H W op(A)
// with M = N <= 32 over a long two-level K (the one-site inner Gram, 2 kappa
// rows over (l, r); the two-site one, 4 kappa rows over (l, beta)).  FP64
// vector arithmetic has the rate of the FP64 matrix cores on this chip, and
// such an output leaves most waves of a 32- or 64-wide MFMA tile idle.
constexpr int GV_RC = 64;  // inner K index per LDS tile
constexpr int GV_MAX = 32; // largest M

// The Gram a descriptor of the form A = B, opA = OP_C, opB = OP_T, K = L
// kinner, weights w[k / wdiv] with wdiv a multiple of kinner (constant over
// the inner index) describes: C[a][a'] = sum_k w conj(A(a, k)) A(a', k) with
// A(a, k) at (k / kinner) kstride + a lda + k % kinner.  One
// workgroup per item and range of the outer K index (split `split` of
// `splits`); each split's partial goes where the GEMM's split-K partials go
// (C + split sSplit, leading dimension ldc), so the same reduction adds them
// up.  FP64 accumulation; the tiles of the range in order, each thread's
// entries of the next tile loaded while the current one is summed.
template <typename T>
__global__ __launch_bounds__(GT) void k_gram_v(const GemmDesc* __restrict__ descs, int splits) {
  __shared__ cpx<double> X[GV_MAX][GV_RC + 1];
  const GemmDesc& d = descs[blockIdx.x / splits];
  const int split = blockIdx.x % splits;
  if (!d.active) return;
  const int m = d.M, kin = d.kinner > 0 ? d.kinner : d.K;
  const int L = kin > 0 ? d.K / kin : 0;
  const int lper = (L + splits - 1) / splits, l0 = split * lper, l1 = min(L, l0 + lper);
  const long long kst = d.kinner > 0 ? d.kstride : 0;
  const cpx<T>* A = reinterpret_cast<const cpx<T>*>(d.A);
  const double* w = reinterpret_cast<const double*>(d.w);
  const int wdiv = d.wdiv > 0 ? d.wdiv : 1;
  const int tid = threadIdx.x, np = m * m;
  constexpr int PPT = GV_MAX * GV_MAX / GT;  // (a, a') pairs per thread
  double ar[PPT], ai[PPT];
#pragma unroll
  for (int p = 0; p < PPT; ++p) ar[p] = ai[p] = 0.0;
  const int nrc = (kin + GV_RC - 1) / GV_RC, ntile = (l1 - l0) * nrc;
  constexpr int EPT = GV_MAX * GV_RC / GT;  // tile entries per thread
  cpx<T> nx[EPT];
  auto fetch = [&](int t) {
    const int l = l0 + t / nrc, r0 = (t % nrc) * GV_RC, rn = min(GV_RC, kin - r0);
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = tid + u * GT, a = e / GV_RC, r = e % GV_RC;
      nx[u] = (a < m && r < rn) ? A[(long long)l * kst + (long long)a * d.lda + r0 + r] : mk<T>((T)0, (T)0);
    }
  };
  if (ntile > 0) fetch(0);
  for (int t = 0; t < ntile; ++t) {
    const int l = l0 + t / nrc, r0 = (t % nrc) * GV_RC, rn = min(GV_RC, kin - r0);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = tid + u * GT, a = e / GV_RC, r = e % GV_RC;
      if (a < m) X[a][r] = mk((double)nx[u].re, (double)nx[u].im);
    }
    __syncthreads();
    if (t + 1 < ntile) fetch(t + 1);
    const double wt = w ? w[(long long)l * kin / wdiv] : 1.0;  // the tile's weight
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      const int q = tid + p * GT;
      if (q < np) {
        const int a = q / m, b = q % m;
        double sr = 0.0, si = 0.0;
        for (int r = 0; r < rn; ++r) {
          const cpx<double> x = X[a][r], y = X[b][r];
          sr += x.re * y.re + x.im * y.im;  // conj(x) y
          si += x.re * y.im - x.im * y.re;
        }
        ar[p] += wt * sr;
        ai[p] += wt * si;
      }
    }
  }
  cpx<double>* C = reinterpret_cast<cpx<double>*>(d.C) + (long long)split * d.sSplit;
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    const int q = tid + p * GT;
    if (q < np) C[(long long)(q / m) * d.ldc + q % m] = mk(ar[p], ai[p]);
  }
}

// ============================================================================
// two-site noisy gate
// ============================================================================
// Order of the two-site update (B_i, B_{i+1} right-canonical, weights lambda
// on the bond left of i):
//   E = F F^dag, F = B_{i+1} as [(m t2)] x [(k2 r)]  -> E = P D P^dag,
//   L_F = P D^(1/2) on the r_F numerically non-zero eigenvalues,
//   th = B_i L_F  (so that the two-site block is th applied to F's row space),
//   H  = lambda^2-weighted Gram of th over (l, beta)  (the inner-index Gram of
//        the gate input, Eq. (9), expressed in the F basis),
//   Gamma from H and the fused operators G_j -> eig -> W (inner truncation,
//        Eqs. (10)-(11)),
//   th2 = W th, C = weighted Gram of th2 -> eig -> new bond (SVD, Sec. II.D).
template <typename T>
__global__ __launch_bounds__(GT) void k_q2_prepare(Ctx2<T>* ctxs, int splitsE) {
  __shared__ cpx<double> sU[64];
  Ctx2<T>& c = ctxs[blockIdx.x];
  build_G(c.g, c.kraus, c.m, c.G, sU);
  if (threadIdx.x != 0) return;
  const int cm = *c.chim, cr = *c.chir, k2 = *c.kap2;
  {  // E = F F^dag with F = B_{i+1} as [(m t2)] x [(k2 r)]
    GemmDesc& d = *c.dGramE;
    void* C = d.C;
    const long long ss = d.sSplit;
    clear_desc(d);
    d.C = C; d.sSplit = ss;
    d.A = c.Bj; d.B = c.Bj; d.opA = OP_N; d.opB = OP_H;
    d.M = d.N = 2 * cm;
    d.K = k2 * cr;
    d.lda = d.ldb = k2 * cr;
    d.ldc = 2 * cm;
    d.splits = splitsE;
    d.herm = 1;
  }
  {
    EigDesc& d = *c.dEigE;
    d.a = c.E; d.lda = 2 * cm; d.n = 2 * cm; d.evals = c.evE; d.evecs = c.vecE; d.trace = c.evE + 2 * cm;
    d.active = 1; d.upper = 1;
  }
}

// r_F, L_F = P D^(1/2), PD = P D^(-1/2); descriptors of th = B_i L_F and of
// the Gram H of th.
template <typename T> __device__ void q2_theta_descs(Ctx2<T>& c, int rF, int splitsH);

template <typename T>
__global__ __launch_bounds__(GT) void k_q2_select_e(Ctx2<T>* ctxs, int splitsH, TruncParams tp) {
  __shared__ int s_rF;
  Ctx2<T>& c = ctxs[blockIdx.x];
  const int cm = *c.chim;
  const int nE = 2 * cm;
  if (threadIdx.x == 0) {
    int rF = 0;
    const double e0 = c.evE[0];
    for (int b = 0; b < nE; ++b) rF += (c.evE[b] > tp.tolE * e0) ? 1 : 0;
    if (rF < 1) rF = 1;
    check_basis(c.disc, c.evE[nE]);
    s_rF = rF;
    c.scratch[1] = rF;
  }
  __syncthreads();
  const int rF = s_rF;
  for (int e = threadIdx.x; e < nE * rF; e += blockDim.x) {
    const int row = e / rF, b = e % rF;
    const cpx<double> p = ld(c.vecE, (long long)row * nE + b);
    const double sq = sqrt(c.evE[b]);
    c.LF[e] = mk<T>((T)(p.re * sq), (T)(p.im * sq));
    st(c.PD, e, mk(p.re / sq, p.im / sq));
  }
  if (threadIdx.x == 0) q2_theta_descs(c, rF, splitsH);
}

// Descriptors of theta = B_i L_F and of the inner Gram H of theta, once r_F
// and L_F are known (one thread).
template <typename T> __device__ void q2_theta_descs(Ctx2<T>& c, int rF, int splitsH) {
  const int k1 = *c.kap1, cl = *c.chil, cm = *c.chim;
  {
    {  // th[(l t1 k1),(t2 b)] = sum_m B_i[(l t1 k1), m] L_F[(m t2), b]
      GemmDesc& d = *c.dTh;
      clear_desc(d);
      d.A = c.Bi; d.B = c.LF; d.C = c.th;
      d.M = cl * 2 * k1; d.K = cm; d.N = 2 * rF;
      d.lda = cm; d.ldb = 2 * rF; d.ldc = 2 * rF;
    }
    {  // H[a][a'] = sum_l lambda_l^2 sum_b conj(th[l][a][b]) th[l][a'][b],
       // a = (t1 k1 t2): th[l] viewed as (4 k1) rows of r_F
      GemmDesc& d = *c.dGramH;
      void* C = d.C;
      const long long ss = d.sSplit;
      clear_desc(d);
      d.C = C; d.sSplit = ss;
      if (c.m <= 1) {
        d.active = 0;
      } else {
        d.A = c.th; d.B = c.th; d.opA = OP_C; d.opB = OP_T;
        d.M = d.N = 4 * k1;
        d.K = cl * rF;
        d.lda = d.ldb = rF;
        d.kinner = rF;
        d.kstride = (long long)4 * k1 * rF;
        d.w = c.laml2; d.wdiv = rF;
        d.ldc = 4 * k1;
        d.splits = splitsH;
      }
    }
  }
}

// The right-factor basis from a pivoted Cholesky factorisation of
// E = F F^H (n = 2 chi_m <= 128) in place of its eigendecomposition: with
// the pivots taken largest first, Pi^T E Pi = L L^H, r = the number of pivots
// above tolE times the first; L_F = Pi L (rows in E's own order) and
// PD = Pi [L1^-H; 0], L1 the leading r x r block, so that PD^H F = L1^-1 F1
// has orthonormal rows and F = L_F (PD^H F) up to the dropped Schur
// complement (weight below n tolE of the first pivot).  One workgroup of
// CH_NT threads per item keeps the upper triangle of E packed in LDS (each
// thread owns up to CH_NE packed entries); a pivot step forms the column
// l = S[:, p] / sqrt(S[p][p]) (zero on earlier pivots) and updates the Schur
// complement S -= l l^H in place, and the columns of L go to the
// eigenvector buffer.  The same LDS then holds X = L1^-1 (packed lower
// triangle, pivot order), built by right-looking elimination with the
// columns of L1 read back from that buffer one step ahead.
constexpr int CH_NT = 1024, CH_NC = 128, CH_NPK = CH_NC * (CH_NC + 1) / 2;
constexpr int CH_NE = (CH_NPK + CH_NT - 1) / CH_NT;

// Candidate (av, ai) ranks above (bv, bi) as a pivot: any candidate above
// none (index n), a NaN above a number (so that it is found and reported),
// else the larger value, ties to the smaller index.
__device__ inline bool chol_better(double av, int ai, double bv, int bi, int n) {
  if (ai >= n) return false;
  if (bi >= n) return true;
  const bool an = av != av, bn = bv != bv;
  if (an != bn) return an;
  if (an) return ai < bi;
  return av > bv || (av == bv && ai < bi);
}

// Wave 0: the largest remaining diagonal entry of rows [0, n) (n <= nmax,
// the length of dg and done) into *piv, *dp (*dp = -1 when every row is a
// pivot already); row `skip` counts as a pivot.
__device__ void chol_pivot(const double* dg, const int* done, int n, int nmax, int skip, int* piv, double* dp) {
  const int lane = threadIdx.x;
  double best = 0.0;
  int bi = n;
  for (int e = lane; e < nmax; e += 64) {
    if (e >= n || done[e] || e == skip) continue;
    if (chol_better(dg[e], e, best, bi, n)) {
      best = dg[e];
      bi = e;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off);
    const int oi = __shfl_xor(bi, off);
    if (chol_better(ob, oi, best, bi, n)) {
      best = ob;
      bi = oi;
    }
  }
  if (lane == 0) {
    *piv = bi;
    *dp = bi < n ? best : -1.0;
  }
}

// Row of packed entry e of an m x m triangle stored row by row, rows of
// length rowlen(i) starting at start[i] (start[m] = the count): the last i
// with start[i] <= e.
__device__ inline int packed_row(const int* start, int m, int e) {
  int lo = 0, hi = m - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename T>
__global__ __launch_bounds__(CH_NT) void k_q2_chol_e(Ctx2<T>* ctxs, int splitsH, TruncParams tp) {
  __shared__ cpx<double> P[CH_NPK];  // S (upper, row i: columns i..n-1), then X (lower, row j: 0..j)
  __shared__ cpx<double> colbuf[CH_NC];
  __shared__ cpx<double> lbuf[2][CH_NC];
  __shared__ double dg[CH_NC];
  __shared__ int done[CH_NC], pivrow[CH_NC], posr[CH_NC], start[CH_NC + 1];
  __shared__ int s_piv;
  __shared__ double s_dp;
  Ctx2<T>& c = ctxs[blockIdx.x];
  const int nE = 2 * *c.chim;
  const int n = nE <= CH_NC ? nE : 0;  // a larger E is reported as a failure below (the host never sends one)
  const int t = threadIdx.x;
  const cpx<double> zero = mk(0.0, 0.0);
  double* Lsc = c.vecE;  // column k of L at Lsc[k n + row]
  const int npk = n * (n + 1) / 2;
  // upper triangle: row i holds columns i..n-1
  if (t <= n) start[t] = t * n - t * (t - 1) / 2;
  if (t < CH_NC) {
    dg[t] = t < n ? c.E[2 * ((long long)t * n + t)] : 0.0;
    done[t] = t < n ? 0 : 1;
    posr[t] = -1;
  }
  __syncthreads();
  int ei[CH_NE], ej[CH_NE];  // (row, column) of this thread's packed entries
#pragma unroll
  for (int q = 0; q < CH_NE; ++q) {
    const int e = t + CH_NT * q;
    ei[q] = ej[q] = 0;
    if (e < npk) {
      const int i = packed_row(start, n, e);
      ei[q] = i;
      ej[q] = i + (e - start[i]);
      P[e] = ld(c.E, (long long)i * n + ej[q]);
    }
  }
  if (t < 64) chol_pivot(dg, done, n, CH_NC, -1, &s_piv, &s_dp);
  __syncthreads();
  const double d0 = s_dp;
  const double thr = tp.tolE * d0;
  bool fail = !(d0 > 0.0 && d0 < 1e300) || n != nE;
  int r = 0;
  for (int k = 0; k < n && !fail; ++k) {
    const int p = s_piv;
    const double dp = s_dp;
    if (!(dp < 1e300)) {  // NaN or overflow in the Schur complement
      fail = true;
      break;
    }
    if (!(dp > thr)) break;
    if (t < n) {  // l = S[:, p] / sqrt(S[p][p]), zero on earlier pivots
      cpx<double> v = zero;
      if (!done[t]) {
        const double inv = 1.0 / sqrt(dp);
        v = t <= p ? inv * P[start[t] + (p - t)] : inv * cconj(P[start[p] + (t - p)]);
      }
      colbuf[t] = v;
      st(Lsc, (long long)k * n + t, v);
      dg[t] -= v.re * v.re + v.im * v.im;
    }
    if (t == 0) {
      pivrow[k] = p;
      posr[p] = k;
    }
    __syncthreads();
    // every read of s_piv, s_dp and done for this step is behind the barrier:
    // wave 0 picks the next pivot while the Schur complement is updated
    if (t < 64) {
      if (t == 0) done[p] = 1;
      chol_pivot(dg, done, n, CH_NC, p, &s_piv, &s_dp);
    }
#pragma unroll
    for (int q = 0; q < CH_NE; ++q) {
      const int e = t + CH_NT * q;
      if (e < npk) {
        const cpx<double> li = colbuf[ei[q]];
        if (li.re != 0.0 || li.im != 0.0) P[e] = P[e] - li * cconj(colbuf[ej[q]]);  // rows of pivots: l = 0
      }
    }
    __syncthreads();
    r = k + 1;
  }
  if (r == 0) fail = true;
  const int rF = fail ? 1 : r;
  if (!fail) {
    // X = L1^-1 (lower triangle, pivot order: row j holds columns 0..j)
    const int nx = r * (r + 1) / 2;
    if (t <= r) start[t] = t * (t + 1) / 2;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < CH_NE; ++q) {
      const int e = t + CH_NT * q;
      ei[q] = ej[q] = 0;
      if (e < nx) {
        const int j = packed_row(start, r, e);
        ei[q] = j;
        ej[q] = e - start[j];
        P[e] = ej[q] == j ? mk(1.0, 0.0) : zero;
      }
    }
    if (t < r) lbuf[0][t] = ld(Lsc, pivrow[t]);
    __syncthreads();
    for (int m = 0; m < r; ++m) {
      const int cur = m & 1;
      if (m + 1 < r && t < r) lbuf[cur ^ 1][t] = ld(Lsc, (long long)(m + 1) * n + pivrow[t]);
      if (t <= m) {  // row m of X, scaled by 1 / L1[m][m]
        const cpx<double> x = (1.0 / lbuf[cur][m].re) * P[start[m] + t];
        P[start[m] + t] = x;
        colbuf[t] = x;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < CH_NE; ++q) {
        const int e = t + CH_NT * q;
        if (e < nx && ei[q] > m && ej[q] <= m) P[e] = P[e] - lbuf[cur][ei[q]] * colbuf[ej[q]];
      }
      __syncthreads();
    }
  }
  for (int e = t; e < nE * rF; e += CH_NT) {
    const int row = e / rF, b = e % rF;
    cpx<double> l = zero, pd = zero;
    if (!fail) {
      l = ld(Lsc, (long long)b * n + row);
      const int j = posr[row];
      if (j >= 0 && j <= b) pd = cconj(P[start[b] + j]);  // conj(X[b][j])
    }
    c.LF[e] = mk<T>((T)l.re, (T)l.im);
    st(c.PD, e, pd);
  }
  if (t == 0) {
    c.scratch[1] = rF;
    if (fail) c.disc[ST_FAIL] += 1.0;
    q2_theta_descs(c, rF, splitsH);
  }
}

// The same factorisation for 128 < n <= 256 (chi_max <= 128), with the
// Schur complement updated in place in E's own buffer (row-major, upper
// triangle) and X = L1^-1 in the bond-Gram eigenvector buffer (row-major,
// lower triangle).  Thread t owns the columns cp = t % 128 and 255 - cp (so
// that every thread holds about the same number of upper-triangle entries)
// in the rows t / 128 + 8 q; each entry is read and written by its owner
// only, apart from the pivot column, which every thread reads after the
// step's barrier.
constexpr int CG_NT = 1024, CG_NC = 256, CG_CP = CG_NC / 2, CG_RP = CG_NT / CG_CP;

template <typename T>
__global__ __launch_bounds__(CG_NT) void k_q2_chol_e_g(Ctx2<T>* ctxs, int splitsH, TruncParams tp) {
  __shared__ cpx<double> colbuf[CG_NC];
  __shared__ cpx<double> lbuf[2][CG_NC];
  __shared__ double dg[CG_NC];
  __shared__ int done[CG_NC], pivrow[CG_NC], posr[CG_NC];
  __shared__ int s_piv;
  __shared__ double s_dp;
  Ctx2<T>& c = ctxs[blockIdx.x];
  const int nE = 2 * *c.chim;
  const int n = nE <= CG_NC ? nE : 0;  // a larger E is reported as a failure below (the host never sends one)
  const int t = threadIdx.x, cp = t % CG_CP, g = t / CG_CP;
  const int cols[2] = {cp, CG_NC - 1 - cp};
  const cpx<double> zero = mk(0.0, 0.0);
  double* S = c.E;       // S[i][j] at S[i n + j], i <= j
  double* Lsc = c.vecE;  // column k of L at Lsc[k n + row]
  double* X = c.vecC;    // X[j][b] at X[j n + b], b <= j
  if (t < CG_NC) {
    dg[t] = t < n ? S[2 * ((long long)t * n + t)] : 0.0;
    done[t] = t < n ? 0 : 1;
    posr[t] = -1;
  }
  __syncthreads();
  if (t < 64) chol_pivot(dg, done, n, CG_NC, -1, &s_piv, &s_dp);
  __syncthreads();
  const double d0 = s_dp;
  const double thr = tp.tolE * d0;
  bool fail = !(d0 > 0.0 && d0 < 1e300) || n != nE;
  int r = 0;
  for (int k = 0; k < n && !fail; ++k) {
    const int p = s_piv;
    const double dp = s_dp;
    if (!(dp < 1e300)) {
      fail = true;
      break;
    }
    if (!(dp > thr)) break;
    if (t < n) {  // l = S[:, p] / sqrt(S[p][p]), zero on earlier pivots
      cpx<double> v = zero;
      if (!done[t]) {
        const double inv = 1.0 / sqrt(dp);
        v = t <= p ? inv * ld(S, (long long)t * n + p) : inv * cconj(ld(S, (long long)p * n + t));
      }
      colbuf[t] = v;
      st(Lsc, (long long)k * n + t, v);
      dg[t] -= v.re * v.re + v.im * v.im;
    }
    if (t == 0) {
      pivrow[k] = p;
      posr[p] = k;
    }
    __syncthreads();
    if (t < 64) {
      if (t == 0) done[p] = 1;
      chol_pivot(dg, done, n, CG_NC, p, &s_piv, &s_dp);
    }
    for (int h = 0; h < 2; ++h) {
      const int j = cols[h];
      if (j >= n) continue;
      const cpx<double> lj = cconj(colbuf[j]);
      if (lj.re == 0.0 && lj.im == 0.0) continue;  // a pivot's column: nothing to subtract
      for (int i = g; i <= j; i += CG_RP) {
        const cpx<double> li = colbuf[i];
        if (li.re != 0.0 || li.im != 0.0) st(S, (long long)i * n + j, ld(S, (long long)i * n + j) - li * lj);
      }
    }
    __syncthreads();
    r = k + 1;
  }
  if (r == 0) fail = true;
  const int rF = fail ? 1 : r;
  if (!fail) {
    // X = L1^-1 (lower triangle, pivot order), right-looking elimination
    for (int h = 0; h < 2; ++h) {
      const int b = cols[h];
      if (b >= r) continue;
      for (int j = b + ((g - b) % CG_RP + CG_RP) % CG_RP; j < r; j += CG_RP)
        st(X, (long long)j * n + b, j == b ? mk(1.0, 0.0) : zero);
    }
    if (t < r) lbuf[0][t] = ld(Lsc, pivrow[t]);
    __syncthreads();
    for (int m = 0; m < r; ++m) {
      const int cur = m & 1;
      if (m + 1 < r && t < r) lbuf[cur ^ 1][t] = ld(Lsc, (long long)(m + 1) * n + pivrow[t]);
      if (t <= m) {  // row m of X, scaled by 1 / L1[m][m]
        const cpx<double> x = (1.0 / lbuf[cur][m].re) * ld(X, (long long)m * n + t);
        st(X, (long long)m * n + t, x);
        colbuf[t] = x;
      }
      __syncthreads();
      for (int h = 0; h < 2; ++h) {
        const int b = cols[h];
        if (b > m || b >= r) continue;
        const cpx<double> xb = colbuf[b];
        // rows j > m owned by this thread: j = g (mod CG_RP)
        for (int j = m + 1 + ((g - m - 1) % CG_RP + CG_RP) % CG_RP; j < r; j += CG_RP)
          st(X, (long long)j * n + b, ld(X, (long long)j * n + b) - lbuf[cur][j] * xb);
      }
      __syncthreads();
    }
  }
  __syncthreads();
  for (int e = t; e < nE * rF; e += CG_NT) {
    const int row = e / rF, b = e % rF;
    cpx<double> l = zero, pd = zero;
    if (!fail) {
      l = ld(Lsc, (long long)b * n + row);
      const int j = posr[row];
      if (j >= 0 && j <= b) pd = cconj(ld(X, (long long)b * n + j));  // conj(X[b][j])
    }
    c.LF[e] = mk<T>((T)l.re, (T)l.im);
    st(c.PD, e, pd);
  }
  if (t == 0) {
    c.scratch[1] = rF;
    if (fail) c.disc[ST_FAIL] += 1.0;
    q2_theta_descs(c, rF, splitsH);
  }
}

template <typename T>
__global__ __launch_bounds__(GT) void k_q2_gamma(Ctx2<T>* ctxs) {
  __shared__ cpx<double> sOm[16 * 16 * 16];  // Omega_{jj'}[t][t'] for m <= 16
  Ctx2<T>& c = ctxs[blockIdx.x];
  const int m = c.m, k1 = *c.kap1;
  if (m <= 1) {
    if (threadIdx.x == 0 && blockIdx.y == 0) c.dEigG->active = 0;
    return;
  }
  const int n = k1 * m;
  const bool om_lds = m <= 16;
  if (om_lds) {
    for (int e = threadIdx.x; e < m * m * 16; e += blockDim.x) {
      const int j = e / (m * 16), j2 = (e / 16) % m, t = (e / 4) % 4, t2 = e % 4;
      cpx<double> om = mk(0.0, 0.0);
      for (int s = 0; s < 4; ++s) om = om + cconj(ld(c.G, j * 16 + s * 4 + t)) * ld(c.G, j2 * 16 + s * 4 + t2);
      sOm[e] = om;
    }
  }
  __syncthreads();
  // Gamma[(kk j),(kk' j')] = sum_{t,t'} Omega_{jj'}[t,t'] H[h(t,kk)][h(t',kk')],
  // h(t, kk) = ((t1 k1 + kk) 2 + t2) with t = 2 t1 + t2; the upper triangle
  // only (the eigensolver reads no more), spread over gridDim.y blocks
  for (int e = threadIdx.x + blockIdx.y * blockDim.x; e < n * n; e += blockDim.x * gridDim.y) {
    const int a = e / n, b = e % n;
    if (b < a) continue;
    const int kk = a / m, j = a % m, kk2 = b / m, j2 = b % m;
    cpx<double> acc = mk(0.0, 0.0);
    for (int t = 0; t < 4; ++t) {
      const int ha = ((t >> 1) * k1 + kk) * 2 + (t & 1);
      for (int t2 = 0; t2 < 4; ++t2) {
        const int hb = ((t2 >> 1) * k1 + kk2) * 2 + (t2 & 1);
        cpx<double> om;
        if (om_lds) {
          om = sOm[((j * m + j2) * 4 + t) * 4 + t2];
        } else {
          om = mk(0.0, 0.0);
          for (int s = 0; s < 4; ++s) om = om + cconj(ld(c.G, j * 16 + s * 4 + t)) * ld(c.G, j2 * 16 + s * 4 + t2);
        }
        acc = acc + om * ld(c.H, (long long)ha * (4 * k1) + hb);
      }
    }
    st(c.Gam, e, acc);
  }
  if (threadIdx.x == 0 && blockIdx.y == 0) {
    EigDesc& d = *c.dEigG;
    d.a = c.Gam; d.lda = n; d.n = n; d.evals = c.evG; d.evecs = c.vecG; d.trace = c.evG + n; d.active = 1;
    d.upper = 1;
  }
}

// kappa' and W; descriptors of th2 = W th, its Gram C and C's eigensolver.
template <typename T>
__global__ __launch_bounds__(GT) void k_q2_select_g(Ctx2<T>* ctxs, int splitsC, TruncParams tp) {
  __shared__ int s_kp;
  __shared__ double s_scale;
  Ctx2<T>& c = ctxs[blockIdx.x];
  const int m = c.m, k1 = *c.kap1, cl = *c.chil;
  const int rF = c.scratch[1];
  if (threadIdx.x == 0) {
    if (m <= 1) {
      s_kp = k1;
      s_scale = 1.0;
    } else {
      double kept, tot;
      const int ng = k1 * m;
      const int kp = select_rank(c.evG, min(ng, tp.kap_max + 1), ng, c.evG[ng], tp.kap_max, tp.kap_cut, &kept, &tot);
      s_kp = kp;
      s_scale = 1.0 / sqrt(kept);
      record_cut(c.disc, c.evG, kp, min(ng, tp.kap_max + 1), tot, kept);
    }
    c.scratch[0] = s_kp;
  }
  __syncthreads();
  const int kp = s_kp;
  const double sc = s_scale;
  // W[(s1 nu s2),(t1 kk t2)] = scale sum_j G_j[(s1 s2),(t1 t2)] V[(kk j), nu]
  const int rows = 4 * kp, cols = 4 * k1;
  for (int e = threadIdx.x; e < rows * cols; e += blockDim.x) {
    const int row = e / cols, col = e % cols;
    const int s1 = row / (2 * kp), nu = (row / 2) % kp, s2 = row % 2;
    const int t1 = col / (2 * k1), kk = (col / 2) % k1, t2 = col % 2;
    const int gs = s1 * 2 + s2, gt = t1 * 2 + t2;
    cpx<double> acc = mk(0.0, 0.0);
    if (m <= 1) {
      if (nu == kk) acc = ld(c.G, gs * 4 + gt);
    } else {
      for (int j = 0; j < m; ++j)
        acc = acc + ld(c.G, j * 16 + gs * 4 + gt) * ld(c.vecG, (long long)(kk * m + j) * (k1 * m) + nu);
    }
    c.W[e] = mk<T>((T)(sc * acc.re), (T)(sc * acc.im));
  }
  if (threadIdx.x == 0) {
    {  // th2[l] = W th[l]
      GemmDesc& d = *c.dTh2;
      clear_desc(d);
      d.A = c.W; d.B = c.th; d.C = c.th2;
      d.M = 4 * kp; d.K = 4 * k1; d.N = rF;
      d.lda = 4 * k1; d.ldb = rF; d.ldc = rF;
      d.nbatch = cl; d.sA = 0; d.sB = (long long)4 * k1 * rF; d.sC = (long long)4 * kp * rF;
    }
    {  // C = th2^H diag(lambda_l^2) th2 over rows (l s1 nu)
      GemmDesc& d = *c.dC;
      void* C = d.C;
      const long long ss = d.sSplit;
      clear_desc(d);
      d.C = C; d.sSplit = ss;
      d.A = c.th2; d.B = c.th2; d.opA = OP_H; d.opB = OP_N;
      d.M = d.N = 2 * rF;
      d.K = cl * 2 * kp;
      d.lda = d.ldb = 2 * rF;
      d.w = c.laml2; d.wdiv = 2 * kp;
      d.ldc = 2 * rF;
      d.splits = splitsC;
      d.herm = 1;
    }
    {
      EigDesc& d = *c.dEigC;
      d.a = c.Cm; d.lda = 2 * rF; d.n = 2 * rF; d.evals = c.evC; d.evecs = c.vecC; d.trace = c.evC + 2 * rF;
      d.active = 1; d.upper = 1;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(GT) void k_q2_select_b(Ctx2<T>* ctxs, TruncParams tp) {
  __shared__ int s_r;
  __shared__ double s_scale;
  Ctx2<T>& c = ctxs[blockIdx.x];
  const int kp = c.scratch[0], rF = c.scratch[1];
  const int cl = *c.chil, cm = *c.chim, cr = *c.chir, k2 = *c.kap2;
  const int n = 2 * rF;
  if (threadIdx.x == 0) {
    double kept, tot;
    const int r = select_rank(c.evC, min(n, tp.chi_max + 1), n, c.evC[n], tp.chi_max, tp.svd_cut, &kept, &tot);
    s_r = r;
    s_scale = 1.0 / sqrt(kept);
    record_cut(c.disc, c.evC, r, min(n, tp.chi_max + 1), tot, kept);
  }
  __syncthreads();
  const int r = s_r;
  const double sc = s_scale;
  for (int v = threadIdx.x; v < r; v += blockDim.x) {
    const double e = c.evC[v] > 0 ? c.evC[v] : 0.0;
    c.lam[v] = sqrt(e) * sc;
    c.lam2[v] = e * sc * sc;
  }
  // Zt[(nu s2)][b] = conj(Z[(s2 rF + b)][nu]),  Zc = Z[:, :r] in working precision
  for (int e = threadIdx.x; e < 2 * r * rF; e += blockDim.x) {
    const int row = e / rF, b = e % rF;
    const int nu = row / 2, s2 = row % 2;
    st(c.Zt, e, cconj(ld(c.vecC, (long long)(s2 * rF + b) * n + nu)));
  }
  for (int e = threadIdx.x; e < n * r; e += blockDim.x) {
    const int row = e / r, nu = e % r;
    const cpx<double> z = ld(c.vecC, (long long)row * n + nu);
    c.Zc[e] = mk<T>((T)z.re, (T)z.im);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    {  // X[(nu s2),(m t2)] = sum_b Zt[(nu s2)][b] conj(PD[(m t2)][b])
      GemmDesc& d = *c.dX;
      clear_desc(d);
      d.A = c.Zt; d.B = c.PD; d.C = c.X;
      d.opB = OP_H;
      d.M = 2 * r; d.K = rF; d.N = 2 * cm;
      d.lda = rF; d.ldb = rF; d.ldc = 2 * cm;
    }
    {  // B_i' = scale th2 Z_r
      GemmDesc& d = c.dOut[0];
      clear_desc(d);
      d.A = c.th2; d.B = c.Zc; d.C = c.Bi_new;
      d.M = cl * 2 * kp; d.K = n; d.N = r;
      d.lda = n; d.ldb = r; d.ldc = r;
      d.alpha = sc;
    }
    {  // B_{i+1}' = X F
      GemmDesc& d = c.dOut[1];
      clear_desc(d);
      d.A = c.X; d.B = c.Bj; d.C = c.Bj_new;
      d.M = 2 * r; d.K = 2 * cm; d.N = k2 * cr;
      d.lda = 2 * cm; d.ldb = k2 * cr; d.ldc = k2 * cr;
    }
    *c.chim = r;
    *c.kap1 = kp;
  }
}

// ============================================================================
// three-site noisy gate (see Ctx3)
// ============================================================================
// Gate operators and the Gram descriptors of the two outer sites.
template <typename T>
__global__ __launch_bounds__(GT) void k_q3_prepare(Ctx3<T>* ctxs, int splitsN, int splitsE) {
  __shared__ cpx<double> sU[64];
  Ctx3<T>& c = ctxs[blockIdx.x];
  build_G(c.g, c.kraus, c.m, c.G, sU);
  if (threadIdx.x != 0) return;
  const int cl = *c.chil, ca = *c.chim1, cb = *c.chim2, cr = *c.chir;
  const int k1 = *c.kap1, k3 = *c.kap3;
  {  // N[(t1 a),(t1' a')] = sum_{l k1} lambda_l^2 conj(Bp) Bp
    GemmDesc& d = *c.dN;
    void* C = d.C;
    const long long ss = d.sSplit;
    clear_desc(d);
    d.C = C; d.sSplit = ss;
    d.A = c.Bp; d.B = c.Bp; d.opA = OP_H; d.opB = OP_N;
    d.M = d.N = 2 * ca;
    d.K = cl * k1;
    d.lda = d.ldb = 2 * ca;
    d.w = c.laml2; d.wdiv = k1;
    d.ldc = 2 * ca;
    d.splits = splitsN;
    d.herm = 1;
    EigDesc& e = *c.eN;
    e.lda = 2 * ca; e.n = 2 * ca; e.evals = c.evN; e.evecs = c.vecN; e.trace = c.evN + 2 * ca; e.active = 1;
    e.upper = 1;
  }
  {  // E3 = F F^H, F = B_{i+2} as [(b t3)] x [(k3 r)]
    GemmDesc& d = *c.dE3;
    void* C = d.C;
    const long long ss = d.sSplit;
    clear_desc(d);
    d.C = C; d.sSplit = ss;
    d.A = c.Bk; d.B = c.Bk; d.opA = OP_N; d.opB = OP_H;
    d.M = d.N = 2 * cb;
    d.K = k3 * cr;
    d.lda = d.ldb = k3 * cr;
    d.ldc = 2 * cb;
    d.splits = splitsE;
    d.herm = 1;
    EigDesc& e = *c.eE3;
    e.lda = 2 * cb; e.n = 2 * cb; e.evals = c.evE3; e.evecs = c.vecE3; e.trace = c.evE3 + 2 * cb; e.active = 1;
    e.upper = 1;
  }
}

// Bp[(l k1), (t1 a)] = B_i[l, t1, k1, a]
template <typename T>
__global__ __launch_bounds__(GT) void k_q3_perm_in(Ctx3<T>* ctxs) {
  Ctx3<T>& c = ctxs[blockIdx.y];
  const int cl = *c.chil, ca = *c.chim1, k1 = *c.kap1;
  const long long total = (long long)cl * 2 * k1 * ca;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int a = (int)(e % ca);
    long long rest = e / ca;
    const int t1 = (int)(rest % 2);
    rest /= 2;
    const int kk = (int)(rest % k1);
    const int l = (int)(rest / k1);
    c.Bp[e] = c.Bi[(((long long)l * 2 + t1) * k1 + kk) * ca + a];
  }
}

// Ranks of N and E3 (eigenvalues above Q3_BASIS_FLOOR times the largest),
// the basis factors, and the descriptors of Xt, Psi and Hin.
template <typename T>
__global__ __launch_bounds__(GT) void k_q3_sel_env(Ctx3<T>* ctxs, int splitsH, double floor) {
  __shared__ int s_r[2];
  Ctx3<T>& c = ctxs[blockIdx.x];
  const int ca = *c.chim1, cb = *c.chim2, k2 = *c.kap2;
  const int nN = 2 * ca, nE = 2 * cb;
  if (threadIdx.x == 0) {
    int rN = 0, r3 = 0;
    for (int b = 0; b < nN; ++b) rN += (c.evN[b] > floor * c.evN[0]) ? 1 : 0;
    for (int b = 0; b < nE; ++b) r3 += (c.evE3[b] > floor * c.evE3[0]) ? 1 : 0;
    s_r[0] = rN < 1 ? 1 : rN;
    s_r[1] = r3 < 1 ? 1 : r3;
    check_basis(c.disc, c.evN[nN]);
    check_basis(c.disc, c.evE3[nE]);
    c.scratch[1] = s_r[0];
    c.scratch[2] = s_r[1];
  }
  __syncthreads();
  const int rN = s_r[0], r3 = s_r[1];
  for (int e = threadIdx.x; e < nN * rN; e += blockDim.x) {
    const int x = e / rN, al = e % rN;
    const cpx<double> p = ld(c.vecN, (long long)x * nN + al);
    const double sq = sqrt(c.evN[al]);
    c.L1[(long long)al * nN + x] = mk<T>((T)(p.re * sq), (T)(-p.im * sq));
    st(c.PND, e, mk(p.re / sq, p.im / sq));
  }
  for (int e = threadIdx.x; e < nE * r3; e += blockDim.x) {
    const int y = e / r3, be = e % r3;
    const cpx<double> p = ld(c.vecE3, (long long)y * nE + be);
    const double sq = sqrt(c.evE3[be]);
    c.L3[e] = mk<T>((T)(p.re * sq), (T)(p.im * sq));
    st(c.PD3, e, mk(p.re / sq, p.im / sq));
  }
  if (threadIdx.x == 0) {
    {  // Xt[(a t2 k2), (t3 beta)] = sum_b B_{i+1}[(a t2 k2), b] L3[(b t3), beta]
      GemmDesc& d = *c.dXt;
      clear_desc(d);
      d.A = c.Bj; d.B = c.L3; d.C = c.Xt;
      d.M = ca * 2 * k2; d.K = cb; d.N = 2 * r3;
      d.lda = cb; d.ldb = 2 * r3; d.ldc = 2 * r3;
    }
    {  // Psi[alpha, t1, :] = sum_a L1[alpha, (t1 a)] Xt[a, :], one batch per t1
      GemmDesc& d = *c.dPsi;
      clear_desc(d);
      d.A = c.L1; d.B = c.Xt; d.C = c.Psi;
      d.M = rN; d.K = ca; d.N = 4 * k2 * r3;
      d.lda = nN; d.ldb = 4 * k2 * r3; d.ldc = 8 * k2 * r3;
      d.nbatch = 2; d.sA = ca; d.sB = 0; d.sC = (long long)4 * k2 * r3;
    }
    {  // Hin[x][x'] = sum_{alpha beta} conj(Psi[alpha][x][beta]) Psi[alpha][x'][beta]
      GemmDesc& d = *c.dHin;
      void* C = d.C;
      const long long ss = d.sSplit;
      clear_desc(d);
      d.C = C; d.sSplit = ss;
      if (c.m <= 1) {
        d.active = 0;
      } else {
        d.A = c.Psi; d.B = c.Psi; d.opA = OP_C; d.opB = OP_T;
        d.M = d.N = 8 * k2;
        d.K = rN * r3;
        d.lda = d.ldb = r3;
        d.kinner = r3;
        d.kstride = (long long)8 * k2 * r3;
        d.ldc = 8 * k2;
        d.splits = splitsH;
      }
    }
  }
}

// Gamma[(k j),(k' j')] = sum_{t,t'} Omega_{jj'}[t,t'] Hin[x(t,k)][x(t',k')],
// Omega_{jj'} = G_j^H G_j' (the 8 x 8 blocks of one (j, j') pair per block),
// x(t, k) = ((t1 2 + t2) k2 + k) 2 + t3.
template <typename T>
__global__ __launch_bounds__(GT) void k_q3_gamma(Ctx3<T>* ctxs) {
  __shared__ cpx<double> sOm[64];
  Ctx3<T>& c = ctxs[blockIdx.y];
  const int m = c.m, k2 = *c.kap2, n = k2 * m;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    EigDesc& d = *c.eG;
    d.a = c.Gam; d.lda = n; d.n = n; d.evals = c.evG; d.evecs = c.vecG; d.trace = c.evG + n;
    d.active = m > 1 ? 1 : 0;
  }
  if (m <= 1 || (int)blockIdx.x >= m * m) return;
  const int j = blockIdx.x / m, j2 = blockIdx.x % m;
  if (threadIdx.x < 64) {
    const int t = threadIdx.x / 8, t2 = threadIdx.x % 8;
    cpx<double> om = mk(0.0, 0.0);
    for (int s = 0; s < 8; ++s) om = om + cconj(ld(c.G, j * 64 + s * 8 + t)) * ld(c.G, j2 * 64 + s * 8 + t2);
    sOm[threadIdx.x] = om;
  }
  __syncthreads();
  const int nh = 8 * k2;
  for (int e = threadIdx.x; e < k2 * k2; e += blockDim.x) {
    const int kk = e / k2, kk2 = e % k2;
    cpx<double> acc = mk(0.0, 0.0);
    for (int t = 0; t < 8; ++t) {
      const int xa = (((t >> 2) * 2 + ((t >> 1) & 1)) * k2 + kk) * 2 + (t & 1);
      for (int t2 = 0; t2 < 8; ++t2) {
        const int xb = (((t2 >> 2) * 2 + ((t2 >> 1) & 1)) * k2 + kk2) * 2 + (t2 & 1);
        acc = acc + sOm[t * 8 + t2] * ld(c.Hin, (long long)xa * nh + xb);
      }
    }
    st(c.Gam, (long long)(kk * m + j) * n + (kk2 * m + j2), acc);
  }
}

// kappa' (Eqs. (10)-(11)) and Qop[(s1 s2 nu s3), (t1 t2 k t3)] =
// sum_j G_j[s, t] V[(k j), nu] / sqrt(kept); descriptors of Psi2 and C1.
template <typename T>
__global__ __launch_bounds__(GT) void k_q3_sel_h(Ctx3<T>* ctxs, int splitsC, TruncParams tp) {
  __shared__ int s_kp;
  __shared__ double s_scale;
  Ctx3<T>& c = ctxs[blockIdx.x];
  const int m = c.m, k2 = *c.kap2, n = k2 * m;
  const int rN = c.scratch[1], r3 = c.scratch[2];
  if (threadIdx.x == 0) {
    if (m <= 1) {
      s_kp = k2;
      s_scale = 1.0;
    } else {
      double kept, tot;
      const int kp = select_rank(c.evG, min(n, tp.kap_max + 1), n, c.evG[n], tp.kap_max, tp.kap_cut, &kept, &tot);
      s_kp = kp;
      s_scale = 1.0 / sqrt(kept);
      record_cut(c.disc, c.evG, kp, min(n, tp.kap_max + 1), tot, kept);
    }
    c.scratch[0] = s_kp;
  }
  __syncthreads();
  const int kp = s_kp;
  const double sc = s_scale;
  const int rows = 8 * kp, cols = 8 * k2;
  for (int e = threadIdx.x; e < rows * cols; e += blockDim.x) {
    const int row = e / cols, col = e % cols;
    const int s1 = row / (4 * kp), s2 = (row / (2 * kp)) % 2, nu = (row / 2) % kp, s3 = row % 2;
    const int t1 = col / (4 * k2), t2 = (col / (2 * k2)) % 2, kk = (col / 2) % k2, t3 = col % 2;
    const int gs = s1 * 4 + s2 * 2 + s3, gt = t1 * 4 + t2 * 2 + t3;
    cpx<double> acc = mk(0.0, 0.0);
    if (m <= 1) {
      if (nu == kk) acc = ld(c.G, gs * 8 + gt);
    } else {
      for (int j = 0; j < m; ++j)
        acc = acc + ld(c.G, j * 64 + gs * 8 + gt) * ld(c.vecG, (long long)(kk * m + j) * n + nu);
    }
    c.Qop[e] = mk<T>((T)(sc * acc.re), (T)(sc * acc.im));
  }
  if (threadIdx.x == 0) {
    {  // Psi2[alpha] = Qop Psi[alpha]
      GemmDesc& d = *c.dPsi2;
      clear_desc(d);
      d.A = c.Qop; d.B = c.Psi; d.C = c.Psi2;
      d.M = rows; d.K = cols; d.N = r3;
      d.lda = cols; d.ldb = r3; d.ldc = r3;
      d.nbatch = rN; d.sA = 0; d.sB = (long long)cols * r3; d.sC = (long long)rows * r3;
    }
    {  // C1 = Psi2 Psi2^H over rows (alpha s1)
      GemmDesc& d = *c.dC1;
      void* C = d.C;
      const long long ss = d.sSplit;
      clear_desc(d);
      d.C = C; d.sSplit = ss;
      d.A = c.Psi2; d.B = c.Psi2; d.opA = OP_N; d.opB = OP_H;
      d.M = d.N = 2 * rN;
      d.K = 4 * kp * r3;
      d.lda = d.ldb = 4 * kp * r3;
      d.ldc = 2 * rN;
      d.splits = splitsC;
      d.herm = 1;
    }
    EigDesc& e = *c.e1;
    e.lda = 2 * rN; e.n = 2 * rN; e.evals = c.ev1; e.evecs = c.vec1; e.trace = c.ev1 + 2 * rN; e.active = 1;
    e.upper = 1;
  }
}

// bond i: rank r1, weights, U1 and U1 S1 / sqrt(kept); descriptors of
// Y1 = P D^-1/2 U1 S1 / sqrt(kept) (FP64), W1 = U1^H Psi2 / sqrt(kept),
// BiP = Bp Y1 and C2 = W1^H W1 over rows (r1 s2 nu).
template <typename T>
__global__ __launch_bounds__(GT) void k_q3_sel_1(Ctx3<T>* ctxs, int splitsC, TruncParams tp) {
  __shared__ int s_r;
  __shared__ double s_kept;
  Ctx3<T>& c = ctxs[blockIdx.x];
  const int cl = *c.chil, ca = *c.chim1, k1 = *c.kap1;
  const int kp = c.scratch[0], rN = c.scratch[1], r3 = c.scratch[2];
  const int n = 2 * rN;
  if (threadIdx.x == 0) {
    double kept, tot;
    const int r = select_rank(c.ev1, min(n, tp.chi_max + 1), n, c.ev1[n], tp.chi_max, tp.svd_cut, &kept, &tot);
    s_r = r;
    s_kept = kept;
    record_cut(c.disc, c.ev1, r, min(n, tp.chi_max + 1), tot, kept);
    c.scratch[3] = r;
    c.kept[0] = kept;
  }
  __syncthreads();
  const int r = s_r;
  const double kept = s_kept, isk = 1.0 / sqrt(kept);
  for (int v = threadIdx.x; v < r; v += blockDim.x) {
    const double e = c.ev1[v] > 0 ? c.ev1[v] : 0.0;
    c.lam1[v] = sqrt(e / kept);
    c.lam1sq[v] = e / kept;
  }
  for (int e = threadIdx.x; e < n * r; e += blockDim.x) {
    const int x = e / r, rho = e % r;
    const cpx<double> u = ld(c.vec1, (long long)x * n + rho);
    const double g = sqrt(c.ev1[rho] > 0 ? c.ev1[rho] : 0.0) * isk;
    c.U1[e] = mk<T>((T)u.re, (T)u.im);
    st(c.U1s, e, mk(u.re * g, u.im * g));
  }
  if (threadIdx.x == 0) {
    {  // Y1[(t1 a), (s1 rho)] = sum_alpha PND[(t1 a), alpha] U1s[(alpha s1), rho]
      GemmDesc& d = *c.dY1;
      clear_desc(d);
      d.A = c.PND; d.B = c.U1s; d.C = c.Y1;
      d.M = 2 * ca; d.K = rN; d.N = 2 * r;
      d.lda = rN; d.ldb = 2 * r; d.ldc = 2 * r;
    }
    {  // W1 = U1^H Psi2 / sqrt(kept)
      GemmDesc& d = *c.dW1;
      clear_desc(d);
      d.A = c.U1; d.B = c.Psi2; d.C = c.W1;
      d.opA = OP_H;
      d.M = r; d.K = n; d.N = 4 * kp * r3;
      d.lda = r; d.ldb = 4 * kp * r3; d.ldc = 4 * kp * r3;
      d.alpha = isk;
    }
    {  // BiP[(l k1), (s1 rho)] = Bp Y1
      GemmDesc& d = *c.dBiP;
      clear_desc(d);
      d.A = c.Bp; d.B = c.Y1; d.C = c.BiP;
      d.M = cl * k1; d.K = 2 * ca; d.N = 2 * r;
      d.lda = 2 * ca; d.ldb = 2 * r; d.ldc = 2 * r;
    }
    {  // C2[(s3 beta), (s3' beta')] = sum_{(rho s2 nu)} conj(W1) W1
      GemmDesc& d = *c.dC2;
      void* C = d.C;
      const long long ss = d.sSplit;
      clear_desc(d);
      d.C = C; d.sSplit = ss;
      d.A = c.W1; d.B = c.W1; d.opA = OP_H; d.opB = OP_N;
      d.M = d.N = 2 * r3;
      d.K = r * 2 * kp;
      d.lda = d.ldb = 2 * r3;
      d.ldc = 2 * r3;
      d.splits = splitsC;
      d.herm = 1;
    }
    EigDesc& e = *c.e2;
    e.lda = 2 * r3; e.n = 2 * r3; e.evals = c.ev2; e.evecs = c.vec2; e.trace = c.ev2 + 2 * r3; e.active = 1;
    e.upper = 1;
  }
}

// B_i'[l, s1, k1, rho] = BiP[(l k1), (s1 rho)]
template <typename T>
__global__ __launch_bounds__(GT) void k_q3_perm_out(Ctx3<T>* ctxs) {
  Ctx3<T>& c = ctxs[blockIdx.y];
  const int cl = *c.chil, k1 = *c.kap1, r = c.scratch[3];
  const long long total = (long long)cl * 2 * k1 * r;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int rho = (int)(e % r);
    long long rest = e / r;
    const int kk = (int)(rest % k1);
    rest /= k1;
    const int s1 = (int)(rest % 2);
    const int l = (int)(rest / 2);
    c.Bi_new[e] = c.BiP[(((long long)l * k1 + kk) * 2 + s1) * r + rho];
  }
}

// bond i+1: rank r2, weights, Z2; descriptors of Y3 = Z2^H (P3 D3^-1/2)^H
// (FP64), B_{i+2}' = Y3 F and B_{i+1}' = W1 Z2 / sqrt(kept) (rows rescaled by
// 1 / lambda' afterwards).
template <typename T>
__global__ __launch_bounds__(GT) void k_q3_sel_2(Ctx3<T>* ctxs, TruncParams tp) {
  __shared__ int s_r;
  __shared__ double s_kept;
  Ctx3<T>& c = ctxs[blockIdx.x];
  const int cb = *c.chim2, cr = *c.chir, k3 = *c.kap3;
  const int kp = c.scratch[0], r3 = c.scratch[2], r1 = c.scratch[3];
  const int n = 2 * r3;
  if (threadIdx.x == 0) {
    double kept, tot;
    const int r = select_rank(c.ev2, min(n, tp.chi_max + 1), n, c.ev2[n], tp.chi_max, tp.svd_cut, &kept, &tot);
    s_r = r;
    s_kept = kept;
    record_cut(c.disc, c.ev2, r, min(n, tp.chi_max + 1), tot, kept);
    c.scratch[4] = r;
    c.kept[1] = kept;
  }
  __syncthreads();
  const int r = s_r;
  const double kept = s_kept;
  for (int v = threadIdx.x; v < r; v += blockDim.x) {
    const double e = c.ev2[v] > 0 ? c.ev2[v] : 0.0;
    c.lam2[v] = sqrt(e / kept);
    c.lam2sq[v] = e / kept;
  }
  // Zt3[(rho s3), beta] = conj(Z2[(s3 beta), rho]),  Z2c = Z2[:, :r]
  for (int e = threadIdx.x; e < 2 * r * r3; e += blockDim.x) {
    const int row = e / r3, be = e % r3;
    const int rho = row / 2, s3 = row % 2;
    st(c.Zt3, e, cconj(ld(c.vec2, (long long)(s3 * r3 + be) * n + rho)));
  }
  for (int e = threadIdx.x; e < n * r; e += blockDim.x) {
    const int y = e / r, rho = e % r;
    const cpx<double> z = ld(c.vec2, (long long)y * n + rho);
    c.Z2c[e] = mk<T>((T)z.re, (T)z.im);
  }
  if (threadIdx.x == 0) {
    {  // Y3[(rho s3), (b t3)] = sum_beta Zt3[(rho s3), beta] conj(PD3[(b t3), beta])
      GemmDesc& d = *c.dY3;
      clear_desc(d);
      d.A = c.Zt3; d.B = c.PD3; d.C = c.Y3;
      d.opB = OP_H;
      d.M = 2 * r; d.K = r3; d.N = 2 * cb;
      d.lda = r3; d.ldb = r3; d.ldc = 2 * cb;
    }
    {  // B_{i+2}'[(rho s3), (k3 r)] = Y3 F
      GemmDesc& d = *c.dBk;
      clear_desc(d);
      d.A = c.Y3; d.B = c.Bk; d.C = c.Bk_new;
      d.M = 2 * r; d.K = 2 * cb; d.N = k3 * cr;
      d.lda = 2 * cb; d.ldb = k3 * cr; d.ldc = k3 * cr;
    }
    {  // B_{i+1}'[(rho1 s2 nu), rho] = W1[(rho1 s2 nu), (s3 beta)] Z2[(s3 beta), rho] / sqrt(kept)
      GemmDesc& d = *c.dBj;
      clear_desc(d);
      d.A = c.W1; d.B = c.Z2c; d.C = c.Bj_new;
      d.M = r1 * 2 * kp; d.K = n; d.N = r;
      d.lda = n; d.ldb = r; d.ldc = r;
      d.alpha = 1.0 / sqrt(kept);
    }
  }
}

// B_{i+1}' rows (rho1, s2, nu) divided by lambda'_rho1; the new dimensions.
template <typename T>
__global__ __launch_bounds__(GT) void k_q3_finish(Ctx3<T>* ctxs) {
  Ctx3<T>& c = ctxs[blockIdx.y];
  const int kp = c.scratch[0], r1 = c.scratch[3], r2 = c.scratch[4];
  const long long row = 2LL * kp * r2;
  const long long total = (long long)r1 * row;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const double f = 1.0 / c.lam1[e / row];
    const cpx<T> v = c.Bj_new[e];
    c.Bj_new[e] = mk<T>((T)(v.re * f), (T)(v.im * f));
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *c.chim1 = r1;
    *c.chim2 = r2;
    *c.kap2 = kp;
  }
}

// ============================================================================
// truncation sweep (Sec. II.D)
// ============================================================================
template <typename T>
__global__ __launch_bounds__(GT) void k_sw_prepare(CtxS<T>* ctxs, int splits) {
  CtxS<T>& c = ctxs[blockIdx.x];
  if (threadIdx.x != 0) return;
  const int l = *c.chil, k = *c.kap, r = *c.chir;
  GemmDesc& d = *c.dG;
  void* C = d.C;
  const long long ss = d.sSplit;
  clear_desc(d);
  d.C = C; d.sSplit = ss;
  d.A = c.A; d.B = c.A;
  d.splits = splits;
  int n;
  if (c.pass == 0) {  // A^H A over rows (l s k): r x r
    n = r;
    d.opA = OP_H; d.opB = OP_N;
    d.M = d.N = r; d.K = l * 2 * k;
    d.lda = d.ldb = r;
  } else {            // A A^H over columns (s k r): l x l
    n = l;
    d.opA = OP_N; d.opB = OP_H;
    d.M = d.N = l; d.K = 2 * k * r;
    d.lda = d.ldb = 2 * k * r;
  }
  d.ldc = n;
  d.herm = 1;
  EigDesc& e = *c.dE;  // a, work and kvec are set by the host (a = the reduced Gram)
  e.lda = n; e.n = n; e.evals = c.ev; e.evecs = c.evec; e.trace = c.ev + n; e.active = 1; e.upper = 1;
}

template <typename T>
__global__ __launch_bounds__(GT) void k_sw_select(CtxS<T>* ctxs, TruncParams tp) {
  __shared__ int s_r;
  __shared__ double s_kept;
  CtxS<T>& c = ctxs[blockIdx.x];
  const int l = *c.chil, k = *c.kap, r = *c.chir;
  const int n = c.pass == 0 ? r : l;
  if (threadIdx.x == 0) {
    if (c.pass == 0) {
      int rr = 0;
      while (rr < n && c.ev[rr] > EIG_FLOOR * c.ev[0] && c.ev[0] > 0) ++rr;
      s_r = rr < 1 ? 1 : rr;
      check_basis(c.disc, c.ev[n]);
      s_kept = 1.0;
    } else {
      double kept, tot;
      const int rr = select_rank(c.ev, min(n, tp.chi_max + 1), n, c.ev[n], tp.chi_max, tp.svd_cut, &kept, &tot);
      s_r = rr;
      s_kept = kept;
      record_cut(c.disc, c.ev, rr, min(n, tp.chi_max + 1), tot, kept);
    }
  }
  __syncthreads();
  const int rr = s_r;
  const double kept = s_kept;
  // P1 (n x rr): V / sqrt(D);  P2: pass 0 (rr x n) sqrt(D) V^H, pass 1 (n x rr) U sqrt(S^2)
  for (int e = threadIdx.x; e < n * rr; e += blockDim.x) {
    const int a = e / rr, b = e % rr;
    const cpx<double> v = ld(c.evec, (long long)a * n + b);
    const double dv = c.ev[b] > 0 ? c.ev[b] : 0.0;
    const double sq = sqrt(dv), is = sq > 0 ? 1.0 / sq : 0.0;
    c.P1[e] = mk<T>((T)(v.re * is), (T)(v.im * is));
    if (c.pass == 0) {
      c.P2[(long long)b * n + a] = mk<T>((T)(v.re * sq), (T)(-v.im * sq));
    } else {
      c.P2[e] = mk<T>((T)(v.re * sq), (T)(v.im * sq));
    }
  }
  if (c.pass == 1) {
    for (int v = threadIdx.x; v < rr; v += blockDim.x) {
      const double e = c.ev[v] > 0 ? c.ev[v] : 0.0;
      c.lam[v] = sqrt(e / kept);
      c.lam2[v] = e / kept;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int o = *c.chio, kn = *c.kapn;
    GemmDesc& a = *c.dA;
    GemmDesc& b = *c.dB;
    clear_desc(a);
    clear_desc(b);
    if (c.pass == 0) {
      // T_i <- A P1: (l s k) x r times r x rr
      a.A = c.A; a.B = c.P1; a.C = c.Anew;
      a.M = l * 2 * k; a.K = r; a.N = rr;
      a.lda = r; a.ldb = rr; a.ldc = rr;
      // T_{i+1} <- P2 T_{i+1}: rr x r times r x (s kn o)
      b.A = c.P2; b.B = c.Bn; b.C = c.Bnnew;
      b.M = rr; b.K = r; b.N = 2 * kn * o;
      b.lda = r; b.ldb = 2 * kn * o; b.ldc = 2 * kn * o;
    } else {
      // T_i <- P1^H A: rr x l times l x (s k r)
      a.A = c.P1; a.B = c.A; a.C = c.Anew;
      a.opA = OP_H;
      a.M = rr; a.K = l; a.N = 2 * k * r;
      a.lda = rr; a.ldb = 2 * k * r; a.ldc = 2 * k * r;
      // T_{i-1} <- T_{i-1} P2: (o s kn) x l times l x rr
      b.A = c.Bn; b.B = c.P2; b.C = c.Bnnew;
      b.M = o * 2 * kn; b.K = l; b.N = rr;
      b.lda = l; b.ldb = rr; b.ldc = rr;
    }
    *c.chib = rr;
  }
}

template <typename T>
__global__ __launch_bounds__(GT) void k_sw_normalize(CtxS<T>* ctxs) {
  __shared__ double red[GT / 64];
  CtxS<T>& c = ctxs[blockIdx.x];
  const long long cnt = (long long)(*c.chil) * 2 * (*c.kap) * (*c.chir);
  double s = 0;
  for (long long e = threadIdx.x; e < cnt; e += blockDim.x) {
    const cpx<T> v = c.Anew[e];
    s += (double)v.re * v.re + (double)v.im * v.im;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  double tot = 0;
  for (int i = 0; i < GT / 64; ++i) tot += red[i];
  const double sc = tot > 0 ? 1.0 / sqrt(tot) : 1.0;
  for (long long e = threadIdx.x; e < cnt; e += blockDim.x) {
    const cpx<T> v = c.Anew[e];
    c.Anew[e] = mk<T>((T)(v.re * sc), (T)(v.im * sc));
  }
}

// ============================================================================
// transfer matrices
// ============================================================================
template <typename T>
__global__ void k_transfer_init(CtxT<T>* ctxs) {
  CtxT<T>& c = ctxs[blockIdx.x];
  if (threadIdx.x == 0) c.Ecur[0] = mk<T>((T)1, (T)0);
}

// BO[l,s',k,r] = sum_s O[s',s] B[l,s,k,r] (B itself when O is the identity); descriptors of Y = E^T BO and
// E' = Y^T conj(B).
template <typename T>
__global__ void k_transfer_prep(CtxT<T>* ctxs) {
  CtxT<T>& c = ctxs[blockIdx.y];
  if (!c.active) {
    if (blockIdx.x == 0 && threadIdx.x == 0) { c.d1->active = 0; c.d2->active = 0; }
    return;
  }
  const int cl = *c.chil, cr = *c.chir, k = *c.kap;
  const double* O = c.ops + 8 * c.site;
  const cpx<T> o00 = mk<T>((T)O[0], (T)O[1]), o01 = mk<T>((T)O[2], (T)O[3]);
  const cpx<T> o10 = mk<T>((T)O[4], (T)O[5]), o11 = mk<T>((T)O[6], (T)O[7]);
  const long long half = (long long)k * cr;
  // an identity factor leaves B as it is: the product reads B itself
  const bool ident = O[0] == 1.0 && O[1] == 0.0 && O[2] == 0.0 && O[3] == 0.0 && O[4] == 0.0 && O[5] == 0.0 &&
                     O[6] == 1.0 && O[7] == 0.0;
  const long long total = ident ? 0 : (long long)cl * half;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long l = e / half, rest = e % half;
    const cpx<T> b0 = c.B[l * 2 * half + rest], b1 = c.B[l * 2 * half + half + rest];
    c.BO[l * 2 * half + rest] = o00 * b0 + o01 * b1;
    c.BO[l * 2 * half + half + rest] = o10 * b0 + o11 * b1;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    GemmDesc& d1 = *c.d1;
    clear_desc(d1);
    d1.A = c.Ecur; d1.B = ident ? c.B : c.BO; d1.C = c.Y;
    d1.opA = OP_T;
    d1.M = cl; d1.K = cl; d1.N = 2 * k * cr;
    d1.lda = cl; d1.ldb = 2 * k * cr; d1.ldc = 2 * k * cr;
    GemmDesc& d2 = *c.d2;
    clear_desc(d2);
    d2.A = c.Y; d2.B = c.B; d2.C = c.Enext;
    d2.opA = OP_T; d2.opB = OP_C;
    d2.M = cr; d2.K = cl * 2 * k; d2.N = cr;
    d2.lda = cr; d2.ldb = cr; d2.ldc = cr;
  }
}

// Descriptors of one right-environment step (one thread per instance).
template <typename T>
__global__ void k_rtransfer_prep(CtxR<T>* ctxs, int n) {
  const int it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= n) return;
  CtxR<T>& c = ctxs[it];
  if (!c.active) {
    c.d3->active = 0;
    c.d4->active = 0;
    return;
  }
  if (c.last) c.Rn[0] = mk<T>((T)1, (T)0);
  const int cl = *c.chil, cr = *c.chir, k = *c.kap;
  GemmDesc& d3 = *c.d3;  // W = conj(B) R_{s+1}^T, (cl 2k) x cr
  clear_desc(d3);
  d3.A = c.B; d3.B = c.Rn; d3.C = c.W;
  d3.opA = OP_C; d3.opB = OP_T;
  d3.M = cl * 2 * k; d3.K = cr; d3.N = cr;
  d3.lda = cr; d3.ldb = cr; d3.ldc = cr;
  GemmDesc& d4 = *c.d4;  // R_s = B W^T over (s k r), cl x cl
  clear_desc(d4);
  d4.A = c.B; d4.B = c.W; d4.C = c.Rs;
  d4.opA = OP_N; d4.opB = OP_T;
  d4.M = cl; d4.K = 2 * k * cr; d4.N = cl;
  d4.lda = 2 * k * cr; d4.ldb = 2 * k * cr; d4.ldc = cl;
}

// out[item] = <E_item, R_item> / E_trace (complex): the left environment
// after the item's last non-identity site contracted with the right
// environment of the same bond (E itself when that bond is the last); the
// trace item of each instance is the identity string.
template <typename T>
__global__ __launch_bounds__(256) void k_transfer_finish(CtxT<T>* ctxs, double* out) {
  __shared__ double sre[256], sim[256];
  const int it = blockIdx.x;
  const CtxT<T>& c = ctxs[it];
  double a, b;
  if (!c.Rfin) {
    a = (double)c.Efinal[0].re;
    b = (double)c.Efinal[0].im;
  } else {
    const int ch = *c.chif;
    double pr = 0, pi = 0;
    for (int e = threadIdx.x; e < ch * ch; e += blockDim.x) {
      const cpx<T> x = c.Efinal[e], y = c.Rfin[e];
      pr += (double)x.re * (double)y.re - (double)x.im * (double)y.im;
      pi += (double)x.re * (double)y.im + (double)x.im * (double)y.re;
    }
    sre[threadIdx.x] = pr;
    sim[threadIdx.x] = pi;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) {
        sre[threadIdx.x] += sre[threadIdx.x + h];
        sim[threadIdx.x] += sim[threadIdx.x + h];
      }
      __syncthreads();
    }
    a = sre[0];
    b = sim[0];
  }
  if (threadIdx.x == 0) {
    if (c.stat && !(a > 0 && a < 1e300)) c.stat[ST_FAIL] += 1.0;  // trace item (NaN fails too)
    double ta = 1.0;  // trace_idx < 0: raw value
    if (c.trace_idx >= 0) ta = (double)ctxs[c.trace_idx].Efinal[0].re;
    out[2 * it] = a / ta;
    out[2 * it + 1] = b / ta;
  }
}

// ============================================================================
// channels: chi -> Lambda -> Kraus
// ============================================================================
__device__ inline cpx<double> pauli_entry(int m, int a, int b, int q) {
  cpx<double> v = mk(1.0, 0.0);
  for (int t = 0; t < q; ++t) {
    const int sh = q - 1 - t;
    const int mt = (m >> (2 * sh)) & 3, at = (a >> sh) & 1, bt = (b >> sh) & 1;
    cpx<double> e;
    switch (mt) {
      case 0: e = mk(at == bt ? 1.0 : 0.0, 0.0); break;
      case 1: e = mk(at != bt ? 1.0 : 0.0, 0.0); break;
      case 2: e = (at == bt) ? mk(0.0, 0.0) : (at == 0 ? mk(0.0, -1.0) : mk(0.0, 1.0)); break;
      default: e = mk(at == bt ? (at == 0 ? 1.0 : -1.0) : 0.0, 0.0); break;
    }
    v = v * e;
  }
  return v;
}

// Lambda[(a b),(c e)] = sum_mn chi_mn sigma_m[a][b] conj(sigma_n[c][e])
__global__ void k_choi(const double* chi, int q, double* lam) {
  const int d = 1 << q, d2 = d * d;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < d2 * d2; e += gridDim.x * blockDim.x) {
    const int x = e / d2, y = e % d2;
    const int a = x / d, b = x % d, c2 = y / d, e2 = y % d;
    cpx<double> acc = mk(0.0, 0.0);
    for (int m = 0; m < d2; ++m) {
      const cpx<double> pm = pauli_entry(m, a, b, q);
      if (pm.re == 0 && pm.im == 0) continue;
      for (int n = 0; n < d2; ++n) {
        const cpx<double> pn = pauli_entry(n, c2, e2, q);
        if (pn.re == 0 && pn.im == 0) continue;
        acc = acc + (ld(chi, (long long)m * d2 + n) * pm) * cconj(pn);
      }
    }
    st(lam, e, acc);
  }
}

// K_i = sqrt(eta_i) unvec(psi_i) for the eta_i above rank_tol * eta_0 and of
// weight >= eps.  info: [0] = kept count, [1] = completeness error of the
// unpruned set, [2] = smallest eigenvalue, [3] = rank.
__global__ void k_kraus_extract(const double* evals, const double* evecs, int q, double eps, double rank_tol,
                                double* kraus, double* info) {
  __shared__ int s_keep[64];
  __shared__ int s_nk, s_rank;
  __shared__ double s_err;
  const int d = 1 << q, d2 = d * d;
  if (threadIdx.x == 0) {
    double tot = 0;
    const double e0 = evals[0];
    int rank = 0;
    for (int i = 0; i < d2; ++i)
      if (evals[i] > rank_tol * e0 && evals[i] > 0) { tot += evals[i]; ++rank; }
    int nk = 0;
    for (int i = 0; i < d2; ++i) {
      if (!(evals[i] > rank_tol * e0 && evals[i] > 0)) continue;
      if (evals[i] / tot < eps) continue;
      s_keep[nk++] = i;
    }
    s_nk = nk;
    s_rank = rank;
    s_err = 0;
  }
  __syncthreads();
  const int nk = s_nk;
  for (int e = threadIdx.x; e < nk * d2; e += blockDim.x) {
    const int kidx = e / d2, x = e % d2;
    const int i = s_keep[kidx];
    const double sq = sqrt(evals[i]);
    const cpx<double> p = ld(evecs, (long long)x * d2 + i);
    st(kraus, e, mk(sq * p.re, sq * p.im));
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // completeness of the full-rank set: sum_i eta_i A_i^dag A_i = I
    double err = 0;
    const double e0 = evals[0];
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) {
        cpx<double> acc = mk(0.0, 0.0);
        for (int i = 0; i < d2; ++i) {
          if (!(evals[i] > rank_tol * e0 && evals[i] > 0)) continue;
          for (int t = 0; t < d; ++t)
            acc = acc + evals[i] * (cconj(ld(evecs, (long long)(t * d + a) * d2 + i)) * ld(evecs, (long long)(t * d + b) * d2 + i));
        }
        if (a == b) acc.re -= 1.0;
        const double v = sqrt(cabs2(acc));
        err = v > err ? v : err;
      }
    info[0] = nk;
    info[1] = err;
    info[2] = evals[d2 - 1];
    info[3] = s_rank;
  }
}

template <typename T>
__global__ void k_copy(const cpx<T>* src, cpx<T>* dst, long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

// ============================================================================
// launch wrappers
// ============================================================================
template <typename T> void launch_q1_prepare(Ctx1<T>* d, int n, int splitsH, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_q1_prepare<T>, dim3(n), dim3(GT), 0, s, d, splitsH);
}
template <typename T> void launch_q1_gamma(Ctx1<T>* d, int n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_q1_gamma<T>, dim3(n), dim3(GT), 0, s, d);
}
template <typename T> void launch_q1_select(Ctx1<T>* d, int n, TruncParams tp, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_q1_select<T>, dim3(n), dim3(GT), 0, s, d, tp);
}
template <typename T> void launch_gram_v(const GemmDesc* d, int n, int splits, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_gram_v<T>, dim3(n * splits), dim3(GT), 0, s, d, splits);
}
template <typename T> void launch_q2_prepare(Ctx2<T>* d, int n, int splitsE, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_q2_prepare<T>, dim3(n), dim3(GT), 0, s, d, splitsE);
}
template <typename T> void launch_q2_select_e(Ctx2<T>* d, int n, int splitsH, TruncParams tp, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_q2_select_e<T>, dim3(n), dim3(GT), 0, s, d, splitsH, tp);
}
template <typename T>
void launch_q2_chol_e(Ctx2<T>* d, int n, int maxn, int splitsH, TruncParams tp, const EigDesc* d_eig,
                      hipStream_t s) {
  if (n <= 0) return;
  const int tok = prof_begin(PC_CHOL_E, s);
  if (maxn <= CH_NC)
    hipLaunchKernelGGL(k_q2_chol_e<T>, dim3(n), dim3(CH_NT), 0, s, d, splitsH, tp);
  else
    hipLaunchKernelGGL(k_q2_chol_e_g<T>, dim3(n), dim3(CG_NT), 0, s, d, splitsH, tp);
  prof_end_chol(tok, PC_CHOL_E, d_eig, n, s);
}

namespace {
bool g_e_chol = true;
bool g_gram_vec = true;
}
void set_e_cholesky(bool on) { g_e_chol = on; }
bool e_cholesky() { return g_e_chol; }
void set_gram_vector(bool on) { g_gram_vec = on; }
bool gram_vector() { return g_gram_vec; }
template <typename T> void launch_q2_gamma(Ctx2<T>* d, int n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_q2_gamma<T>, dim3(n, 4), dim3(GT), 0, s, d);
}
template <typename T> void launch_q2_select_g(Ctx2<T>* d, int n, int splitsC, TruncParams tp, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_q2_select_g<T>, dim3(n), dim3(GT), 0, s, d, splitsC, tp);
}
template <typename T> void launch_q2_select_b(Ctx2<T>* d, int n, TruncParams tp, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_q2_select_b<T>, dim3(n), dim3(GT), 0, s, d, tp);
}
template <typename T> void launch_q3_prepare(Ctx3<T>* d, int n, int splitsN, int splitsE, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_q3_prepare<T>, dim3(n), dim3(GT), 0, s, d, splitsN, splitsE);
}
template <typename T> void launch_q3_perm_in(Ctx3<T>* d, int n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_q3_perm_in<T>, dim3(256, n), dim3(GT), 0, s, d);
}
template <typename T> void launch_q3_sel_env(Ctx3<T>* d, int n, int splitsH, double floor, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_q3_sel_env<T>, dim3(n), dim3(GT), 0, s, d, splitsH, floor);
}
template <typename T> void launch_q3_gamma(Ctx3<T>* d, int n, int mmax, hipStream_t s) {
  const int pairs = mmax > 1 ? mmax * mmax : 1;
  if (n > 0) hipLaunchKernelGGL(k_q3_gamma<T>, dim3(pairs, n), dim3(GT), 0, s, d);
}
template <typename T> void launch_q3_sel_h(Ctx3<T>* d, int n, int splitsC, TruncParams tp, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_q3_sel_h<T>, dim3(n), dim3(GT), 0, s, d, splitsC, tp);
}
template <typename T> void launch_q3_sel_1(Ctx3<T>* d, int n, int splitsC, TruncParams tp, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_q3_sel_1<T>, dim3(n), dim3(GT), 0, s, d, splitsC, tp);
}
template <typename T> void launch_q3_perm_out(Ctx3<T>* d, int n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_q3_perm_out<T>, dim3(256, n), dim3(GT), 0, s, d);
}
template <typename T> void launch_q3_sel_2(Ctx3<T>* d, int n, TruncParams tp, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_q3_sel_2<T>, dim3(n), dim3(GT), 0, s, d, tp);
}
template <typename T> void launch_q3_finish(Ctx3<T>* d, int n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_q3_finish<T>, dim3(128, n), dim3(GT), 0, s, d);
}
template <typename T> void launch_sw_prepare(CtxS<T>* d, int n, int splits, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_sw_prepare<T>, dim3(n), dim3(GT), 0, s, d, splits);
}
template <typename T> void launch_sw_select(CtxS<T>* d, int n, TruncParams tp, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_sw_select<T>, dim3(n), dim3(GT), 0, s, d, tp);
}
template <typename T> void launch_sw_normalize(CtxS<T>* d, int n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_sw_normalize<T>, dim3(n), dim3(GT), 0, s, d);
}
template <typename T> void launch_transfer_init(CtxT<T>* d, int n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_transfer_init<T>, dim3(n), dim3(64), 0, s, d);
}
template <typename T> void launch_transfer_prep(CtxT<T>* d, int n, int maxElems, hipStream_t s) {
  if (n <= 0) return;
  int bx = (maxElems + 255) / 256;
  if (bx < 1) bx = 1;
  if (bx > 64) bx = 64;
  hipLaunchKernelGGL(k_transfer_prep<T>, dim3(bx, n), dim3(256), 0, s, d);
}
template <typename T> void launch_transfer_finish(CtxT<T>* d, int n, double* out, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_transfer_finish<T>, dim3(n), dim3(256), 0, s, d, out);
}
template <typename T> void launch_rtransfer_prep(CtxR<T>* d, int n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_rtransfer_prep<T>, dim3((n + 63) / 64), dim3(64), 0, s, d, n);
}
void launch_choi(const double* chi, int q, double* lam, hipStream_t s) {
  hipLaunchKernelGGL(k_choi, dim3(16), dim3(256), 0, s, chi, q, lam);
}
void launch_kraus_extract(const double* evals, const double* evecs, int q, double eps, double rank_tol,
                          double* kraus, double* info, hipStream_t s) {
  hipLaunchKernelGGL(k_kraus_extract, dim3(1), dim3(256), 0, s, evals, evecs, q, eps, rank_tol, kraus, info);
}
template <typename T> void launch_copy_site(const cpx<T>* src, cpx<T>* dst, long long n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_copy<T>, dim3(256), dim3(256), 0, s, src, dst, n);
}

#define INST(T)                                                                               \
  template void launch_q1_prepare<T>(Ctx1<T>*, int, int, hipStream_t);                        \
  template void launch_q1_gamma<T>(Ctx1<T>*, int, hipStream_t);                               \
  template void launch_q1_select<T>(Ctx1<T>*, int, TruncParams, hipStream_t);                 \
  template void launch_gram_v<T>(const GemmDesc*, int, int, hipStream_t);                     \
  template void launch_q2_prepare<T>(Ctx2<T>*, int, int, hipStream_t);                        \
  template void launch_q2_select_e<T>(Ctx2<T>*, int, int, TruncParams, hipStream_t);          \
  template void launch_q2_chol_e<T>(Ctx2<T>*, int, int, int, TruncParams, const EigDesc*, hipStream_t); \
  template void launch_q2_gamma<T>(Ctx2<T>*, int, hipStream_t);                               \
  template void launch_q2_select_g<T>(Ctx2<T>*, int, int, TruncParams, hipStream_t);          \
  template void launch_q2_select_b<T>(Ctx2<T>*, int, TruncParams, hipStream_t);              \
  template void launch_q3_prepare<T>(Ctx3<T>*, int, int, int, hipStream_t);                   \
  template void launch_q3_perm_in<T>(Ctx3<T>*, int, hipStream_t);                             \
  template void launch_q3_sel_env<T>(Ctx3<T>*, int, int, double, hipStream_t);                \
  template void launch_q3_gamma<T>(Ctx3<T>*, int, int, hipStream_t);                          \
  template void launch_q3_sel_h<T>(Ctx3<T>*, int, int, TruncParams, hipStream_t);             \
  template void launch_q3_sel_1<T>(Ctx3<T>*, int, int, TruncParams, hipStream_t);             \
  template void launch_q3_perm_out<T>(Ctx3<T>*, int, hipStream_t);                            \
  template void launch_q3_sel_2<T>(Ctx3<T>*, int, TruncParams, hipStream_t);                  \
  template void launch_q3_finish<T>(Ctx3<T>*, int, hipStream_t);                              \
  template void launch_sw_prepare<T>(CtxS<T>*, int, int, hipStream_t);                        \
  template void launch_sw_select<T>(CtxS<T>*, int, TruncParams, hipStream_t);                 \
  template void launch_sw_normalize<T>(CtxS<T>*, int, hipStream_t);                           \
  template void launch_transfer_init<T>(CtxT<T>*, int, hipStream_t);                          \
  template void launch_transfer_prep<T>(CtxT<T>*, int, int, hipStream_t);                     \
  template void launch_transfer_finish<T>(CtxT<T>*, int, double*, hipStream_t);          \
  template void launch_rtransfer_prep<T>(CtxR<T>*, int, hipStream_t);                      \
  template void launch_copy_site<T>(const cpx<T>*, cpx<T>*, long long, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace mpdo
