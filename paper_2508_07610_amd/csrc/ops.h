// Per-item contexts of the MPDO update kernels and their launch wrappers.
#pragma once
#include "common.h"

namespace mpdo {

// How a kernel builds the ideal unitary of a gate: a fixed matrix or a
// rotation whose angle is scale * params[pidx] (scale alone if pidx < 0).
enum GateKind : int { GK_FIXED = 0, GK_RX = 1, GK_RY = 2, GK_RZ = 3, GK_ZZPHASE = 4, GK_SWAPZZ = 5 };

struct GateSrc {
  int kind, q, pidx, pad;
  double scale;
  const double* params;   // device, may be null
  const double* ufix;     // device, 2^q x 2^q complex (GK_FIXED; null = identity)
};

// One-site noisy gate: B'[l,s,(k j),r] = sum_t G_j[s,t] B[l,t,k,r], inner
// truncation from the lambda^2-weighted Gram matrix, projection.
template <typename T> struct Ctx1 {
  GateSrc g;
  const double* kraus;    // m x 2 x 2 complex (device) or null (m = 1)
  int m;
  int force;              // truncate the inner index even when m = 1
  const cpx<T>* Bold;
  cpx<T>* Bnew;
  const double* laml2;    // squared weights of the left bond
  const int* chil;
  const int* chir;
  int* kap;
  double* disc;           // the site's truncation record (StatField)
  double* G;              // m x 2 x 2 complex: G_j = K_j U
  double* H;              // (2k)^2 Gram over (l, r)
  double* Gam;            // (k m)^2
  double* ev;
  double* evec;
  cpx<T>* W;              // (2k') x (2k)
  GemmDesc* dH;
  EigDesc* dE;
  GemmDesc* dA;
};

// Two-site noisy gate on (i, i+1).
template <typename T> struct Ctx2 {
  GateSrc g;
  const double* kraus;    // m x 4 x 4 complex or null
  int m, pad;
  const cpx<T>* Bi;
  const cpx<T>* Bj;
  cpx<T>* Bi_new;
  cpx<T>* Bj_new;
  const double* laml2;    // squared weights of bond i-1
  double* lam;            // weights of bond i (output)
  double* lam2;
  const int* chil;
  int* chim;
  const int* chir;
  int* kap1;
  const int* kap2;
  double* disc;           // the site's truncation record (StatField)
  int* scratch;           // [0] = kappa', [1] = r_F
  double* G;              // m x 4 x 4
  double* H;              // (4 k1)^2
  double* E;              // (2 chim)^2
  double* Gam;            // (k1 m)^2
  double* evG; double* vecG;
  double* evE; double* vecE;
  double* evC; double* vecC;
  cpx<T>* W;              // (4 k') x (4 k1)
  cpx<T>* LF;             // (2 chim) x r_F
  double* PD;             // (2 chim) x r_F
  cpx<T>* th;             // (2 k1 chil) x (2 r_F)
  cpx<T>* th2;            // (2 k' chil) x (2 r_F)
  double* Cm;             // (2 r_F)^2
  double* Zt;             // (2 r) x r_F
  cpx<T>* Zc;             // (2 r_F) x r
  cpx<T>* X;              // (2 r) x (2 chim)
  GemmDesc* dGramE;       // E = F F^dag
  EigDesc* dEigE;
  GemmDesc* dGramH;       // H from th (lambda^2-weighted)
  EigDesc* dEigG;         // Gamma
  GemmDesc* dTh;
  GemmDesc* dTh2;
  GemmDesc* dC;
  EigDesc* dEigC;
  GemmDesc* dX;
  GemmDesc* dOut;         // 2: B_i, B_{i+1}
};

// Three-site noisy gate on (i, i+1, i+2), the Kraus index joining the inner
// index of the middle site.  The passive indices of the outer sites, (l k1)
// of site i (weighted by lambda_l) and (k3 r) of site i+2, are replaced by
// orthonormal bases of their spans, taken from the Gram eigendecompositions
//   N  = (Lambda B_i)^H (Lambda B_i) over (l k1), columns (t1 a):  P D P^H,
//   E3 = F F^H with F = B_{i+2} as [(b t3)] x [(k3 r)]:            P3 D3 P3^H,
// so that Lambda Psi = Q1 Psi^ Q3 with Q1, Q3 isometries and the reduced block
//   Psi^[alpha, (t1 t2 k2 t3), beta] = sum_a L1[alpha, (t1 a)] Xt[(a t2 k2), (t3 beta)],
//   L1 = sqrt(D) P^H,  Xt = B_{i+1} L3,  L3 = P3 sqrt(D3)
// (at most 2 chi_a x 8 kappa x 2 chi_b).  Every Gram matrix of the gate output
// is then a Gram matrix of the reduced block:
//   Hin = Gram of Psi^ over (alpha, beta) with the middle indices open -> Gamma
//         (fused operators, Eqs. (9)-(11)) -> kappa' and the operator Qop;
//   Psi2 = Qop Psi^;  C1 = Psi2 Psi2^H over rows (alpha s1): bond i, at most
//         4 chi; W1 = U1^H Psi2 / sqrt(kept) = lambda' V1;
//   C2 = W1^H W1 over columns (s3 beta): bond i+1, at most 4 chi.
// New tensors:  B_i' = Bp (P D^-1/2 U1 S1) / sqrt(kept1),
//   B_{i+1}' = lambda'^-1 W1 Z2 / sqrt(kept2),  B_{i+2}' = (Z2^H D3^-1/2 P3^H) F,
// the small factors in parentheses formed in FP64.
// N is weighted by lambda^2, so its spectrum spans that of the bond weights:
// its basis keeps every direction above this fraction of the largest
// eigenvalue (the factors P D^-1/2 and sqrt(D) P^H enter only as balanced
// products), where the Gram floor of the truncation rule would drop weight.
constexpr double Q3_BASIS_FLOOR = 1e-18;

template <typename T> struct Ctx3 {
  GateSrc g;
  const double* kraus;    // m x 8 x 8 complex or null
  int m, pad;
  const cpx<T>* Bi;
  const cpx<T>* Bj;
  const cpx<T>* Bk;
  cpx<T>* Bi_new;
  cpx<T>* Bj_new;
  cpx<T>* Bk_new;
  const double* laml2;    // squared weights of bond i-1
  double* lam1;           // weights of bond i (output)
  double* lam1sq;
  double* lam2;           // weights of bond i+1 (output)
  double* lam2sq;
  const int* chil;
  int* chim1;
  int* chim2;
  const int* chir;
  const int* kap1;
  int* kap2;
  const int* kap3;
  double* disc;           // the site's truncation record (StatField)
  int* scratch;           // [0] kappa', [1] r_N, [2] r_3, [3] bond i, [4] bond i+1
  double* kept;           // [0] kept weight at bond i, [1] at bond i+1
  double* G;              // m x 8 x 8
  cpx<T>* Bp;             // B_i as (l k1) x (t1 a)
  double* N;  double* evN;  double* vecN;
  double* E3; double* evE3; double* vecE3;
  cpx<T>* L1;             // r_N x (t1 a)
  double* PND;            // (t1 a) x r_N: P D^-1/2
  cpx<T>* L3;             // (b t3) x r_3
  double* PD3;            // (b t3) x r_3: P3 D3^-1/2
  cpx<T>* Xt;             // (a t2 k2) x (t3 beta)
  cpx<T>* Psi;            // alpha x (t1 t2 k2 t3) x beta
  double* Hin;            // (8 k2)^2
  double* Gam; double* evG; double* vecG;
  cpx<T>* Qop;            // (s1 s2 nu s3) x (t1 t2 k2 t3)
  cpx<T>* Psi2;           // alpha x (s1 s2 nu s3) x beta
  double* C1; double* ev1; double* vec1;
  cpx<T>* U1;             // (alpha s1) x r1
  double* U1s;            // (alpha s1) x r1, columns scaled by sqrt(eta / kept)
  cpx<T>* W1;             // r1 x (s2 nu s3 beta)
  cpx<T>* Y1;             // (t1 a) x (s1 r1)
  cpx<T>* BiP;            // (l k1) x (s1 r1)
  double* C2; double* ev2; double* vec2;
  double* Zt3;            // (r2 s3) x beta
  cpx<T>* Z2c;            // (s3 beta) x r2
  cpx<T>* Y3;             // (r2 s3) x (b t3)
  GemmDesc* dN; GemmDesc* dE3; GemmDesc* dXt; GemmDesc* dPsi; GemmDesc* dHin; GemmDesc* dPsi2;
  GemmDesc* dC1; GemmDesc* dY1; GemmDesc* dW1; GemmDesc* dBiP; GemmDesc* dC2; GemmDesc* dY3;
  GemmDesc* dBk; GemmDesc* dBj;
  EigDesc* eN; EigDesc* eE3; EigDesc* eG; EigDesc* e1; EigDesc* e2;
};

// One step of the truncation sweep (Sec. II.D) on one instance.
//  pass 0, left to right: A = T_i as (l s k) x r; A^H A = V D V^H on the
//    eigenvalues above the numerical floor; T_i <- A V D^(-1/2) (orthonormal
//    columns), T_{i+1} <- D^(1/2) V^H T_{i+1}.
//  pass 1, right to left: A = T_i as l x (s k r); A A^H = U S^2 U^H, rank r
//    by the truncation rule; T_i <- S^(-1) U_r^H A (orthonormal rows),
//    T_{i-1} <- T_{i-1} U_r S_r, bond weights S_r / sqrt(kept weight).
template <typename T> struct CtxS {
  int pass, pad;
  const cpx<T>* A;        // T_i
  cpx<T>* Anew;
  const cpx<T>* Bn;       // the neighbour: T_{i+1} (pass 0) or T_{i-1} (pass 1)
  cpx<T>* Bnnew;
  const int* chil;        // bonds and inner dimension of site i
  const int* chir;
  const int* kap;
  int* chib;              // the bond shared with the neighbour (rewritten)
  const int* chio;        // the neighbour's other bond
  const int* kapn;        // the neighbour's inner dimension
  double* lam;            // weights of the shared bond (pass 1)
  double* lam2;
  double* disc;           // the site's truncation record (StatField)
  double* ev;
  double* evec;
  cpx<T>* P1;             // pass 0: V D^(-1/2);  pass 1: U_r S_r^(-1)
  cpx<T>* P2;             // pass 0: D^(1/2) V^H; pass 1: U_r S_r
  GemmDesc* dG;
  EigDesc* dE;
  GemmDesc* dA;
  GemmDesc* dB;
};

// Transfer-matrix item: E'[r, r'] = sum E[l, l'] B[l,s,k,r] O[s',s] conj(B[l',s',k,r']).
template <typename T> struct CtxT {
  const double* ops;      // n x 2 x 2 complex of this item's product operator
  const cpx<T>* B;        // site tensor of the current step
  const int* chil;
  const int* chir;
  const int* kap;
  cpx<T>* Ecur;
  cpx<T>* Enext;
  cpx<T>* BO;
  cpx<T>* Y;
  cpx<T>* Efinal;         // the item's last left environment
  const cpx<T>* Rfin;     // right environment Efinal is contracted with (null: Efinal is 1 x 1)
  const int* chif;        // bond dimension of Efinal and Rfin
  GemmDesc* d1;
  GemmDesc* d2;
  double* stat;           // trace item: the instance's first site record (a
                          // non-finite or non-positive trace counts as a failure)
  int site, active, trace_idx, pad;
};

// Right environment R_s[l, l'] = sum B_s[l, x] W[l', x] with
// W[(l' s k), r] = sum_r' conj(B_s[(l' s k), r']) R_{s+1}[r, r'] (R_n = [1]).
template <typename T> struct CtxR {
  const cpx<T>* B;
  const int* chil;
  const int* chir;
  const int* kap;
  cpx<T>* Rn;  // R_{s+1}
  cpx<T>* Rs;  // R_s
  cpx<T>* W;
  GemmDesc* d3;
  GemmDesc* d4;
  int active, last;  // last: s is the last site (R_{s+1} = [1] is written here)
};

struct TruncParams {
  int chi_max, kap_max;
  double svd_cut, kap_cut;
  double tolE;            // relative eigenvalue floor of the right-factor Gram
};

template <typename T> void launch_q1_prepare(Ctx1<T>* d_ctx, int n, int splitsH, hipStream_t s);
template <typename T> void launch_q1_gamma(Ctx1<T>* d_ctx, int n, hipStream_t s);
template <typename T> void launch_q1_select(Ctx1<T>* d_ctx, int n, TruncParams tp, hipStream_t s);
// a weighted Gram (A = B, opA = OP_C, opB = OP_T, two-level K) with M = N <=
// GV_MAX = 32 on the vector units, split partials where the GEMM writes them
template <typename T> void launch_gram_v(const GemmDesc* d_descs, int n, int splits, hipStream_t s);

template <typename T> void launch_q2_prepare(Ctx2<T>* d_ctx, int n, int splitsE, hipStream_t s);
template <typename T> void launch_q2_select_e(Ctx2<T>* d_ctx, int n, int splitsH, TruncParams tp, hipStream_t s);
// The right-factor basis of the two-site update from a pivoted Cholesky
// factorisation of E instead of launch_eigh + launch_q2_select_e; maxn
// (= 2 chi_max) bounds E's size: up to 128 the matrix is held in LDS, up to
// 256 it is updated in place in global memory.  d_eig: the items' EigDesc of
// E (for the profiler).
template <typename T>
void launch_q2_chol_e(Ctx2<T>* d_ctx, int n, int maxn, int splitsH, TruncParams tp, const EigDesc* d_eig,
                      hipStream_t s);
// Process-wide choice of that route (default on).
void set_e_cholesky(bool on);
bool e_cholesky();
// the one- and two-site inner Grams on the vector units when their size
// (2 kappa_max, 4 kappa_max) is at most GV_ROWS (default on) rather than on
// the GEMM kernel: a 16 x 16 Gram fills a quarter of the 32 x 32 MFMA tile
// (vector units faster on the C2 step); a 32 x 32 one fills it (MFMA faster)
constexpr int GV_ROWS = 16;
void set_gram_vector(bool on);
bool gram_vector();
template <typename T> void launch_q2_gamma(Ctx2<T>* d_ctx, int n, hipStream_t s);
template <typename T> void launch_q2_select_g(Ctx2<T>* d_ctx, int n, int splitsC, TruncParams tp, hipStream_t s);
template <typename T> void launch_q2_select_b(Ctx2<T>* d_ctx, int n, TruncParams tp, hipStream_t s);

template <typename T> void launch_q3_prepare(Ctx3<T>* d_ctx, int n, int splitsN, int splitsE, hipStream_t s);
template <typename T> void launch_q3_perm_in(Ctx3<T>* d_ctx, int n, hipStream_t s);
template <typename T> void launch_q3_sel_env(Ctx3<T>* d_ctx, int n, int splitsH, double floor, hipStream_t s);
template <typename T> void launch_q3_gamma(Ctx3<T>* d_ctx, int n, int mmax, hipStream_t s);
template <typename T> void launch_q3_sel_h(Ctx3<T>* d_ctx, int n, int splitsC, TruncParams tp, hipStream_t s);
template <typename T> void launch_q3_sel_1(Ctx3<T>* d_ctx, int n, int splitsC, TruncParams tp, hipStream_t s);
template <typename T> void launch_q3_perm_out(Ctx3<T>* d_ctx, int n, hipStream_t s);
template <typename T> void launch_q3_sel_2(Ctx3<T>* d_ctx, int n, TruncParams tp, hipStream_t s);
template <typename T> void launch_q3_finish(Ctx3<T>* d_ctx, int n, hipStream_t s);

template <typename T> void launch_sw_prepare(CtxS<T>* d_ctx, int n, int splits, hipStream_t s);
template <typename T> void launch_sw_select(CtxS<T>* d_ctx, int n, TruncParams tp, hipStream_t s);
// T_0 <- T_0 / ||T_0|| (Anew of each item is the instance's T_0)
template <typename T> void launch_sw_normalize(CtxS<T>* d_ctx, int n, hipStream_t s);

template <typename T> void launch_transfer_prep(CtxT<T>* d_ctx, int n, int maxElems, hipStream_t s);
template <typename T> void launch_transfer_init(CtxT<T>* d_ctx, int n, hipStream_t s);
template <typename T> void launch_transfer_finish(CtxT<T>* d_ctx, int n, double* out, hipStream_t s);
template <typename T> void launch_rtransfer_prep(CtxR<T>* d_ctx, int n, hipStream_t s);

// chi -> Lambda (Eqs. (13)-(14)) and Kraus extraction (Eq. (16)).
void launch_choi(const double* chi, int q, double* lam, hipStream_t s);
void launch_kraus_extract(const double* evals, const double* evecs, int q, double eps, double rank_tol,
                          double* kraus, double* info, hipStream_t s);

// Right-orthonormalisation helpers of the truncation sweep.
template <typename T> void launch_copy_site(const cpx<T>* src, cpx<T>* dst, long long n, hipStream_t s);

}  // namespace mpdo
