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
  double* disc;
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
  double* disc;
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
// index of the middle site: the three-site block is contracted, the fused
// operators applied, the middle inner index truncated, and the block split
// twice (bond i, then bond i+1) by Gram eigendecompositions.
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
  double* disc;
  int* scratch;           // [0] kappa', [1] bond i, [2] bond i+1
  double* G;              // m x 8 x 8
  cpx<T>* X;              // B_{i+1} B_{i+2}
  cpx<T>* Phi;            // (l t1 k1) x (t2 k2 t3 k3 r)
  cpx<T>* Psi;            // (l s1 k1) x (s2 (k2 j) s3 k3 r)
  cpx<T>* Psi2;           // (l s1 k1) x (s2 nu s3 k3 r)
  double* H;  double* evH; double* vecH;
  cpx<T>* P;              // (k2 m) x kappa'
  double* G1; double* ev1; double* vec1;
  cpx<T>* Q1;             // (l s1 k1) x r1
  cpx<T>* V1;             // r1 x (s2 nu s3 k3 r)
  double* G2; double* ev2; double* vec2;
  cpx<T>* Q2;             // (r1 s2 nu) x r2
  GemmDesc* dX; GemmDesc* dPhi; GemmDesc* dH; GemmDesc* dProj; GemmDesc* dG1; GemmDesc* dV1;
  GemmDesc* dG2; GemmDesc* dTk;
  EigDesc* dEH; EigDesc* dE1; EigDesc* dE2;
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
  double* disc;
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
  cpx<T>* Efinal;         // where the 1 x 1 result ends up
  GemmDesc* d1;
  GemmDesc* d2;
  int site, active, trace_idx, pad;
};

struct TruncParams {
  int chi_max, kap_max;
  double svd_cut, kap_cut;
  double tolE;            // relative eigenvalue floor of the right-factor Gram
};

template <typename T> void launch_q1_prepare(Ctx1<T>* d_ctx, int n, int splitsH, hipStream_t s);
template <typename T> void launch_q1_gamma(Ctx1<T>* d_ctx, int n, hipStream_t s);
template <typename T> void launch_q1_select(Ctx1<T>* d_ctx, int n, TruncParams tp, hipStream_t s);

template <typename T> void launch_q2_prepare(Ctx2<T>* d_ctx, int n, int splitsE, hipStream_t s);
template <typename T> void launch_q2_select_e(Ctx2<T>* d_ctx, int n, int splitsH, TruncParams tp, hipStream_t s);
template <typename T> void launch_q2_gamma(Ctx2<T>* d_ctx, int n, hipStream_t s);
template <typename T> void launch_q2_select_g(Ctx2<T>* d_ctx, int n, int splitsC, TruncParams tp, hipStream_t s);
template <typename T> void launch_q2_select_b(Ctx2<T>* d_ctx, int n, TruncParams tp, hipStream_t s);

template <typename T> void launch_q3_prepare(Ctx3<T>* d_ctx, int n, int splitsH, hipStream_t s);
template <typename T> void launch_q3_apply(Ctx3<T>* d_ctx, int n, hipStream_t s);
template <typename T> void launch_q3_select_h(Ctx3<T>* d_ctx, int n, int splitsG, TruncParams tp, hipStream_t s);
template <typename T> void launch_q3_scale1(Ctx3<T>* d_ctx, int n, hipStream_t s);
template <typename T> void launch_q3_select_1(Ctx3<T>* d_ctx, int n, int splitsG, TruncParams tp, hipStream_t s);
template <typename T> void launch_q3_scale2(Ctx3<T>* d_ctx, int n, hipStream_t s);
template <typename T> void launch_q3_select_2(Ctx3<T>* d_ctx, int n, TruncParams tp, hipStream_t s);

template <typename T> void launch_sw_prepare(CtxS<T>* d_ctx, int n, int splits, hipStream_t s);
template <typename T> void launch_sw_select(CtxS<T>* d_ctx, int n, TruncParams tp, hipStream_t s);
// T_0 <- T_0 / ||T_0|| (Anew of each item is the instance's T_0)
template <typename T> void launch_sw_normalize(CtxS<T>* d_ctx, int n, hipStream_t s);

template <typename T> void launch_transfer_prep(CtxT<T>* d_ctx, int n, int maxElems, hipStream_t s);
template <typename T> void launch_transfer_init(CtxT<T>* d_ctx, int n, hipStream_t s);
template <typename T> void launch_transfer_finish(CtxT<T>* d_ctx, int n, double* out, hipStream_t s);

// chi -> Lambda (Eqs. (13)-(14)) and Kraus extraction (Eq. (16)).
void launch_choi(const double* chi, int q, double* lam, hipStream_t s);
void launch_kraus_extract(const double* evals, const double* evecs, int q, double eps, double rank_tol,
                          double* kraus, double* info, hipStream_t s);

// Right-orthonormalisation helpers of the truncation sweep.
template <typename T> void launch_copy_site(const cpx<T>* src, cpx<T>* dst, long long n, hipStream_t s);

}  // namespace mpdo
