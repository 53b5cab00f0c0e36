// Dense density matrix of a small MPDO (n <= 12), for verification
// (Eqs. (6)-(7)).
//
// rho = Psi Psi^H with Psi the purification (physical indices s, inner
// indices k).  Per site the tensor M[(l s r), (l' s' r')] =
// sum_k B[l, s, k, r] conj(B[l', s', k, r']) (one GEMM over k) is absorbed
// into an accumulated block X[(S S'), (b b')]: the left half from the left
// edge, the right half from the right edge, so that neither block exceeds
// 4^(n/2) chi^2 entries; one final GEMM over the middle bond pair (b b')
// joins them.  Every contraction is a GEMM of the library (FP64) between
// index permutations.
#include <cstring>
#include <vector>

#include "engine.h"
#include "kernels.h"

namespace mpdo {
namespace {

struct Perm {
  int nd, conj;
  long long total;
  long long dims[6];   // output dimensions, row-major
  long long sstr[6];   // source stride of each output dimension
};

template <typename Tin>
__global__ void k_permute(const cpx<Tin>* __restrict__ src, cpx<double>* __restrict__ dst, Perm p) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < p.total;
       e += (long long)gridDim.x * blockDim.x) {
    long long rest = e, off = 0;
    for (int d = p.nd - 1; d >= 0; --d) {
      const long long i = rest % p.dims[d];
      rest /= p.dims[d];
      off += i * p.sstr[d];
    }
    const cpx<Tin> v = src[off];
    dst[e] = mk((double)v.re, p.conj ? -(double)v.im : (double)v.im);
  }
}

// x[(b b'), (l l')] = delta(b, l) delta(b', l') for b, l < c (c = 1: x = [1])
__global__ void k_identity_pairs(cpx<double>* x, int c) {
  const long long n2 = (long long)c * c, total = n2 * n2;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x)
    x[e] = mk(e / n2 == e % n2 ? 1.0 : 0.0, 0.0);
}

template <typename Tin>
void permute(const cpx<Tin>* src, cpx<double>* dst, std::vector<long long> dims, std::vector<long long> sstr,
             bool conj, hipStream_t s) {
  Perm p;
  std::memset(&p, 0, sizeof(p));
  p.nd = (int)dims.size();
  p.conj = conj ? 1 : 0;
  p.total = 1;
  for (int d = 0; d < p.nd; ++d) {
    p.dims[d] = dims[d];
    p.sstr[d] = sstr[d];
    p.total *= dims[d];
  }
  const long long blocks = std::min<long long>((p.total + 255) / 256, 8192);
  hipLaunchKernelGGL(k_permute<Tin>, dim3((unsigned)std::max<long long>(1, blocks)), dim3(256), 0, s, src, dst, p);
}

}  // namespace

// C = op(A) op(B) in FP64 with a one-item descriptor in `dd` (herm: C is
// Hermitian and only its upper triangle of tiles is computed); synchronises s.
void gemm_once(DevBuf& dd, const cpx<double>* A, const cpx<double>* B, cpx<double>* C, int M, int N, int K, int opA,
               int opB, int lda, int ldb, int ldc, hipStream_t s, bool herm) {
  GemmDesc d;
  std::memset(&d, 0, sizeof(d));
  d.A = A; d.B = B; d.C = C;
  d.M = M; d.N = N; d.K = K;
  d.lda = lda; d.ldb = ldb; d.ldc = ldc;
  d.opA = opA; d.opB = opB;
  d.nbatch = 1; d.splits = 1; d.wdiv = 1; d.active = 1; d.alpha = 1.0;
  d.herm = herm ? 1 : 0;
  dd.alloc(sizeof(GemmDesc));
  hip_check(hipMemcpyAsync(dd.p, &d, sizeof(d), hipMemcpyHostToDevice, s), "descriptor");
  launch_gemm<double, double, double>(dd.as<GemmDesc>(), 1, 1, 1, herm ? gemm_tiles_herm(N) : gemm_tiles(M, N), s);
  hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");  // dd is reused by the next call
}

namespace {
void gemm(DevBuf& dd, const cpx<double>* A, const cpx<double>* B, cpx<double>* C, int M, int N, int K, int opA,
          int opB, int lda, int ldb, int ldc, hipStream_t s) {
  gemm_once(dd, A, B, C, M, N, K, opA, opB, lda, ldb, ldc, s, false);
}
}  // namespace

template <typename T> void Engine<T>::to_dense(int b, double* host, bool device_out) {
  const int n = nq_[b];
  std::vector<int> bonds, inner;
  double disc;
  dims(b, bonds, inner, disc);
  std::vector<long long> chi(n + 1, 1);
  for (int i = 1; i < n; ++i) chi[i] = bonds[i - 1];
  const int m = n / 2;
  // workspace: the largest block (left: 4^j chi_j^2 for j <= m, right:
  // 4^(n-j) chi_j^2 for j >= m; a product Y has the size of the next block),
  // transfer tensor (4 chi^4) and the final 4^n
  long long big = 1LL << (2 * n);
  for (int j = 0; j <= m; ++j) big = std::max(big, (1LL << (2 * j)) * chi[j] * chi[j]);
  for (int j = m; j <= n; ++j) big = std::max(big, (1LL << (2 * (n - j))) * chi[j] * chi[j]);
  for (int i = 0; i < n; ++i) big = std::max(big, 4 * chi[i] * chi[i] * chi[i + 1] * chi[i + 1]);
  if (big * 16 * 5 > (16LL << 30)) throw Error{6 /*MPDO_EUNSUPPORTED*/, "dense state: workspace would exceed 16 GiB"};
  DevBuf bufX, bufY, bufM, bufMp, bufBk, bufL, dd;
  bufX.alloc(big * 16); bufY.alloc(big * 16); bufM.alloc(big * 16); bufMp.alloc(big * 16);
  bufL.alloc(big * 16); dd.alloc(sizeof(GemmDesc));
  size_t bk = 16;
  for (int i = 0; i < n; ++i) bk = std::max(bk, (size_t)(chi[i] * 2 * inner[i] * chi[i + 1]) * 16);
  bufBk.alloc(bk);
  auto X = bufX.as<cpx<double>>(), Y = bufY.as<cpx<double>>(), Mf = bufM.as<cpx<double>>(),
       Mp = bufMp.as<cpx<double>>(), Bk = bufBk.as<cpx<double>>();
  // transfer tensor of site i into Mf[(l s r), (l' s' r')]
  auto transfer = [&](int i) {
    const long long L = chi[i], K = inner[i], R = chi[i + 1];
    const cpx<T>* B = site(b, i, par_[soff_[b] + i]);
    permute<T>(B, Bk, {L, 2, R, K}, {2 * K * R, K * R, 1, R}, false, st_);
    gemm(dd, Bk, Bk, Mf, (int)(2 * L * R), (int)(2 * L * R), (int)K, OP_N, OP_H, (int)K, (int)K,
         (int)(2 * L * R), st_);
  };
  // left half: X[(S S'), (l l')], S over sites 0..j-1
  long long S = 1;
  hipLaunchKernelGGL(k_identity_pairs, dim3(1), dim3(64), 0, st_, X, 1);  // X = [1]
  for (int i = 0; i < m; ++i) {
    const long long L = chi[i], R = chi[i + 1];
    transfer(i);
    // Mp[(l l'), (s s' r r')]
    permute<double>(Mf, Mp, {L, L, 2, 2, R, R}, {2 * R * 2 * L * R, 2 * R, R * 2 * L * R, R, 2 * L * R, 1}, false, st_);
    // Y[(S S'), (s s' r r')] = X Mp
    gemm(dd, X, Mp, Y, (int)(S * S), (int)(4 * R * R), (int)(L * L), OP_N, OP_N, (int)(L * L), (int)(4 * R * R),
         (int)(4 * R * R), st_);
    // X[(S s), (S' s'), r, r']
    permute<double>(Y, X, {S, 2, S, 2, R, R}, {S * 4 * R * R, 2 * R * R, 4 * R * R, R * R, R, 1}, false, st_);
    S *= 2;
  }
  hip_check(hipMemcpyAsync(bufL.p, X, (size_t)(S * S * chi[m] * chi[m]) * 16, hipMemcpyDeviceToDevice, st_), "copy");
  const long long SL = S;
  // right half: X[(S S'), (r r')], S over sites j..n-1, built from the right edge
  S = 1;
  hipLaunchKernelGGL(k_identity_pairs, dim3(1), dim3(64), 0, st_, X, 1);
  for (int i = n - 1; i >= m; --i) {
    const long long L = chi[i], R = chi[i + 1];
    transfer(i);
    // Mp[(s s' l l'), (r r')]
    permute<double>(Mf, Mp, {2, 2, L, L, R, R}, {R * 2 * L * R, R, 2 * R * 2 * L * R, 2 * R, 2 * L * R, 1}, false, st_);
    // Y[(s s' l l'), (S S')] = Mp X^T
    gemm(dd, Mp, X, Y, (int)(4 * L * L), (int)(S * S), (int)(R * R), OP_N, OP_T, (int)(R * R), (int)(R * R),
         (int)(S * S), st_);
    // X[(s S), (s' S'), l, l']
    permute<double>(Y, X, {2, S, 2, S, L, L}, {2 * L * L * S * S, S, L * L * S * S, 1, L * S * S, S * S}, false,
                    st_);
    S *= 2;
  }
  const long long SR = S, cm = chi[m];
  // R[(S_L S_L'), (S_R S_R')] = X_L X_R^T over (b b')
  gemm(dd, bufL.as<cpx<double>>(), X, Y, (int)(SL * SL), (int)(SR * SR), (int)(cm * cm), OP_N, OP_T, (int)(cm * cm),
       (int)(cm * cm), (int)(SR * SR), st_);
  // rho[(S_L S_R), (S_L' S_R')]
  permute<double>(Y, Mf, {SL, SR, SL, SR}, {SL * SR * SR, SR, SR * SR, 1}, false, st_);
  hip_check(hipMemcpyAsync(host, Mf, (size_t)(SL * SR) * (SL * SR) * 16,
                           device_out ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st_), "rho");
  hip_check(hipStreamSynchronize(st_), "hipStreamSynchronize");
}

template void Engine<double>::to_dense(int, double*, bool);
template void Engine<float>::to_dense(int, double*, bool);

}  // namespace mpdo
