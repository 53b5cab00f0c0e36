// Computational-basis measurement of an MPDO: exact sampling by sequential
// conditionals (the bitstring distributions the paper compares in Sec. IV.A,
// Eq. (18)).
//
// rho = Psi Psi^H with the purification Psi = B_0 B_1 ... B_{n-1},
// B_i[l, s, k, r].  Right environments R_i[l, l'] = sum B_i[l, x] W_i[l', x]
// with W_i[(l' s k), r] = sum_r' conj(B_i[(l' s k), r']) R_{i+1}[r, r']
// (R_n = [1]) are formed once per state, so no canonical form is assumed.
// Each shot carries a left environment E (chi x chi) normalised to the
// probability of its prefix; at site i
//   Y = E^T B_i,                         Y[l', (s k r)]
//   p_s = sum_{l' k r} Y[l', s, k, r] W_i[l', s, k, r],
// the bit is 0 when the shot's uniform u_i < p_0 / (p_0 + p_1), else 1, and
//   E' = Y_s^T conj(B_i,s) / p_s
// (the rows (l', s, k) of Y and B_i with s fixed: a two-level K index).
// Every contraction is a GEMM of the library; the shots of a chunk run as
// one batched launch per site and step.
#include <algorithm>
#include <cstring>
#include <vector>

#include "engine.h"
#include "kernels.h"

namespace mpdo {
namespace {

template <typename T> struct CtxSamp {
  const cpx<T>* Y;      // this shot's Y
  const cpx<T>* W;      // W_i of the site
  const cpx<T>* B;      // B_i
  cpx<T>* E;            // this shot's environment (output of d2)
  GemmDesc* d2;         // written here
  const double* u;      // this shot's uniforms (n)
  unsigned char* bits;  // this shot's bits (n)
  double* pz;           // this shot's probability
  int* fail;            // set when p_0 + p_1 is not positive
  int site, cl, k, cr;
};

// p_0, p_1, the bit and the descriptor of E' = Y_s^T conj(B_s) / p_s
template <typename T>
__global__ __launch_bounds__(256) void k_sample_select(const CtxSamp<T>* ctxs) {
  const CtxSamp<T>& c = ctxs[blockIdx.x];
  __shared__ double red[2][8];
  const long long half = (long long)c.k * c.cr, total = (long long)c.cl * 2 * half;
  double p[2] = {0.0, 0.0};
  for (long long e = threadIdx.x; e < total; e += blockDim.x) {
    const int s = (int)((e / half) & 1);
    const cpx<T> y = c.Y[e], w = c.W[e];
    p[s] += (double)y.re * (double)w.re - (double)y.im * (double)w.im;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int h = 0; h < 2; ++h) {
    double v = p[h];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[h][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double p0 = 0, p1 = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    p0 += red[0][w];
    p1 += red[1][w];
  }
  p0 = fmax(p0, 0.0);  // rounding can leave a vanishing branch slightly negative
  p1 = fmax(p1, 0.0);
  const double tot = p0 + p1;
  int s = 0;
  double ps = 1.0;
  if (!(tot > 0.0)) {
    *c.fail = 1;
  } else {
    s = c.u[c.site] < p0 / tot ? 0 : 1;
    ps = s ? p1 : p0;
    *c.pz *= ps / tot;
  }
  c.bits[c.site] = (unsigned char)s;
  GemmDesc& d = *c.d2;
  d.A = reinterpret_cast<const double*>(c.Y + (long long)s * half);
  d.B = reinterpret_cast<const double*>(c.B + (long long)s * half);
  d.C = reinterpret_cast<double*>(c.E);
  d.w = nullptr; d.kstride = 2 * c.k; d.kinner = c.k;
  d.sA = d.sB = d.sC = d.sSplit = 0;
  d.M = c.cr; d.N = c.cr; d.K = c.cl * c.k;
  d.lda = c.cr; d.ldb = c.cr; d.ldc = c.cr;
  d.wdiv = 1; d.nbatch = 1; d.splits = 1;
  d.opA = OP_T; d.opB = OP_C; d.beta = 0; d.active = 1; d.herm = 0;
  d.alpha = ps > 0.0 ? 1.0 / ps : 1.0;
}

template <typename T> __global__ void k_sample_init(cpx<T>* E, long long stride, int nshots, double* pz) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nshots) return;
  E[(long long)b * stride] = mk<T>((T)1, (T)0);
  pz[b] = 1.0;
}

template <typename T> __global__ void k_one(cpx<T>* R) { R[0] = mk<T>((T)1, (T)0); }

GemmDesc desc(const void* A, const void* B, void* C, int M, int N, int K, int opA, int opB, int lda, int ldb,
              int ldc) {
  GemmDesc d;
  std::memset(&d, 0, sizeof(d));
  d.A = reinterpret_cast<const double*>(A);
  d.B = reinterpret_cast<const double*>(B);
  d.C = reinterpret_cast<double*>(C);
  d.M = M; d.N = N; d.K = K;
  d.lda = lda; d.ldb = ldb; d.ldc = ldc;
  d.opA = opA; d.opB = opB;
  d.nbatch = 1; d.splits = 1; d.wdiv = 1; d.active = 1; d.alpha = 1.0;
  return d;
}
}  // namespace

template <typename T>
void Engine<T>::sample(int b, const double* u_host, int nshots, unsigned char* bits_host, double* pz_host) {
  const int n = nq_[b];
  std::vector<int> bonds, inner;
  double disc;
  dims(b, bonds, inner, disc);
  std::vector<int> chi(n + 1, 1);
  for (int i = 1; i < n; ++i) chi[i] = bonds[i - 1];
  std::vector<long long> woff(n + 1, 0);  // W_i offsets (elements)
  long long ymax = 1;
  for (int i = 0; i < n; ++i) {
    const long long sz = (long long)chi[i] * 2 * inner[i] * chi[i + 1];
    woff[i + 1] = woff[i] + sz;
    ymax = std::max(ymax, sz);
  }
  const int cx = cfg_.chi_max;
  // ---- right environments and W_i (one pass from the right) ----
  DevBuf bufW, bufR, dR;
  bufW.alloc((size_t)woff[n] * sizeof(cpx<T>));
  bufR.alloc((size_t)2 * cx * cx * sizeof(cpx<T>));
  dR.alloc(sizeof(GemmDesc) * 2 * n);
  cpx<T>* W = bufW.as<cpx<T>>();
  cpx<T>* R[2] = {bufR.as<cpx<T>>(), bufR.as<cpx<T>>() + (size_t)cx * cx};
  std::vector<GemmDesc> hR(2 * n);
  for (int i = n - 1, q = 0; i >= 0; --i, ++q) {
    const int L = chi[i], K2 = 2 * inner[i], Rr = chi[i + 1];
    const cpx<T>* B = site(b, i, par_[soff_[b] + i]);
    const cpx<T>* Rn = R[q & 1];  // R_{i+1}
    cpx<T>* Ri = R[(q + 1) & 1];
    // W_i[(l s k), r] = sum_r' conj(B[(l s k), r']) R_{i+1}[r, r']
    hR[2 * q] = desc(B, Rn, W + woff[i], L * K2, Rr, Rr, OP_C, OP_T, Rr, Rr, Rr);
    // R_i[l, l'] = sum_x B[l, x] W_i[l', x]
    hR[2 * q + 1] = desc(B, W + woff[i], Ri, L, L, K2 * Rr, OP_N, OP_T, K2 * Rr, K2 * Rr, L);
  }
  hip_check(hipMemcpyAsync(dR.p, hR.data(), sizeof(GemmDesc) * 2 * n, hipMemcpyHostToDevice, st_), "descriptors");
  hipLaunchKernelGGL(k_one<T>, dim3(1), dim3(1), 0, st_, R[0]);  // R_n = [1]
  for (int q = 0; q < n; ++q) {
    const int i = n - 1 - q;
    launch_gemm<T, T, T>(dR.as<GemmDesc>() + 2 * q, 1, 1, 1, gemm_tiles(chi[i] * 2 * inner[i], chi[i + 1]), st_);
    launch_gemm<T, T, T>(dR.as<GemmDesc>() + 2 * q + 1, 1, 1, 1, gemm_tiles(chi[i], chi[i]), st_);
  }
  // ---- shots, in chunks that keep the per-shot buffers near 2 GiB ----
  const size_t per_shot = ((size_t)cx * cx + (size_t)ymax) * sizeof(cpx<T>);
  const int chunk = (int)std::max<size_t>(1, std::min<size_t>((size_t)nshots, (2ULL << 30) / per_shot));
  DevBuf bufE, bufY, bufU, bufBits, bufPz, bufFail, dD1, dD2, dCtx;
  bufE.alloc((size_t)chunk * cx * cx * sizeof(cpx<T>));
  bufY.alloc((size_t)chunk * ymax * sizeof(cpx<T>));
  bufU.alloc((size_t)chunk * n * sizeof(double));
  bufBits.alloc((size_t)chunk * n);
  bufPz.alloc((size_t)chunk * sizeof(double));
  bufFail.alloc(sizeof(int));
  dD1.alloc(sizeof(GemmDesc) * (size_t)chunk * n);
  dD2.alloc(sizeof(GemmDesc) * (size_t)chunk);
  dCtx.alloc(sizeof(CtxSamp<T>) * (size_t)chunk * n);
  int fail = 0;
  hip_check(hipMemcpyAsync(bufFail.p, &fail, sizeof(int), hipMemcpyHostToDevice, st_), "flag");
  std::vector<GemmDesc> h1((size_t)chunk * n);
  std::vector<CtxSamp<T>> hc((size_t)chunk * n);
  for (int s0 = 0; s0 < nshots; s0 += chunk) {
    const int cs = std::min(chunk, nshots - s0);
    for (int i = 0; i < n; ++i) {
      const int L = chi[i], K2 = 2 * inner[i], Rr = chi[i + 1];
      const cpx<T>* B = site(b, i, par_[soff_[b] + i]);
      for (int t = 0; t < cs; ++t) {
        cpx<T>* E = bufE.as<cpx<T>>() + (size_t)t * cx * cx;
        cpx<T>* Y = bufY.as<cpx<T>>() + (size_t)t * ymax;
        // Y = E^T B_i  (E: L x L, B_i: L x (2 k r))
        h1[(size_t)i * cs + t] = desc(E, B, Y, L, K2 * Rr, L, OP_T, OP_N, L, K2 * Rr, K2 * Rr);
        CtxSamp<T>& c = hc[(size_t)i * cs + t];
        c.Y = Y;
        c.W = W + woff[i];
        c.B = B;
        c.E = E;
        c.d2 = dD2.as<GemmDesc>() + t;
        c.u = bufU.as<double>() + (size_t)t * n;
        c.bits = bufBits.as<unsigned char>() + (size_t)t * n;
        c.pz = bufPz.as<double>() + t;
        c.fail = bufFail.as<int>();
        c.site = i;
        c.cl = L;
        c.k = inner[i];
        c.cr = Rr;
      }
    }
    hip_check(hipMemcpyAsync(dD1.p, h1.data(), sizeof(GemmDesc) * (size_t)cs * n, hipMemcpyHostToDevice, st_),
              "descriptors");
    hip_check(hipMemcpyAsync(dCtx.p, hc.data(), sizeof(CtxSamp<T>) * (size_t)cs * n, hipMemcpyHostToDevice, st_),
              "contexts");
    hip_check(hipMemcpyAsync(bufU.p, u_host + (size_t)s0 * n, sizeof(double) * (size_t)cs * n,
                             hipMemcpyHostToDevice, st_), "uniforms");
    hipLaunchKernelGGL(k_sample_init<T>, dim3((cs + 255) / 256), dim3(256), 0, st_, bufE.as<cpx<T>>(),
                       (long long)cx * cx, cs, bufPz.as<double>());
    for (int i = 0; i < n; ++i) {
      launch_gemm<T, T, T>(dD1.as<GemmDesc>() + (size_t)i * cs, cs, 1, 1, gemm_tiles(chi[i], 2 * inner[i] * chi[i + 1]),
                           st_);
      hipLaunchKernelGGL(k_sample_select<T>, dim3(cs), dim3(256), 0, st_, dCtx.as<CtxSamp<T>>() + (size_t)i * cs);
      launch_gemm<T, T, T>(dD2.as<GemmDesc>(), cs, 1, 1, gemm_tiles(chi[i + 1], chi[i + 1]), st_);
    }
    hip_check(hipGetLastError(), "launch (sample)");
    hip_check(hipMemcpyAsync(bits_host + (size_t)s0 * n, bufBits.p, (size_t)cs * n, hipMemcpyDeviceToHost, st_),
              "bits");
    std::vector<double> pz(cs);
    hip_check(hipMemcpyAsync(pz.data(), bufPz.p, sizeof(double) * cs, hipMemcpyDeviceToHost, st_), "pz");
    hip_check(hipMemcpyAsync(&fail, bufFail.p, sizeof(int), hipMemcpyDeviceToHost, st_), "flag");
    hip_check(hipStreamSynchronize(st_), "hipStreamSynchronize");
    if (pz_host) std::memcpy(pz_host + s0, pz.data(), sizeof(double) * cs);
    if (fail) throw Error{5 /*MPDO_ENOTCONV*/, "sampling: a prefix has zero probability (state not normalisable)"};
  }
}

template void Engine<double>::sample(int, const double*, int, unsigned char*, double*);
template void Engine<float>::sample(int, const double*, int, unsigned char*, double*);

}  // namespace mpdo
