// Surrogate multilayer perceptron: forward, backward and Adam on the gfx950
// matrix cores in bfloat16 with FP32 accumulation, and two loops that run
// entirely in the library (minibatch training, input-gradient ascent).
//
// Network (widths d_0 .. d_L): z_l = W_l h_{l-1} + b_l, h_l = GELU(z_l) for
// hidden layers (exact erf form), y = z_L; loss = mean (y - t)^2.  Operands
// of every matrix product (inputs, hidden activations, weights, gradients
// with respect to z) are bfloat16, rounded to nearest-even from FP32; biases,
// pre-activations, gradients and the Adam state are FP32, with FP32 master
// weights.  Matrix products use v_mfma_f32_16x16x16_bf16: 64 x 64 tiles per
// workgroup of four waves, each wave a 32 x 32 quadrant of 2 x 2 MFMA blocks,
// operand tiles staged in LDS with the K index contiguous, and the bias /
// activation / rounding epilogues fused into the product kernel.  The
// weight gradients (K = batch rows, few output tiles) are split over K into
// partial sums, which also carry the bias gradients; one pass adds them up.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mpdo.h"
#include "engine.h"

namespace mpdo {
namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// K slices of 16 (one MFMA step between two barriers); slices of 32 and 64
// made a training step of the 168-256-256-256-12 network at batch 512 slower
// (0.22 -> 0.23 and 0.28 ms).
constexpr int MT = 64, KT = 16, MTH = 256, KP = KT + 4;

__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)(u >> 16);  // inf / nan
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

enum Epi : int {
  EPI_STORE = 0,   // C = acc
  EPI_HIDDEN = 1,  // z = acc + bias[col] -> Z (FP32), h = GELU(z) -> Hb (bf16)
  EPI_OUT = 2,     // y = acc + bias[col] -> C
  EPI_ACTGRAD = 3, // g = acc * GELU'(aux[row][col]) -> C (FP32) and Hb (bf16)
  EPI_OUTGRAD = 4  // y = acc + bias[col] -> C; the MSE cotangent 2 (y - aux) scale -> C2 (FP32), Hb (bf16)
};

struct MlpGemm {
  const uint16_t* A;
  const uint16_t* B;
  int M, N, K, lda, ldb, transA, transB;
  float* C;
  int ldc;
  uint16_t* Hb;
  const float* bias;
  const float* aux;
  // split over K (grid dimension y): split s covers k in [s kper, (s + 1) kper)
  // and writes C + s sC; kper = K without a split
  int kper;
  long long sC;
  // optional (transA only): colout[s sC + i] = sum over the split's k of
  // colsrc[k ldcol + i] (FP32), from the workgroups of the first column tile
  const float* colsrc;
  float* colout;
  float* C2;    // EPI_OUTGRAD: the cotangent
  float scale;  // EPI_OUTGRAD: 1 / (rows x outputs)
};

// C[M x N] = op(A)[M x K] op(B)[K x N]: op(A)[i][k] = transA ? A[k lda + i] : A[i lda + k],
// op(B)[k][j] = transB ? B[j ldb + k] : B[k ldb + j].
// One output tile (bx) of one K range (by) of the product g, epilogue epi
// (uniform per workgroup).
__device__ void mlp_gemm_tile(const MlpGemm& g, int epi, int bx, int by) {
  __shared__ __attribute__((aligned(16))) uint16_t As[MT][KP];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[MT][KP];  // [n][k]
  __shared__ float red[MTH / MT][MT];
  const int tilesN = (g.N + MT - 1) / MT;
  const int m0 = (bx / tilesN) * MT, n0 = (bx % tilesN) * MT;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1, li = lane & 15, lg = lane >> 4;
  const int kb = by * g.kper, ke = min(g.K, kb + g.kper);
  // with transA each thread stages one row m0 + tid % MT of op(A) (MT divides MTH)
  const bool colsum = g.colsrc != nullptr && (bx % tilesN) == 0;
  float csum = 0.0f;
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0, 0, 0, 0};
  for (int k0 = kb; k0 < ke; k0 += KT) {
#pragma unroll
    for (int it = 0; it < (MT * KT) / MTH; ++it) {
      const int idx = tid + it * MTH;
      int mm, kk;
      if (g.transA) { mm = idx % MT; kk = idx / MT; }
      else { kk = idx % KT; mm = idx / KT; }
      const int m = m0 + mm, k = k0 + kk;
      uint16_t v = 0;
      if (m < g.M && k < ke) {
        v = g.transA ? g.A[(long long)k * g.lda + m] : g.A[(long long)m * g.lda + k];
        if (colsum) csum += g.colsrc[(long long)k * g.lda + m];
      }
      As[mm][kk] = v;
    }
#pragma unroll
    for (int it = 0; it < (MT * KT) / MTH; ++it) {
      const int idx = tid + it * MTH;
      int nn, kk;
      if (g.transB) { kk = idx % KT; nn = idx / KT; }
      else { nn = idx % MT; kk = idx / MT; }
      const int n = n0 + nn, k = k0 + kk;
      uint16_t v = 0;
      if (n < g.N && k < ke) v = g.transB ? g.B[(long long)n * g.ldb + k] : g.B[(long long)k * g.ldb + n];
      Bs[nn][kk] = v;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KT; ks += 16) {
      s4 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const s4*>(&As[wm * 32 + i * 16 + li][ks + 4 * lg]);
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const s4*>(&Bs[wn * 32 + j * 16 + li][ks + 4 * lg]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  if (colsum) {  // uniform per workgroup
    red[tid / MT][tid % MT] = csum;
    __syncthreads();
    if (tid < MT && m0 + tid < g.M) {
      float t = 0;
#pragma unroll
      for (int r = 0; r < MTH / MT; ++r) t += red[r][tid];
      g.colout[by * g.sC + m0 + tid] = t;
    }
  }
  float* C = g.C + by * g.sC;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * 32 + i * 16 + 4 * lg + v;
        const int col = n0 + wn * 32 + j * 16 + li;
        if (row >= g.M || col >= g.N) continue;
        const float x = acc[i][j][v];
        const long long o = (long long)row * g.ldc + col;
        if (epi == EPI_STORE) {
          C[o] = x;
        } else if (epi == EPI_HIDDEN) {
          const float z = x + g.bias[col];
          C[o] = z;
          g.Hb[o] = f2bf(gelu(z));
        } else if (epi == EPI_OUT) {
          C[o] = x + g.bias[col];
        } else if (epi == EPI_OUTGRAD) {
          const float y = x + g.bias[col];
          C[o] = y;
          const float d = y - g.aux[o];
          const float v = 2.0f * d * g.scale;
          g.C2[o] = v;
          g.Hb[o] = f2bf(v);
        } else {
          const float gz = x * gelu_grad(g.aux[o]);
          C[o] = gz;
          g.Hb[o] = f2bf(gz);
        }
      }
}

template <int EPI>
__global__ __launch_bounds__(MTH) void k_mlp_gemm(MlpGemm g) {
  mlp_gemm_tile(g, EPI, blockIdx.x, blockIdx.y);
}

// Two independent products in one launch (grid z = 0, 1): blocks beyond a
// product's tiles or K ranges return.
__global__ __launch_bounds__(MTH) void k_mlp_gemm_pair(MlpGemm g0, int epi0, int tiles0, int splits0, MlpGemm g1,
                                                       int epi1, int tiles1, int splits1) {
  if (blockIdx.z == 0) {
    if ((int)blockIdx.x < tiles0 && (int)blockIdx.y < splits0) mlp_gemm_tile(g0, epi0, blockIdx.x, blockIdx.y);
  } else {
    if ((int)blockIdx.x < tiles1 && (int)blockIdx.y < splits1) mlp_gemm_tile(g1, epi1, blockIdx.x, blockIdx.y);
  }
}

__global__ void k_to_bf16(const float* __restrict__ x, uint16_t* __restrict__ y, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = f2bf(x[i]);
}

// g = 2 (y - t) / count; loss partials per block
__global__ void k_out_grad(const float* __restrict__ y, const float* __restrict__ t, long long n, float inv,
                           float* __restrict__ g, uint16_t* __restrict__ gb, float* __restrict__ part) {
  __shared__ float red[256];
  float s = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float d = y[i] - t[i];
    s += d * d;
    const float v = 2.0f * d * inv;
    g[i] = v;
    gb[i] = f2bf(v);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// copies a given output cotangent into the gradient buffers
__global__ void k_set_grad(const float* __restrict__ gy, long long n, float* __restrict__ g,
                           uint16_t* __restrict__ gb) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    g[i] = gy[i];
    gb[i] = f2bf(gy[i]);
  }
}

// grad[i] = sum over the splits of part[s np + i]
__global__ void k_grad_reduce(const float* __restrict__ part, long long np, int splits, float* __restrict__ grad) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < np; i += (long long)gridDim.x * blockDim.x) {
    float t = 0;
    for (int s = 0; s < splits; ++s) t += part[s * np + i];
    grad[i] = t;
  }
}

// Adam on the FP32 master parameters; refreshes the bf16 weight copies.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ grad, float* __restrict__ m,
                       float* __restrict__ v, uint16_t* __restrict__ pb, long long n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float gr = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gr;
    const float vi = b2 * v[i] + (1.0f - b2) * gr * gr;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    p[i] = pi;
    pb[i] = f2bf(pi);
  }
}

// The split reduction of k_grad_reduce followed by the update of k_adam, in
// one pass (same arithmetic; the summed gradient is still written to grad).
__global__ void k_reduce_adam(const float* __restrict__ part, int splits, float* __restrict__ p,
                              float* __restrict__ grad, float* __restrict__ m, float* __restrict__ v,
                              uint16_t* __restrict__ pb, long long n, float lr, float b1, float b2, float eps,
                              float c1, float c2) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    float gr = 0;
    for (int s = 0; s < splits; ++s) gr += part[s * n + i];
    grad[i] = gr;
    const float mi = b1 * m[i] + (1.0f - b1) * gr;
    const float vi = b2 * v[i] + (1.0f - b2) * gr * gr;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    p[i] = pi;
    pb[i] = f2bf(pi);
  }
}

// SplitMix64 (Steele, Lea and Flood, 2014): the k-th output (k >= 1) of the
// generator seeded with `seed` is the finalizer applied to seed + k * gamma.
__device__ inline uint64_t splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Minibatch of a training loop: row b of step `step` is dataset row
// splitmix64(seed, step * batch + b + 1) mod nrows; inputs to bf16, targets
// copied (FP32).
__global__ void k_gather(const float* __restrict__ x, const float* __restrict__ t, long long nrows, int d0, int dL,
                         int batch, uint64_t seed, long long step, uint16_t* __restrict__ xb,
                         float* __restrict__ tg) {
  const int b = blockIdx.x;
  const long long r = (long long)(splitmix64(seed, (uint64_t)(step * batch + b + 1)) % (uint64_t)nrows);
  for (int j = threadIdx.x; j < d0; j += blockDim.x) xb[(long long)b * d0 + j] = f2bf(x[r * d0 + j]);
  for (int j = threadIdx.x; j < dL; j += blockDim.x) tg[(long long)b * dL + j] = t[r * dL + j];
}

// One Adam ascent step on the first nfree entries of the input row xa (the
// rest are held): xa += lr mhat / (sqrt(vhat) + eps) with the gradient dx;
// the row is recorded in rec and its bf16 copy refreshed for the next pass.
__global__ void k_ascend(float* __restrict__ xa, const float* __restrict__ dx, float* __restrict__ m,
                         float* __restrict__ v, int d0, int nfree, float lr, float b1, float b2, float eps, float c1,
                         float c2, float* __restrict__ rec, uint16_t* __restrict__ xb) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d0; i += gridDim.x * blockDim.x) {
    float xi = xa[i];
    if (i < nfree) {
      const float gr = dx[i];
      const float mi = b1 * m[i] + (1.0f - b1) * gr;
      const float vi = b2 * v[i] + (1.0f - b2) * gr * gr;
      m[i] = mi;
      v[i] = vi;
      xi += lr * (mi * c1) / (sqrtf(vi * c2) + eps);
      xa[i] = xi;
    }
    rec[i] = xi;
    xb[i] = f2bf(xi);
  }
}

__global__ void k_fill(float* __restrict__ p, int n, float val) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = val;
}

// output cotangent: one-hot at column `col` for a single row
__global__ void k_onehot(int n, int col, float* __restrict__ g, uint16_t* __restrict__ gb) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    g[i] = i == col ? 1.0f : 0.0f;
    gb[i] = f2bf(i == col ? 1.0f : 0.0f);
  }
}

int tiles_of(const MlpGemm& g) { return ((g.M + MT - 1) / MT) * ((g.N + MT - 1) / MT); }

// splits: number of K ranges (grid dimension y); g.kper and g.sC must match
template <int EPI> void gemm(MlpGemm g, hipStream_t s, int splits = 1) {
  const int tiles = tiles_of(g);
  if (splits <= 1) g.kper = g.K;
  if (tiles > 0 && g.K > 0)
    hipLaunchKernelGGL(k_mlp_gemm<EPI>, dim3(tiles, splits > 1 ? splits : 1), dim3(MTH), 0, s, g);
}

// Two independent products (epilogues e0, e1; K splits s0, s1) in one launch.
void gemm_pair(MlpGemm g0, int e0, int s0, MlpGemm g1, int e1, int s1, hipStream_t s) {
  if (s0 <= 1) { g0.kper = g0.K; s0 = 1; }
  if (s1 <= 1) { g1.kper = g1.K; s1 = 1; }
  const int t0 = g0.K > 0 ? tiles_of(g0) : 0, t1 = g1.K > 0 ? tiles_of(g1) : 0;
  const int tx = t0 > t1 ? t0 : t1, sy = s0 > s1 ? s0 : s1;
  if (tx > 0)
    hipLaunchKernelGGL(k_mlp_gemm_pair, dim3(tx, sy, 2), dim3(MTH), 0, s, g0, e0, t0, s0, g1, e1, t1, s1);
}

// K split of the weight-gradient products: ranges of a multiple of KT rows,
// at most SPLIT_MAX of them, about 32 rows each
constexpr int SPLIT_MAX = 16;
void split_of(int batch, int* splits, int* kper) {
  int s = batch / 32;
  s = s < 1 ? 1 : (s > SPLIT_MAX ? SPLIT_MAX : s);
  int k = (batch + s - 1) / s;
  k = (k + KT - 1) / KT * KT;
  *kper = k;
  *splits = (batch + k - 1) / k;
}

int grid_for(long long n) {
  long long b = (n + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

}  // namespace
}  // namespace mpdo

using namespace mpdo;

struct mpdo_mlp_s {
  std::vector<int> w;            // widths d_0 .. d_L
  int L = 0, max_batch = 0;
  long long np = 0;
  std::vector<long long> woff, boff;
  hipStream_t st = nullptr;
  DevBuf p, g, m, v, pb;         // FP32 params / grads / Adam moments; bf16 params
  DevBuf xb;                     // input, bf16
  DevBuf z, hb, gz, gzb, dx, part;
  DevBuf gpart;                  // split partial gradients, SPLIT_MAX x np
  DevBuf yb, tb;                 // outputs and gathered targets of the training loop (max_batch x d_L)
  DevBuf xa, am, av, dxa;        // ascent: input row, its Adam moments, its gradient (d_0 each)
  std::vector<long long> zoff;   // per layer offsets into z / hb / gz / gzb (max_batch x d_l)
  long long step = 0;
  long long ascent_step = 0;     // Adam steps of the ascent since its last reset
};

namespace {
mpdo_status mfail(int st, const std::string& msg) { return (mpdo_status)set_last_error(st, msg); }

// Forward pass for `batch` rows of the bf16 input already in xb into y (FP32,
// device). With targets tgt (batch x d_L) the last product also writes the
// MSE output cotangent 2 (y - tgt) / (batch d_L) into gz/gzb of the last layer.
void mlp_forward_xb(mpdo_mlp_s* h, int batch, float* y, const float* tgt = nullptr) {
  const int L = h->L;
  const uint16_t* in = h->xb.as<uint16_t>();
  for (int l = 0; l < L; ++l) {
    MlpGemm g{};
    g.A = in; g.lda = h->w[l];
    g.B = h->pb.as<uint16_t>() + h->woff[l]; g.ldb = h->w[l]; g.transB = 1;  // W_l^T
    g.M = batch; g.N = h->w[l + 1]; g.K = h->w[l];
    g.bias = h->p.as<float>() + h->boff[l];
    g.ldc = h->w[l + 1];
    if (l + 1 < L) {
      g.C = h->z.as<float>() + h->zoff[l];
      g.Hb = h->hb.as<uint16_t>() + h->zoff[l];
      gemm<EPI_HIDDEN>(g, h->st);
      in = g.Hb;
    } else if (tgt) {
      g.C = y;
      g.aux = tgt;
      g.C2 = h->gz.as<float>() + h->zoff[l];
      g.Hb = h->gzb.as<uint16_t>() + h->zoff[l];
      g.scale = 1.0f / (float)((long long)batch * h->w[L]);
      gemm<EPI_OUTGRAD>(g, h->st);
    } else {
      g.C = y;
      gemm<EPI_OUT>(g, h->st);
    }
  }
}

// Forward pass for `batch` rows of x (FP32, device) into y (FP32, device).
void mlp_forward(mpdo_mlp_s* h, const float* x, int batch, float* y) {
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_for((long long)batch * h->w[0])), dim3(256), 0, h->st, x,
                     h->xb.as<uint16_t>(), (long long)batch * h->w[0]);
  mlp_forward_xb(h, batch, y);
}

// Backward pass from the output cotangent already in gz/gzb of the last
// layer: with params, weight and bias gradients of each layer as split
// partial sums in gpart (split over the batch); input gradient into dx (if
// set). The weight-gradient product of a layer and the product for the
// cotangent of the layer below read the same inputs and write disjoint
// buffers, so they share one launch. Returns the number of splits.
int mlp_backward_parts(mpdo_mlp_s* h, int batch, float* dx, bool params) {
  const int L = h->L;
  int splits = 1, kper = batch;
  split_of(batch, &splits, &kper);
  float* part = h->gpart.as<float>();
  for (int l = L - 1; l >= 0; --l) {
    const uint16_t* gb = h->gzb.as<uint16_t>() + h->zoff[l];
    const float* gf = h->gz.as<float>() + h->zoff[l];
    const uint16_t* hin = l == 0 ? h->xb.as<uint16_t>() : h->hb.as<uint16_t>() + h->zoff[l - 1];
    // dW_l = G^T H_{l-1}: (d_l x B)(B x d_{l-1}); db_l = G^T 1 alongside
    MlpGemm gw{};
    gw.A = gb; gw.lda = h->w[l + 1]; gw.transA = 1;
    gw.B = hin; gw.ldb = h->w[l];
    gw.M = h->w[l + 1]; gw.N = h->w[l]; gw.K = batch;
    gw.C = part + h->woff[l]; gw.ldc = h->w[l];
    gw.kper = kper;
    gw.sC = h->np;
    gw.colsrc = gf;
    gw.colout = part + h->boff[l];
    const bool need_da = l > 0 || dx;
    if (!need_da) {
      if (params) gemm<EPI_STORE>(gw, h->st, splits);
      break;
    }
    // dA = G W_l: (B x d_l)(d_l x d_{l-1}); times GELU'(z_{l-1}) for hidden inputs
    MlpGemm ga{};
    ga.A = gb; ga.lda = h->w[l + 1];
    ga.B = h->pb.as<uint16_t>() + h->woff[l]; ga.ldb = h->w[l];
    ga.M = batch; ga.N = h->w[l]; ga.K = h->w[l + 1];
    ga.ldc = h->w[l];
    int ea = EPI_STORE;
    if (l > 0) {
      ga.C = h->gz.as<float>() + h->zoff[l - 1];
      ga.Hb = h->gzb.as<uint16_t>() + h->zoff[l - 1];
      ga.aux = h->z.as<float>() + h->zoff[l - 1];
      ea = EPI_ACTGRAD;
    } else {
      ga.C = dx;
    }
    if (params) {
      gemm_pair(gw, EPI_STORE, splits, ga, ea, 1, h->st);
    } else if (ea == EPI_ACTGRAD) {
      gemm<EPI_ACTGRAD>(ga, h->st);
    } else {
      gemm<EPI_STORE>(ga, h->st);
    }
  }
  return splits;
}

// mlp_backward_parts, then the split partial sums added up into h->g.
void mlp_backward(mpdo_mlp_s* h, int batch, float* dx, bool params = true) {
  const int splits = mlp_backward_parts(h, batch, dx, params);
  if (params)
    hipLaunchKernelGGL(k_grad_reduce, dim3(grid_for(h->np)), dim3(256), 0, h->st, h->gpart.as<float>(), h->np,
                       splits, h->g.as<float>());
}

void adam_step(mpdo_mlp_s* h, float lr, float beta1, float beta2, float eps) {
  h->step += 1;
  const float c1 = 1.0f / (1.0f - std::pow(beta1, (float)h->step));
  const float c2 = 1.0f / (1.0f - std::pow(beta2, (float)h->step));
  hipLaunchKernelGGL(k_adam, dim3(grid_for(h->np)), dim3(256), 0, h->st, h->p.as<float>(), h->g.as<float>(),
                     h->m.as<float>(), h->v.as<float>(), h->pb.as<uint16_t>(), h->np, lr, beta1, beta2, eps, c1,
                     c2);
}

void refresh_bf16(mpdo_mlp_s* h) {
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(h->np)), dim3(256), 0, h->st, h->p.as<float>(),
                     h->pb.as<uint16_t>(), h->np);
}

#define MGUARD_BEGIN try {
#define MGUARD_END                                                    \
  }                                                                   \
  catch (const Error& e) {                                            \
    return mfail(e.status, e.msg);                                    \
  }                                                                   \
  catch (...) {                                                       \
    return mfail(MPDO_EDEVICE, "internal error");                     \
  }

const char* check_batch(mpdo_mlp_s* h, int batch) {
  if (!h) return "null network";
  if (batch < 1 || batch > h->max_batch) return "batch must be in [1, max_batch]";
  return nullptr;
}
}  // namespace

extern "C" {

mpdo_status mpdo_mlp_create(const int32_t* widths, int32_t nlayers, int32_t max_batch, void* hip_stream,
                            mpdo_mlp_t* out) {
  if (!out) return mfail(MPDO_EINVAL, "null out");
  *out = nullptr;
  if (!widths || nlayers < 1 || nlayers > 16) return mfail(MPDO_EINVAL, "nlayers must be in [1, 16]");
  if (max_batch < 1 || max_batch > (1 << 20)) return mfail(MPDO_EINVAL, "max_batch must be in [1, 2^20]");
  for (int l = 0; l <= nlayers; ++l)
    if (widths[l] < 1 || widths[l] > 8192) return mfail(MPDO_EINVAL, "widths must be in [1, 8192]");
  MGUARD_BEGIN
  auto* h = new mpdo_mlp_s();
  h->L = nlayers;
  h->max_batch = max_batch;
  h->st = reinterpret_cast<hipStream_t>(hip_stream);
  h->w.assign(widths, widths + nlayers + 1);
  long long off = 0, zo = 0;
  for (int l = 0; l < nlayers; ++l) {
    h->woff.push_back(off);
    off += (long long)h->w[l + 1] * h->w[l];
    h->boff.push_back(off);
    off += h->w[l + 1];
    h->zoff.push_back(zo);
    zo += (long long)max_batch * h->w[l + 1];
  }
  h->np = off;
  try {
    h->p.alloc(off * 4);
    h->g.alloc(off * 4);
    h->m.alloc(off * 4);
    h->v.alloc(off * 4);
    h->pb.alloc(off * 2);
    h->xb.alloc((size_t)max_batch * h->w[0] * 2);
    h->z.alloc(zo * 4);
    h->hb.alloc(zo * 2);
    h->gz.alloc(zo * 4);
    h->gzb.alloc(zo * 2);
    h->part.alloc(1024 * 4);
    h->gpart.alloc((size_t)SPLIT_MAX * off * 4);
    h->yb.alloc((size_t)max_batch * h->w[nlayers] * 4);
    h->tb.alloc((size_t)max_batch * h->w[nlayers] * 4);
    h->xa.alloc((size_t)h->w[0] * 4);
    h->am.alloc((size_t)h->w[0] * 4);
    h->av.alloc((size_t)h->w[0] * 4);
    h->dxa.alloc((size_t)h->w[0] * 4);
    hip_check(hipMemsetAsync(h->p.p, 0, off * 4, h->st), "memset");
    hip_check(hipMemsetAsync(h->m.p, 0, off * 4, h->st), "memset");
    hip_check(hipMemsetAsync(h->v.p, 0, off * 4, h->st), "memset");
    refresh_bf16(h);
    hip_check(hipStreamSynchronize(h->st), "sync");
  } catch (...) {
    delete h;
    throw;
  }
  *out = h;
  return MPDO_OK;
  MGUARD_END
}

mpdo_status mpdo_mlp_destroy(mpdo_mlp_t h) {
  if (!h) return MPDO_OK;
  (void)hipStreamSynchronize(h->st);
  delete h;
  return MPDO_OK;
}

mpdo_status mpdo_mlp_info(mpdo_mlp_t h, int64_t* nparams) {
  if (!h || !nparams) return mfail(MPDO_EINVAL, "null argument");
  *nparams = h->np;
  return MPDO_OK;
}

mpdo_status mpdo_mlp_set_params(mpdo_mlp_t h, const float* host) {
  if (!h || !host) return mfail(MPDO_EINVAL, "null argument");
  MGUARD_BEGIN
  hip_check(hipMemcpyAsync(h->p.p, host, h->np * 4, hipMemcpyHostToDevice, h->st), "params");
  hip_check(hipMemsetAsync(h->m.p, 0, h->np * 4, h->st), "memset");
  hip_check(hipMemsetAsync(h->v.p, 0, h->np * 4, h->st), "memset");
  h->step = 0;
  refresh_bf16(h);
  hip_check(hipStreamSynchronize(h->st), "sync");
  return MPDO_OK;
  MGUARD_END
}

mpdo_status mpdo_mlp_get_params(mpdo_mlp_t h, float* host) {
  if (!h || !host) return mfail(MPDO_EINVAL, "null argument");
  MGUARD_BEGIN
  hip_check(hipMemcpyAsync(host, h->p.p, h->np * 4, hipMemcpyDeviceToHost, h->st), "params");
  hip_check(hipStreamSynchronize(h->st), "sync");
  return MPDO_OK;
  MGUARD_END
}

mpdo_status mpdo_mlp_forward(mpdo_mlp_t h, const float* x_dev, int32_t batch, float* y_dev) {
  if (const char* why = check_batch(h, batch)) return mfail(MPDO_EINVAL, why);
  if (!x_dev || !y_dev) return mfail(MPDO_EINVAL, "null buffer");
  MGUARD_BEGIN
  mlp_forward(h, x_dev, batch, y_dev);
  hip_check(hipGetLastError(), "launch (mlp forward)");
  return MPDO_OK;
  MGUARD_END
}

mpdo_status mpdo_mlp_backward(mpdo_mlp_t h, const float* x_dev, const float* t_dev, const float* gy_dev,
                              int32_t batch, float* y_dev, float* grad_dev, float* dx_dev, float* loss) {
  if (const char* why = check_batch(h, batch)) return mfail(MPDO_EINVAL, why);
  if (!x_dev || !y_dev) return mfail(MPDO_EINVAL, "null buffer");
  if ((t_dev == nullptr) == (gy_dev == nullptr)) return mfail(MPDO_EINVAL, "give exactly one of t_dev, gy_dev");
  MGUARD_BEGIN
  mlp_forward(h, x_dev, batch, y_dev);
  const int L = h->L;
  const long long n = (long long)batch * h->w[L];
  float* gl = h->gz.as<float>() + h->zoff[L - 1];
  uint16_t* glb = h->gzb.as<uint16_t>() + h->zoff[L - 1];
  const int blocks = grid_for(n);
  if (t_dev) {
    hipLaunchKernelGGL(k_out_grad, dim3(blocks), dim3(256), 0, h->st, y_dev, t_dev, n, 1.0f / (float)n, gl, glb,
                       h->part.as<float>());
  } else {
    hipLaunchKernelGGL(k_set_grad, dim3(blocks), dim3(256), 0, h->st, gy_dev, n, gl, glb);
  }
  mlp_backward(h, batch, dx_dev);
  if (grad_dev)
    hip_check(hipMemcpyAsync(grad_dev, h->g.p, h->np * 4, hipMemcpyDeviceToDevice, h->st), "grad copy");
  hip_check(hipGetLastError(), "launch (mlp backward)");
  if (loss) {
    *loss = 0;
    if (t_dev) {
      std::vector<float> part(blocks);
      hip_check(hipMemcpyAsync(part.data(), h->part.p, blocks * 4, hipMemcpyDeviceToHost, h->st), "loss");
      hip_check(hipStreamSynchronize(h->st), "sync");
      double s = 0;
      for (float x : part) s += x;
      *loss = (float)(s / (double)n);
    }
  }
  return MPDO_OK;
  MGUARD_END
}

mpdo_status mpdo_mlp_adam(mpdo_mlp_t h, float lr, float beta1, float beta2, float eps) {
  if (!h) return mfail(MPDO_EINVAL, "null network");
  if (!(lr >= 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return mfail(MPDO_EINVAL, "bad Adam hyper-parameters");
  MGUARD_BEGIN
  adam_step(h, lr, beta1, beta2, eps);
  hip_check(hipGetLastError(), "launch (adam)");
  return MPDO_OK;
  MGUARD_END
}

mpdo_status mpdo_mlp_fit(mpdo_mlp_t h, const float* x_dev, const float* t_dev, int64_t nrows, int32_t batch,
                         int32_t steps, float lr, int32_t cosine, uint64_t seed, float* loss) {
  if (const char* why = check_batch(h, batch)) return mfail(MPDO_EINVAL, why);
  if (!x_dev || !t_dev) return mfail(MPDO_EINVAL, "null buffer");
  if (nrows < 1) return mfail(MPDO_EINVAL, "nrows must be >= 1");
  if (steps < 0) return mfail(MPDO_EINVAL, "steps must be >= 0");
  if (!(lr >= 0)) return mfail(MPDO_EINVAL, "lr must be >= 0");
  MGUARD_BEGIN
  const int L = h->L, d0 = h->w[0], dL = h->w[L];
  const long long n = (long long)batch * dL;
  float* gl = h->gz.as<float>() + h->zoff[L - 1];
  uint16_t* glb = h->gzb.as<uint16_t>() + h->zoff[L - 1];
  const int blocks = grid_for(n);
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int s = 0; s < steps; ++s) {
    hipLaunchKernelGGL(k_gather, dim3(batch), dim3(64), 0, h->st, x_dev, t_dev, (long long)nrows, d0, dL, batch,
                       seed, (long long)s, h->xb.as<uint16_t>(), h->tb.as<float>());
    if (loss && s + 1 == steps) {  // the last step also leaves the loss partials
      mlp_forward_xb(h, batch, h->yb.as<float>());
      hipLaunchKernelGGL(k_out_grad, dim3(blocks), dim3(256), 0, h->st, h->yb.as<float>(), h->tb.as<float>(), n,
                         1.0f / (float)n, gl, glb, h->part.as<float>());
    } else {
      mlp_forward_xb(h, batch, h->yb.as<float>(), h->tb.as<float>());
    }
    const int splits = mlp_backward_parts(h, batch, nullptr, true);
    const float lr_s = cosine ? lr * 0.5f * (1.0f + std::cos(3.14159265358979f * (float)s / (float)steps)) : lr;
    h->step += 1;
    const float c1 = 1.0f / (1.0f - std::pow(b1, (float)h->step));
    const float c2 = 1.0f / (1.0f - std::pow(b2, (float)h->step));
    hipLaunchKernelGGL(k_reduce_adam, dim3(grid_for(h->np)), dim3(256), 0, h->st, h->gpart.as<float>(), splits,
                       h->p.as<float>(), h->g.as<float>(), h->m.as<float>(), h->v.as<float>(),
                       h->pb.as<uint16_t>(), h->np, lr_s, b1, b2, eps, c1, c2);
  }
  hip_check(hipGetLastError(), "launch (mlp fit)");
  if (loss) {
    *loss = 0;
    if (steps > 0) {
      std::vector<float> part(blocks);
      hip_check(hipMemcpyAsync(part.data(), h->part.p, blocks * 4, hipMemcpyDeviceToHost, h->st), "loss");
      hip_check(hipStreamSynchronize(h->st), "sync");
      double t = 0;
      for (float x : part) t += x;
      *loss = (float)(t / (double)n);
    }
  }
  return MPDO_OK;
  MGUARD_END
}

mpdo_status mpdo_mlp_ascend(mpdo_mlp_t h, const float* x0_dev, int32_t nfree, int32_t out_index, int32_t steps,
                            float lr, float beta1, float beta2, float eps, int32_t reset, float* xs_dev) {
  if (!h) return mfail(MPDO_EINVAL, "null network");
  if (!x0_dev || (steps > 0 && !xs_dev)) return mfail(MPDO_EINVAL, "null buffer");
  const int L = h->L, d0 = h->w[0];
  if (nfree < 0 || nfree > d0) return mfail(MPDO_EINVAL, "nfree must be in [0, d_0]");
  if (out_index < 0 || out_index >= h->w[L]) return mfail(MPDO_EINVAL, "out_index must be in [0, d_L)");
  if (steps < 0) return mfail(MPDO_EINVAL, "steps must be >= 0");
  if (!(lr >= 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return mfail(MPDO_EINVAL, "bad Adam hyper-parameters");
  MGUARD_BEGIN
  if (reset) {
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(256), 0, h->st, h->am.as<float>(), d0, 0.0f);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(256), 0, h->st, h->av.as<float>(), d0, 0.0f);
    h->ascent_step = 0;
  }
  hip_check(hipMemcpyAsync(h->xa.p, x0_dev, (size_t)d0 * 4, hipMemcpyDeviceToDevice, h->st), "ascent input");
  hipLaunchKernelGGL(k_to_bf16, dim3(1), dim3(256), 0, h->st, h->xa.as<float>(), h->xb.as<uint16_t>(),
                     (long long)d0);
  // the forward pass does not touch the output cotangent, so it is set once
  hipLaunchKernelGGL(k_onehot, dim3(1), dim3(256), 0, h->st, h->w[L], out_index,
                     h->gz.as<float>() + h->zoff[L - 1], h->gzb.as<uint16_t>() + h->zoff[L - 1]);
  for (int s = 0; s < steps; ++s) {
    mlp_forward_xb(h, 1, h->yb.as<float>());
    mlp_backward(h, 1, h->dxa.as<float>(), false);
    h->ascent_step += 1;
    const float c1 = 1.0f / (1.0f - std::pow(beta1, (float)h->ascent_step));
    const float c2 = 1.0f / (1.0f - std::pow(beta2, (float)h->ascent_step));
    hipLaunchKernelGGL(k_ascend, dim3(1), dim3(256), 0, h->st, h->xa.as<float>(), h->dxa.as<float>(),
                       h->am.as<float>(), h->av.as<float>(), d0, nfree, lr, beta1, beta2, eps, c1, c2,
                       xs_dev + (long long)s * d0, h->xb.as<uint16_t>());
  }
  hip_check(hipGetLastError(), "launch (mlp ascend)");
  return MPDO_OK;
  MGUARD_END
}

}  // extern "C"
