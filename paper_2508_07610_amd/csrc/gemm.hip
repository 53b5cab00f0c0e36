// Batched complex GEMM on the gfx950 matrix cores (MFMA), ragged shapes read
// on the device.  Used for every contraction of the MPDO update: the two-site
// contraction, the Gram matrices of the inner and bond truncations, the
// projections and the transfer matrices.
//
// A complex product is four real MFMA products on split real/imaginary
// planes staged in LDS:  Re += Ar Br - Ai Bi,  Im += Ar Bi + Ai Br.
// Tiles of 64 x 64 (or 32 x 32 for products with small outputs and long K)
// per workgroup of four waves; each wave owns a quadrant made of 16 x 16
// MFMA blocks; the next K slice is fetched into registers while the current
// one is multiplied.  At these sizes the products are latency-bound rather
// than MFMA-bound, so the design favours occupancy: short K slices and a
// register budget of four waves per SIMD.
#include <cmath>

#include "common.h"
#include "kernels.h"
#include "profile.h"

namespace mpdo {

// Operand layout of both 16x16x4 MFMAs: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16].  Output: lane l holds column l % 16; accumulator
// element v is row row(l / 16, v), which differs between the two types.
template <typename Tc> struct Mfma;
template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static inline v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int g, int v) { return g + 4 * v; }
};
template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static inline v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int g, int v) { return 4 * g + v; }
};

// Operands are read through global-address-space pointers (the descriptors
// hold generic ones), so their loads are not tied to the LDS wait counter.
#define GLB __attribute__((address_space(1)))

namespace {
// K slice of 8: the kernel is latency-bound at small tiles, so the slice is
// kept short to fit four waves per SIMD (four workgroups per CU).
constexpr int BK = 8, NTHR = 256, PAD = 4;
constexpr int NXCD = 8;  // accelerator complex dies of the MI355X

__device__ inline long long kaddr(int k, int kinner, long long kstride) {
  return (long long)(k / kinner) * kstride + (k % kinner);
}

// Staging of one BK-deep slice of op(A) (T x BK) or op(B) (BK x T): each
// thread holds E = T * BK / NTHR elements in registers between the global
// loads (issued one slice ahead) and the LDS stores.
template <typename Tin, typename Tc, int T> struct Slice {
  static constexpr int E = T * BK / NTHR;
  Tc re[E], im[E];
  // kfast: the K index is contiguous in memory for this operand
  __device__ void load(const GLB cpx<Tin>* X, int ld, bool kfast, bool conj, int r0, int R, int k0, int kend,
                       int kinner, long long kstride, const GLB double* w, int wdiv, bool two) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int it = 0; it < E; ++it) {
      const int idx = tid + it * NTHR;
      int rr, kk;
      if (kfast) { kk = idx % BK; rr = idx / BK; }
      else { rr = idx % T; kk = idx / T; }
      const int r = r0 + rr, k = k0 + kk;
      Tc vr = 0, vi = 0;
      if (r < R && k < kend) {
        const long long ka = two ? kaddr(k, kinner, kstride) : (long long)k;  // uniform branch
        const GLB cpx<Tin>* px = kfast ? X + ((long long)r * ld + ka) : X + (ka * ld + r);
        const cpx<Tin> v = mk<Tin>(px->re, px->im);
        vr = (Tc)v.re;
        vi = conj ? -(Tc)v.im : (Tc)v.im;
        if (w) {
          const Tc sw = (Tc)w[wdiv == 1 ? k : k / wdiv];
          vr *= sw;
          vi *= sw;
        }
      }
      re[it] = vr;
      im[it] = vi;
    }
  }
  __device__ void store(Tc (*Sre)[T + PAD], Tc (*Sim)[T + PAD], bool kfast) const {
    const int tid = threadIdx.x;
#pragma unroll
    for (int it = 0; it < E; ++it) {
      const int idx = tid + it * NTHR;
      int rr, kk;
      if (kfast) { kk = idx % BK; rr = idx / BK; }
      else { rr = idx % T; kk = idx / T; }
      Sre[kk][rr] = re[it];
      Sim[kk][rr] = im[it];
    }
  }
};
}  // namespace

// Tile TM x TN per workgroup of four waves in a 2 x 2 arrangement; each wave
// computes (TM/2) x (TN/2) from 16 x 16 MFMA blocks.  The next K slice is
// loaded into registers while the current one is multiplied from LDS.  The
// 32 x 32 tiles (small outputs, long K) fit eight waves per SIMD, the 64 x 64
// tiles four (the FP64 three-product form, with its third accumulator set,
// fits three and seven).
//
// Two forms of the complex product: G3 = false, four real products per
// complex one (Re = Ar Br - Ai Bi, Im = Ar Bi + Ai Br); G3 = true, three
// (Gauss: P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi); Re = P1 - P2,
// Im = P3 - P1 - P2), a quarter fewer MFMAs for a third accumulator set.
template <typename Tin, typename Tc, typename Tout, int TM, int TN, bool G3>
__global__ __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(
    (G3 && sizeof(Tc) == 8) ? (TM == 64 ? 3 : 7) : (TM == 32 ? 8 : 4),
    (G3 && sizeof(Tc) == 8) ? (TM == 64 ? 3 : 7) : (TM == 32 ? 8 : 4))))
void k_gemm(const GemmDesc* __restrict__ descs, int maxBatch, int maxSplits, int maxTiles, long long nblocks,
            int nitems, int groups) {
  typedef typename Mfma<Tc>::v4 v4;
  constexpr int FM = TM / 32, FN = TN / 32;  // 16 x 16 blocks per wave and dimension
  __shared__ Tc As_re[BK][TM + PAD], As_im[BK][TM + PAD];
  __shared__ Tc Bs_re[BK][TN + PAD], Bs_im[BK][TN + PAD];

  // Workgroups are dealt to the XCDs round-robin (block b runs on XCD b % 8);
  // renumber so that each XCD takes a contiguous range of (item, batch,
  // split, tile), keeping the tiles that share operands in one L2.
  const long long per_xcd = (nblocks + NXCD - 1) / NXCD;
  long long bid = (long long)(blockIdx.x % NXCD) * per_xcd + blockIdx.x / NXCD;
  if (bid >= nblocks) return;
  // Items with fewer tiles than maxTiles leave blocks with nothing to do.
  // Workgroups reach the CUs of an XCD in a fixed rotation, so a block
  // position that is idle in every group would leave the same CUs idle for
  // the whole launch; rotating the tile order by the group index spreads the
  // idle positions over all CUs.
  const long long grp = bid / maxTiles;
  const int tile = (int)((bid + grp) % maxTiles);
  bid = grp;
  const int split = (int)(bid % maxSplits);
  bid /= maxSplits;
  const int batch = (int)(bid % maxBatch);
  int item = (int)(bid / maxBatch);
  // A launch of `groups` descriptor groups of nitems / groups items each
  // (different products, e.g. the two outputs of a split) visits them
  // interleaved, so that every XCD's contiguous range holds items of each
  // group rather than one group's items only.
  if (groups > 1) item = (item % groups) * (nitems / groups) + item / groups;
  const GemmDesc& d = descs[item];
  if (!d.active || batch >= d.nbatch || split >= d.splits) return;
  const int M = d.M, N = d.N, K = d.K;
  // this item's tiles are a prefix of the tile range
  const int tilesN = (N + TN - 1) / TN;
  int tm, tn;
  if (d.herm) {
    // Hermitian (square) C: only the tiles on and above the diagonal, numbered
    // row by row, so no block of the launch is spent on the lower triangle
    if (tile >= tilesN * (tilesN + 1) / 2) return;
    tm = 0;
    int rest = tile;
    while (rest >= tilesN - tm) {
      rest -= tilesN - tm;
      ++tm;
    }
    tn = tm + rest;
  } else {
    if (tile >= ((M + TM - 1) / TM) * tilesN) return;
    tm = tile / tilesN;
    tn = tile % tilesN;
  }
  const int m0 = tm * TM, n0 = tn * TN;

  const GLB cpx<Tin>* A = (const GLB cpx<Tin>*)(d.A) + (long long)batch * d.sA;
  const GLB cpx<Tin>* B = (const GLB cpx<Tin>*)(d.B) + (long long)batch * d.sB;
  GLB cpx<Tout>* C = (GLB cpx<Tout>*)(d.C) + (long long)batch * d.sC + (long long)split * d.sSplit;
  const int opA = d.opA, opB = d.opB, lda = d.lda, ldb = d.ldb;
  const int kinner = d.kinner > 0 ? d.kinner : (K > 0 ? K : 1);
  const long long kstride = d.kinner > 0 ? d.kstride : (long long)kinner;
  const GLB double* w = (const GLB double*)d.w;
  const bool two = d.kinner > 0 && d.kinner < K;
  const int wdiv = d.wdiv > 0 ? d.wdiv : 1;

  int kper = (K + d.splits - 1) / d.splits;
  kper = (kper + BK - 1) / BK * BK;
  const int kbeg = split * kper;
  const int kend = min(K, kbeg + kper);

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, lk = lane >> 4;

  // four-product form: acc_re, acc_im; three-product form: acc_re = P1,
  // acc_im = P2, acc_s = P3
  v4 acc_re[FM][FN], acc_im[FM][FN], acc_s[G3 ? FM : 1][G3 ? FN : 1];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      acc_re[i][j] = v4{0, 0, 0, 0};
      acc_im[i][j] = v4{0, 0, 0, 0};
      if (G3) acc_s[G3 ? i : 0][G3 ? j : 0] = v4{0, 0, 0, 0};
    }

  const bool aKfast = (opA == OP_N || opA == OP_C);
  const bool aConj = (opA == OP_C || opA == OP_H);
  const bool bKfast = (opB == OP_T || opB == OP_H);
  const bool bConj = (opB == OP_C || opB == OP_H);

  Slice<Tin, Tc, TM> sa;
  Slice<Tin, Tc, TN> sb;
  if (kbeg < kend) {
    sa.load(A, lda, aKfast, aConj, m0, M, kbeg, kend, kinner, kstride, w, wdiv, two);
    sb.load(B, ldb, bKfast, bConj, n0, N, kbeg, kend, kinner, kstride, nullptr, 1, two);
  }
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    sa.store(As_re, As_im, aKfast);
    sb.store(Bs_re, Bs_im, bKfast);
    __syncthreads();
    if (k0 + BK < kend) {  // next slice in flight during the products below
      sa.load(A, lda, aKfast, aConj, m0, M, k0 + BK, kend, kinner, kstride, w, wdiv, two);
      sb.load(B, ldb, bKfast, bConj, n0, N, k0 + BK, kend, kinner, kstride, nullptr, 1, two);
    }
#pragma unroll 1
    for (int kb = 0; kb < BK; kb += 4) {
      Tc ar[FM], ai[FM], br[FN], bi[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        ar[i] = As_re[kb + lk][wm * (TM / 2) + i * 16 + li];
        ai[i] = As_im[kb + lk][wm * (TM / 2) + i * 16 + li];
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        br[j] = Bs_re[kb + lk][wn * (TN / 2) + j * 16 + li];
        bi[j] = Bs_im[kb + lk][wn * (TN / 2) + j * 16 + li];
      }
      if (G3) {
        Tc as[FM], bs[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) as[i] = ar[i] + ai[i];
#pragma unroll
        for (int j = 0; j < FN; ++j) bs[j] = br[j] + bi[j];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            acc_re[i][j] = Mfma<Tc>::mma(ar[i], br[j], acc_re[i][j]);
            acc_im[i][j] = Mfma<Tc>::mma(ai[i], bi[j], acc_im[i][j]);
            acc_s[G3 ? i : 0][G3 ? j : 0] = Mfma<Tc>::mma(as[i], bs[j], acc_s[G3 ? i : 0][G3 ? j : 0]);
          }
      } else {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            acc_re[i][j] = Mfma<Tc>::mma(ar[i], br[j], acc_re[i][j]);
            acc_re[i][j] = Mfma<Tc>::mma(-ai[i], bi[j], acc_re[i][j]);
            acc_im[i][j] = Mfma<Tc>::mma(ar[i], bi[j], acc_im[i][j]);
            acc_im[i][j] = Mfma<Tc>::mma(ai[i], br[j], acc_im[i][j]);
          }
      }
    }
    __syncthreads();
  }
  if (G3) {  // Re = P1 - P2, Im = P3 - P1 - P2
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const v4 p1 = acc_re[i][j], p2 = acc_im[i][j];
        acc_re[i][j] = p1 - p2;
        acc_im[i][j] = acc_s[G3 ? i : 0][G3 ? j : 0] - p1 - p2;
      }
  }

  const Tc alpha = (Tc)d.alpha;
  const int ldc = d.ldc;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * (TM / 2) + i * 16 + Mfma<Tc>::row(lk, v);
        const int col = n0 + wn * (TN / 2) + j * 16 + li;
        if (row < M && col < N) {
          GLB cpx<Tout>* p = C + (long long)row * ldc + col;
          cpx<Tc> r = mk<Tc>(alpha * acc_re[i][j][v], alpha * acc_im[i][j][v]);
          if (d.beta) r = r + mk<Tc>((Tc)p->re, (Tc)p->im);
          const cpx<Tout> o = mk<Tout>((Tout)r.re, (Tout)r.im);
          p->re = o.re;
          p->im = o.im;
        }
      }
}

// Sum the split-K partial products: out[i] = sum_s parts[s * sSplit + i]
// over a dense M x N block (complex double).
__global__ void k_reduce_splits(const GemmDesc* __restrict__ descs, double* const* __restrict__ outs,
                                int maxCount) {
  const GemmDesc& d = descs[blockIdx.y];
  if (!d.active) return;
  double* out = outs[blockIdx.y];
  const int count = d.M * d.ldc;
  const cpx<double>* parts = reinterpret_cast<const cpx<double>*>(d.C);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < count && e < maxCount;
       e += gridDim.x * blockDim.x) {
    const int row = e / d.ldc, col = e % d.ldc;
    if (col >= d.N || (d.herm && row > col)) continue;
    double re = 0, im = 0;
    for (int s = 0; s < d.splits; ++s) {
      const cpx<double> v = parts[(long long)s * d.sSplit + e];
      re += v.re;
      im += v.im;
    }
    out[2 * (long long)e] = re;
    out[2 * (long long)e + 1] = im;
    (void)row;
  }
}

int gemm_tiles(int maxM, int maxN, int tile) { return ((maxM + tile - 1) / tile) * ((maxN + tile - 1) / tile); }

namespace {
// complex-product form (3 or 4 real products) per MFMA precision and tile
// FP32: three products (measured faster: 98 against 87 TFLOP/s on 16 products
// of 512 x 512 x 1024); FP64: four (the three-product kernel's third
// accumulator set costs a wave per SIMD: 46 against 51 TFLOP/s)
int g_form[2][2] = {{3, 3}, {4, 4}};  // [fp64][tile == 64]
}
int gemm_form(bool fp64, int tile) { return g_form[fp64 ? 1 : 0][tile == 64 ? 1 : 0]; }
void set_gemm_form(bool fp64, int tile, int form) { g_form[fp64 ? 1 : 0][tile == 64 ? 1 : 0] = form == 3 ? 3 : 4; }

int gemm_tiles_herm(int maxN, int tile) {
  const int t = (maxN + tile - 1) / tile;
  return t * (t + 1) / 2;
}

namespace {
SiteTune g_site[GS_N];
}
void set_site_tune(int site, const SiteTune& t) {
  if (site >= 0 && site < GS_N) g_site[site] = t;
}
SiteTune get_site_tune(int site) { return (site >= 0 && site < GS_N) ? g_site[site] : SiteTune{}; }
int tuned_tile(int site, int dflt) {
  const int t = get_site_tune(site).tile;
  return (t == 32 || t == 64) ? t : dflt;
}
int tuned_splits(int site, int dflt) {
  const double f = get_site_tune(site).split_scale;
  if (!(f > 0)) return dflt;
  const int s = (int)std::lround(dflt * f);
  return s < 1 ? 1 : (s > 64 ? 64 : s);
}

template <typename Tin, typename Tc, typename Tout>
void launch_gemm(const GemmDesc* d_descs, int nitems, int maxBatch, int maxSplits, int maxTiles, hipStream_t s,
                 int tile, int site, int groups) {
  if (nitems <= 0 || maxTiles <= 0) return;
  if (groups < 1 || nitems % groups != 0) groups = 1;
  const long long blocks = (long long)nitems * maxBatch * maxSplits * maxTiles;
  if (blocks <= 0) return;
  const long long grid = (blocks + NXCD - 1) / NXCD * NXCD;
  const int cls = sizeof(Tc) == 8 ? PC_GEMM_F64 : PC_GEMM_F32;
  if (site >= 0) prof_set_site(site);
  const int tok = prof_begin(cls, s);
  prof_set_site(GS_OTHER);  // a call site labels only the launch that follows it
  const int sf = get_site_tune(site).form;
  const bool g3 = (sf == 3 || sf == 4) ? sf == 3 : gemm_form(sizeof(Tc) == 8, tile) == 3;
  if (tile == 32) {
    if (g3)
      hipLaunchKernelGGL((k_gemm<Tin, Tc, Tout, 32, 32, true>), dim3((unsigned)grid), dim3(NTHR), 0, s, d_descs,
                         maxBatch, maxSplits, maxTiles, blocks, nitems, groups);
    else
      hipLaunchKernelGGL((k_gemm<Tin, Tc, Tout, 32, 32, false>), dim3((unsigned)grid), dim3(NTHR), 0, s, d_descs,
                         maxBatch, maxSplits, maxTiles, blocks, nitems, groups);
  } else {
    if (g3)
      hipLaunchKernelGGL((k_gemm<Tin, Tc, Tout, 64, 64, true>), dim3((unsigned)grid), dim3(NTHR), 0, s, d_descs,
                         maxBatch, maxSplits, maxTiles, blocks, nitems, groups);
    else
      hipLaunchKernelGGL((k_gemm<Tin, Tc, Tout, 64, 64, false>), dim3((unsigned)grid), dim3(NTHR), 0, s, d_descs,
                         maxBatch, maxSplits, maxTiles, blocks, nitems, groups);
  }
  prof_end_gemm(tok, cls, d_descs, nitems, (int)sizeof(cpx<Tin>), (int)sizeof(cpx<Tout>), s);
}

void launch_reduce_splits(const GemmDesc* d_descs, double* const* d_outs, int nitems, int maxCount,
                          hipStream_t s) {
  if (nitems <= 0) return;
  const int threads = 256;
  const int bx = (maxCount + threads - 1) / threads;
  hipLaunchKernelGGL(k_reduce_splits, dim3(bx > 4096 ? 4096 : bx, nitems), dim3(threads), 0, s, d_descs,
                     d_outs, maxCount);
}

template void launch_gemm<double, double, double>(const GemmDesc*, int, int, int, int, hipStream_t, int, int, int);
template void launch_gemm<float, float, float>(const GemmDesc*, int, int, int, int, hipStream_t, int, int, int);
template void launch_gemm<float, double, double>(const GemmDesc*, int, int, int, int, hipStream_t, int, int, int);
template void launch_gemm<double, double, float>(const GemmDesc*, int, int, int, int, hipStream_t, int, int, int);

}  // namespace mpdo
