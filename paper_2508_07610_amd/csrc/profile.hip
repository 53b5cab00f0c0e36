// Kernel timing and algorithmic-work accounting (see profile.h).  The
// accounting kernels are one block each; a launch's work is summed over its
// descriptors in parallel and added to the class counters by one thread
// (launches on one stream are ordered, so the updates do not race).
#include <mutex>
#include <vector>

#include "profile.h"

namespace mpdo {

namespace {

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  int cls = 0;
  int site = -1;
};

// device counters: flops[PC_NCLASS], bytes[PC_NCLASS], then flops and bytes per GEMM site
constexpr int NCOUNT = 2 * PC_NCLASS + 2 * GS_N;

struct Prof {
  std::mutex mu;
  bool on = false;
  std::vector<EventPair> ev;
  int launches[PC_NCLASS] = {};
  int site_launches[GS_N] = {};
  double* dcount = nullptr;
};

thread_local int t_site = GS_OTHER;

Prof& P() {
  static Prof p;
  return p;
}

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return true;
  return st != hipStreamCaptureStatusNone;
}

constexpr int AT = 256;  // accounting threads (one block)

__device__ void block_add(double f, double b, double* __restrict__ flops, double* __restrict__ bytes) {
  __shared__ double sf[AT], sb[AT];
  sf[threadIdx.x] = f;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int off = AT / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      sf[threadIdx.x] += sf[threadIdx.x + off];
      sb[threadIdx.x] += sb[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *flops += sf[0];
    *bytes += sb[0];
  }
}

__global__ __launch_bounds__(AT) void k_account_gemm(const GemmDesc* __restrict__ d, int n, int in_bytes,
                                                     int out_bytes, double* __restrict__ flops,
                                                     double* __restrict__ bytes) {
  double f = 0, b = 0;
  for (int i = threadIdx.x; i < n; i += AT) {
    if (!d[i].active) continue;
    const double nb = d[i].nbatch > 0 ? d[i].nbatch : 1;
    const double M = d[i].M, N = d[i].N, K = d[i].K;
    const double MN = d[i].herm ? 0.5 * M * (M + 1) : M * N;  // Hermitian C: its upper triangle
    f += 8.0 * MN * K * nb;
    b += nb * (in_bytes * (M * K + K * N) + out_bytes * MN);
  }
  block_add(f, b, flops, bytes);
}

__global__ __launch_bounds__(AT) void k_account_eig(const EigDesc* __restrict__ d, int n, int nlo, int nhi,
                                                    double* __restrict__ flops, double* __restrict__ bytes) {
  double f = 0, b = 0;
  for (int i = threadIdx.x; i < n; i += AT) {
    if (!d[i].active || d[i].n < nlo || d[i].n > nhi) continue;
    const double m = d[i].n;
    const double k = d[i].kvec < d[i].n ? d[i].kvec : d[i].n;
    f += 16.0 / 3.0 * m * m * m + 8.0 * m * m * k;
    b += 16.0 * m * m + 16.0 * m * k;
  }
  block_add(f, b, flops, bytes);
}

__global__ __launch_bounds__(AT) void k_account_chol(const EigDesc* __restrict__ d, int n,
                                                     double* __restrict__ flops, double* __restrict__ bytes) {
  double f = 0, b = 0;
  for (int i = threadIdx.x; i < n; i += AT) {
    if (!d[i].active) continue;
    const double m = d[i].n;
    f += 8.0 / 3.0 * m * m * m;
    b += 48.0 * m * m;
  }
  block_add(f, b, flops, bytes);
}

}  // namespace

bool prof_enabled() { return P().on; }

void prof_reset(bool on) {
  Prof& p = P();
  std::lock_guard<std::mutex> g(p.mu);
  (void)hipDeviceSynchronize();
  for (auto& e : p.ev) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  p.ev.clear();
  for (int c = 0; c < PC_NCLASS; ++c) p.launches[c] = 0;
  for (int c = 0; c < GS_N; ++c) p.site_launches[c] = 0;
  if (!p.dcount && hipMalloc(&p.dcount, sizeof(double) * NCOUNT) != hipSuccess) p.dcount = nullptr;
  if (p.dcount) (void)hipMemset(p.dcount, 0, sizeof(double) * NCOUNT);
  p.on = on && p.dcount != nullptr;
}

int prof_begin(int cls, hipStream_t s) {
  Prof& p = P();
  if (!p.on || capturing(s)) return -1;
  std::lock_guard<std::mutex> g(p.mu);
  EventPair e;
  e.cls = cls;
  if (cls == PC_GEMM_F64 || cls == PC_GEMM_F32) e.site = t_site;
  if (hipEventCreate(&e.a) != hipSuccess) return -1;
  if (hipEventCreate(&e.b) != hipSuccess) {
    (void)hipEventDestroy(e.a);
    return -1;
  }
  (void)hipEventRecord(e.a, s);
  p.ev.push_back(e);
  return (int)p.ev.size() - 1;
}

static void end_common(int token, int cls, hipStream_t s) {
  Prof& p = P();
  std::lock_guard<std::mutex> g(p.mu);
  (void)hipEventRecord(p.ev[token].b, s);
  p.launches[cls] += 1;
  if (p.ev[token].site >= 0) p.site_launches[p.ev[token].site] += 1;
}

void prof_set_site(int site) { t_site = (site >= 0 && site < GS_N) ? site : GS_OTHER; }

void prof_end_gemm(int token, int cls, const GemmDesc* d_descs, int nitems, int in_bytes, int out_bytes,
                   hipStream_t s) {
  if (token < 0) return;
  end_common(token, cls, s);
  double* c = P().dcount;
  hipLaunchKernelGGL(k_account_gemm, dim3(1), dim3(AT), 0, s, d_descs, nitems, in_bytes, out_bytes, c + cls,
                     c + PC_NCLASS + cls);
  const int site = P().ev[token].site;
  if (site >= 0)
    hipLaunchKernelGGL(k_account_gemm, dim3(1), dim3(AT), 0, s, d_descs, nitems, in_bytes, out_bytes,
                       c + 2 * PC_NCLASS + site, c + 2 * PC_NCLASS + GS_N + site);
}

void prof_end_eig(int token, int cls, const EigDesc* d_descs, int nitems, int nlo, int nhi, hipStream_t s) {
  if (token < 0) return;
  end_common(token, cls, s);
  double* c = P().dcount;
  hipLaunchKernelGGL(k_account_eig, dim3(1), dim3(AT), 0, s, d_descs, nitems, nlo, nhi, c + cls,
                     c + PC_NCLASS + cls);
}

void prof_end_chol(int token, int cls, const EigDesc* d_descs, int nitems, hipStream_t s) {
  if (token < 0) return;
  end_common(token, cls, s);
  double* c = P().dcount;
  hipLaunchKernelGGL(k_account_chol, dim3(1), dim3(AT), 0, s, d_descs, nitems, c + cls, c + PC_NCLASS + cls);
}

void prof_read(int cls, int* launches, double* ms, double* flops, double* bytes) {
  Prof& p = P();
  std::lock_guard<std::mutex> g(p.mu);
  (void)hipDeviceSynchronize();
  double t = 0;
  for (auto& e : p.ev) {
    if (e.cls != cls) continue;
    float x = 0;
    if (hipEventElapsedTime(&x, e.a, e.b) == hipSuccess) t += x;
  }
  double h[NCOUNT] = {0};
  if (p.dcount) (void)hipMemcpy(h, p.dcount, sizeof(h), hipMemcpyDeviceToHost);
  if (launches) *launches = p.launches[cls];
  if (ms) *ms = t;
  if (flops) *flops = h[cls];
  if (bytes) *bytes = h[PC_NCLASS + cls];
}

void prof_read_site(int site, int* launches, double* ms, double* flops) {
  Prof& p = P();
  std::lock_guard<std::mutex> g(p.mu);
  (void)hipDeviceSynchronize();
  double t = 0;
  for (auto& e : p.ev) {
    if (e.site != site) continue;
    float x = 0;
    if (hipEventElapsedTime(&x, e.a, e.b) == hipSuccess) t += x;
  }
  double h[NCOUNT] = {0};
  if (p.dcount) (void)hipMemcpy(h, p.dcount, sizeof(h), hipMemcpyDeviceToHost);
  if (launches) *launches = p.site_launches[site];
  if (ms) *ms = t;
  if (flops) *flops = h[2 * PC_NCLASS + site];
}

}  // namespace mpdo
