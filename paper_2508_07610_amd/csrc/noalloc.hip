// Allocation-free chi -> Kraus conversion: the kernels of
// mpdo_channel_from_chi (Choi matrix, eigensolver, Kraus extraction) with
// their scratch in a file-scope device array instead of allocated buffers,
// and device inputs and outputs, so the call allocates nothing and every
// step is a kernel on the caller's stream (capturable into a HIP graph).
#include <mutex>

#include "../../include/mpdo_noalloc.h"
#include "common.h"
#include "engine.h"
#include "kernels.h"
#include "ops.h"

namespace mpdo {
namespace {

// 512 KiB per device: a three-qubit channel needs 53,464 doubles (Choi
// matrix, eigenvectors and eigensolver work of a 64 x 64 problem).
constexpr long long SCRATCH_DOUBLES = 1LL << 16;
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_scratch[MAX_DEVICES] = {};

// Device address of this device's copy of `scratch` (looked up once per
// device, with the device current).
double* scratch_ptr(int dev) {
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
    g_scratch[dev] = reinterpret_cast<double*>(p);
  }
  return g_scratch[dev];
}

struct Parts {
  long long lam, ev, vec, work, desc, status, total;
};

Parts parts(int d2) {
  Parts p;
  long long o = 0;
  auto take = [&](long long n) {
    const long long at = o;
    o += (n + 31) / 32 * 32;  // 256-byte pieces
    return at;
  };
  p.lam = take(2LL * d2 * d2);
  p.ev = take(d2 + 1);
  p.vec = take(2LL * d2 * d2);
  p.work = take(eig_work_doubles(d2));
  p.desc = take((sizeof(EigDesc) + 7) / 8);
  p.status = take(1);
  p.total = o;
  return p;
}

// The eigensolver's descriptor, written on the device (no host copy).
__global__ void k_noalloc_desc(EigDesc* d, double* a, double* ev, double* vec, double* work, int n) {
  EigDesc e;
  e.a = a;
  e.evals = ev;
  e.evecs = vec;
  e.work = work;
  e.trace = ev + n;
  e.vfloor = 0;
  e.n = n;
  e.lda = n;
  e.kvec = n;
  e.active = 1;
  e.upper = 0;
  e.upad = 0;
  *d = e;
}

}  // namespace
}  // namespace mpdo

using namespace mpdo;

extern "C" mpdo_status mpdo_kraus_from_chi_noalloc(const double* chi_dev, int32_t q, double eps, double* kraus_dev,
                                                   double* info_dev, void* hip_stream) {
  if (!chi_dev || !kraus_dev || !info_dev) return (mpdo_status)set_last_error(MPDO_EINVAL, "null pointer");
  if (q < 1 || q > 3) return (mpdo_status)set_last_error(MPDO_EINVAL, "q must be 1, 2 or 3");
  if (!(eps >= 0 && eps < 1)) return (mpdo_status)set_last_error(MPDO_EINVAL, "eps must be in [0, 1)");
  const int d2 = 1 << (2 * q);
  const Parts p = parts(d2);
  if (p.total > SCRATCH_DOUBLES)
    return (mpdo_status)set_last_error(MPDO_EINVAL, "the problem needs " + std::to_string(p.total) +
                                                         " doubles of scratch, above the maximum of " +
                                                         std::to_string(SCRATCH_DOUBLES));
  try {
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= MAX_DEVICES) return (mpdo_status)set_last_error(MPDO_EINVAL, "device index too large");
    double* s = scratch_ptr(dev);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    EigDesc* desc = reinterpret_cast<EigDesc*>(s + p.desc);
    hipLaunchKernelGGL(k_noalloc_desc, dim3(1), dim3(1), 0, st, desc, s + p.lam, s + p.ev, s + p.vec, s + p.work, d2);
    launch_choi(chi_dev, q, s + p.lam, st);
    launch_eigh(desc, 1, d2, reinterpret_cast<int*>(s + p.status), st);
    launch_kraus_extract(s + p.ev, s + p.vec, q, eps, 1e-13, kraus_dev, info_dev, st);
    hip_check(hipGetLastError(), "launch (kraus_from_chi_noalloc)");
  } catch (const Error& e) {
    return (mpdo_status)set_last_error(e.status, e.msg);
  } catch (...) {
    return (mpdo_status)set_last_error(MPDO_EDEVICE, "internal error");
  }
  return MPDO_OK;
}
