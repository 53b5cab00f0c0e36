// Host runtime of libmpdo: device state of MPDO instances and the launch
// sequences that apply a sublayer of noisy gates (Eq. (8)) with inner and
// bond truncation (Eqs. (9)-(11), Sec. II.D), observables by transfer
// matrices (Eqs. (6)-(7)) and the canonicalise-then-truncate sweep.
//
// Gauge: every site tensor B[l, s, k, r] is right-orthonormal and every bond
// carries its weights lambda, so the environment of a site or of a pair of
// neighbouring sites is diag(lambda_left^2) (x) identity.  Gates on disjoint
// sites are therefore independent and a whole sublayer runs as one launch
// sequence over all its gates (and all instances of a batch).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <stdexcept>

#include "engine.h"
#include "kernels.h"
#include "profile.h"

namespace mpdo {

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error{4 /*MPDO_EDEVICE*/, std::string(what) + ": " + hipGetErrorString(e)};
}

namespace {
thread_local const DeviceAllocator* t_alloc = nullptr;

// Free blocks of the library's caches: device blocks per device, pinned
// host blocks in one list, keyed by size.
constexpr int MAX_DEV = 64;
std::mutex g_cache_mu;
std::multimap<size_t, void*> g_dev_free[MAX_DEV];
std::multimap<size_t, void*> g_pin_free;

void* take_fitting(std::multimap<size_t, void*>& m, size_t n, size_t* got) {
  auto it = m.lower_bound(n);
  if (it == m.end() || it->first > 2 * n + (1 << 20)) return nullptr;
  void* p = it->second;
  *got = it->first;
  m.erase(it);
  return p;
}
}  // namespace

const DeviceAllocator* current_allocator() { return t_alloc; }
AllocScope::AllocScope(const DeviceAllocator* a) : prev(t_alloc) { t_alloc = (a && a->alloc) ? a : nullptr; }
AllocScope::~AllocScope() { t_alloc = prev; }

void release_cached_memory() {
  std::lock_guard<std::mutex> g(g_cache_mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (int d = 0; d < MAX_DEV; ++d) {
    if (g_dev_free[d].empty()) continue;
    (void)hipSetDevice(d);
    for (auto& kv : g_dev_free[d]) (void)hipFree(kv.second);
    g_dev_free[d].clear();
  }
  (void)hipSetDevice(cur);
  for (auto& kv : g_pin_free) (void)hipHostFree(kv.second);
  g_pin_free.clear();
}

size_t cached_device_bytes() {
  std::lock_guard<std::mutex> g(g_cache_mu);
  size_t t = 0;
  for (int d = 0; d < MAX_DEV; ++d)
    for (auto& kv : g_dev_free[d]) t += kv.first;
  return t;
}

void* pinned_get(size_t n, size_t* got) {
  {
    std::lock_guard<std::mutex> g(g_cache_mu);
    if (void* p = take_fitting(g_pin_free, n, got)) return p;
  }
  void* p = nullptr;
  hip_check(hipHostMalloc(&p, n, hipHostMallocDefault), "hipHostMalloc");
  *got = n;
  return p;
}

void pinned_put(void* p, size_t n) {
  if (!p) return;
  std::lock_guard<std::mutex> g(g_cache_mu);
  g_pin_free.emplace(n, p);
}

void DevBuf::release() {
  if (!p) return;
  // the block may still be read by queued work: wait for the device before
  // it can be handed out again (hipFree would wait the same way)
  (void)hipDeviceSynchronize();
  if (from.alloc) {
    if (from.free) from.free(p, from.ctx);
  } else if (device >= 0 && device < MAX_DEV) {
    std::lock_guard<std::mutex> g(g_cache_mu);
    g_dev_free[device].emplace(bytes, p);
  } else {
    (void)hipFree(p);
  }
  p = nullptr;
  bytes = 0;
}

DevBuf::~DevBuf() { release(); }

void DevBuf::alloc(size_t n) {
  if (n <= bytes && p) return;
  release();
  if (n == 0) n = 256;
  n = (n + 255) & ~size_t(255);
  int dev = 0;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  const DeviceAllocator* a = current_allocator();
  if (a) {
    p = a->alloc(n, a->ctx);
    if (!p) throw Error{3 /*MPDO_ENOMEM*/, "caller allocator refused " + std::to_string(n) + " bytes"};
    from = *a;
    device = dev;
    bytes = n;
    return;
  }
  from = DeviceAllocator{};
  device = dev;
  if (dev >= 0 && dev < MAX_DEV) {
    std::lock_guard<std::mutex> g(g_cache_mu);
    size_t got = 0;
    if (void* q = take_fitting(g_dev_free[dev], n, &got)) {
      p = q;
      bytes = got;
      return;
    }
  }
  if (hipMalloc(&p, n) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
    release_cached_memory();   // give the cache back to the driver and try once more
    if (hipMalloc(&p, n) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      throw Error{3 /*MPDO_ENOMEM*/, "device allocation of " + std::to_string(n) + " bytes failed"};
    }
  }
  bytes = n;
}

HostStage::~HostStage() {
  if (done) {
    (void)hipEventSynchronize(done);
    (void)hipEventDestroy(done);
  }
  pinned_put(p, bytes);
}

void* HostStage::get(size_t n) {
  if (done) hip_check(hipEventSynchronize(done), "hipEventSynchronize");
  else hip_check(hipEventCreateWithFlags(&done, hipEventDisableTiming), "hipEventCreate");
  if (n > bytes) {
    pinned_put(p, bytes);
    p = nullptr;
    bytes = 0;
    p = pinned_get(std::max<size_t>(n, 1 << 20), &bytes);
  }
  return p;
}

namespace {
// Offsets of the pieces of one upload (descriptors, contexts) or of the
// per-item workspace, 256-byte aligned.
struct Layout {
  size_t off = 0;
  size_t add(size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  }
};

template <typename X> X* at(void* base, size_t off) { return reinterpret_cast<X*>(reinterpret_cast<char*>(base) + off); }

__global__ void k_init_sites_kernel(double* base, long long nsites, long long stride_doubles) {
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < nsites; s += (long long)gridDim.x * blockDim.x)
    base[s * stride_doubles] = 1.0;
}
__global__ void k_gather_pairs(const double* src, const int* idx, int n, double* dst) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) {
    dst[2 * k] = src[2 * idx[k]];
    dst[2 * k + 1] = src[2 * idx[k] + 1];
  }
}
__global__ void k_init_sites_kernel_f(float* base, long long nsites, long long stride_floats) {
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < nsites; s += (long long)gridDim.x * blockDim.x)
    base[s * stride_floats] = 1.0f;
}
}  // namespace

template <typename T>
Engine<T>::Engine(const Config& cfg, const std::vector<int>& nq, hipStream_t s) : cfg_(cfg), nq_(nq), st_(s) {
  soff_.resize(nq_.size() + 1, 0);
  for (size_t b = 0; b < nq_.size(); ++b) soff_[b + 1] = soff_[b] + nq_[b];
  nsites_ = soff_.back();
  cap_site_ = (size_t)cfg_.chi_max * 2 * cfg_.kap_max * cfg_.chi_max;
  sites_.alloc((size_t)nsites_ * 2 * cap_site_ * sizeof(cpx<T>));
  hip_check(hipMemsetAsync(sites_.p, 0, sites_.bytes, st_), "hipMemsetAsync");
  if (sizeof(T) == 8)
    hipLaunchKernelGGL(k_init_sites_kernel, dim3(64), dim3(256), 0, st_, sites_.as<double>(), (long long)nsites_,
                       (long long)(2 * cap_site_ * 2));
  else
    hipLaunchKernelGGL(k_init_sites_kernel_f, dim3(64), dim3(256), 0, st_, sites_.as<float>(), (long long)nsites_,
                       (long long)(2 * cap_site_ * 2));
  par_.assign(nsites_, 0);
  std::vector<double> ones((size_t)nsites_ * cfg_.chi_max, 1.0);
  lam_.alloc(ones.size() * sizeof(double));
  lam2_.alloc(ones.size() * sizeof(double));
  hip_check(hipMemcpyAsync(lam_.p, ones.data(), ones.size() * sizeof(double), hipMemcpyHostToDevice, st_), "copy");
  hip_check(hipMemcpyAsync(lam2_.p, ones.data(), ones.size() * sizeof(double), hipMemcpyHostToDevice, st_), "copy");
  one_.alloc(sizeof(double));
  hip_check(hipMemcpyAsync(one_.p, ones.data(), sizeof(double), hipMemcpyHostToDevice, st_), "copy");
  std::vector<int> d(nsites_ + nq_.size() + nsites_, 1);
  dims_.alloc(d.size() * sizeof(int));
  hip_check(hipMemcpyAsync(dims_.p, d.data(), d.size() * sizeof(int), hipMemcpyHostToDevice, st_), "copy");
  std::vector<double> z((size_t)nsites_ * ST_W, 0.0);
  for (int i = 0; i < nsites_; ++i) z[(size_t)i * ST_W + ST_GAP] = 1e300;
  disc_.alloc(z.size() * sizeof(double));
  hip_check(hipMemcpyAsync(disc_.p, z.data(), z.size() * sizeof(double), hipMemcpyHostToDevice, st_), "copy");
  hip_check(hipStreamSynchronize(st_), "hipStreamSynchronize");
}

template <typename T> int Engine<T>::splits_for(long long K) const {
  long long s = (K + 2047) / 2048;
  if (s < 1) s = 1;
  if (s > 64) s = 64;
  return (int)s;
}

template <typename T>
bool Engine<T>::reserve(Upload& up, size_t bytes, size_t work_bytes, int items, char*& h, char*& dv) {
  const size_t ab = (bytes + 255) & ~size_t(255);
  if (up.dry) {
    up.cursor += ab;
    up.work_need = std::max(up.work_need, work_bytes);
    up.max_items = std::max(up.max_items, items);
    return false;
  }
  if (up.immediate) {
    work_.alloc(work_bytes);
    sweeps_.alloc(sizeof(int) * 2 * std::max(1, items));
    blob_.alloc(bytes);
    h = reinterpret_cast<char*>(stage_.get(bytes));
    dv = reinterpret_cast<char*>(blob_.p);
  } else {
    if (work_.bytes < work_bytes || sweeps_.bytes < sizeof(int) * 2 * (size_t)items)
      throw Error{4, "capture workspace was not prepared"};
    h = up.host + up.cursor;
    dv = up.dev + up.cursor;
    up.cursor += ab;
  }
  std::memset(h, 0, bytes);
  return true;
}

template <typename T> void Engine<T>::commit(Upload& up, char* h, char* dv, size_t bytes) {
  if (!up.immediate) return;  // the whole image is copied before the first kernel
  hip_check(hipMemcpyAsync(dv, h, bytes, hipMemcpyHostToDevice, st_), "upload");
  hip_check(hipEventRecord(stage_.done, st_), "hipEventRecord");
}

template <typename T> void Engine<T>::prepare_capture(const Upload& dry) {
  work_.alloc(dry.work_need);
  sweeps_.alloc(sizeof(int) * 2 * std::max(1, dry.max_items));
}

template <typename T> void Engine<T>::run_sublayer(const std::vector<GateOp>& ops) {
  Upload up;
  run_sublayer(ops, up);
}

namespace {
std::atomic<int> g_fail_next{0};
}
void inject_update_failure(int status) { g_fail_next.store(status); }

template <typename T> void Engine<T>::run_sublayer(const std::vector<GateOp>& ops, Upload& up) {
  if (!ops.empty()) {
    if (const int f = g_fail_next.exchange(0)) throw Error{f, "injected failure before a sublayer"};
  }
  std::vector<const GateOp*> one, two, three;
  for (const GateOp& g : ops) {
    if (g.q == 1) one.push_back(&g);
    else if (g.q == 2) two.push_back(&g);
    else three.push_back(&g);
  }
  // chunks bounded by a workspace budget
  const size_t budget = (size_t)8 << 30;
  const int kx = cfg_.kap_max, cx = cfg_.chi_max, mm = std::max(1, cfg_.mmax);
  const size_t per2 = (size_t)(2 * kx * cx) * (4 * cx) * sizeof(cpx<T>) * 2 +
                      (size_t)(4 * cx) * (4 * cx) * 16 * 4 + (size_t)(kx * mm) * (kx * mm) * 16 * 3 + (1 << 20);
  const int chunk2 = (int)std::max<size_t>(1, budget / per2);
  for (size_t a = 0; a < one.size(); a += 4096)
    run_1q(std::vector<const GateOp*>(one.begin() + a, one.begin() + std::min(one.size(), a + 4096)), up);
  for (size_t a = 0; a < two.size(); a += chunk2)
    run_2q(std::vector<const GateOp*>(two.begin() + a, two.begin() + std::min(two.size(), a + chunk2)), up);
  for (size_t a = 0; a < three.size(); a += 8)
    run_3q(std::vector<const GateOp*>(three.begin() + a, three.begin() + std::min(three.size(), a + 8)), up);
}

template <typename T>
void Engine<T>::run_1q(const std::vector<const GateOp*>& ops, Upload& up, bool force, const TruncParams* tpo) {
  const int n = (int)ops.size();
  if (n == 0) return;
  const int kx = cfg_.kap_max, cx = cfg_.chi_max;
  int m1 = 1;
  for (auto* g : ops) m1 = std::max(m1, g->ch ? g->ch->m : 1);
  // (2k)^2 Gram over chi^2 terms: small output, long K -> 32 x 32 tiles, more splits
  const int tileH = tuned_tile(GS_Q1_GRAM, 2 * kx <= 32 ? 32 : 64);
  const int splitsH = tuned_splits(GS_Q1_GRAM, splits_for((long long)cx * cx * (tileH == 32 ? 4 : 1)));
  const int ng = kx * m1;  // largest Gamma
  // ---- workspace layout per item ----
  Layout w;
  const size_t oG = w.add((size_t)m1 * 4 * 16);
  const size_t oH = w.add((size_t)4 * kx * kx * 16);
  const size_t oHp = w.add((size_t)splitsH * 4 * kx * kx * 16);
  const size_t oGam = w.add((size_t)ng * ng * 16);
  const size_t oEv = w.add((size_t)(ng + 1) * 8);
  const size_t oVec = w.add((size_t)ng * ng * 16);
  const size_t oWk = w.add((size_t)eig_work_doubles(ng) * 8);
  const size_t oW = w.add((size_t)4 * kx * kx * sizeof(cpx<T>));
  const size_t per = w.off;
  // ---- upload layout ----
  Layout u;
  const size_t uCtx = u.add(sizeof(Ctx1<T>) * n);
  const size_t uH = u.add(sizeof(GemmDesc) * n);
  const size_t uE = u.add(sizeof(EigDesc) * n);
  const size_t uA = u.add(sizeof(GemmDesc) * n);
  const size_t uOut = u.add(sizeof(double*) * n);
  const size_t uU = u.add(sizeof(double) * 8 * n);
  char *h = nullptr, *dv = nullptr;
  if (!reserve(up, u.off, per * n, n, h, dv)) return;
  char* wk = reinterpret_cast<char*>(work_.p);
  for (int it = 0; it < n; ++it) {
    const GateOp& g = *ops[it];
    char* base = wk + per * it;
    Ctx1<T>& c = at<Ctx1<T>>(h, uCtx)[it];
    double* uslot = at<double>(h, uU) + 8 * it;
    c.g.kind = g.kind; c.g.q = 1; c.g.pidx = g.pidx; c.g.scale = g.scale; c.g.params = g.params;
    c.g.ufix = g.ufix;
    if (g.has_u) {
      std::memcpy(uslot, g.uhost, 8 * sizeof(double));
      c.g.ufix = reinterpret_cast<const double*>(dv + uU) + 8 * it;
    }
    c.kraus = g.ch ? g.ch->kraus.as<double>() : nullptr;
    c.m = g.ch ? g.ch->m : 1;
    c.force = force ? 1 : 0;
    const int b = g.inst, i = g.site;
    const int p = par_[soff_[b] + i];
    c.Bold = site(b, i, p);
    c.Bnew = site(b, i, 1 - p);
    c.laml2 = laml2(b, i);
    c.chil = chi_ptr(b, i);
    c.chir = chi_ptr(b, i + 1);
    c.kap = kap_ptr(b, i);
    c.disc = disc_ptr(b, i);
    c.G = at<double>(base, oG);
    c.H = at<double>(base, oH);
    c.Gam = at<double>(base, oGam);
    c.ev = at<double>(base, oEv);
    c.evec = at<double>(base, oVec);
    c.W = at<cpx<T>>(base, oW);
    c.dH = reinterpret_cast<GemmDesc*>(dv + uH) + it;
    c.dE = reinterpret_cast<EigDesc*>(dv + uE) + it;
    c.dA = reinterpret_cast<GemmDesc*>(dv + uA) + it;
    GemmDesc& dh = at<GemmDesc>(h, uH)[it];
    dh.C = at<double>(base, oHp);
    dh.sSplit = (long long)4 * kx * kx;
    EigDesc& de = at<EigDesc>(h, uE)[it];
    de.work = at<double>(base, oWk);
    de.kvec = kx;
    at<double*>(h, uOut)[it] = c.H;
  }
  commit(up, h, dv, u.off);
  Ctx1<T>* dctx = reinterpret_cast<Ctx1<T>*>(dv + uCtx);
  TruncParams tp{cfg_.chi_max, cfg_.kap_max, cfg_.svd_cut, cfg_.kap_cut, cfg_.tolE};
  if (tpo) tp = *tpo;
  // at most GV_ROWS rows: the Gram on the vector units
  const bool vec = gram_vector() && 2 * kx <= GV_ROWS;
  launch_q1_prepare<T>(dctx, n, splitsH, st_);
  if (vec)
    launch_gram_v<T>(reinterpret_cast<GemmDesc*>(dv + uH), n, splitsH, st_);
  else
    launch_gemm_site<T, double, double>(GS_Q1_GRAM, reinterpret_cast<GemmDesc*>(dv + uH), n, 1, splitsH,
                            [&](int tl) { return gemm_tiles(2 * kx, 2 * kx, tl); }, st_, tileH);
  launch_reduce_splits(reinterpret_cast<GemmDesc*>(dv + uH), reinterpret_cast<double**>(dv + uOut), n,
                       4 * kx * kx, st_);
  launch_q1_gamma<T>(dctx, n, st_);
  launch_eigh(reinterpret_cast<EigDesc*>(dv + uE), n, ng, sweeps_.as<int>(), st_);
  launch_q1_select<T>(dctx, n, tp, st_);
  launch_gemm_site<T, T, T>(GS_Q1_PROJ, reinterpret_cast<GemmDesc*>(dv + uA), n, cx, 1,
                          [&](int tl) { return gemm_tiles(2 * kx, cx, tl); }, st_, 64);
  hip_check(hipGetLastError(), "launch (1q sublayer)");
  for (auto* g : ops) par_[soff_[g->inst] + g->site] ^= 1;
}

template <typename T> void Engine<T>::run_2q(const std::vector<const GateOp*>& ops, Upload& up) {
  const int n = (int)ops.size();
  if (n == 0) return;
  const int kx = cfg_.kap_max, cx = cfg_.chi_max;
  int m2 = 1;
  for (auto* g : ops) m2 = std::max(m2, g->ch ? g->ch->m : 1);
  const int tileH0 = 4 * kx <= 32 ? 32 : 64;  // default tile of the H Gram and of theta''
  const int tileH = tuned_tile(GS_Q2_GRAM_H, tileH0);
  const int splitsH = tuned_splits(GS_Q2_GRAM_H, splits_for((long long)cx * 2 * cx * (tileH == 32 ? 4 : 1)));
  const int splitsE = tuned_splits(GS_Q2_GRAM_E, splits_for((long long)kx * cx));
  const int splitsC = tuned_splits(GS_Q2_GRAM_C, splits_for((long long)2 * kx * cx));
  const int ng = kx * m2;
  const long long thetaN = (long long)2 * kx * cx;
  Layout w;
  const size_t oG = w.add((size_t)m2 * 16 * 16);
  const size_t oH = w.add((size_t)16 * kx * kx * 16);
  const size_t oHp = w.add((size_t)splitsH * 16 * kx * kx * 16);
  const size_t oE = w.add((size_t)4 * cx * cx * 16);
  const size_t oEp = w.add((size_t)splitsE * 4 * cx * cx * 16);
  const size_t oGam = w.add((size_t)ng * ng * 16);
  const size_t oEvG = w.add((size_t)(ng + 1) * 8);
  const size_t oVecG = w.add((size_t)ng * ng * 16);
  const size_t oWkG = w.add((size_t)eig_work_doubles(ng) * 8);
  const size_t oEvE = w.add((size_t)(2 * cx + 1) * 8);
  const size_t oVecE = w.add((size_t)4 * cx * cx * 16);
  const size_t oWkE = w.add((size_t)eig_work_doubles(2 * cx) * 8);
  const size_t oEvC = w.add((size_t)(4 * cx + 1) * 8);
  const size_t oVecC = w.add((size_t)16 * cx * cx * 16);
  const size_t oWkC = w.add((size_t)eig_work_doubles(4 * cx) * 8);
  const size_t oW = w.add((size_t)16 * kx * kx * sizeof(cpx<T>));
  const size_t oLF = w.add((size_t)4 * cx * cx * sizeof(cpx<T>));
  const size_t oPD = w.add((size_t)4 * cx * cx * 16);
  const size_t oTh = w.add((size_t)thetaN * 4 * cx * sizeof(cpx<T>));
  const size_t oTh2 = w.add((size_t)thetaN * 4 * cx * sizeof(cpx<T>));
  const size_t oCm = w.add((size_t)16 * cx * cx * 16);
  const size_t oCp = w.add((size_t)splitsC * 16 * cx * cx * 16);
  const size_t oZt = w.add((size_t)4 * cx * cx * 16);
  const size_t oZc = w.add((size_t)4 * cx * cx * sizeof(cpx<T>));
  const size_t oX = w.add((size_t)4 * cx * cx * sizeof(cpx<T>));
  const size_t oScr = w.add(16);
  const size_t per = w.off;
  Layout u;
  const size_t uCtx = u.add(sizeof(Ctx2<T>) * n);
  const size_t uGramE = u.add(sizeof(GemmDesc) * n);
  const size_t uEigE = u.add(sizeof(EigDesc) * n);
  const size_t uGramH = u.add(sizeof(GemmDesc) * n);
  const size_t uEigG = u.add(sizeof(EigDesc) * n);
  const size_t uTh = u.add(sizeof(GemmDesc) * n);
  const size_t uTh2 = u.add(sizeof(GemmDesc) * n);
  const size_t uC = u.add(sizeof(GemmDesc) * n);
  const size_t uEigC = u.add(sizeof(EigDesc) * n);
  const size_t uX = u.add(sizeof(GemmDesc) * n);
  const size_t uOut = u.add(sizeof(GemmDesc) * 2 * n);
  const size_t uOutsE = u.add(sizeof(double*) * n);
  const size_t uOutsH = u.add(sizeof(double*) * n);
  const size_t uOutsC = u.add(sizeof(double*) * n);
  const size_t uU = u.add(sizeof(double) * 32 * n);
  char *h = nullptr, *dv = nullptr;
  if (!reserve(up, u.off, per * n, 2 * n, h, dv)) return;
  char* wk = reinterpret_cast<char*>(work_.p);
  for (int it = 0; it < n; ++it) {
    const GateOp& g = *ops[it];
    char* base = wk + per * it;
    Ctx2<T>& c = at<Ctx2<T>>(h, uCtx)[it];
    double* uslot = at<double>(h, uU) + 32 * it;
    c.g.kind = g.kind; c.g.q = 2; c.g.pidx = g.pidx; c.g.scale = g.scale; c.g.params = g.params;
    c.g.ufix = g.ufix;
    if (g.has_u) {
      std::memcpy(uslot, g.uhost, 32 * sizeof(double));
      c.g.ufix = reinterpret_cast<const double*>(dv + uU) + 32 * it;
    }
    c.kraus = g.ch ? g.ch->kraus.as<double>() : nullptr;
    c.m = g.ch ? g.ch->m : 1;
    const int b = g.inst, i = g.site;
    const int pi = par_[soff_[b] + i], pj = par_[soff_[b] + i + 1];
    c.Bi = site(b, i, pi);
    c.Bj = site(b, i + 1, pj);
    c.Bi_new = site(b, i, 1 - pi);
    c.Bj_new = site(b, i + 1, 1 - pj);
    c.laml2 = laml2(b, i);
    c.lam = lam_ptr(b, i);
    c.lam2 = lam2_ptr(b, i);
    c.chil = chi_ptr(b, i);
    c.chim = chi_ptr(b, i + 1);
    c.chir = chi_ptr(b, i + 2);
    c.kap1 = kap_ptr(b, i);
    c.kap2 = kap_ptr(b, i + 1);
    c.disc = disc_ptr(b, i);
    c.scratch = at<int>(base, oScr);
    c.G = at<double>(base, oG);
    c.H = at<double>(base, oH);
    c.E = at<double>(base, oE);
    c.Gam = at<double>(base, oGam);
    c.evG = at<double>(base, oEvG);
    c.vecG = at<double>(base, oVecG);
    c.evE = at<double>(base, oEvE);
    c.vecE = at<double>(base, oVecE);
    c.evC = at<double>(base, oEvC);
    c.vecC = at<double>(base, oVecC);
    c.W = at<cpx<T>>(base, oW);
    c.LF = at<cpx<T>>(base, oLF);
    c.PD = at<double>(base, oPD);
    c.th = at<cpx<T>>(base, oTh);
    c.th2 = at<cpx<T>>(base, oTh2);
    c.Cm = at<double>(base, oCm);
    c.Zt = at<double>(base, oZt);
    c.Zc = at<cpx<T>>(base, oZc);
    c.X = at<cpx<T>>(base, oX);
    c.dGramE = reinterpret_cast<GemmDesc*>(dv + uGramE) + it;
    c.dEigE = reinterpret_cast<EigDesc*>(dv + uEigE) + it;
    c.dGramH = reinterpret_cast<GemmDesc*>(dv + uGramH) + it;
    c.dEigG = reinterpret_cast<EigDesc*>(dv + uEigG) + it;
    c.dTh = reinterpret_cast<GemmDesc*>(dv + uTh) + it;
    c.dTh2 = reinterpret_cast<GemmDesc*>(dv + uTh2) + it;
    c.dC = reinterpret_cast<GemmDesc*>(dv + uC) + it;
    c.dEigC = reinterpret_cast<EigDesc*>(dv + uEigC) + it;
    c.dX = reinterpret_cast<GemmDesc*>(dv + uX) + it;
    c.dOut = reinterpret_cast<GemmDesc*>(dv + uOut) + 2 * it;
    GemmDesc& hgE = at<GemmDesc>(h, uGramE)[it];
    hgE.C = at<double>(base, oEp);
    hgE.sSplit = (long long)4 * cx * cx;
    GemmDesc& hgH = at<GemmDesc>(h, uGramH)[it];
    hgH.C = at<double>(base, oHp);
    hgH.sSplit = (long long)16 * kx * kx;
    EigDesc& heE = at<EigDesc>(h, uEigE)[it];
    heE.work = at<double>(base, oWkE);
    heE.kvec = 2 * cx;  // every eigenpair of the right-factor Gram
    EigDesc& heG = at<EigDesc>(h, uEigG)[it];
    heG.work = at<double>(base, oWkG);
    heG.kvec = kx;
    GemmDesc& hc = at<GemmDesc>(h, uC)[it];
    hc.C = at<double>(base, oCp);
    hc.sSplit = (long long)16 * cx * cx;
    at<EigDesc>(h, uEigC)[it].work = at<double>(base, oWkC);
    at<EigDesc>(h, uEigC)[it].kvec = cx;
    at<double*>(h, uOutsE)[it] = c.E;
    at<double*>(h, uOutsH)[it] = c.H;
    at<double*>(h, uOutsC)[it] = c.Cm;
  }
  commit(up, h, dv, u.off);
  Ctx2<T>* dctx = reinterpret_cast<Ctx2<T>*>(dv + uCtx);
  TruncParams tp{cfg_.chi_max, cfg_.kap_max, cfg_.svd_cut, cfg_.kap_cut, cfg_.tolE};
  int* status = sweeps_.as<int>();
  launch_q2_prepare<T>(dctx, n, splitsE, st_);
  launch_gemm_site<T, double, double>(GS_Q2_GRAM_E, reinterpret_cast<GemmDesc*>(dv + uGramE), n, 1, splitsE,
                          [&](int tl) { return gemm_tiles_herm(2 * cx, tl); }, st_, 64);
  launch_reduce_splits(reinterpret_cast<GemmDesc*>(dv + uGramE), reinterpret_cast<double**>(dv + uOutsE), n,
                       4 * cx * cx, st_);
  if (e_cholesky() && 2 * cx <= 256) {
    launch_q2_chol_e<T>(dctx, n, 2 * cx, splitsH, tp, reinterpret_cast<EigDesc*>(dv + uEigE), st_);
  } else {
    launch_eigh(reinterpret_cast<EigDesc*>(dv + uEigE), n, 2 * cx, status, st_);
    launch_q2_select_e<T>(dctx, n, splitsH, tp, st_);
  }
  launch_gemm_site<T, T, T>(GS_Q2_THETA, reinterpret_cast<GemmDesc*>(dv + uTh), n, 1, 1,
                          [&](int tl) { return gemm_tiles((int)thetaN, 4 * cx, tl); }, st_, 64);
  if (gram_vector() && 4 * kx <= GV_ROWS)  // the inner Gram on the vector units
    launch_gram_v<T>(reinterpret_cast<GemmDesc*>(dv + uGramH), n, splitsH, st_);
  else
    launch_gemm_site<T, double, double>(GS_Q2_GRAM_H, reinterpret_cast<GemmDesc*>(dv + uGramH), n, 1, splitsH,
                            [&](int tl) { return gemm_tiles(4 * kx, 4 * kx, tl); }, st_, tileH);
  launch_reduce_splits(reinterpret_cast<GemmDesc*>(dv + uGramH), reinterpret_cast<double**>(dv + uOutsH), n,
                       16 * kx * kx, st_);
  launch_q2_gamma<T>(dctx, n, st_);
  launch_eigh(reinterpret_cast<EigDesc*>(dv + uEigG), n, ng, status + n, st_);
  launch_q2_select_g<T>(dctx, n, splitsC, tp, st_);
  launch_gemm_site<T, T, T>(GS_Q2_THETA2, reinterpret_cast<GemmDesc*>(dv + uTh2), n, cx, 1,
                          [&](int tl) { return gemm_tiles(4 * kx, 2 * cx, tl); }, st_, tileH0);
  launch_gemm_site<T, double, double>(GS_Q2_GRAM_C, reinterpret_cast<GemmDesc*>(dv + uC), n, 1, splitsC,
                          [&](int tl) { return gemm_tiles_herm(4 * cx, tl); }, st_, 64);
  launch_reduce_splits(reinterpret_cast<GemmDesc*>(dv + uC), reinterpret_cast<double**>(dv + uOutsC), n,
                       16 * cx * cx, st_);
  launch_eigh(reinterpret_cast<EigDesc*>(dv + uEigC), n, 4 * cx, status + 2 * n, st_);
  launch_q2_select_b<T>(dctx, n, tp, st_);
  launch_gemm_site<double, double, T>(GS_Q2_X, reinterpret_cast<GemmDesc*>(dv + uX), n, 1, 1,
                          [&](int tl) { return gemm_tiles(2 * cx, 2 * cx, tl); }, st_, 64);
  // B_i' (at most thetaN x cx) and B_{i+1}' (at most 2 cx x kx cx) share a launch
  launch_gemm_site<T, T, T>(GS_Q2_OUT, reinterpret_cast<GemmDesc*>(dv + uOut), 2 * n, 1, 1,
                          [&](int tl) { return std::max(gemm_tiles((int)thetaN, cx, tl), gemm_tiles(2 * cx, kx * cx, tl)); }, st_, 64);
  hip_check(hipGetLastError(), "launch (2q sublayer)");
  for (auto* g : ops) {
    par_[soff_[g->inst] + g->site] ^= 1;
    par_[soff_[g->inst] + g->site + 1] ^= 1;
  }
}

template <typename T>
void Engine<T>::expect(const std::vector<int>& inst, const std::vector<const double*>& ops_host, double* out_dev,
                       bool raw) {
  Upload up;
  expect(inst, ops_host, out_dev, raw, up);
}

template <typename T>
void Engine<T>::expect(const std::vector<int>& inst, const std::vector<const double*>& ops_host, double* out_dev,
                       bool raw, Upload& up) {
  // items: per instance a trace item (identity) followed by its observables,
  // in the order given (inst[] must be grouped by instance).
  struct It { int b; const double* ops; int trace; };
  std::vector<It> items;
  int last = -1, trace_idx = 0;
  std::vector<int> result_index;  // item index of each requested observable
  for (size_t k = 0; k < inst.size(); ++k) {
    if (inst[k] != last) {
      trace_idx = (int)items.size();
      items.push_back({inst[k], nullptr, trace_idx});
      last = inst[k];
    }
    result_index.push_back((int)items.size());
    items.push_back({inst[k], ops_host[k], trace_idx});
  }
  const int n = (int)items.size();
  int nmax = 0;
  for (auto& it : items) nmax = std::max(nmax, nq_[it.b]);
  // Each observable only needs the sites between its first and last
  // non-identity factor: the left environment before the first comes from
  // the instance's identity (trace) sweep, which keeps every L_s, and the
  // environment after the last is the right environment R_{last+1} of the
  // instance, from one right sweep.
  std::vector<int> fst(n), lst(n), slot(n);  // non-identity range of each item
  int ninst = 0;
  for (int it = 0; it < n; ++it) {
    const int nb = nq_[items[it].b];
    if (!items[it].ops) {  // the trace item: every site, recorded
      slot[it] = ninst++;
      fst[it] = 0;
      lst[it] = nb - 1;
      continue;
    }
    slot[it] = slot[items[it].trace];
    fst[it] = nb;
    lst[it] = -1;
    for (int s = 0; s < nb; ++s) {
      const double* o = items[it].ops + 8 * s;
      const bool id = o[0] == 1.0 && o[1] == 0.0 && o[2] == 0.0 && o[3] == 0.0 && o[4] == 0.0 && o[5] == 0.0 &&
                      o[6] == 1.0 && o[7] == 0.0;
      if (!id) {
        fst[it] = std::min(fst[it], s);
        lst[it] = s;
      }
    }
  }
  const int cx = cfg_.chi_max;
  Layout w;  // per item
  const size_t oE0 = w.add((size_t)cx * cx * sizeof(cpx<T>));
  const size_t oE1 = w.add((size_t)cx * cx * sizeof(cpx<T>));
  const size_t oBO = w.add(cap_site_ * sizeof(cpx<T>));
  const size_t oY = w.add(cap_site_ * sizeof(cpx<T>));
  const size_t per = w.off;
  Layout v;  // per instance: L_0 .. L_nmax, R_0 .. R_nmax, W
  const size_t oL = v.add((size_t)(nmax + 1) * cx * cx * sizeof(cpx<T>));
  const size_t oR = v.add((size_t)(nmax + 1) * cx * cx * sizeof(cpx<T>));
  const size_t oW = v.add(cap_site_ * sizeof(cpx<T>));
  const size_t env = v.off;
  const int nr = std::max(1, nmax - 1);  // right-sweep steps
  Layout u;
  const size_t uCtx = u.add(sizeof(CtxT<T>) * (size_t)nmax * n);
  const size_t uD1 = u.add(sizeof(GemmDesc) * (size_t)nmax * n);
  const size_t uD2 = u.add(sizeof(GemmDesc) * (size_t)nmax * n);
  const size_t uCtxR = u.add(sizeof(CtxR<T>) * (size_t)nr * ninst);
  const size_t uD3 = u.add(sizeof(GemmDesc) * (size_t)nr * ninst);
  const size_t uD4 = u.add(sizeof(GemmDesc) * (size_t)nr * ninst);
  const size_t uOps = u.add(sizeof(double) * 8 * (size_t)nmax * n);
  const size_t uRes = u.add(sizeof(double) * 2 * n);
  const size_t uIdx = u.add(sizeof(int) * result_index.size());
  char *h = nullptr, *dv = nullptr;
  if (!reserve(up, u.off, per * n + env * ninst, 0, h, dv)) return;
  char* wk = reinterpret_cast<char*>(work_.p);
  char* ebase = wk + per * n;
  auto Lp = [&](int it, int s) { return at<cpx<T>>(ebase + env * slot[it], oL) + (size_t)s * cx * cx; };
  auto Rp = [&](int it, int s) { return at<cpx<T>>(ebase + env * slot[it], oR) + (size_t)s * cx * cx; };
  std::memcpy(h + uIdx, result_index.data(), sizeof(int) * result_index.size());
  for (int it = 0; it < n; ++it) {
    const int b = items[it].b, nb = nq_[b];
    const bool rec = !items[it].ops, any = fst[it] <= lst[it];
    double* ops = at<double>(h, uOps) + 8 * (size_t)nmax * it;
    for (int s = 0; s < nb; ++s) {
      if (items[it].ops) {
        std::memcpy(ops + 8 * s, items[it].ops + 8 * s, 8 * sizeof(double));
      } else {
        const double id[8] = {1, 0, 0, 0, 0, 0, 1, 0};
        std::memcpy(ops + 8 * s, id, sizeof(id));
      }
    }
    char* base = wk + per * it;
    cpx<T>* E[2] = {at<cpx<T>>(base, oE0), at<cpx<T>>(base, oE1)};
    cpx<T>* efin = rec || !any ? Lp(it, nb) : E[(lst[it] - fst[it]) & 1];
    const bool rfin = !rec && any && lst[it] + 1 < nb;
    for (int s = 0; s < nmax; ++s) {
      CtxT<T>& c = at<CtxT<T>>(h, uCtx)[(size_t)s * n + it];
      c.ops = reinterpret_cast<const double*>(dv + uOps) + 8 * (size_t)nmax * it;
      c.site = s;
      c.active = s < nb && s >= fst[it] && s <= lst[it];
      c.trace_idx = raw ? -1 : items[it].trace;
      c.stat = rec ? disc_ptr(b, 0) : nullptr;
      if (rec) {
        c.Ecur = Lp(it, s);
        c.Enext = Lp(it, s + 1);
      } else {
        c.Ecur = s == fst[it] ? Lp(it, s) : (s > fst[it] ? E[(s - 1 - fst[it]) & 1] : E[0]);
        c.Enext = E[(s - fst[it]) & 1];
      }
      c.Efinal = efin;
      c.Rfin = rfin ? Rp(it, lst[it] + 1) : nullptr;
      c.chif = rfin ? chi_ptr(b, lst[it] + 1) : nullptr;
      c.BO = at<cpx<T>>(base, oBO);
      c.Y = at<cpx<T>>(base, oY);
      c.d1 = reinterpret_cast<GemmDesc*>(dv + uD1) + (size_t)s * n + it;
      c.d2 = reinterpret_cast<GemmDesc*>(dv + uD2) + (size_t)s * n + it;
      if (s < nb) {
        c.B = site(b, s, par_[soff_[b] + s]);
        c.chil = chi_ptr(b, s);
        c.chir = chi_ptr(b, s + 1);
        c.kap = kap_ptr(b, s);
      } else {
        c.B = nullptr;
        c.chil = c.chir = c.kap = nullptr;
      }
    }
    if (!rec) continue;
    // right sweep of this instance: step t builds R_s, s = nb - 1 - t (s >= 1)
    for (int t = 0; t < nr; ++t) {
      CtxR<T>& r = at<CtxR<T>>(h, uCtxR)[(size_t)t * ninst + slot[it]];
      const int s = nb - 1 - t;
      r.d3 = reinterpret_cast<GemmDesc*>(dv + uD3) + (size_t)t * ninst + slot[it];
      r.d4 = reinterpret_cast<GemmDesc*>(dv + uD4) + (size_t)t * ninst + slot[it];
      r.active = s >= 1;
      r.last = t == 0;
      if (s >= 1) {
        r.B = site(b, s, par_[soff_[b] + s]);
        r.chil = chi_ptr(b, s);
        r.chir = chi_ptr(b, s + 1);
        r.kap = kap_ptr(b, s);
        r.Rn = Rp(it, s + 1);
        r.Rs = Rp(it, s);
        r.W = at<cpx<T>>(ebase + env * slot[it], oW);
      }
    }
  }
  commit(up, h, dv, u.off);
  CtxT<T>* dctx = reinterpret_cast<CtxT<T>*>(dv + uCtx);
  CtxR<T>* rctx = reinterpret_cast<CtxR<T>*>(dv + uCtxR);
  launch_transfer_init<T>(dctx, n, st_);
  for (int t = 0; t < nmax - 1; ++t) {
    launch_rtransfer_prep<T>(rctx + (size_t)t * ninst, ninst, st_);
    launch_gemm_site<T, T, T>(GS_TRANSFER_R, reinterpret_cast<GemmDesc*>(dv + uD3) + (size_t)t * ninst, ninst, 1, 1,
                            [&](int tl) { return gemm_tiles((int)(2 * cfg_.kap_max * cx), cx, tl); }, st_, 64);
    launch_gemm_site<T, T, T>(GS_TRANSFER_R, reinterpret_cast<GemmDesc*>(dv + uD4) + (size_t)t * ninst, ninst, 1, 1,
                            [&](int tl) { return gemm_tiles(cx, cx, tl); }, st_, 32);
  }
  for (int s = 0; s < nmax; ++s) {
    launch_transfer_prep<T>(dctx + (size_t)s * n, n, (int)cap_site_ / 2, st_);
    launch_gemm_site<T, T, T>(GS_TRANSFER_L, reinterpret_cast<GemmDesc*>(dv + uD1) + (size_t)s * n, n, 1, 1,
                            [&](int tl) { return gemm_tiles(cx, (int)(2 * cfg_.kap_max * cx), tl); }, st_, 64);
    // one cx x cx output over a long K per item: 32 x 32 tiles fill the CUs
    launch_gemm_site<T, T, T>(GS_TRANSFER_L, reinterpret_cast<GemmDesc*>(dv + uD2) + (size_t)s * n, n, 1, 1,
                            [&](int tl) { return gemm_tiles(cx, cx, tl); }, st_, 32);
  }
  double* res = reinterpret_cast<double*>(dv + uRes);
  launch_transfer_finish<T>(dctx, n, res, st_);
  // gather the requested observables in order
  const int nres = (int)result_index.size();
  hipLaunchKernelGGL(k_gather_pairs, dim3((nres + 255) / 256), dim3(256), 0, st_, res,
                     reinterpret_cast<const int*>(dv + uIdx), nres, out_dev);
  hip_check(hipGetLastError(), "launch (transfer)");
}

template <typename T>
void Engine<T>::dims(int b, std::vector<int>& bonds, std::vector<int>& inner, double& disc) {
  const int nb = nq_[b];
  std::vector<int> chi(nb + 1), kap(nb);
  std::vector<double> d((size_t)nb * ST_W);
  hip_check(hipMemcpyAsync(chi.data(), chi_ptr(b, 0), sizeof(int) * (nb + 1), hipMemcpyDeviceToHost, st_), "dims");
  hip_check(hipMemcpyAsync(kap.data(), kap_ptr(b, 0), sizeof(int) * nb, hipMemcpyDeviceToHost, st_), "dims");
  hip_check(hipMemcpyAsync(d.data(), disc_ptr(b, 0), sizeof(double) * nb * ST_W, hipMemcpyDeviceToHost, st_), "dims");
  hip_check(hipStreamSynchronize(st_), "hipStreamSynchronize");
  bonds.assign(chi.begin() + 1, chi.end() - 1);
  inner = kap;
  disc = 0;
  for (int i = 0; i < nb; ++i) disc += d[(size_t)i * ST_W + ST_DISC];
}

template <typename T> InstStats Engine<T>::stats(int b) {
  const int nb = nq_[b];
  std::vector<double> d((size_t)nb * ST_W);
  hip_check(hipMemcpyAsync(d.data(), disc_ptr(b, 0), sizeof(double) * nb * ST_W, hipMemcpyDeviceToHost, st_), "stats");
  hip_check(hipStreamSynchronize(st_), "hipStreamSynchronize");
  InstStats r;
  r.min_gap = 1e300;
  for (int i = 0; i < nb; ++i) {
    const double* x = &d[(size_t)i * ST_W];
    r.discarded += x[ST_DISC];
    r.max_discarded = std::max(r.max_discarded, x[ST_MAXD]);
    r.cuts += (long long)x[ST_CUTS];
    r.min_gap = std::min(r.min_gap, x[ST_GAP]);
    r.failures += (long long)x[ST_FAIL];
  }
  return r;
}

template <typename T> long long Engine<T>::failures() {
  std::vector<double> d((size_t)nsites_ * ST_W);
  hip_check(hipMemcpyAsync(d.data(), disc_.p, sizeof(double) * d.size(), hipMemcpyDeviceToHost, st_), "stats");
  hip_check(hipStreamSynchronize(st_), "hipStreamSynchronize");
  long long f = 0;
  for (int i = 0; i < nsites_; ++i) f += (long long)d[(size_t)i * ST_W + ST_FAIL];
  return f;
}

template <typename T> std::vector<double> Engine<T>::bond_weights(int b, int bond) {
  std::vector<int> bonds, inner;
  double disc;
  dims(b, bonds, inner, disc);
  const int len = bonds[bond];
  std::vector<double> v(len);
  hip_check(hipMemcpy(v.data(), lam_ptr(b, bond), sizeof(double) * len, hipMemcpyDeviceToHost), "lambda");
  return v;
}

// Three-site noisy gates (see Ctx3).  Requires kap_max m <= EIG_NMAX (the
// Gamma eigenproblem of the middle inner index); every other eigenproblem has
// size at most 4 chi_max.
template <typename T> void Engine<T>::run_3q(const std::vector<const GateOp*>& ops, Upload& up) {
  const int n = (int)ops.size();
  if (n == 0) return;
  const int kx = cfg_.kap_max, cx = cfg_.chi_max;
  int m3 = 1;
  for (auto* g : ops) m3 = std::max(m3, g->ch ? g->ch->m : 1);
  const int ng = kx * m3;
  if (ng > EIG_NMAX)
    throw Error{6 /*MPDO_EUNSUPPORTED*/, "3-site channels need kappa_max * (Kraus operators) <= 1024"};
  const int n2 = 2 * cx, n4 = 4 * cx, nh = 8 * kx;
  const size_t sT = sizeof(cpx<T>);
  const int spN = tuned_splits(GS_Q3_GRAM_NE, splits_for((long long)cx * kx));
  const int spE = tuned_splits(GS_Q3_GRAM_NE, splits_for((long long)kx * cx));
  const int spH = tuned_splits(GS_Q3_GRAM_H, splits_for((long long)n2 * n2));
  const int spC1 = tuned_splits(GS_Q3_GRAM_C1, splits_for((long long)nh * n2));
  const int spC2 = tuned_splits(GS_Q3_GRAM_C2, splits_for((long long)cx * 2 * kx));
  Layout w;
  const size_t oG = w.add((size_t)m3 * 64 * 16);
  const size_t oBp = w.add((size_t)cx * kx * n2 * sT);
  const size_t oN = w.add((size_t)n2 * n2 * 16), oNp = w.add((size_t)spN * n2 * n2 * 16);
  const size_t oEvN = w.add((size_t)(n2 + 1) * 8), oVecN = w.add((size_t)n2 * n2 * 16);
  const size_t oWkN = w.add((size_t)eig_work_doubles(n2) * 8);
  const size_t oE3 = w.add((size_t)n2 * n2 * 16), oE3p = w.add((size_t)spE * n2 * n2 * 16);
  const size_t oEvE = w.add((size_t)(n2 + 1) * 8), oVecE = w.add((size_t)n2 * n2 * 16);
  const size_t oWkE = w.add((size_t)eig_work_doubles(n2) * 8);
  const size_t oL1 = w.add((size_t)n2 * n2 * sT), oPND = w.add((size_t)n2 * n2 * 16);
  const size_t oL3 = w.add((size_t)n2 * n2 * sT), oPD3 = w.add((size_t)n2 * n2 * 16);
  const size_t oXt = w.add((size_t)cx * 2 * kx * n4 * sT);
  const size_t oPsi = w.add((size_t)n2 * nh * n2 * sT);
  const size_t oHin = w.add((size_t)nh * nh * 16), oHinp = w.add((size_t)spH * nh * nh * 16);
  const size_t oGam = w.add((size_t)ng * ng * 16), oEvG = w.add((size_t)(ng + 1) * 8);
  const size_t oVecG = w.add((size_t)ng * ng * 16), oWkG = w.add((size_t)eig_work_doubles(ng) * 8);
  const size_t oQop = w.add((size_t)nh * nh * sT);
  const size_t oPsi2 = w.add((size_t)n2 * nh * n2 * sT);
  const size_t oC1 = w.add((size_t)n4 * n4 * 16), oC1p = w.add((size_t)spC1 * n4 * n4 * 16);
  const size_t oEv1 = w.add((size_t)(n4 + 1) * 8), oVec1 = w.add((size_t)n4 * n4 * 16);
  const size_t oWk1 = w.add((size_t)eig_work_doubles(n4) * 8);
  const size_t oU1 = w.add((size_t)n4 * cx * sT), oU1s = w.add((size_t)n4 * cx * 16);
  const size_t oW1 = w.add((size_t)cx * 4 * kx * n2 * sT);
  const size_t oY1 = w.add((size_t)n2 * n2 * sT);
  const size_t oBiP = w.add((size_t)cx * kx * n2 * sT);
  const size_t oC2 = w.add((size_t)n4 * n4 * 16), oC2p = w.add((size_t)spC2 * n4 * n4 * 16);
  const size_t oEv2 = w.add((size_t)(n4 + 1) * 8), oVec2 = w.add((size_t)n4 * n4 * 16);
  const size_t oWk2 = w.add((size_t)eig_work_doubles(n4) * 8);
  const size_t oZt3 = w.add((size_t)n2 * n2 * 16), oZ2c = w.add((size_t)n4 * cx * sT);
  const size_t oY3 = w.add((size_t)n2 * n2 * sT);
  const size_t oScr = w.add(64), oKept = w.add(16);
  const size_t per = w.off;
  if (n > 1 && per * n > ((size_t)8 << 30)) {  // workspace budget: split the group
    const int h = n / 2;
    run_3q(std::vector<const GateOp*>(ops.begin(), ops.begin() + h), up);
    run_3q(std::vector<const GateOp*>(ops.begin() + h, ops.end()), up);
    return;
  }
  // descriptor kinds (item it of kind k at k n + it; kinds launched together are adjacent)
  enum { gN, gE3, gXt, gPsi, gHin, gPsi2, gC1, gY1, gW1, gBiP, gC2, gY3, gBk, gBj, gCount };
  enum { eN, eE3, eG, e1, e2, eCount };
  Layout u;
  const size_t uCtx = u.add(sizeof(Ctx3<T>) * n);
  const size_t uG = u.add(sizeof(GemmDesc) * gCount * n);
  const size_t uE = u.add(sizeof(EigDesc) * eCount * n);
  const size_t uOuts = u.add(sizeof(double*) * 5 * n);  // N E3 | Hin | C1 | C2
  const size_t uU = u.add(sizeof(double) * 128 * n);
  char *h = nullptr, *dv = nullptr;
  if (!reserve(up, u.off, per * n, 3 * n, h, dv)) return;
  char* wk = reinterpret_cast<char*>(work_.p);
  GemmDesc* dG = reinterpret_cast<GemmDesc*>(dv + uG);
  EigDesc* dE = reinterpret_cast<EigDesc*>(dv + uE);
  GemmDesc* hd = at<GemmDesc>(h, uG);
  EigDesc* he = at<EigDesc>(h, uE);
  double** outs = at<double*>(h, uOuts);
  for (int it = 0; it < n; ++it) {
    const GateOp& g = *ops[it];
    char* base = wk + per * it;
    Ctx3<T>& c = at<Ctx3<T>>(h, uCtx)[it];
    double* uslot = at<double>(h, uU) + 128 * it;
    c.g.kind = g.kind; c.g.q = 3; c.g.pidx = g.pidx; c.g.scale = g.scale; c.g.params = g.params;
    c.g.ufix = g.ufix;
    if (g.has_u) {
      std::memcpy(uslot, g.uhost, 128 * sizeof(double));
      c.g.ufix = reinterpret_cast<const double*>(dv + uU) + 128 * it;
    }
    c.kraus = g.ch ? g.ch->kraus.as<double>() : nullptr;
    c.m = g.ch ? g.ch->m : 1;
    const int b = g.inst, i = g.site;
    const int p0 = par_[soff_[b] + i], p1 = par_[soff_[b] + i + 1], p2 = par_[soff_[b] + i + 2];
    c.Bi = site(b, i, p0);
    c.Bj = site(b, i + 1, p1);
    c.Bk = site(b, i + 2, p2);
    c.Bi_new = site(b, i, 1 - p0);
    c.Bj_new = site(b, i + 1, 1 - p1);
    c.Bk_new = site(b, i + 2, 1 - p2);
    c.laml2 = laml2(b, i);
    c.lam1 = lam_ptr(b, i);
    c.lam1sq = lam2_ptr(b, i);
    c.lam2 = lam_ptr(b, i + 1);
    c.lam2sq = lam2_ptr(b, i + 1);
    c.chil = chi_ptr(b, i);
    c.chim1 = chi_ptr(b, i + 1);
    c.chim2 = chi_ptr(b, i + 2);
    c.chir = chi_ptr(b, i + 3);
    c.kap1 = kap_ptr(b, i);
    c.kap2 = kap_ptr(b, i + 1);
    c.kap3 = kap_ptr(b, i + 2);
    c.disc = disc_ptr(b, i);
    c.scratch = at<int>(base, oScr);
    c.kept = at<double>(base, oKept);
    c.G = at<double>(base, oG);
    c.Bp = at<cpx<T>>(base, oBp);
    c.N = at<double>(base, oN); c.evN = at<double>(base, oEvN); c.vecN = at<double>(base, oVecN);
    c.E3 = at<double>(base, oE3); c.evE3 = at<double>(base, oEvE); c.vecE3 = at<double>(base, oVecE);
    c.L1 = at<cpx<T>>(base, oL1); c.PND = at<double>(base, oPND);
    c.L3 = at<cpx<T>>(base, oL3); c.PD3 = at<double>(base, oPD3);
    c.Xt = at<cpx<T>>(base, oXt);
    c.Psi = at<cpx<T>>(base, oPsi);
    c.Hin = at<double>(base, oHin);
    c.Gam = at<double>(base, oGam); c.evG = at<double>(base, oEvG); c.vecG = at<double>(base, oVecG);
    c.Qop = at<cpx<T>>(base, oQop);
    c.Psi2 = at<cpx<T>>(base, oPsi2);
    c.C1 = at<double>(base, oC1); c.ev1 = at<double>(base, oEv1); c.vec1 = at<double>(base, oVec1);
    c.U1 = at<cpx<T>>(base, oU1); c.U1s = at<double>(base, oU1s);
    c.W1 = at<cpx<T>>(base, oW1);
    c.Y1 = at<cpx<T>>(base, oY1);
    c.BiP = at<cpx<T>>(base, oBiP);
    c.C2 = at<double>(base, oC2); c.ev2 = at<double>(base, oEv2); c.vec2 = at<double>(base, oVec2);
    c.Zt3 = at<double>(base, oZt3); c.Z2c = at<cpx<T>>(base, oZ2c);
    c.Y3 = at<cpx<T>>(base, oY3);
    c.dN = dG + gN * n + it; c.dE3 = dG + gE3 * n + it; c.dXt = dG + gXt * n + it; c.dPsi = dG + gPsi * n + it;
    c.dHin = dG + gHin * n + it; c.dPsi2 = dG + gPsi2 * n + it; c.dC1 = dG + gC1 * n + it;
    c.dY1 = dG + gY1 * n + it; c.dW1 = dG + gW1 * n + it; c.dBiP = dG + gBiP * n + it;
    c.dC2 = dG + gC2 * n + it; c.dY3 = dG + gY3 * n + it; c.dBk = dG + gBk * n + it; c.dBj = dG + gBj * n + it;
    c.eN = dE + eN * n + it; c.eE3 = dE + eE3 * n + it; c.eG = dE + eG * n + it;
    c.e1 = dE + e1 * n + it; c.e2 = dE + e2 * n + it;
    // split-K partial buffers of the Gram products (kept by the device-side descriptor setup)
    hd[gN * n + it].C = at<double>(base, oNp);    hd[gN * n + it].sSplit = (long long)n2 * n2;
    hd[gE3 * n + it].C = at<double>(base, oE3p);  hd[gE3 * n + it].sSplit = (long long)n2 * n2;
    hd[gHin * n + it].C = at<double>(base, oHinp); hd[gHin * n + it].sSplit = (long long)nh * nh;
    hd[gC1 * n + it].C = at<double>(base, oC1p);  hd[gC1 * n + it].sSplit = (long long)n4 * n4;
    hd[gC2 * n + it].C = at<double>(base, oC2p);  hd[gC2 * n + it].sSplit = (long long)n4 * n4;
    he[eN * n + it].a = c.N;   he[eN * n + it].work = at<double>(base, oWkN);  he[eN * n + it].kvec = n2;
    he[eE3 * n + it].a = c.E3; he[eE3 * n + it].work = at<double>(base, oWkE); he[eE3 * n + it].kvec = n2;
    he[eN * n + it].vfloor = Q3_BASIS_FLOOR;
    he[eE3 * n + it].vfloor = Q3_BASIS_FLOOR;
    he[eG * n + it].a = c.Gam; he[eG * n + it].work = at<double>(base, oWkG);  he[eG * n + it].kvec = kx;
    he[e1 * n + it].a = c.C1;  he[e1 * n + it].work = at<double>(base, oWk1);  he[e1 * n + it].kvec = cx;
    he[e2 * n + it].a = c.C2;  he[e2 * n + it].work = at<double>(base, oWk2);  he[e2 * n + it].kvec = cx;
    outs[it] = c.N;
    outs[n + it] = c.E3;
    outs[2 * n + it] = c.Hin;
    outs[3 * n + it] = c.C1;
    outs[4 * n + it] = c.C2;
  }
  commit(up, h, dv, u.off);
  Ctx3<T>* dctx = reinterpret_cast<Ctx3<T>*>(dv + uCtx);
  double** douts = reinterpret_cast<double**>(dv + uOuts);
  TruncParams tp{cfg_.chi_max, cfg_.kap_max, cfg_.svd_cut, cfg_.kap_cut, cfg_.tolE};
  int* status = sweeps_.as<int>();
  // outer bases
  launch_q3_prepare<T>(dctx, n, spN, spE, st_);
  launch_q3_perm_in<T>(dctx, n, st_);
  launch_gemm_site<T, double, double>(GS_Q3_GRAM_NE, dG + gN * n, 2 * n, 1, std::max(spN, spE),
                          [&](int tl) { return gemm_tiles_herm(n2, tl); }, st_, 64, 2);
  launch_reduce_splits(dG + gN * n, douts, 2 * n, n2 * n2, st_);
  launch_eigh(dE + eN * n, 2 * n, n2, status, st_);
  launch_q3_sel_env<T>(dctx, n, spH, Q3_BASIS_FLOOR, st_);
  // reduced block, middle inner truncation
  launch_gemm_site<T, T, T>(GS_Q3_XT, dG + gXt * n, n, 1, 1,
                          [&](int tl) { return gemm_tiles(cx * 2 * kx, n4, tl); }, st_, 64);
  launch_gemm_site<T, T, T>(GS_Q3_PSI, dG + gPsi * n, n, 2, 1,
                          [&](int tl) { return gemm_tiles(n2, 4 * kx * n2, tl); }, st_, 64);
  launch_gemm_site<T, double, double>(GS_Q3_GRAM_H, dG + gHin * n, n, 1, spH,
                          [&](int tl) { return gemm_tiles(nh, nh, tl); }, st_, 64);
  launch_reduce_splits(dG + gHin * n, douts + 2 * n, n, nh * nh, st_);
  launch_q3_gamma<T>(dctx, n, m3, st_);
  launch_eigh(dE + eG * n, n, ng, status + 2 * n, st_);
  launch_q3_sel_h<T>(dctx, n, spC1, tp, st_);
  launch_gemm_site<T, T, T>(GS_Q3_PSI2, dG + gPsi2 * n, n, n2, 1,
                          [&](int tl) { return gemm_tiles(nh, n2, tl); }, st_, 64);
  // bond i
  launch_gemm_site<T, double, double>(GS_Q3_GRAM_C1, dG + gC1 * n, n, 1, spC1,
                          [&](int tl) { return gemm_tiles_herm(n4, tl); }, st_, 64);
  launch_reduce_splits(dG + gC1 * n, douts + 3 * n, n, n4 * n4, st_);
  launch_eigh(dE + e1 * n, n, n4, status + 3 * n, st_);
  launch_q3_sel_1<T>(dctx, n, spC2, tp, st_);
  launch_gemm_site<double, double, T>(GS_Q3_Y1, dG + gY1 * n, n, 1, 1,
                          [&](int tl) { return gemm_tiles(n2, n2, tl); }, st_, 64);
  launch_gemm_site<T, T, T>(GS_Q3_W1, dG + gW1 * n, 2 * n, 1, 1,
                          [&](int tl) { return std::max(gemm_tiles(cx, 4 * kx * n2, tl), gemm_tiles(cx * kx, n2, tl)); }, st_, 64, 2);
  launch_q3_perm_out<T>(dctx, n, st_);
  // bond i+1
  launch_gemm_site<T, double, double>(GS_Q3_GRAM_C2, dG + gC2 * n, n, 1, spC2,
                          [&](int tl) { return gemm_tiles_herm(n4, tl); }, st_, 64);
  launch_reduce_splits(dG + gC2 * n, douts + 4 * n, n, n4 * n4, st_);
  launch_eigh(dE + e2 * n, n, n4, status + 4 * n, st_);
  launch_q3_sel_2<T>(dctx, n, tp, st_);
  launch_gemm_site<double, double, T>(GS_Q3_Y3, dG + gY3 * n, n, 1, 1,
                          [&](int tl) { return gemm_tiles(n2, n2, tl); }, st_, 64);
  launch_gemm_site<T, T, T>(GS_Q3_OUT, dG + gBk * n, 2 * n, 1, 1,
                          [&](int tl) { return std::max(gemm_tiles(n2, kx * cx, tl), gemm_tiles(2 * kx * cx, cx, tl)); }, st_, 64, 2);
  launch_q3_finish<T>(dctx, n, st_);
  hip_check(hipGetLastError(), "launch (3-site sublayer)");
  for (auto* g : ops)
    for (int t = 0; t < 3; ++t) par_[soff_[g->inst] + g->site + t] ^= 1;
}

// One sweep step (pass 0: site -> site + 1, pass 1: site -> site - 1) on the
// instances `inst`.
template <typename T>
void Engine<T>::sweep_step(const std::vector<int>& inst, int pass, int si, const TruncParams& tp) {
  const int n = (int)inst.size();
  if (n == 0) return;
  const int kx = cfg_.kap_max, cx = cfg_.chi_max;
  const int splits = tuned_splits(GS_SWEEP_GRAM, splits_for((long long)2 * kx * cx));
  Layout w;
  const size_t oG = w.add((size_t)cx * cx * 16);
  const size_t oGp = w.add((size_t)splits * cx * cx * 16);
  const size_t oEv = w.add((size_t)(cx + 1) * 8);
  const size_t oVec = w.add((size_t)cx * cx * 16);
  const size_t oWk = w.add((size_t)eig_work_doubles(cx) * 8);
  const size_t oP1 = w.add((size_t)cx * cx * sizeof(cpx<T>));
  const size_t oP2 = w.add((size_t)cx * cx * sizeof(cpx<T>));
  const size_t per = w.off;
  Layout u;
  const size_t uCtx = u.add(sizeof(CtxS<T>) * n);
  const size_t uG = u.add(sizeof(GemmDesc) * n);
  const size_t uE = u.add(sizeof(EigDesc) * n);
  const size_t uA = u.add(sizeof(GemmDesc) * 2 * n);
  const size_t uOut = u.add(sizeof(double*) * n);
  Upload up;
  char *h = nullptr, *dv = nullptr;
  if (!reserve(up, u.off, per * n, n, h, dv)) return;
  char* wk = reinterpret_cast<char*>(work_.p);
  const int nb = pass == 0 ? si + 1 : si - 1;
  for (int it = 0; it < n; ++it) {
    const int b = inst[it];
    char* base = wk + per * it;
    CtxS<T>& c = at<CtxS<T>>(h, uCtx)[it];
    const int pi = par_[soff_[b] + si], pn = par_[soff_[b] + nb];
    c.pass = pass;
    c.A = site(b, si, pi);
    c.Anew = site(b, si, 1 - pi);
    c.Bn = site(b, nb, pn);
    c.Bnnew = site(b, nb, 1 - pn);
    c.chil = chi_ptr(b, si);
    c.chir = chi_ptr(b, si + 1);
    c.kap = kap_ptr(b, si);
    c.chib = pass == 0 ? chi_ptr(b, si + 1) : chi_ptr(b, si);
    c.chio = pass == 0 ? chi_ptr(b, si + 2) : chi_ptr(b, si - 1);
    c.kapn = kap_ptr(b, nb);
    c.lam = pass == 1 ? lam_ptr(b, si - 1) : nullptr;
    c.lam2 = pass == 1 ? lam2_ptr(b, si - 1) : nullptr;
    c.disc = disc_ptr(b, si);
    c.ev = at<double>(base, oEv);
    c.evec = at<double>(base, oVec);
    c.P1 = at<cpx<T>>(base, oP1);
    c.P2 = at<cpx<T>>(base, oP2);
    c.dG = reinterpret_cast<GemmDesc*>(dv + uG) + it;
    c.dE = reinterpret_cast<EigDesc*>(dv + uE) + it;
    c.dA = reinterpret_cast<GemmDesc*>(dv + uA) + 2 * it;
    c.dB = c.dA + 1;
    GemmDesc& g = at<GemmDesc>(h, uG)[it];
    g.C = at<double>(base, oGp);
    g.sSplit = (long long)cx * cx;
    EigDesc& e = at<EigDesc>(h, uE)[it];
    e.a = at<double>(base, oG);
    e.work = at<double>(base, oWk);
    e.kvec = cx;
    at<double*>(h, uOut)[it] = at<double>(base, oG);
  }
  commit(up, h, dv, u.off);
  CtxS<T>* dctx = reinterpret_cast<CtxS<T>*>(dv + uCtx);
  launch_sw_prepare<T>(dctx, n, splits, st_);
  launch_gemm_site<T, double, double>(GS_SWEEP_GRAM, reinterpret_cast<GemmDesc*>(dv + uG), n, 1, splits,
                          [&](int tl) { return gemm_tiles_herm(cx, tl); }, st_, 64);
  launch_reduce_splits(reinterpret_cast<GemmDesc*>(dv + uG), reinterpret_cast<double**>(dv + uOut), n, cx * cx,
                       st_);
  launch_eigh(reinterpret_cast<EigDesc*>(dv + uE), n, cx, sweeps_.as<int>(), st_);
  launch_sw_select<T>(dctx, n, tp, st_);
  const int tiles = std::max(gemm_tiles(2 * kx * cx, cx), gemm_tiles(cx, 2 * kx * cx));
  const int tiles32 = std::max(gemm_tiles(2 * kx * cx, cx, 32), gemm_tiles(cx, 2 * kx * cx, 32));
  launch_gemm_site<T, T, T>(GS_SWEEP_OUT, reinterpret_cast<GemmDesc*>(dv + uA), 2 * n, 1, 1,
                          [&](int tl) { return tl == 64 ? tiles : tiles32; }, st_, 64);
  hip_check(hipGetLastError(), "launch (truncation sweep)");
  for (int b : inst) {
    par_[soff_[b] + si] ^= 1;
    par_[soff_[b] + nb] ^= 1;
  }
}

// The truncation sweep of Sec. II.D on instance b: orthonormalise from left
// to right, SVD from right to left with the bond rule (chi_max, cut), then
// truncate every inner index to kap_max.  Returns the discarded weight.
template <typename T> double Engine<T>::truncate_sweep(int b, int chi_max, int kap_max, double cut) {
  std::vector<int> b0, b1;
  double d0 = 0, d1 = 0;
  dims(b, b0, b1, d0);
  const int n = nq_[b];
  const std::vector<int> one{b};
  TruncParams tp{chi_max, kap_max, cut, cfg_.kap_cut, cfg_.tolE};
  for (int i = 0; i + 1 < n; ++i) sweep_step(one, 0, i, tp);
  for (int i = n - 1; i >= 1; --i) sweep_step(one, 1, i, tp);
  {  // normalise the first site
    Upload up;
    char *h = nullptr, *dv = nullptr;
    if (reserve(up, sizeof(CtxS<T>), 0, 1, h, dv)) {
      CtxS<T>& c = *reinterpret_cast<CtxS<T>*>(h);
      c.Anew = site(b, 0, par_[soff_[b]]);
      c.chil = chi_ptr(b, 0);
      c.chir = chi_ptr(b, 1);
      c.kap = kap_ptr(b, 0);
      commit(up, h, dv, sizeof(CtxS<T>));
      launch_sw_normalize<T>(reinterpret_cast<CtxS<T>*>(dv), 1, st_);
      hip_check(hipGetLastError(), "launch (normalise)");
    }
  }
  {  // inner truncation of every site (identity operators, forced)
    std::vector<GateOp> ops(n);
    std::vector<const GateOp*> ptrs;
    for (int i = 0; i < n; ++i) {
      ops[i].inst = b;
      ops[i].site = i;
      ops[i].q = 1;
      ops[i].kind = 0;
      ops[i].pidx = -1;
      ops[i].scale = 1.0;
      ops[i].params = nullptr;
      ops[i].ufix = nullptr;
      ops[i].has_u = false;
      ops[i].ch = nullptr;
      ptrs.push_back(&ops[i]);
    }
    Upload up;
    run_1q(ptrs, up, true, &tp);
  }
  dims(b, b0, b1, d1);
  return d1 - d0;
}

template class Engine<double>;
template class Engine<float>;

}  // namespace mpdo
