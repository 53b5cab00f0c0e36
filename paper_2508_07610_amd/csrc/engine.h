// Host-side runtime of libmpdo: device state of one or many MPDO instances
// and the launch sequences of a sublayer of noisy gates on disjoint sites.
#pragma once
#include <string>
#include <vector>

#include "common.h"
#include "ops.h"

namespace mpdo {

struct Error {
  int status;
  std::string msg;
};

// Makes the next run_sublayer of any engine throw Error{status} before it
// launches anything (tests of the error paths; 0 cancels).
void inject_update_failure(int status);

void hip_check(hipError_t e, const char* what);
// Records the message returned by mpdo_last_error() and passes the status through.
int set_last_error(int status, const std::string& msg);

// Where device memory comes from.  A caller may supply an allocator (the
// alloc/free hooks of mpdo_config, e.g. a framework's caching allocator);
// otherwise blocks come from the library's own cache: a freed block is kept
// per device and handed to the next request it fits (at most twice its
// size), so repeated runs of the same shapes allocate nothing after the
// first.  mpdo_release_cached_memory() returns the cache to the driver.
struct DeviceAllocator {
  void* (*alloc)(size_t bytes, void* ctx) = nullptr;
  void (*free)(void* ptr, void* ctx) = nullptr;
  void* ctx = nullptr;
};
// The allocator of the running entry point (set by an AllocScope; none: the cache).
const DeviceAllocator* current_allocator();
struct AllocScope {
  const DeviceAllocator* prev;
  explicit AllocScope(const DeviceAllocator* a);
  ~AllocScope();
};
void release_cached_memory();
size_t cached_device_bytes();
// Pinned host blocks from the same kind of cache.
void* pinned_get(size_t n, size_t* got);
void pinned_put(void* p, size_t n);

// Device allocation owned by the runtime (freed on destruction, through the
// allocator it came from).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DeviceAllocator from;   // hooks of the allocation (alloc == null: the cache)
  int device = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf();
  void alloc(size_t n);   // (re)allocates when n > bytes; contents are lost
  void release();
  template <typename X> X* as() const { return reinterpret_cast<X*>(p); }
};

// Pinned host staging area for descriptor uploads.
struct HostStage {
  void* p = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
  ~HostStage();
  void* get(size_t n);    // waits until the previous upload finished
};

// C = op(A) op(B) in FP64, one item (descriptor staged in `dd`); herm: C is
// Hermitian and only its upper triangle of tiles is written.  Synchronises s.
void gemm_once(DevBuf& dd, const cpx<double>* A, const cpx<double>* B, cpx<double>* C, int M, int N, int K, int opA,
               int opB, int lda, int ldb, int ldc, hipStream_t s, bool herm);

struct InstStats {
  double discarded = 0, max_discarded = 0, min_gap = 0;
  long long cuts = 0, failures = 0;
};

struct Channel {
  int q = 0, m = 0;
  DevBuf kraus;           // m x d x d complex double
  std::vector<double> host_kraus;
  double completeness_err = 0, min_eig = 0;
};

// A gate of a sublayer: sites [site, site + q), ideal gate source, channel.
struct GateOp {
  int inst = 0, site = 0, q = 1;
  int kind = GK_FIXED, pidx = -1;
  double scale = 1.0;
  const double* params = nullptr;  // device
  const double* ufix = nullptr;    // device (filled by the executor from `uhost`)
  double uhost[2 * 64];
  bool has_u = false;
  const Channel* ch = nullptr;
};

struct Config {
  int chi_max = 16, kap_max = 4, mmax = 16;
  double svd_cut = 1e-14, kap_cut = 1e-14;
  double tolE = 1e-13;
};

// Where the descriptors of the launch sequences go.  Immediate mode (the
// default) copies each sequence's descriptors to the device right before
// its kernels.  For graph capture a run is planned twice: a dry pass that
// only measures the descriptor bytes and the workspace, then a pass that
// writes every sequence's descriptors into one host image (`host`, pinned)
// of one device blob (`dev`) and launches the kernels; the image is copied
// to the device by a single copy issued before the first kernel.
struct Upload {
  bool dry = false;
  bool immediate = true;
  char* host = nullptr;
  char* dev = nullptr;
  size_t cursor = 0;
  size_t work_need = 0;
  int max_items = 0;
};

template <typename T> class Engine {
 public:
  Engine(const Config& cfg, const std::vector<int>& nq, hipStream_t s);
  ~Engine() = default;

  // One group of gates on pairwise disjoint sites (any mix of 1q and 2q).
  void run_sublayer(const std::vector<GateOp>& ops);
  void run_sublayer(const std::vector<GateOp>& ops, Upload& up);
  // Tr(O_k rho) / Tr rho for product operators; ops_host: per item n x 4 complex.
  // Results (complex) are written to out_dev (device, 2 doubles per item, items
  // of all instances concatenated in the order given).
  void expect(const std::vector<int>& inst, const std::vector<const double*>& ops_host, double* out_dev,
              bool raw = false);
  void expect(const std::vector<int>& inst, const std::vector<const double*>& ops_host, double* out_dev,
              bool raw, Upload& up);
  // Allocate the workspace and status buffers measured by a dry pass.
  void prepare_capture(const Upload& dry);
  // The Sec. II.D sweep on instance b.
  double truncate_sweep(int b, int chi_max, int kap_max, double cut);

  void dims(int b, std::vector<int>& bonds, std::vector<int>& inner, double& disc);
  // truncation statistics of instance b (reads the per-site records)
  InstStats stats(int b);
  // numerical failures recorded on the device, summed over all instances
  long long failures();
  // site tensor of instance b, site i (current buffer): for host-side tests
  void* site_ptr(int b, int i) { return site(b, i, par_[soff_[b] + i]); }
  std::vector<double> bond_weights(int b, int bond);
  // rho of instance b (n <= 12) as 2^n x 2^n complex doubles into `out`
  // (host memory, or device memory when device_out)
  void to_dense(int b, double* out, bool device_out = false);
  // nshots bitstrings by sequential conditionals (u: nshots x n uniforms,
  // host; bits: nshots x n, host; pz: probability of each, host or null)
  void sample(int b, const double* u_host, int nshots, unsigned char* bits_host, double* pz_host);

  const Config& config() const { return cfg_; }
  int nq(int b) const { return nq_[b]; }
  int ninst() const { return (int)nq_.size(); }
  hipStream_t stream() const { return st_; }

  // capture support: sizes of the upload blobs must not change during capture
  bool capturing = false;

 private:
  Config cfg_;
  std::vector<int> nq_, soff_;
  int nsites_ = 0;
  hipStream_t st_;
  size_t cap_site_ = 0;
  DevBuf sites_, lam_, lam2_, one_, dims_, disc_;
  std::vector<int> par_;
  DevBuf work_, blob_;
  HostStage stage_;
  DevBuf sweeps_;

  cpx<T>* site(int b, int i, int p) const {
    return sites_.as<cpx<T>>() + ((size_t)(soff_[b] + i) * 2 + p) * cap_site_;
  }
  int* chi_ptr(int b, int i) const { return dims_.as<int>() + soff_[b] + b + i; }  // bond left of site i
  int* kap_ptr(int b, int i) const { return dims_.as<int>() + nsites_ + (int)nq_.size() + soff_[b] + i; }
  double* lam_ptr(int b, int bond) const { return lam_.as<double>() + (size_t)(soff_[b] + bond) * cfg_.chi_max; }
  double* lam2_ptr(int b, int bond) const { return lam2_.as<double>() + (size_t)(soff_[b] + bond) * cfg_.chi_max; }
  const double* laml2(int b, int i) const { return i == 0 ? one_.as<double>() : lam2_ptr(b, i - 1); }
  double* disc_ptr(int b, int i) const { return disc_.as<double>() + (size_t)(soff_[b] + i) * ST_W; }

  // force: truncate the inner index even for unitary ops; tpo overrides the
  // truncation parameters of the configuration.
  void run_1q(const std::vector<const GateOp*>& ops, Upload& up, bool force = false,
              const TruncParams* tpo = nullptr);
  void sweep_step(const std::vector<int>& inst, int pass, int site, const TruncParams& tp);
  void run_2q(const std::vector<const GateOp*>& ops, Upload& up);
  void run_3q(const std::vector<const GateOp*>& ops, Upload& up);
  int splits_for(long long K) const;
  // descriptor space of `bytes` (host image h, device address dv); false in a dry pass
  bool reserve(Upload& up, size_t bytes, size_t work_bytes, int items, char*& h, char*& dv);
  void commit(Upload& up, char* h, char* dv, size_t bytes);
};

}  // namespace mpdo
