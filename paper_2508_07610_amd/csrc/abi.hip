// C ABI of libmpdo (declared in include/mpdo.h).  Argument checking, the
// gate queue that groups gates on disjoint sites into sublayers, and the
// translation of host inputs into device work.  No exception crosses the ABI.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mpdo.h"
#include "engine.h"
#include "kernels.h"
#include "mpo.h"
#include "ops.h"
#include "profile.h"

using namespace mpdo;

namespace {
thread_local std::string g_err;

mpdo_status fail(int st, const std::string& msg) {
  g_err = msg;
  return (mpdo_status)st;
}
}  // namespace

int mpdo::set_last_error(int st, const std::string& msg) {
  g_err = msg;
  return st;
}

namespace {

struct AnyEngine {
  std::unique_ptr<Engine<double>> d;
  std::unique_ptr<Engine<float>> f;
  void run_sublayer(const std::vector<GateOp>& ops) { d ? d->run_sublayer(ops) : f->run_sublayer(ops); }
  void expect(const std::vector<int>& inst, const std::vector<const double*>& ops, double* out, bool raw = false) {
    d ? d->expect(inst, ops, out, raw) : f->expect(inst, ops, out, raw);
  }
  void dims(int b, std::vector<int>& bo, std::vector<int>& in, double& disc) {
    d ? d->dims(b, bo, in, disc) : f->dims(b, bo, in, disc);
  }
  std::vector<double> bond_weights(int b, int bond) { return d ? d->bond_weights(b, bond) : f->bond_weights(b, bond); }
  void to_dense(int b, double* host) { d ? d->to_dense(b, host, false) : f->to_dense(b, host, false); }
  void sample(int b, const double* u, int ns, unsigned char* bits, double* pz) {
    d ? d->sample(b, u, ns, bits, pz) : f->sample(b, u, ns, bits, pz);
  }
  double truncate_sweep(int b, int c, int k, double cut) {
    return d ? d->truncate_sweep(b, c, k, cut) : f->truncate_sweep(b, c, k, cut);
  }
  InstStats stats(int b) { return d ? d->stats(b) : f->stats(b); }
  // rho of instance b as local density tensors
  void load_mpo(int b, MpoState& m) {
    std::vector<int> bo, in;
    double disc;
    dims(b, bo, in, disc);
    for (int i = 0; i < m.n; ++i) {
      const int l = i ? bo[i - 1] : 1, r = i + 1 < m.n ? bo[i] : 1;
      if (d) m.load_site<double>(i, reinterpret_cast<const cpx<double>*>(d->site_ptr(b, i)), l, in[i], r);
      else m.load_site<float>(i, reinterpret_cast<const cpx<float>*>(f->site_ptr(b, i)), l, in[i], r);
    }
  }
  long long failures() { return d ? d->failures() : f->failures(); }
};

Config make_config(const mpdo_config* cfg) {
  Config c;
  c.chi_max = cfg->chi_max;
  c.kap_max = cfg->kappa_max;
  c.mmax = cfg->max_kraus;
  c.svd_cut = cfg->svd_cutoff;
  c.kap_cut = cfg->kappa_cutoff;
  return c;
}

const char* check_config(const mpdo_config* cfg, bool need_n) {
  if (!cfg) return "null config";
  if (need_n && (cfg->n < 1 || cfg->n > 64)) return "n must be in [1, 64]";
  if (cfg->chi_max < 1 || cfg->chi_max > 128) return "chi_max must be in [1, 128]";
  if (cfg->kappa_max < 1 || cfg->kappa_max > 64) return "kappa_max must be in [1, 64]";
  if (cfg->max_kraus < 1 || cfg->max_kraus > 64) return "max_kraus must be in [1, 64]";
  if ((long long)cfg->kappa_max * cfg->max_kraus > EIG_NMAX) return "kappa_max * max_kraus must be <= 1024";
  if (!(cfg->svd_cutoff >= 0 && cfg->svd_cutoff < 1)) return "svd_cutoff must be in [0, 1)";
  if (!(cfg->kappa_cutoff >= 0 && cfg->kappa_cutoff < 1)) return "kappa_cutoff must be in [0, 1)";
  if (cfg->prec != MPDO_C128 && cfg->prec != MPDO_C64_MIXED) return "prec must be MPDO_C128 or MPDO_C64_MIXED";
  return nullptr;
}

DeviceAllocator hooks_of(const mpdo_config* cfg) {
  DeviceAllocator a;
  if (cfg && cfg->alloc && cfg->free) {
    a.alloc = cfg->alloc;
    a.free = cfg->free;
    a.ctx = cfg->alloc_ctx;
  }
  return a;
}

#define GUARD_BEGIN try {
#define GUARD_END                                                     \
  }                                                                   \
  catch (const Error& e) {                                            \
    return fail(e.status, e.msg);                                     \
  }                                                                   \
  catch (const std::exception& e) {                                   \
    return fail(MPDO_EDEVICE, std::string("internal error: ") + e.what()); \
  }                                                                   \
  catch (...) {                                                       \
    return fail(MPDO_EDEVICE, "internal error");                      \
  }

// Handle entry points: allocations go through the handle's allocator, and
// an error once work has started makes the handle unusable.
#define HANDLE_CHECK(h)                                                      \
  if (!(h)) return fail(MPDO_EINVAL, "null handle");                         \
  if ((h)->dead) return fail(MPDO_EDEVICE, "handle is unusable after an earlier error: " + (h)->why);
#define GUARD_BEGIN_H(h)                                                     \
  AllocScope alloc_scope_((h)->alloc.alloc ? &(h)->alloc : nullptr);         \
  try {
#define GUARD_END_H(h)                                                       \
  }                                                                          \
  catch (const Error& e) {                                                   \
    return mark_dead((h), e.status, e.msg);                                  \
  }                                                                          \
  catch (const std::exception& e) {                                          \
    return mark_dead((h), MPDO_EDEVICE, std::string("internal error: ") + e.what()); \
  }                                                                          \
  catch (...) {                                                              \
    return mark_dead((h), MPDO_EDEVICE, "internal error");                   \
  }
}  // namespace

struct mpdo_s {
  mpdo_config cfg;
  DeviceAllocator alloc;
  hipStream_t st = nullptr;
  AnyEngine eng;
  std::vector<GateOp> pending;
  std::vector<char> busy;
  bool dead = false;        // an error after device work started
  std::string why;
};

struct mpdo_chan_s {
  Channel ch;
};

static mpdo_status mark_dead(mpdo_t h, int st, const std::string& msg) {
  h->dead = true;
  h->why = msg;
  return fail(st, msg);
}

static mpdo_status flush_queue(mpdo_t h) {
  if (h->pending.empty()) return MPDO_OK;
  std::vector<GateOp> ops;
  ops.swap(h->pending);
  std::fill(h->busy.begin(), h->busy.end(), 0);
  h->eng.run_sublayer(ops);
  return MPDO_OK;
}

// After a synchronising call: a numerical failure recorded on the device
// (see mpdo.h) is an error of this call.
static void check_health(mpdo_t h) {
  const long long f = h->eng.failures();
  if (f > 0)
    throw Error{MPDO_ENOTCONV, std::to_string(f) +
                                   " numerical failure(s) in truncations (non-finite weights, an eigenpair above its "
                                   "residual bound, or a non-positive trace)"};
}

extern "C" {

const char* mpdo_last_error(void) { return g_err.c_str(); }

const char* mpdo_version(void) { return "libmpdo 0.1 (gfx950)"; }

mpdo_status mpdo_create(const mpdo_config* cfg, void* hip_stream, mpdo_t* out) {
  if (!out) return fail(MPDO_EINVAL, "null output pointer");
  *out = nullptr;
  if (const char* why = check_config(cfg, true)) return fail(MPDO_EINVAL, why);
  if ((cfg->alloc == nullptr) != (cfg->free == nullptr)) return fail(MPDO_EINVAL, "set both allocator hooks or none");
  std::unique_ptr<mpdo_s> h(new mpdo_s());
  h->cfg = *cfg;
  h->alloc = hooks_of(cfg);
  AllocScope scope(h->alloc.alloc ? &h->alloc : nullptr);
  GUARD_BEGIN
  h->st = reinterpret_cast<hipStream_t>(hip_stream);
  const Config c = make_config(cfg);
  std::vector<int> nq(1, cfg->n);
  if (cfg->prec == MPDO_C128) h->eng.d.reset(new Engine<double>(c, nq, h->st));
  else h->eng.f.reset(new Engine<float>(c, nq, h->st));
  h->busy.assign(cfg->n, 0);
  *out = h.release();
  return MPDO_OK;
  GUARD_END
}

mpdo_status mpdo_destroy(mpdo_t h) {
  if (!h) return MPDO_OK;
  GUARD_BEGIN
  if (h->st) (void)hipStreamSynchronize(h->st);
  else (void)hipDeviceSynchronize();
  delete h;
  return MPDO_OK;
  GUARD_END
}

mpdo_status mpdo_channel_from_chi(const double* chi, int32_t q, double eps, void* hip_stream, mpdo_chan_t* out) {
  if (!out) return fail(MPDO_EINVAL, "null output pointer");
  *out = nullptr;
  if (!chi) return fail(MPDO_EINVAL, "null chi");
  if (q < 1 || q > 3) return fail(MPDO_EINVAL, "q must be 1, 2 or 3");
  if (!(eps >= 0 && eps < 1)) return fail(MPDO_EINVAL, "eps must be in [0, 1)");
  const int d2 = 1 << (2 * q);
  double scale = 0;
  for (int e = 0; e < d2 * d2; ++e) {
    if (!std::isfinite(chi[2 * e]) || !std::isfinite(chi[2 * e + 1])) return fail(MPDO_EINVAL, "chi is not finite");
    scale = std::max(scale, std::hypot(chi[2 * e], chi[2 * e + 1]));
  }
  for (int a = 0; a < d2; ++a)
    for (int b = 0; b < d2; ++b) {
      const double dr = chi[2 * (a * d2 + b)] - chi[2 * (b * d2 + a)];
      const double di = chi[2 * (a * d2 + b) + 1] + chi[2 * (b * d2 + a) + 1];
      if (std::hypot(dr, di) > 1e-10 * std::max(1.0, scale)) return fail(MPDO_EINVAL, "chi is not Hermitian");
    }
  GUARD_BEGIN
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  std::unique_ptr<mpdo_chan_s> c(new mpdo_chan_s());
  DevBuf dchi, dlam, dev, dvec, dwork, dinfo, ddesc, dkr;
  dchi.alloc(sizeof(double) * 2 * d2 * d2);
  dlam.alloc(sizeof(double) * 2 * d2 * d2);
  dev.alloc(sizeof(double) * (d2 + 1));
  dvec.alloc(sizeof(double) * 2 * d2 * d2);
  dwork.alloc(sizeof(double) * eig_work_doubles(d2));
  dinfo.alloc(sizeof(double) * 4);
  dkr.alloc(sizeof(double) * 2 * d2 * d2);
  ddesc.alloc(sizeof(EigDesc));
  hip_check(hipMemcpyAsync(dchi.p, chi, sizeof(double) * 2 * d2 * d2, hipMemcpyHostToDevice, st), "upload chi");
  EigDesc ed;
  std::memset(&ed, 0, sizeof(ed));
  ed.a = dlam.as<double>(); ed.lda = d2; ed.n = d2; ed.evals = dev.as<double>(); ed.evecs = dvec.as<double>();
  ed.work = dwork.as<double>(); ed.trace = dev.as<double>() + d2; ed.kvec = d2; ed.active = 1;
  hip_check(hipMemcpyAsync(ddesc.p, &ed, sizeof(ed), hipMemcpyHostToDevice, st), "upload desc");
  launch_choi(dchi.as<double>(), q, dlam.as<double>(), st);
  DevBuf dsw;
  dsw.alloc(sizeof(int));
  launch_eigh(ddesc.as<EigDesc>(), 1, d2, dsw.as<int>(), st);
  launch_kraus_extract(dev.as<double>(), dvec.as<double>(), q, eps, 1e-13, dkr.as<double>(), dinfo.as<double>(), st);
  double info[4];
  int sweeps = 0;
  hip_check(hipMemcpyAsync(info, dinfo.p, sizeof(info), hipMemcpyDeviceToHost, st), "info");
  hip_check(hipMemcpyAsync(&sweeps, dsw.p, sizeof(int), hipMemcpyDeviceToHost, st), "info");
  hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
  if (sweeps != 1) return fail(MPDO_EDEVICE, "Choi eigensolver did not run");
  if (!(info[1] <= 1e-8)) return fail(MPDO_ENOTCPTP, "sum K^dag K differs from I by " + std::to_string(info[1]));
  const int m = (int)info[0];
  if (m < 1) return fail(MPDO_ENOTCPTP, "no Kraus operator kept");
  const int d = 1 << q;
  c->ch.q = q;
  c->ch.m = m;
  c->ch.completeness_err = info[1];
  c->ch.min_eig = info[2];
  c->ch.kraus.alloc(sizeof(double) * 2 * m * d * d);
  hip_check(hipMemcpyAsync(c->ch.kraus.p, dkr.p, sizeof(double) * 2 * m * d * d, hipMemcpyDeviceToDevice, st), "kraus");
  c->ch.host_kraus.resize((size_t)2 * m * d * d);
  hip_check(hipMemcpyAsync(c->ch.host_kraus.data(), dkr.p, sizeof(double) * 2 * m * d * d, hipMemcpyDeviceToHost, st),
            "kraus");
  hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
  *out = c.release();
  return MPDO_OK;
  GUARD_END
}

mpdo_status mpdo_channel_info(mpdo_chan_t ch, int32_t* q, int32_t* nkraus, double* kraus_out) {
  if (!ch) return fail(MPDO_EINVAL, "null channel");
  if (q) *q = ch->ch.q;
  if (nkraus) *nkraus = ch->ch.m;
  if (kraus_out) std::memcpy(kraus_out, ch->ch.host_kraus.data(), ch->ch.host_kraus.size() * sizeof(double));
  return MPDO_OK;
}

mpdo_status mpdo_channel_destroy(mpdo_chan_t ch) {
  GUARD_BEGIN
  if (ch) {
    (void)hipDeviceSynchronize();
    delete ch;
  }
  return MPDO_OK;
  GUARD_END
}

static mpdo_status enqueue(mpdo_t h, const int32_t* sites, int32_t q, const double* U, mpdo_chan_t ch) {
  HANDLE_CHECK(h)
  if (!sites) return fail(MPDO_EINVAL, "null sites");
  if (q < 1 || q > 3) return fail(MPDO_EINVAL, "q must be 1, 2 or 3");
  const int n = h->cfg.n;
  for (int t = 0; t < q; ++t) {
    if (sites[t] < 0 || sites[t] >= n) return fail(MPDO_EINVAL, "site out of range");
    if (t > 0 && sites[t] != sites[t - 1] + 1) return fail(MPDO_EINVAL, "sites must be ascending and adjacent");
  }
  if (ch && ch->ch.q != q) return fail(MPDO_EINVAL, "channel arity differs from the number of sites");
  if (ch && ch->ch.m > h->cfg.max_kraus) return fail(MPDO_EINVAL, "channel has more Kraus operators than max_kraus");
  const int d = 1 << q;
  if (U) {
    for (int e = 0; e < 2 * d * d; ++e)
      if (!std::isfinite(U[e])) return fail(MPDO_EINVAL, "U is not finite");
  }
  GUARD_BEGIN_H(h)
  for (int t = 0; t < q; ++t)
    if (h->busy[sites[t]]) {
      flush_queue(h);
      break;
    }
  GateOp g;
  g.inst = 0;
  g.site = sites[0];
  g.q = q;
  g.kind = GK_FIXED;
  g.ch = ch ? &ch->ch : nullptr;
  if (U) {
    std::memcpy(g.uhost, U, sizeof(double) * 2 * d * d);
    g.has_u = true;
  }
  h->pending.push_back(g);
  for (int t = 0; t < q; ++t) h->busy[sites[t]] = 1;
  return MPDO_OK;
  GUARD_END_H(h)
}

mpdo_status mpdo_apply_gate(mpdo_t h, const int32_t* sites, int32_t q, const double* U) {
  if (!U) return fail(MPDO_EINVAL, "null U");
  return enqueue(h, sites, q, U, nullptr);
}

mpdo_status mpdo_apply_channel(mpdo_t h, const int32_t* sites, int32_t q, const double* U, mpdo_chan_t ch) {
  if (!ch) return fail(MPDO_EINVAL, "null channel");
  return enqueue(h, sites, q, U, ch);
}

mpdo_status mpdo_flush(mpdo_t h) {
  HANDLE_CHECK(h)
  GUARD_BEGIN_H(h)
  return flush_queue(h);
  GUARD_END_H(h)
}

mpdo_status mpdo_truncate(mpdo_t h, int32_t chi_max, int32_t kappa_max, double cutoff, double* discarded) {
  HANDLE_CHECK(h)
  if (chi_max < 1 || chi_max > h->cfg.chi_max) return fail(MPDO_EINVAL, "chi_max out of range");
  if (kappa_max < 1 || kappa_max > h->cfg.kappa_max) return fail(MPDO_EINVAL, "kappa_max out of range");
  if (!(cutoff >= 0 && cutoff < 1)) return fail(MPDO_EINVAL, "cutoff must be in [0, 1)");
  GUARD_BEGIN_H(h)
  flush_queue(h);
  const double d = h->eng.truncate_sweep(0, chi_max, kappa_max, cutoff);
  check_health(h);
  if (discarded) *discarded = d;
  return MPDO_OK;
  GUARD_END_H(h)
}

static mpdo_status expect_ops(mpdo_t h, const std::vector<std::vector<double>>& ops, double* out, bool raw) {
  flush_queue(h);
  std::vector<int> inst(ops.size(), 0);
  std::vector<const double*> p;
  for (auto& o : ops) p.push_back(o.data());
  DevBuf res;
  res.alloc(sizeof(double) * 2 * ops.size());
  h->eng.expect(inst, p, res.as<double>(), raw);
  hip_check(hipMemcpyAsync(out, res.p, sizeof(double) * 2 * ops.size(), hipMemcpyDeviceToHost, h->st), "result");
  hip_check(hipStreamSynchronize(h->st), "hipStreamSynchronize");
  check_health(h);
  return MPDO_OK;
}

static void pauli2x2(char c, double* o) {
  const double I[8] = {1, 0, 0, 0, 0, 0, 1, 0};
  const double X[8] = {0, 0, 1, 0, 1, 0, 0, 0};
  const double Y[8] = {0, 0, 0, -1, 0, 1, 0, 0};
  const double Z[8] = {1, 0, 0, 0, 0, 0, -1, 0};
  const double* s = c == 'X' ? X : c == 'Y' ? Y : c == 'Z' ? Z : I;
  std::memcpy(o, s, sizeof(I));
}

mpdo_status mpdo_expect(mpdo_t h, const char* pauli, double* re, double* im) {
  HANDLE_CHECK(h)
  if (!pauli) return fail(MPDO_EINVAL, "null argument");
  const int n = h->cfg.n;
  if ((int)std::strlen(pauli) != n) return fail(MPDO_EINVAL, "Pauli string length differs from n");
  for (int i = 0; i < n; ++i)
    if (!std::strchr("IXYZ", pauli[i]) || pauli[i] == 0) return fail(MPDO_EINVAL, "Pauli string must use IXYZ");
  GUARD_BEGIN_H(h)
  std::vector<std::vector<double>> ops(1, std::vector<double>(8 * n));
  for (int i = 0; i < n; ++i) pauli2x2(pauli[i], ops[0].data() + 8 * i);
  double out[2];
  expect_ops(h, ops, out, false);
  if (re) *re = out[0];
  if (im) *im = out[1];
  return MPDO_OK;
  GUARD_END_H(h)
}

mpdo_status mpdo_expect_products(mpdo_t h, const double* ops, int32_t nops, double* out) {
  HANDLE_CHECK(h)
  if (!ops || !out) return fail(MPDO_EINVAL, "null argument");
  if (nops < 1) return fail(MPDO_EINVAL, "nops must be >= 1");
  const int n = h->cfg.n;
  GUARD_BEGIN_H(h)
  std::vector<std::vector<double>> v(nops, std::vector<double>(8 * n));
  for (int k = 0; k < nops; ++k) std::memcpy(v[k].data(), ops + (size_t)8 * n * k, sizeof(double) * 8 * n);
  return expect_ops(h, v, out, false);
  GUARD_END_H(h)
}

mpdo_status mpdo_fidelity_ghz(mpdo_t h, double* f) {
  HANDLE_CHECK(h)
  if (!f) return fail(MPDO_EINVAL, "null argument");
  const int n = h->cfg.n;
  GUARD_BEGIN_H(h)
  // Tr(|0..0><0..0| rho), Tr(|1..1><1..1| rho), Tr(|1..1><0..0| rho) = rho_{0..0,1..1}
  const double P0[8] = {1, 0, 0, 0, 0, 0, 0, 0}, P1[8] = {0, 0, 0, 0, 0, 0, 1, 0}, UP[8] = {0, 0, 0, 0, 1, 0, 0, 0};
  std::vector<std::vector<double>> ops(3, std::vector<double>(8 * n));
  for (int i = 0; i < n; ++i) {
    std::memcpy(ops[0].data() + 8 * i, P0, sizeof(P0));
    std::memcpy(ops[1].data() + 8 * i, P1, sizeof(P1));
    std::memcpy(ops[2].data() + 8 * i, UP, sizeof(UP));
  }
  double out[6];
  expect_ops(h, ops, out, false);
  *f = 0.5 * (out[0] + out[2] + 2 * out[4]);
  return MPDO_OK;
  GUARD_END_H(h)
}

mpdo_status mpdo_trace(mpdo_t h, double* tr) {
  HANDLE_CHECK(h)
  if (!tr) return fail(MPDO_EINVAL, "null argument");
  const int n = h->cfg.n;
  GUARD_BEGIN_H(h)
  std::vector<std::vector<double>> ops(1, std::vector<double>(8 * n));
  for (int i = 0; i < n; ++i) pauli2x2('I', ops[0].data() + 8 * i);
  double out[2];
  expect_ops(h, ops, out, true);
  *tr = out[0];
  return MPDO_OK;
  GUARD_END_H(h)
}

mpdo_status mpdo_dims(mpdo_t h, int32_t* bonds, int32_t* inner, double* discarded) {
  if (!h) return fail(MPDO_EINVAL, "null handle");
  const bool was_dead = h->dead;
  GUARD_BEGIN_H(h)
  if (!was_dead) flush_queue(h);   // an unusable handle reports its state as it is
  std::vector<int> b, k;
  double d;
  h->eng.dims(0, b, k, d);
  if (bonds) std::memcpy(bonds, b.data(), sizeof(int) * b.size());
  if (inner) std::memcpy(inner, k.data(), sizeof(int) * k.size());
  if (discarded) *discarded = d;
  if (!was_dead) check_health(h);
  return MPDO_OK;
  GUARD_END_H(h)
}

mpdo_status mpdo_stats(mpdo_t h, mpdo_stats_t* out) {
  if (!h || !out) return fail(MPDO_EINVAL, "null argument");
  const bool was_dead = h->dead;
  GUARD_BEGIN_H(h)
  std::memset(out, 0, sizeof(*out));
  double tr = std::nan("");
  if (!was_dead) {
    flush_queue(h);
    const int n = h->cfg.n;
    std::vector<std::vector<double>> ops(1, std::vector<double>(8 * n));
    for (int i = 0; i < n; ++i) pauli2x2('I', ops[0].data() + 8 * i);
    std::vector<int> inst(1, 0);
    std::vector<const double*> p(1, ops[0].data());
    DevBuf res;
    res.alloc(sizeof(double) * 2);
    h->eng.expect(inst, p, res.as<double>(), true);
    double v[2];
    hip_check(hipMemcpyAsync(v, res.p, sizeof(v), hipMemcpyDeviceToHost, h->st), "trace");
    hip_check(hipStreamSynchronize(h->st), "hipStreamSynchronize");
    tr = v[0];
  }
  const InstStats st = h->eng.stats(0);
  std::vector<int> b, k;
  double d;
  h->eng.dims(0, b, k, d);
  out->truncations = st.cuts;
  out->failures = st.failures;
  out->discarded = st.discarded;
  out->max_discarded = st.max_discarded;
  out->min_gap = st.min_gap;
  out->trace = tr;
  out->max_bond = b.empty() ? 1 : *std::max_element(b.begin(), b.end());
  out->max_inner = k.empty() ? 1 : *std::max_element(k.begin(), k.end());
  if (st.failures > 0 && !h->dead) {
    h->dead = true;
    h->why = "numerical failure recorded on the device";
  }
  return MPDO_OK;
  GUARD_END_H(h)
}

mpdo_status mpdo_release_cached_memory(size_t* cached) {
  GUARD_BEGIN
  if (cached) *cached = cached_device_bytes();
  release_cached_memory();
  return MPDO_OK;
  GUARD_END
}

mpdo_status mpdo_to_dense(mpdo_t h, double* rho) {
  HANDLE_CHECK(h)
  if (!rho) return fail(MPDO_EINVAL, "null argument");
  if (h->cfg.n > 12) return fail(MPDO_EINVAL, "dense state needs n <= 12");
  GUARD_BEGIN_H(h)
  flush_queue(h);
  h->eng.to_dense(0, rho);
  check_health(h);
  return MPDO_OK;
  GUARD_END_H(h)
}

mpdo_status mpdo_probabilities(mpdo_t h, const uint8_t* bits, int32_t nz, double* p) {
  HANDLE_CHECK(h)
  if (!bits || !p) return fail(MPDO_EINVAL, "null argument");
  if (nz < 1) return fail(MPDO_EINVAL, "nz must be >= 1");
  const int n = h->cfg.n;
  for (long long e = 0; e < (long long)nz * n; ++e)
    if (bits[e] > 1) return fail(MPDO_EINVAL, "bits must be 0 or 1");
  GUARD_BEGIN_H(h)
  // <z| rho |z> / Tr rho: the product of the projectors |z_i><z_i|
  const double P0[8] = {1, 0, 0, 0, 0, 0, 0, 0}, P1[8] = {0, 0, 0, 0, 0, 0, 1, 0};
  std::vector<std::vector<double>> ops(nz, std::vector<double>(8 * n));
  for (int z = 0; z < nz; ++z)
    for (int i = 0; i < n; ++i) std::memcpy(ops[z].data() + 8 * i, bits[(size_t)z * n + i] ? P1 : P0, sizeof(P0));
  std::vector<double> out(2 * (size_t)nz);
  expect_ops(h, ops, out.data(), false);
  for (int z = 0; z < nz; ++z) p[z] = out[2 * (size_t)z];
  return MPDO_OK;
  GUARD_END_H(h)
}

mpdo_status mpdo_sample(mpdo_t h, const double* u, int32_t nshots, uint8_t* bits, double* pz) {
  HANDLE_CHECK(h)
  if (!u || !bits) return fail(MPDO_EINVAL, "null argument");
  if (nshots < 1) return fail(MPDO_EINVAL, "nshots must be >= 1");
  const int n = h->cfg.n;
  for (long long e = 0; e < (long long)nshots * n; ++e)
    if (!(u[e] >= 0.0 && u[e] < 1.0)) return fail(MPDO_EINVAL, "uniforms must lie in [0, 1)");
  GUARD_BEGIN_H(h)
  flush_queue(h);
  h->eng.sample(0, u, nshots, bits, pz);
  check_health(h);
  return MPDO_OK;
  GUARD_END_H(h)
}

mpdo_status mpdo_bond_weights(mpdo_t h, int32_t b, double* out, int32_t cap, int32_t* len) {
  HANDLE_CHECK(h)
  if (!out || !len) return fail(MPDO_EINVAL, "null argument");
  if (b < 0 || b >= h->cfg.n - 1) return fail(MPDO_EINVAL, "bond out of range");
  GUARD_BEGIN_H(h)
  flush_queue(h);
  std::vector<double> v = h->eng.bond_weights(0, b);
  check_health(h);
  *len = (int)v.size();
  std::memcpy(out, v.data(), sizeof(double) * std::min<size_t>(v.size(), cap));
  return MPDO_OK;
  GUARD_END_H(h)
}

}  // extern "C"

namespace {
// Runs a batch on an engine of real type T: sublayers merged across instances,
// then the observables; with use_graph the whole sequence is one HIP graph.
template <typename T>
void batch_exec(const Config& c, const std::vector<int>& nq, const std::vector<std::vector<GateOp>>& layers,
                const std::vector<int>& oinst, const std::vector<const double*>& oops, double* out_dev,
                bool use_graph, hipStream_t user_st, double* rho_dev = nullptr) {
  // graph capture needs a real stream: use a private one when given NULL
  struct OwnStream {
    hipStream_t s = nullptr;
    ~OwnStream() { if (s) (void)hipStreamDestroy(s); }
  } own;
  hipStream_t st = user_st;
  if (use_graph && !st) {
    hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
    hip_check(hipStreamCreate(&own.s), "hipStreamCreate");
    st = own.s;
  }
  Engine<T> eng(c, nq, st);
  if (rho_dev) {  // dense state of every instance, offsets by the prefix sum of 4^n
    for (const auto& L : layers) eng.run_sublayer(L);
    long long off = 0;
    for (size_t b = 0; b < nq.size(); ++b) {
      eng.to_dense((int)b, rho_dev + 2 * off, true);
      off += 1LL << (2 * nq[b]);
    }
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    if (const long long f = eng.failures())
      throw Error{MPDO_ENOTCONV, std::to_string(f) + " numerical failure(s) in the batch's truncations"};
    return;
  }
  if (!use_graph) {
    for (const auto& L : layers) eng.run_sublayer(L);
    if (!oinst.empty()) eng.expect(oinst, oops, out_dev);
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    if (const long long f = eng.failures())
      throw Error{MPDO_ENOTCONV, std::to_string(f) + " numerical failure(s) in the batch's truncations"};
    return;
  }
  Upload dry;
  dry.dry = true;
  for (const auto& L : layers) eng.run_sublayer(L, dry);
  if (!oinst.empty()) eng.expect(oinst, oops, out_dev, false, dry);
  eng.prepare_capture(dry);
  const size_t bytes = std::max<size_t>(dry.cursor, 256);
  size_t hbytes = 0;
  void* himg = pinned_get(bytes, &hbytes);
  struct HostFree {
    void* p;
    size_t n;
    hipStream_t s;
    ~HostFree() {
      (void)hipStreamSynchronize(s);
      pinned_put(p, n);
    }
  } guard{himg, hbytes, st};
  DevBuf dimg;
  dimg.alloc(bytes);
  hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
  Upload real;
  real.immediate = false;
  real.host = reinterpret_cast<char*>(himg);
  real.dev = reinterpret_cast<char*>(dimg.p);
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  try {
    // the image is filled below, before the graph is launched
    hip_check(hipMemcpyAsync(dimg.p, himg, bytes, hipMemcpyHostToDevice, st), "capture upload");
    for (const auto& L : layers) eng.run_sublayer(L, real);
    if (!oinst.empty()) eng.expect(oinst, oops, out_dev, false, real);
  } catch (...) {
    hipGraph_t g2 = nullptr;
    (void)hipStreamEndCapture(st, &g2);
    if (g2) (void)hipGraphDestroy(g2);
    throw;
  }
  hip_check(hipStreamEndCapture(st, &graph), "hipStreamEndCapture");
  hip_check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
  const hipError_t le = hipGraphLaunch(exec, st);
  const hipError_t se = hipStreamSynchronize(st);
  (void)hipGraphExecDestroy(exec);
  (void)hipGraphDestroy(graph);
  hip_check(le, "hipGraphLaunch");
  hip_check(se, "hipStreamSynchronize");
  if (const long long f = eng.failures())
    throw Error{MPDO_ENOTCONV, std::to_string(f) + " numerical failure(s) in the batch's truncations"};
}
}  // namespace

extern "C" {

static mpdo_status batch_common(const mpdo_config* cfg, const mpdo_program* progs, int32_t ninst,
                                const double* params_dev, int32_t param_stride, const double* fixed_u, int32_t nfixed,
                                const mpdo_chan_t* chans, int32_t nchans, double* out_dev, int32_t use_graph,
                                void* hip_stream, double* rho_dev);

mpdo_status mpdo_batch_run(const mpdo_config* cfg, const mpdo_program* progs, int32_t ninst,
                           const double* params_dev, int32_t param_stride, const double* fixed_u, int32_t nfixed,
                           const mpdo_chan_t* chans, int32_t nchans, double* out_dev, int32_t use_graph,
                           void* hip_stream) {
  return batch_common(cfg, progs, ninst, params_dev, param_stride, fixed_u, nfixed, chans, nchans, out_dev,
                      use_graph, hip_stream, nullptr);
}

mpdo_status mpdo_batch_run_dense(const mpdo_config* cfg, const mpdo_program* progs, int32_t ninst,
                                 const double* params_dev, int32_t param_stride, const double* fixed_u,
                                 int32_t nfixed, const mpdo_chan_t* chans, int32_t nchans, double* rho_dev,
                                 void* hip_stream) {
  if (!rho_dev) return fail(MPDO_EINVAL, "null rho_dev");
  if (progs && ninst >= 1)
    for (int b = 0; b < ninst; ++b)
      if (progs[b].n > 12) return fail(MPDO_EINVAL, "dense states need n <= 12");
  return batch_common(cfg, progs, ninst, params_dev, param_stride, fixed_u, nfixed, chans, nchans, nullptr, 0,
                      hip_stream, rho_dev);
}

}  // extern "C"

static mpdo_status batch_common(const mpdo_config* cfg, const mpdo_program* progs, int32_t ninst,
                                const double* params_dev, int32_t param_stride, const double* fixed_u, int32_t nfixed,
                                const mpdo_chan_t* chans, int32_t nchans, double* out_dev, int32_t use_graph,
                                void* hip_stream, double* rho_dev) {
  if (const char* why = check_config(cfg, false)) return fail(MPDO_EINVAL, why);
  if (!progs || ninst < 1) return fail(MPDO_EINVAL, "no programs");
  if (nfixed < 0 || nchans < 0 || param_stride < 0) return fail(MPDO_EINVAL, "negative count");
  if (nfixed > 0 && !fixed_u) return fail(MPDO_EINVAL, "null fixed_u");
  if (nchans > 0 && !chans) return fail(MPDO_EINVAL, "null chans");
  for (int c = 0; c < nchans; ++c)
    if (!chans[c]) return fail(MPDO_EINVAL, "null channel handle");
  long long total_obs = 0;
  for (int b = 0; b < ninst; ++b) {
    const mpdo_program& p = progs[b];
    if (p.n < 1 || p.n > 64) return fail(MPDO_EINVAL, "program qubit count must be in [1, 64]");
    if (p.nops < 0 || (p.nops > 0 && !p.ops)) return fail(MPDO_EINVAL, "bad op list");
    if (p.nobs < 0 || (p.nobs > 0 && !p.obs)) return fail(MPDO_EINVAL, "bad observable list");
    total_obs += p.nobs;
    for (int j = 0; j < p.nops; ++j) {
      const mpdo_op& o = p.ops[j];
      if (o.q < 1 || o.q > 3) return fail(MPDO_EINVAL, "op arity must be 1, 2 or 3");
      if (o.q == 3 && (o.kind != MPDO_G_FIXED || o.fixed != -1))
        return fail(MPDO_EINVAL, "3-site ops carry no gate matrix (kind MPDO_G_FIXED, fixed = -1)");
      if (o.site < 0 || o.site + o.q > p.n) return fail(MPDO_EINVAL, "op site out of range");
      const bool k1 = o.kind == MPDO_G_RX || o.kind == MPDO_G_RY || o.kind == MPDO_G_RZ;
      const bool k2 = o.kind == MPDO_G_ZZPHASE || o.kind == MPDO_G_SWAPZZ;
      if (o.kind != MPDO_G_FIXED && !((k1 && o.q == 1) || (k2 && o.q == 2)))
        return fail(MPDO_EINVAL, "gate kind does not match its arity");
      if (o.kind == MPDO_G_FIXED && (o.fixed < -1 || o.fixed >= nfixed)) return fail(MPDO_EINVAL, "bad fixed index");
      if (o.param >= 0 && (!params_dev || o.param >= param_stride)) return fail(MPDO_EINVAL, "bad parameter index");
      if (!std::isfinite(o.scale)) return fail(MPDO_EINVAL, "scale is not finite");
      if (o.chan >= nchans || o.chan < -1) return fail(MPDO_EINVAL, "bad channel index");
      if (o.chan >= 0) {
        if (chans[o.chan]->ch.q != o.q) return fail(MPDO_EINVAL, "channel arity differs from the op's");
        if (chans[o.chan]->ch.m > cfg->max_kraus) return fail(MPDO_EINVAL, "channel exceeds max_kraus");
      }
    }
  }
  if (total_obs > 0 && !out_dev && !rho_dev) return fail(MPDO_EINVAL, "null out_dev");
  if ((cfg->alloc == nullptr) != (cfg->free == nullptr)) return fail(MPDO_EINVAL, "set both allocator hooks or none");
  const DeviceAllocator hooks = hooks_of(cfg);
  AllocScope scope(hooks.alloc ? &hooks : nullptr);
  GUARD_BEGIN
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  // fixed gates: a 4x4 slot and its compact top-left 2x2 per entry
  DevBuf dfix;
  std::vector<double> hfix((size_t)std::max(1, nfixed) * 40, 0.0);
  for (int f = 0; f < nfixed; ++f) {
    std::memcpy(&hfix[(size_t)f * 40], fixed_u + (size_t)f * 32, 32 * sizeof(double));
    for (int r = 0; r < 2; ++r)
      for (int cc = 0; cc < 2; ++cc) {
        hfix[(size_t)f * 40 + 32 + 2 * (2 * r + cc)] = fixed_u[(size_t)f * 32 + 2 * (4 * r + cc)];
        hfix[(size_t)f * 40 + 32 + 2 * (2 * r + cc) + 1] = fixed_u[(size_t)f * 32 + 2 * (4 * r + cc) + 1];
      }
  }
  dfix.alloc(hfix.size() * sizeof(double));
  hip_check(hipMemcpy(dfix.p, hfix.data(), hfix.size() * sizeof(double), hipMemcpyHostToDevice), "fixed gates");
  // sublayers: per instance, an op goes to the first group after the last
  // group that touches one of its sites; groups of all instances merge
  std::vector<std::vector<GateOp>> layers;
  std::vector<int> nq(ninst);
  for (int b = 0; b < ninst; ++b) {
    const mpdo_program& p = progs[b];
    nq[b] = p.n;
    std::vector<int> last(p.n, -1);
    for (int j = 0; j < p.nops; ++j) {
      const mpdo_op& o = p.ops[j];
      int g = 0;
      for (int t = 0; t < o.q; ++t) g = std::max(g, last[o.site + t] + 1);
      for (int t = 0; t < o.q; ++t) last[o.site + t] = g;
      if ((int)layers.size() <= g) layers.resize(g + 1);
      GateOp op;
      op.inst = b;
      op.site = o.site;
      op.q = o.q;
      op.kind = o.kind;
      op.pidx = o.param;
      op.scale = o.scale;
      op.params = o.param >= 0 ? params_dev + (size_t)b * param_stride : nullptr;
      if (o.kind == MPDO_G_FIXED && o.fixed >= 0)
        op.ufix = dfix.as<double>() + (size_t)o.fixed * 40 + (o.q == 1 ? 32 : 0);
      op.ch = o.chan >= 0 ? &chans[o.chan]->ch : nullptr;
      layers[g].push_back(op);
    }
  }
  std::vector<int> oinst;
  std::vector<const double*> oops;
  for (int b = 0; b < ninst; ++b)
    for (int k = 0; k < progs[b].nobs; ++k) {
      oinst.push_back(b);
      oops.push_back(progs[b].obs + (size_t)k * progs[b].n * 8);
    }
  const Config c = make_config(cfg);
  if (cfg->prec == MPDO_C128) batch_exec<double>(c, nq, layers, oinst, oops, out_dev, use_graph != 0, st, rho_dev);
  else batch_exec<float>(c, nq, layers, oinst, oops, out_dev, use_graph != 0, st, rho_dev);
  return MPDO_OK;
  GUARD_END
}

extern "C" {

}  // extern "C"

extern "C" {

mpdo_status mpdo_tune_set(int32_t site, int32_t tile, int32_t form, double split_scale) {
  if (site < 1 || site >= GS_N) return fail(MPDO_EINVAL, "site must be in 1..24");
  if (tile != 0 && tile != 32 && tile != 64) return fail(MPDO_EINVAL, "tile must be 0, 32 or 64");
  if (form != 0 && form != 3 && form != 4) return fail(MPDO_EINVAL, "form must be 0, 3 or 4");
  if (!(split_scale >= 0 && split_scale <= 16)) return fail(MPDO_EINVAL, "split_scale must be in [0, 16]");
  SiteTune t;
  t.tile = tile;
  t.form = form;
  t.split_scale = split_scale;
  set_site_tune(site, t);
  return MPDO_OK;
}

mpdo_status mpdo_tune_get(int32_t site, int32_t* tile, int32_t* form, double* split_scale) {
  if (site < 1 || site >= GS_N) return fail(MPDO_EINVAL, "site must be in 1..24");
  const SiteTune t = get_site_tune(site);
  if (tile) *tile = t.tile;
  if (form) *form = t.form;
  if (split_scale) *split_scale = t.split_scale;
  return MPDO_OK;
}

mpdo_status mpdo_profile_enable(int32_t on) {
  GUARD_BEGIN
  prof_reset(on != 0);
  return MPDO_OK;
  GUARD_END
}

mpdo_status mpdo_profile_read(int32_t cls, int32_t* launches, double* ms, double* flops, double* bytes) {
  if (cls < 0 || cls >= PC_NCLASS) return fail(MPDO_EINVAL, "unknown profile class");
  GUARD_BEGIN
  prof_read(cls, launches, ms, flops, bytes);
  return MPDO_OK;
  GUARD_END
}

}  // extern "C"

// ---------------------------------------------------------------------------
// kernel-level test entry points (include/mpdo_testing.h)
// ---------------------------------------------------------------------------
#include "../../include/mpdo_testing.h"

namespace {
template <typename Tin> std::vector<Tin> to_prec(const double* a, size_t n) {
  std::vector<Tin> v(n);
  for (size_t i = 0; i < n; ++i) v[i] = (Tin)a[i];
  return v;
}
}  // namespace

extern "C" mpdo_status mpdo_test_gemm(int32_t prec, int32_t opA, int32_t opB, int32_t M, int32_t N, int32_t K,
                                      const double* A, int32_t rowsA, int32_t lda, const double* B, int32_t rowsB,
                                      int32_t ldb, const double* w, int32_t wdiv, int32_t splits, double alpha,
                                      double* C, int32_t tile, int32_t herm) {
  if (prec < 0 || prec > 2 || opA < 0 || opA > 3 || opB < 0 || opB > 3) return fail(MPDO_EINVAL, "bad mode");
  if (tile != 64 && tile != 32) return fail(MPDO_EINVAL, "tile must be 64 or 32");
  if (herm != 0 && (herm != 1 || M != N)) return fail(MPDO_EINVAL, "herm needs a square C");
  if (M < 1 || N < 1 || K < 1 || rowsA < 1 || rowsB < 1 || lda < 1 || ldb < 1 || splits < 1 || splits > 64)
    return fail(MPDO_EINVAL, "bad size");
  if (!A || !B || !C) return fail(MPDO_EINVAL, "null buffer");
  if (w && wdiv < 1) return fail(MPDO_EINVAL, "bad wdiv");
  // bounds of op(A), op(B) inside the given buffers
  const bool at = (opA == 1 || opA == 3), bt = (opB == 1 || opB == 3);
  if (at ? (K > rowsA || M > lda) : (M > rowsA || K > lda)) return fail(MPDO_EINVAL, "A too small");
  if (bt ? (N > rowsB || K > ldb) : (K > rowsB || N > ldb)) return fail(MPDO_EINVAL, "B too small");
  GUARD_BEGIN
  hipStream_t st = nullptr;
  const size_t na = (size_t)2 * rowsA * lda, nb = (size_t)2 * rowsB * ldb;
  const size_t esz = prec == 0 ? 8 : 4;
  DevBuf dA, dB, dC, dW, dD;
  dA.alloc(na * esz);
  dB.alloc(nb * esz);
  const size_t outsz = prec == 1 ? 4 : 8;
  dC.alloc((size_t)2 * M * N * splits * outsz);
  if (herm) hip_check(hipMemset(dC.p, 0, (size_t)2 * M * N * splits * outsz), "C");  // tiles left unwritten
  if (prec == 0) {
    hip_check(hipMemcpy(dA.p, A, na * 8, hipMemcpyHostToDevice), "A");
    hip_check(hipMemcpy(dB.p, B, nb * 8, hipMemcpyHostToDevice), "B");
  } else {
    auto a = to_prec<float>(A, na), b = to_prec<float>(B, nb);
    hip_check(hipMemcpy(dA.p, a.data(), na * 4, hipMemcpyHostToDevice), "A");
    hip_check(hipMemcpy(dB.p, b.data(), nb * 4, hipMemcpyHostToDevice), "B");
  }
  const int nw = w ? (at ? rowsA : lda) : 0;
  if (w) {
    const int kmax = (K + wdiv - 1) / wdiv;
    dW.alloc(sizeof(double) * std::max(nw, kmax));
    hip_check(hipMemcpy(dW.p, w, sizeof(double) * kmax, hipMemcpyHostToDevice), "w");
  }
  GemmDesc d;
  std::memset(&d, 0, sizeof(d));
  d.A = dA.p; d.B = dB.p; d.C = dC.p; d.w = w ? dW.as<double>() : nullptr;
  d.M = M; d.N = N; d.K = K; d.lda = lda; d.ldb = ldb; d.ldc = N; d.wdiv = w ? wdiv : 1;
  d.nbatch = 1; d.splits = splits; d.sSplit = (long long)M * N; d.opA = opA; d.opB = opB; d.active = 1;
  d.alpha = alpha;
  d.herm = herm;
  dD.alloc(sizeof(GemmDesc));
  hip_check(hipMemcpy(dD.p, &d, sizeof(d), hipMemcpyHostToDevice), "desc");
  const int tiles = herm ? gemm_tiles_herm(N, tile) : gemm_tiles(M, N, tile);
  if (prec == 0) launch_gemm<double, double, double>(dD.as<GemmDesc>(), 1, 1, splits, tiles, st, tile);
  else if (prec == 1) launch_gemm<float, float, float>(dD.as<GemmDesc>(), 1, 1, splits, tiles, st, tile);
  else launch_gemm<float, double, double>(dD.as<GemmDesc>(), 1, 1, splits, tiles, st, tile);
  hip_check(hipGetLastError(), "launch");
  hip_check(hipDeviceSynchronize(), "sync");
  const size_t nc = (size_t)2 * M * N;
  std::vector<double> out(nc, 0.0);
  if (prec == 1) {
    std::vector<float> f(nc * splits);
    hip_check(hipMemcpy(f.data(), dC.p, f.size() * 4, hipMemcpyDeviceToHost), "C");
    for (int s = 0; s < splits; ++s)
      for (size_t i = 0; i < nc; ++i) out[i] += f[s * nc + i];
  } else {
    std::vector<double> f(nc * splits);
    hip_check(hipMemcpy(f.data(), dC.p, f.size() * 8, hipMemcpyDeviceToHost), "C");
    for (int s = 0; s < splits; ++s)
      for (size_t i = 0; i < nc; ++i) out[i] += f[s * nc + i];
  }
  std::memcpy(C, out.data(), nc * sizeof(double));
  return MPDO_OK;
  GUARD_END
}

namespace {
template <typename T> __global__ void k_fill_test(T* p, size_t n, unsigned seed) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    unsigned h = (unsigned)i * 2654435761u ^ seed;
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    p[i] = (T)((double)(h & 0xFFFF) / 65536.0 - 0.5);
  }
}

template <typename T>
void gemm_rate(int M, int N, int K, int items, int reps, double* ms) {
  const size_t ea = (size_t)2 * M * K, eb = (size_t)2 * K * N, ec = (size_t)2 * M * N;
  DevBuf dA, dB, dC, dD;
  dA.alloc(ea * items * sizeof(T));
  dB.alloc(eb * items * sizeof(T));
  dC.alloc(ec * items * sizeof(T));
  hipLaunchKernelGGL(k_fill_test<T>, dim3(4096), dim3(256), 0, nullptr, dA.as<T>(), ea * items, 11u);
  hipLaunchKernelGGL(k_fill_test<T>, dim3(4096), dim3(256), 0, nullptr, dB.as<T>(), eb * items, 23u);
  std::vector<GemmDesc> hd(items);
  for (int i = 0; i < items; ++i) {
    GemmDesc& d = hd[i];
    std::memset(&d, 0, sizeof(d));
    d.A = reinterpret_cast<const double*>(dA.as<T>() + ea * i);
    d.B = reinterpret_cast<const double*>(dB.as<T>() + eb * i);
    d.C = reinterpret_cast<double*>(dC.as<T>() + ec * i);
    d.M = M; d.N = N; d.K = K; d.lda = K; d.ldb = N; d.ldc = N;
    d.nbatch = 1; d.splits = 1; d.wdiv = 1; d.active = 1; d.alpha = 1.0;
  }
  dD.alloc(sizeof(GemmDesc) * items);
  hip_check(hipMemcpy(dD.p, hd.data(), sizeof(GemmDesc) * items, hipMemcpyHostToDevice), "descriptors");
  hipEvent_t e0, e1;
  hip_check(hipEventCreate(&e0), "event");
  hip_check(hipEventCreate(&e1), "event");
  const int tiles = gemm_tiles(M, N, 64);
  launch_gemm<T, T, T>(dD.as<GemmDesc>(), items, 1, 1, tiles, nullptr);
  hip_check(hipEventRecord(e0, nullptr), "event");
  for (int r = 0; r < reps; ++r) launch_gemm<T, T, T>(dD.as<GemmDesc>(), items, 1, 1, tiles, nullptr);
  hip_check(hipEventRecord(e1, nullptr), "event");
  hip_check(hipEventSynchronize(e1), "event");
  hip_check(hipGetLastError(), "launch");
  float t = 0;
  hip_check(hipEventElapsedTime(&t, e0, e1), "event");
  hip_check(hipEventDestroy(e0), "event");
  hip_check(hipEventDestroy(e1), "event");
  *ms = (double)t / reps;
}
}  // namespace

extern "C" mpdo_status mpdo_test_gemm_rate(int32_t prec, int32_t M, int32_t N, int32_t K, int32_t items, int32_t reps,
                                           double* ms) {
  if (prec < 0 || prec > 1) return fail(MPDO_EINVAL, "prec must be 0 or 1");
  if (M < 1 || N < 1 || K < 1 || items < 1 || reps < 1 || reps > 1000 || !ms) return fail(MPDO_EINVAL, "bad size");
  const double bytes = 2.0 * (prec == 0 ? 8 : 4) * items * ((double)M * K + (double)K * N + (double)M * N);
  if (bytes > 32.0 * (1ULL << 30)) return fail(MPDO_EINVAL, "operands above 32 GiB");
  GUARD_BEGIN
  if (prec == 0) gemm_rate<double>(M, N, K, items, reps, ms);
  else gemm_rate<float>(M, N, K, items, reps, ms);
  return MPDO_OK;
  GUARD_END
}

extern "C" mpdo_status mpdo_test_eigh(int32_t n, int32_t kvec, const double* A, double* evals, double* evecs,
                                      double* trace) {
  if (n < 1 || n > EIG_NMAX) return fail(MPDO_EINVAL, "n must be in [1, 1024]");
  if (kvec < 0) return fail(MPDO_EINVAL, "kvec must be >= 0");
  if (!A || !evals || !evecs) return fail(MPDO_EINVAL, "null buffer");
  GUARD_BEGIN
  DevBuf da, de, dv, dw, dd, ds;
  const size_t nn = (size_t)2 * n * n;
  da.alloc(nn * 8);
  de.alloc((size_t)(n + 1) * 8);
  dv.alloc(nn * 8);
  dw.alloc((size_t)eig_work_doubles(n) * 8);
  ds.alloc(sizeof(int));
  hip_check(hipMemcpy(da.p, A, nn * 8, hipMemcpyHostToDevice), "A");
  hip_check(hipMemset(dv.p, 0, nn * 8), "zero");
  hip_check(hipMemset(ds.p, 0, sizeof(int)), "zero");
  EigDesc d;
  std::memset(&d, 0, sizeof(d));
  d.a = da.as<double>(); d.lda = n; d.n = n; d.evals = de.as<double>(); d.evecs = dv.as<double>();
  d.work = dw.as<double>(); d.trace = de.as<double>() + n; d.kvec = kvec; d.active = 1;
  dd.alloc(sizeof(d));
  hip_check(hipMemcpy(dd.p, &d, sizeof(d), hipMemcpyHostToDevice), "desc");
  launch_eigh(dd.as<EigDesc>(), 1, n, ds.as<int>(), nullptr);
  hip_check(hipGetLastError(), "launch");
  hip_check(hipDeviceSynchronize(), "sync");
  hip_check(hipMemcpy(evals, de.p, (size_t)n * 8, hipMemcpyDeviceToHost), "evals");
  hip_check(hipMemcpy(evecs, dv.p, nn * 8, hipMemcpyDeviceToHost), "evecs");
  int ran = 0;
  hip_check(hipMemcpy(&ran, ds.p, sizeof(int), hipMemcpyDeviceToHost), "status");
  if (trace) hip_check(hipMemcpy(trace, de.as<double>() + n, 8, hipMemcpyDeviceToHost), "trace");
  if (ran != 1) return fail(MPDO_EDEVICE, "eigensolver kernel did not run");
  return MPDO_OK;
  GUARD_END
}

extern "C" mpdo_status mpdo_test_eig_residual_bound(double rtol) {
  if (!std::isfinite(rtol)) return fail(MPDO_EINVAL, "rtol must be finite");
  GUARD_BEGIN
  hip_check(set_eig_residual_bound(rtol), "hipMemcpyToSymbol");
  return MPDO_OK;
  GUARD_END
}

extern "C" mpdo_status mpdo_test_fail_next_update(int32_t status) {
  if (status < 0 || status > MPDO_EUNSUPPORTED) return fail(MPDO_EINVAL, "unknown status");
  inject_update_failure(status);
  return MPDO_OK;
}

extern "C" mpdo_status mpdo_test_profile_site(int32_t site, int32_t* launches, double* ms, double* flops) {
  if (site < 0 || site >= GS_N) return fail(MPDO_EINVAL, "unknown GEMM site");
  GUARD_BEGIN
  prof_read_site(site, launches, ms, flops);
  return MPDO_OK;
  GUARD_END
}

extern "C" mpdo_status mpdo_test_gemm_form(int32_t prec, int32_t tile, int32_t form, int32_t* previous) {
  if (prec < 0 || prec > 1 || (tile != 32 && tile != 64) || (form != 3 && form != 4))
    return fail(MPDO_EINVAL, "prec 0/1, tile 32/64, form 3/4");
  if (previous) *previous = gemm_form(prec == 0, tile);
  set_gemm_form(prec == 0, tile, form);
  return MPDO_OK;
}

extern "C" mpdo_status mpdo_test_e_cholesky(int32_t on, int32_t* previous) {
  if (on != 0 && on != 1) return fail(MPDO_EINVAL, "on must be 0 or 1");
  if (previous) *previous = e_cholesky() ? 1 : 0;
  set_e_cholesky(on != 0);
  return MPDO_OK;
}

extern "C" mpdo_status mpdo_test_eig_band(int32_t on, int32_t* previous) {
  if (on != 0 && on != 1) return fail(MPDO_EINVAL, "on must be 0 or 1");
  if (previous) *previous = eig_band() ? 1 : 0;
  set_eig_band(on != 0);
  return MPDO_OK;
}

extern "C" mpdo_status mpdo_test_gram_vector(int32_t on, int32_t* previous) {
  if (on != 0 && on != 1) return fail(MPDO_EINVAL, "on must be 0 or 1");
  if (previous) *previous = gram_vector() ? 1 : 0;
  set_gram_vector(on != 0);
  return MPDO_OK;
}

extern "C" mpdo_status mpdo_test_eig_coop(int32_t on, int32_t* previous) {
  if (on != 0 && on != 1) return fail(MPDO_EINVAL, "on must be 0 or 1");
  if (previous) *previous = eig_coop() ? 1 : 0;
  set_eig_coop(on != 0);
  return MPDO_OK;
}

// ---- error mitigation on an MPO of rho ----

struct mpdo_mpo_s {
  DeviceAllocator alloc;
  std::unique_ptr<MpoState> m;
  bool dead = false;
  std::string why;
};

static mpdo_status mark_dead_mpo(mpdo_mpo_t h, int st, const std::string& msg) {
  h->dead = true;
  h->why = msg;
  return fail(st, msg);
}

#define MPO_CHECK(h)                                                         \
  if (!(h)) return fail(MPDO_EINVAL, "null MPO handle");                     \
  if ((h)->dead) return fail(MPDO_EDEVICE, "MPO handle is unusable after an earlier error: " + (h)->why);
#define MPO_GUARD_END(h)                                                     \
  }                                                                          \
  catch (const Error& e) {                                                   \
    return mark_dead_mpo((h), e.status, e.msg);                              \
  }                                                                          \
  catch (const std::exception& e) {                                          \
    return mark_dead_mpo((h), MPDO_EDEVICE, std::string("internal error: ") + e.what()); \
  }                                                                          \
  catch (...) {                                                              \
    return mark_dead_mpo((h), MPDO_EDEVICE, "internal error");               \
  }

extern "C" {

mpdo_status mpdo_mpo_from_state(mpdo_t h, int32_t d_max, double cutoff, mpdo_mpo_t* out) {
  if (!out) return fail(MPDO_EINVAL, "null output pointer");
  *out = nullptr;
  HANDLE_CHECK(h)
  if (d_max < 1 || d_max > 256) return fail(MPDO_EINVAL, "d_max must be in [1, 256]");
  if (!(cutoff >= 0 && cutoff < 1)) return fail(MPDO_EINVAL, "cutoff must be in [0, 1)");
  std::unique_ptr<mpdo_mpo_s> m(new mpdo_mpo_s);
  m->alloc = h->alloc;
  GUARD_BEGIN_H(h)
  flush_queue(h);
  check_health(h);
  std::vector<int> bo, in;
  double disc;
  h->eng.dims(0, bo, in, disc);
  for (int x : bo)
    if (x > 32) return fail(MPDO_EUNSUPPORTED, "MPO of a state with a bond above 32 (MPO bond above 1024)");
  m->m.reset(new MpoState(h->cfg.n, d_max, cutoff, h->st));
  h->eng.load_mpo(0, *m->m);
  hip_check(hipStreamSynchronize(h->st), "hipStreamSynchronize");
  *out = m.release();
  return MPDO_OK;
  GUARD_END_H(h)
}

mpdo_status mpdo_mpo_destroy(mpdo_mpo_t m) {
  if (!m) return MPDO_OK;
  GUARD_BEGIN
  AllocScope scope(m->alloc.alloc ? &m->alloc : nullptr);
  (void)hipDeviceSynchronize();
  delete m;
  return MPDO_OK;
  GUARD_END
}

mpdo_status mpdo_mpo_apply_gate(mpdo_mpo_t m, int32_t site, int32_t q, const double* U, int32_t inverse) {
  MPO_CHECK(m)
  if (!U) return fail(MPDO_EINVAL, "null gate");
  if (q < 1 || q > 2) return fail(MPDO_EINVAL, "q must be 1 or 2");
  if (site < 0 || site + q > m->m->n) return fail(MPDO_EINVAL, "sites out of range");
  for (int e = 0; e < 2 << (2 * q); ++e)
    if (!std::isfinite(U[e])) return fail(MPDO_EINVAL, "non-finite gate entry");
  AllocScope alloc_scope_(m->alloc.alloc ? &m->alloc : nullptr);
  try {
    m->m->gate_superop(U, q, inverse != 0);
    m->m->apply(site, q);
    hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
    return MPDO_OK;
  MPO_GUARD_END(m)
}

mpdo_status mpdo_mpo_apply_channel(mpdo_mpo_t m, int32_t site, mpdo_chan_t ch, int32_t inverse) {
  MPO_CHECK(m)
  if (!ch) return fail(MPDO_EINVAL, "null channel");
  const int q = ch->ch.q;
  if (q > 2) return fail(MPDO_EUNSUPPORTED, "MPO maps act on at most two sites");
  if (site < 0 || site + q > m->m->n) return fail(MPDO_EINVAL, "sites out of range");
  AllocScope alloc_scope_(m->alloc.alloc ? &m->alloc : nullptr);
  try {
    m->m->superop(ch->ch.kraus.as<double>(), ch->ch.m, q, false, inverse != 0);
    m->m->apply(site, q);
    hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
    return MPDO_OK;
  MPO_GUARD_END(m)
}

mpdo_status mpdo_mpo_expect(mpdo_mpo_t m, const double* ops, int32_t nops, double* out) {
  MPO_CHECK(m)
  if (!ops || !out) return fail(MPDO_EINVAL, "null argument");
  if (nops < 1) return fail(MPDO_EINVAL, "nops must be >= 1");
  AllocScope alloc_scope_(m->alloc.alloc ? &m->alloc : nullptr);
  try {
    m->m->expect(ops, nops, out);
    return MPDO_OK;
  MPO_GUARD_END(m)
}

mpdo_status mpdo_mpo_dims(mpdo_mpo_t m, int32_t* bonds, double* discarded) {
  MPO_CHECK(m)
  const auto& D = m->m->bonds();
  if (bonds)
    for (int i = 1; i < m->m->n; ++i) bonds[i - 1] = D[i];
  if (discarded) *discarded = m->m->discarded;
  return MPDO_OK;
}

mpdo_status mpdo_mpo_to_dense(mpdo_mpo_t m, double* rho) {
  MPO_CHECK(m)
  if (!rho) return fail(MPDO_EINVAL, "null argument");
  if (m->m->n > 12) return fail(MPDO_EINVAL, "dense rho needs n <= 12");
  AllocScope alloc_scope_(m->alloc.alloc ? &m->alloc : nullptr);
  try {
    m->m->to_dense(rho);
    return MPDO_OK;
  MPO_GUARD_END(m)
}

}  // extern "C"
