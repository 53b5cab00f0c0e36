// rho as a matrix product operator of the paper's local density tensors
// (Eq. (6)) and the maps of error mitigation by the inverse of a noisy
// process (Sec. V); the device side of the mpdo_mpo_* entry points.
#pragma once
#include <memory>
#include <vector>

#include "common.h"
#include "engine.h"

namespace mpdo {

class MpoState {
 public:
  // n sites, bond limit dmax, discarded-weight cutoff of the two-site splits,
  // all work on stream s.
  MpoState(int n, int dmax, double cutoff, hipStream_t s);
  // Site i from an MPDO site tensor B[l, 2, k, r] (device):
  // R[(a a'), (p p'), (b b')] = sum_n B[a, p, n, b] conj(B[a', p', n, b']).
  template <typename T> void load_site(int i, const cpx<T>* B, int l, int k, int r);
  // The superoperator sum_j K_j (x) conj(K_j) of m Kraus operators on q
  // qubits (device, m x 2^q x 2^q complex double) in pair order; adj: of the
  // K_j^dagger; inverse: its matrix inverse (throws MPDO_ENOTCONV when singular).
  void superop(const double* K, int m, int q, bool adj, bool inverse);
  // The superoperator of a gate U (host, 2^q x 2^q complex), of U^dagger when adj.
  void gate_superop(const double* U, int q, bool adj);
  // Applies the last superop to site `site` (q = 1) or to sites site and
  // site + 1 (q = 2, then split again with the bond rule).
  void apply(int site, int q);
  // Tr(O rho) for nops product operators (host, nops x n x 2 x 2 complex);
  // out: nops complex values (host).
  void expect(const double* ops, int nops, double* out);
  // The dense rho, row-major 2^n x 2^n complex (host), n <= 12.
  void to_dense(double* out);
  const std::vector<int>& bonds() const { return D; }
  double discarded = 0;
  int n, dmax;
  double cutoff;

 private:
  hipStream_t st;
  std::vector<int> D;
  std::vector<std::unique_ptr<DevBuf>> R;
  DevBuf tA, tB, tG, ev, vec, work, status, desc, edesc, sop, okf, obuf, res, ubuf;
};

}  // namespace mpdo
