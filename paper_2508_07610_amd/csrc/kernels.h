// Launch wrappers of the libmpdo kernels (all asynchronous on stream s).
#pragma once
#include "common.h"

namespace mpdo {

// Batched complex GEMM (see GemmDesc).  The grid covers nitems x maxBatch x
// maxSplits x maxTiles output tiles of tile x tile (tile = 64 or 32); an item
// uses the first ceil(M/tile) ceil(N/tile) tiles of its range, so maxTiles
// must bound that count for every item (gemm_tiles of the largest M and N).
// An item with herm set (square, Hermitian C) computes only the tiles on and
// above the diagonal, ceil(N/tile) (ceil(N/tile) + 1) / 2 of them: a launch
// of such items needs only gemm_tiles_herm of the largest N.
// Tin: input precision, Tc: MFMA precision, Tout: output precision.
// groups > 1: the descriptors form `groups` consecutive groups of
// nitems / groups (different products of each item); the launch visits them
// interleaved so that every XCD takes a share of each group.
int gemm_tiles(int maxM, int maxN, int tile = 64);
// Complex-product form of the launches of one MFMA precision and tile size:
// 4 (four real products) or 3 (Gauss's three); process-wide, default 4.
int gemm_form(bool fp64, int tile);
void set_gemm_form(bool fp64, int tile, int form);
int gemm_tiles_herm(int maxN, int tile = 64);
template <typename Tin, typename Tc, typename Tout>
void launch_gemm(const GemmDesc* d_descs, int nitems, int maxBatch, int maxSplits, int maxTiles, hipStream_t s,
                 int tile = 64, int site = -1, int groups = 1);

// Per call site of the MPDO update (a GemmSite of profile.h), the settings
// an autotuner may choose: the tile edge (32 or 64), the complex-product form
// (3 or 4) and a factor on the split-K count; 0 keeps the built-in choice.
struct SiteTune {
  int tile = 0;
  int form = 0;
  double split_scale = 0;
};
void set_site_tune(int site, const SiteTune& t);
SiteTune get_site_tune(int site);
int tuned_tile(int site, int dflt);
int tuned_splits(int site, int dflt);

// A call site's launch: its tuned tile (else `dflt_tile`), the tile count for
// that tile from tiles_of(tile), and its tuned form.
template <typename Tin, typename Tc, typename Tout, typename F>
void launch_gemm_site(int site, const GemmDesc* d_descs, int nitems, int maxBatch, int maxSplits, F tiles_of,
                      hipStream_t s, int dflt_tile = 64, int groups = 1) {
  const int tile = tuned_tile(site, dflt_tile);
  launch_gemm<Tin, Tc, Tout>(d_descs, nitems, maxBatch, maxSplits, tiles_of(tile), s, tile, site, groups);
}

// out[item] = sum over splits of the partial products of descs[item]
// (complex double, dense M x ldc).
void launch_reduce_splits(const GemmDesc* d_descs, double* const* d_outs, int nitems, int maxCount,
                          hipStream_t s);

// Batched Hermitian eigensolver (FP64, Householder tridiagonalisation,
// multisection, inverse iteration), one workgroup per problem; maxn bounds
// every item's n.  d_status[item] is set to 1 when the item's workgroup ran.
// An eigenpair whose tridiagonal residual ||(T - lambda) z|| exceeds
// 1e-9 ||T||, or a non-finite spectrum, sets the item's trace to NaN.
void launch_eigh(const EigDesc* d_descs, int nitems, int maxn, int* d_status, hipStream_t s);
// 128 < n <= 256 through the two-stage (band) reduction or the one-stage
// panel reduction (the default); process-wide.
void set_eig_band(bool on);
bool eig_band();
// launches of at most 32 matrices with n > 128: several workgroups share each
// matrix during the Householder reduction (default on)
void set_eig_coop(bool on);
bool eig_coop();
// Overrides the residual bound on the current device (0 restores 1e-9).
hipError_t set_eig_residual_bound(double rtol);

}  // namespace mpdo
