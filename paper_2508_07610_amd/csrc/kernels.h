// Launch wrappers of the libmpdo kernels (all asynchronous on stream s).
#pragma once
#include "common.h"

namespace mpdo {

// Batched complex GEMM (see GemmDesc).  The grid covers nitems x maxBatch x
// maxSplits x tiles of a maxM x maxN output; items with smaller shapes exit
// early.  Tin: input precision, Tc: MFMA precision, Tout: output precision.
template <typename Tin, typename Tc, typename Tout>
void launch_gemm(const GemmDesc* d_descs, int nitems, int maxBatch, int maxSplits, int maxM, int maxN,
                 hipStream_t s);

// out[item] = sum over splits of the partial products of descs[item]
// (complex double, dense M x ldc).
void launch_reduce_splits(const GemmDesc* d_descs, double* const* d_outs, int nitems, int maxCount,
                          hipStream_t s);

// Batched Hermitian eigensolver (Jacobi, FP64), one workgroup per problem.
// d_sweeps[item] receives the sweep count (negative: not converged).
void launch_eigh(const EigDesc* d_descs, int nitems, int maxn, int* d_sweeps, hipStream_t s);

}  // namespace mpdo
