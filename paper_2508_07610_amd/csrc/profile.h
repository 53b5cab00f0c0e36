// Kernel timing and work accounting behind mpdo_profile_enable /
// mpdo_profile_read.  While enabled, each compute launch is bracketed by two
// HIP events recorded on the launch's own stream, and a one-thread kernel
// queued right after it adds the launch's algorithmic work (from the
// device-side shapes of its descriptors) to per-class counters.  Launches on
// a stream that is being captured into a graph are not profiled.
#pragma once
#include "common.h"

namespace mpdo {

enum ProfClass : int {
  PC_GEMM_F64 = 0,   // contractions / Gram matrices on FP64 MFMA
  PC_GEMM_F32 = 1,   // contractions on FP32 MFMA (mixed precision)
  PC_EIG_REG = 2,    // Hermitian eigensolver, matrix in registers (n <= 128)
  PC_EIG_GLOBAL = 3, // Hermitian eigensolver, matrix in global memory
  PC_NCLASS = 4
};

// Returns an opaque token (>= 0) if the launch is profiled, else -1.
int prof_begin(int cls, hipStream_t s);
// Algorithmic work of a GEMM launch: 8 M N K flops per complex product and
// the bytes of reading op(A), op(B) and writing C once, per active item.
void prof_end_gemm(int token, int cls, const GemmDesc* d_descs, int nitems, int in_bytes, int out_bytes,
                   hipStream_t s);
// Eigensolver work: 16/3 n^3 (tridiagonalisation) + 8 n^2 k (back-
// transformation of k = min(kvec, n) vectors) flops; bytes = reading A and
// writing the k vectors.  Items outside [nlo, nhi] are skipped.
void prof_end_eig(int token, int cls, const EigDesc* d_descs, int nitems, int nlo, int nhi, hipStream_t s);

bool prof_enabled();
void prof_reset(bool on);
// Sums of one class; synchronises the device.
void prof_read(int cls, int* launches, double* ms, double* flops, double* bytes);

}  // namespace mpdo
