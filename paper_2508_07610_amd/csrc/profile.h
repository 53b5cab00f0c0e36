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
  PC_EIG_BAND = 4,   // Hermitian eigensolver, two-stage through a band (128 < n <= 256)
  PC_CHOL_E = 5,     // pivoted Cholesky of the two-site right-factor Gram and its triangular inverse
  PC_NCLASS = 6
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
// Pivoted Cholesky of an n x n Hermitian matrix and the inverse of its
// triangular factor (n from the item's EigDesc): 8/3 n^3 flops (4/3 n^3
// each); bytes = reading the matrix and writing two n x n factors.
void prof_end_chol(int token, int cls, const EigDesc* d_descs, int nitems, hipStream_t s);

// Call site of the following GEMM launches on this thread (a label of the
// contraction, see GemmSite); each site's time and work are also summed.
enum GemmSite : int {
  GS_OTHER = 0,
  GS_Q1_GRAM = 1, GS_Q1_PROJ = 2,
  GS_Q2_GRAM_E = 3, GS_Q2_THETA = 4, GS_Q2_GRAM_H = 5, GS_Q2_THETA2 = 6, GS_Q2_GRAM_C = 7, GS_Q2_X = 8,
  GS_Q2_OUT = 9,
  GS_TRANSFER_R = 10, GS_TRANSFER_L = 11,
  GS_Q3_GRAM_NE = 12, GS_Q3_XT = 13, GS_Q3_PSI = 14, GS_Q3_GRAM_H = 15, GS_Q3_PSI2 = 16, GS_Q3_GRAM_C1 = 17,
  GS_Q3_Y1 = 18, GS_Q3_W1 = 19, GS_Q3_GRAM_C2 = 20, GS_Q3_Y3 = 21, GS_Q3_OUT = 22,
  GS_SWEEP_GRAM = 23, GS_SWEEP_OUT = 24,
  GS_N = 25
};
void prof_set_site(int site);
// Sums of one GEMM call site (both precisions); synchronises the device.
void prof_read_site(int site, int* launches, double* ms, double* flops);

bool prof_enabled();
void prof_reset(bool on);
// Sums of one class; synchronises the device.
void prof_read(int cls, int* launches, double* ms, double* flops, double* bytes);

}  // namespace mpdo
