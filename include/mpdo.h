/*
 * libmpdo -- QPT-assisted matrix product density operator simulator for
 * AMD Instinct MI355X (gfx950).  C ABI.
 *
 * The operations follow the problem statement of arXiv 2508.07610:
 *   - a noisy n-qubit state as a matrix product density operator (MPDO):
 *     site tensors T[l, p, n, r] with physical p, noise/inner n and bond
 *     indices l, r (Sec. II.C, Eq. (5)); rho is the sum over the inner
 *     indices of the tensor product with the conjugate copy (Eqs. (6)-(7));
 *   - process-tomography channels given as a Pauli chi-matrix, converted to
 *     Kraus operators through the Choi matrix (Sec. III, Eqs. (12)-(16));
 *   - noisy gates K_i = N_i K~ contracted into the state, the new noise
 *     index joining a site's inner index (Eq. (8), Fig. fig_mpdoSingle);
 *   - truncation of the inner index (SVD, Eqs. (9)-(11)) and of the bonds
 *     (canonical form, then SVD; Sec. II.D);
 *   - observables from transfer-matrix contractions (Eqs. (6)-(7)), the
 *     MaxCut objective (Eq. (20)) and state fidelities.
 *
 * Conventions (all entry points):
 *   - Complex numbers are interleaved (re, im) doubles on the host.
 *   - Matrices are row-major.  A q-qubit operator acts on (s_1 ... s_q) with
 *     s_1 the lowest site and the most significant index bit; qubit 0 is
 *     the leftmost site.
 *   - Pauli order is I, X, Y, Z; the q-qubit Pauli index is
 *     m = sum_t m_t 4^(q-1-t), t = 0 the lowest site.
 *   - Host buffers passed in are owned by the caller and only read during
 *     the call.  Handles own their device memory, released by the matching
 *     destroy call.  It comes from the caller's allocator when the config
 *     supplies one (alloc/free hooks, e.g. a framework's caching allocator),
 *     else from the library's cache of device blocks: a released block is
 *     kept and reused by later requests of up to its size (so repeated
 *     mpdo_batch_run calls of the same shapes allocate nothing after the
 *     first); mpdo_release_cached_memory() returns the cache to the driver.
 *   - Work is enqueued on the HIP stream given at creation (NULL = the
 *     default stream).  Calls that return host values synchronise that
 *     stream; others may return before the GPU work finishes.
 *   - A handle is not thread-safe.
 *   - Errors.  Argument errors (EINVAL, ENOTCPTP) are detected before any
 *     work starts: the call changes nothing.  Any error after work on the
 *     device has started (EDEVICE: a HIP call failed; ENOMEM; ENOTCONV: a
 *     numerical failure, see below) makes the handle unusable: that call and
 *     every later call on the handle except mpdo_destroy, mpdo_stats and
 *     mpdo_dims return an error (EDEVICE after the first).  Queued gates run
 *     when a call needs the state, so a failure in a queued gate is reported
 *     by the next call that synchronises (expect, trace, dims, truncate,
 *     to_dense, probabilities, sample, bond_weights, stats).
 *     mpdo_last_error() describes the last error of the calling thread.
 *   - Numerical failures (ENOTCONV) are detected on the device and checked
 *     at every synchronising call: a non-finite weight in a truncation, an
 *     eigenpair of a Gram matrix whose tridiagonal residual exceeds
 *     1e-9 ||T||, a non-finite or non-positive Tr(rho).
 */
#ifndef MPDO_H
#define MPDO_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MPDO_OK = 0,
  MPDO_EINVAL = 1,        /* bad argument: sites, sizes, null pointers       */
  MPDO_ENOTCPTP = 2,      /* chi does not describe a trace-preserving map    */
  MPDO_ENOMEM = 3,        /* device allocation failed                        */
  MPDO_EDEVICE = 4,       /* a HIP call failed; the handle is unusable       */
  MPDO_ENOTCONV = 5,      /* a numerical failure: an eigenpair above its
                             residual bound, non-finite weights or trace    */
  MPDO_EUNSUPPORTED = 6   /* valid but not implemented in this build         */
} mpdo_status;

typedef enum {
  MPDO_C128 = 0,          /* complex128 everywhere                            */
  MPDO_C64_MIXED = 1      /* complex64 tensors and contractions (FP32 MFMA);
                             Gram matrices, eigensolvers, truncation and
                             normalisation in FP64                            */
} mpdo_prec;

typedef struct {
  int32_t n;              /* qubits (sites), 1 <= n <= 64                     */
  int32_t chi_max;        /* bond dimension limit chi (Sec. II.D), 1..128     */
  int32_t kappa_max;      /* inner (noise) dimension limit kappa (Eq. (10)),
                             1..64                                            */
  int32_t max_kraus;      /* largest Kraus count of any channel that will be
                             applied (sizes the workspace), >= 1;
                             kappa_max * max_kraus <= 1024                    */
  double svd_cutoff;      /* bond truncation: drop the smallest singular
                             values whose summed squares are <= cutoff times
                             the total, then cap at chi_max                   */
  double kappa_cutoff;    /* same rule for the inner index                    */
  int32_t prec;           /* mpdo_prec                                        */
  /* Optional device allocator for every allocation the call or the handle
   * makes (both hooks set, or alloc NULL for the library's cache).  alloc
   * returns device memory of at least `bytes` bytes on the current device,
   * or NULL (the call then fails with ENOMEM); free releases it.  Memory is
   * released only after the device has finished the work that uses it. */
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* alloc_ctx;
} mpdo_config;

typedef struct mpdo_s* mpdo_t;
typedef struct mpdo_chan_s* mpdo_chan_t;

/* Last error message of the calling thread ("" if none). */
const char* mpdo_last_error(void);

/* Library version string. */
const char* mpdo_version(void);

/* Create the state rho = |0...0><0...0| for cfg->n qubits on the current HIP
 * device.  `hip_stream` is a hipStream_t (NULL = default stream).
 * Returns EINVAL for invalid sizes, ENOMEM if the tensors do not fit. */
mpdo_status mpdo_create(const mpdo_config* cfg, void* hip_stream, mpdo_t* out);

/* Release a state and its device memory.  NULL is accepted. */
mpdo_status mpdo_destroy(mpdo_t h);

/* Convert a process matrix to Kraus operators on the GPU (Sec. III):
 * Lambda = sum_mn chi_mn |sigma_m>><<sigma_n| (Eqs. (13)-(14)), Lambda =
 * sum_i eta_i |psi_i><psi_i| (Eq. (15)), K_i = sqrt(eta_i) unvec(psi_i)
 * (Eq. (16)), eigenvalues in descending order, negative ones clipped,
 * operators of weight eta_i / sum eta below `eps` dropped (Sec. III,
 * pruning "by descending eigenvalue magnitude").
 *   chi: host, 4^q x 4^q complex, interleaved, row-major, q in {1, 2, 3}.
 *   Returns ENOTCPTP if sum_i K_i^dag K_i differs from the identity by more
 *   than 1e-8 (before pruning), EINVAL for bad q or non-Hermitian chi. */
mpdo_status mpdo_channel_from_chi(const double* chi, int32_t q, double eps,
                                  void* hip_stream, mpdo_chan_t* out);

/* Number of Kraus operators and qubits of a channel; optionally copy the
 * operators to `kraus_out` (host, nkraus x 2^q x 2^q complex, may be NULL). */
mpdo_status mpdo_channel_info(mpdo_chan_t ch, int32_t* q, int32_t* nkraus,
                              double* kraus_out);

mpdo_status mpdo_channel_destroy(mpdo_chan_t ch);

/* Apply the ideal gate U (host, 2^q x 2^q complex) on `sites` (q ascending
 * adjacent sites, q in {1, 2, 3}).  A 2- or 3-qubit gate re-splits the block
 * by SVD with bond truncation. */
mpdo_status mpdo_apply_gate(mpdo_t h, const int32_t* sites, int32_t q, const double* U);

/* Apply the noisy gate "U then channel": operators G_i = K_i U (Eq. (8));
 * U may be NULL (identity).  The Kraus index joins the inner index of the
 * lowest site (q <= 2) or the middle site (q = 3); that inner index is then
 * truncated (Eqs. (9)-(11)) and the touched bonds are re-split by SVD with
 * truncation.  q in {1, 2, 3}; sites ascending and adjacent. */
mpdo_status mpdo_apply_channel(mpdo_t h, const int32_t* sites, int32_t q,
                               const double* U, mpdo_chan_t ch);

/* Finish all queued gates (gates on disjoint sites are grouped into one
 * launch sequence; this call forces the queue out). */
mpdo_status mpdo_flush(mpdo_t h);

/* The truncation sweep of Sec. II.D: orthonormalise from left to right,
 * then SVD from right to left truncating every bond to chi_max with the
 * cutoff rule, then truncate every inner index to kappa_max.  Writes the
 * summed discarded weight to *discarded (may be NULL). */
mpdo_status mpdo_truncate(mpdo_t h, int32_t chi_max, int32_t kappa_max,
                          double cutoff, double* discarded);

/* Tr(P rho) / Tr(rho) for a Pauli string of length n over "IXYZ". */
mpdo_status mpdo_expect(mpdo_t h, const char* pauli, double* re, double* im);

/* Tr(O rho) / Tr(rho) for a batch of product operators:
 * ops: host, nops x n x 2 x 2 complex (operator k on site i at
 * ops + ((k n + i) 4) 2 doubles); out: host, nops complex. */
mpdo_status mpdo_expect_products(mpdo_t h, const double* ops, int32_t nops, double* out);

/* <GHZ| rho |GHZ> / Tr rho with |GHZ> = (|0..0> + |1..1>)/sqrt(2). */
mpdo_status mpdo_fidelity_ghz(mpdo_t h, double* f);

/* Tr(rho) (after the library's normalisation it is 1 up to truncation). */
mpdo_status mpdo_trace(mpdo_t h, double* tr);

/* Current dimensions: bonds (n-1 ints, may be NULL), inner (n ints, may be
 * NULL), and the summed discarded weight of all truncations (may be NULL). */
mpdo_status mpdo_dims(mpdo_t h, int32_t* bonds, int32_t* inner, double* discarded);

/* Bond weights lambda of bond b (between sites b and b+1): writes up to
 * `cap` doubles and the count to *len. */
mpdo_status mpdo_bond_weights(mpdo_t h, int32_t b, double* out, int32_t cap, int32_t* len);

/* Truncation statistics of a state (metrics for diagnosing truncated
 * results; the rule is the one of mpdo_config):
 *   truncations: inner and bond truncations applied so far;
 *   discarded: summed discarded weight, each truncation's dropped fraction
 *     of its Gram trace (Eq. (10): the squared Frobenius error of the
 *     truncated site, relative);
 *   max_discarded: the largest single one;
 *   min_gap: smallest relative gap eta_{r-1} / eta_r - 1 between the last
 *     kept and the first dropped eigenvalue over all truncations that
 *     dropped weight (1e300 if none): a cut inside a near-degenerate
 *     multiplet makes a truncated result depend on rounding;
 *   trace: Tr(rho) of the current state, unnormalised (its drift from 1
 *     measures accumulated rounding and pruning);
 *   failures: numerical failures detected on the device (nonzero means the
 *     handle has reported ENOTCONV);
 *   max_bond, max_inner: largest bond and inner dimension.
 * Works on an unusable handle too (then trace is NaN). */
typedef struct {
  int64_t truncations;
  int64_t failures;
  double discarded;
  double max_discarded;
  double min_gap;
  double trace;
  int32_t max_bond;
  int32_t max_inner;
} mpdo_stats_t;
mpdo_status mpdo_stats(mpdo_t h, mpdo_stats_t* out);

/* Return the library's cache of released device and pinned host blocks to
 * the driver (blocks held by live handles stay).  *cached (may be NULL)
 * receives the device bytes the cache held. */
mpdo_status mpdo_release_cached_memory(size_t* cached);

/* The dense density matrix (Eqs. (6)-(7): the per-site tensors summed over
 * the inner index, contracted along the chain) for n <= 12: rho is host
 * memory of 2^n x 2^n complex doubles, row-major, qubit 0 the most
 * significant bit of the row and column indices.  For verification: the
 * contraction runs on the device in FP64 (in both precisions) and needs
 * about 5 x 16 x max(4^(n/2) chi^2, 4 chi^4, 4^n) bytes of scratch;
 * EUNSUPPORTED above 16 GiB, EINVAL for n > 12. */
mpdo_status mpdo_to_dense(mpdo_t h, double* rho);

/* Computational-basis measurement (the bitstring distributions compared in
 * Sec. IV.A, whose distance there is the Jensen-Shannon divergence, Eq. (18)).
 *
 * mpdo_probabilities: p[z] = <z| rho |z> / Tr rho for nz bitstrings.
 * bits: host, nz x n bytes, each 0 or 1 (bits[z n + i] is qubit i of string
 * z, qubit 0 first); p: host, nz doubles.  EINVAL for a byte above 1.
 *
 * mpdo_sample: nshots bitstrings drawn by sequential conditionals: qubit i
 * of shot t is 0 when u[t n + i] < P(z_i = 0 | z_0 .. z_{i-1}), else 1.  The
 * random numbers are the caller's: u is host memory of nshots x n uniforms
 * in [0, 1) (EINVAL otherwise), so a draw is reproducible.  bits: host,
 * nshots x n bytes (output); pz: host, nshots doubles, the probability
 * P(z) / Tr rho of each drawn string (the product of its conditionals), or
 * NULL.  The conditionals come from left environments of the shots and right
 * environments of the state, contracted on the device in the handle's
 * precision; ENOTCONV if a prefix has no weight. */
mpdo_status mpdo_probabilities(mpdo_t h, const uint8_t* bits, int32_t nz, double* p);
mpdo_status mpdo_sample(mpdo_t h, const double* u, int32_t nshots, uint8_t* bits, double* pz);

/* ---------------------------------------------------------------------------
 * Batched execution: many independent instances (parameter points, graphs of
 * different sizes) advanced together, every sublayer of every instance in
 * one launch sequence, the whole run captured in one HIP graph.
 * ------------------------------------------------------------------------- */

typedef enum {
  MPDO_G_FIXED = 0,   /* U given in the program                              */
  MPDO_G_RX = 1,      /* exp(-i a X / 2), a = scale * param                  */
  MPDO_G_RY = 2,
  MPDO_G_RZ = 3,
  MPDO_G_ZZPHASE = 4, /* exp(-i a (1 - Z Z) / 2) (Eq. (21) cost term)        */
  MPDO_G_SWAPZZ = 5   /* SWAP . exp(-i a (1 - Z Z) / 2)                      */
} mpdo_gate_kind;

typedef struct {
  int32_t q;            /* 1, 2 or 3 (3: kind MPDO_G_FIXED with fixed = -1,
                           i.e. a three-site channel without a gate)          */
  int32_t site;         /* lowest site                                         */
  int32_t kind;         /* mpdo_gate_kind                                      */
  int32_t param;        /* index into the instance's parameter row, or -1      */
  double scale;         /* angle = scale * param value                         */
  int32_t chan;         /* channel slot (index into `chans`), or -1            */
  int32_t fixed;        /* for MPDO_G_FIXED: index into `fixed_u`, or -1 for
                           the identity                                        */
} mpdo_op;

typedef struct {
  int32_t n;            /* qubits of this instance                            */
  int32_t nops;
  const mpdo_op* ops;   /* host                                                */
  int32_t nobs;         /* observables: product operators                     */
  const double* obs;    /* host, nobs x n x 2 x 2 complex                      */
} mpdo_program;

/* Run `ninst` programs to completion and write, for instance b, its nobs
 * expectation values Tr(O rho)/Tr(rho) as complex doubles to
 * out_dev + 2 * (obs_offset[b] + k), where obs_offset is the prefix sum of
 * nobs.  params_dev: device doubles, instance b's parameter row at
 * params_dev + b * param_stride.  fixed_u: host, nfixed 4x4 complex
 * (2-qubit) or 2x2 (1-qubit, stored in the top-left of a 4x4 slot).
 * chans: channel handles.  cfg: chi_max, kappa_max, cutoffs, precision for
 * all instances (cfg->n ignored).  Gates are grouped per instance into
 * sublayers on disjoint sites (an op joins the first group after the last
 * one touching its sites) and the k-th sublayers of all instances run as one
 * ragged launch sequence.  `use_graph` != 0 captures the whole run (one
 * descriptor upload, every sublayer, the observables) into one HIP graph and
 * launches it once; with hip_stream NULL a private stream is used for the
 * capture.  The call returns when the results are in out_dev.  Returns
 * EINVAL for malformed programs, ENOTCONV (after writing the results) when
 * a numerical failure was detected in any instance.  Device memory comes
 * from cfg's allocator or the library's cache (no driver allocation once
 * a run of the same shapes has been made). */
mpdo_status mpdo_batch_run(const mpdo_config* cfg, const mpdo_program* progs, int32_t ninst,
                           const double* params_dev, int32_t param_stride,
                           const double* fixed_u, int32_t nfixed,
                           const mpdo_chan_t* chans, int32_t nchans,
                           double* out_dev, int32_t use_graph, void* hip_stream);

/* As mpdo_batch_run (launch by launch; observables of the programs are
 * ignored), then the dense density matrix of every instance, as
 * mpdo_to_dense computes it (unnormalised, FP64), to device memory: instance
 * b's 2^n x 2^n complex matrix at rho_dev + 2 * off_b doubles, off_b the sum
 * of 4^n over the earlier instances.  For verification workloads with
 * n <= 12 (EINVAL above), such as the fidelity study of Sec. IV.C. */
mpdo_status mpdo_batch_run_dense(const mpdo_config* cfg, const mpdo_program* progs, int32_t ninst,
                                 const double* params_dev, int32_t param_stride,
                                 const double* fixed_u, int32_t nfixed,
                                 const mpdo_chan_t* chans, int32_t nchans,
                                 double* rho_dev, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Kernel profiling (process-wide, not thread-safe).  While enabled, every
 * launch of the library's compute kernels on a stream that is not being
 * captured into a graph is bracketed by two HIP events recorded on that
 * stream, and the launch's algorithmic work, computed on the device from the
 * shapes its descriptors hold when it runs, is added to per-class counters:
 *   GEMM classes: 8 M N K flops per complex product; bytes of reading op(A)
 *     and op(B) and writing C once;
 *   eigensolver classes: 16/3 n^3 + 8 n^2 k flops (Householder
 *     tridiagonalisation, back-transformation of k vectors); bytes of reading
 *     the matrix and writing k vectors.
 * ------------------------------------------------------------------------- */
typedef enum {
  MPDO_PROF_GEMM_F64 = 0,   /* complex GEMMs on FP64 MFMA                     */
  MPDO_PROF_GEMM_F32 = 1,   /* complex GEMMs on FP32 MFMA (mixed precision)   */
  MPDO_PROF_EIG_REG = 2,    /* eigensolver, n <= 128 (register-resident)      */
  MPDO_PROF_EIG_GLOBAL = 3, /* eigensolver, one-stage, matrix in global memory */
  MPDO_PROF_EIG_BAND = 4,   /* eigensolver, 128 < n <= 256, through a band    */
  MPDO_PROF_CHOL = 5,       /* pivoted Cholesky of the right-factor Gram      */
  MPDO_PROF_NCLASS = 6
} mpdo_prof_class;

/* Reset the counters (synchronises the device) and switch profiling on
 * (on != 0) or off. */
mpdo_status mpdo_profile_enable(int32_t on);

/* Totals of one class since the last reset: launches, summed event time in
 * milliseconds, algorithmic flops and bytes (any pointer may be NULL).
 * Synchronises the device.  EINVAL for an unknown class. */
mpdo_status mpdo_profile_read(int32_t cls, int32_t* launches, double* ms, double* flops, double* bytes);

/* ---------------------------------------------------------------------------
 * GEMM tuning (process-wide; an autotuner times candidates and sets them).
 * The contractions of the MPDO update are grouped by call site:
 *   1-2 one-site update: Gram, projection; 3-9 two-site update: E Gram,
 *   theta, H Gram, theta'', C Gram, X, outputs; 10-11 right and left transfer
 *   steps; 12-22 three-site update (N/E3 Grams, Xt, Psi, H Gram, Psi2, C1
 *   Gram, Y1, W1, C2 Gram, Y3, outputs); 23-24 truncation sweep (Gram,
 *   outputs).
 * Per site: tile edge (32 or 64), complex-product form (4: four real MFMA
 * products per complex product; 3: Gauss's three, P1 = Ar Br, P2 = Ai Bi,
 * P3 = (Ar + Ai)(Br + Bi), Re = P1 - P2, Im = P3 - P1 - P2) and a factor on
 * the split-K count of the Gram sites; 0 keeps the library's built-in choice.
 * Settings apply to launches issued after the call (a captured graph keeps
 * the settings of its capture).  EINVAL for a site outside 1..24 or values
 * outside those sets (split_scale in [0, 16]).
 * ------------------------------------------------------------------------- */
mpdo_status mpdo_tune_set(int32_t site, int32_t tile, int32_t form, double split_scale);
mpdo_status mpdo_tune_get(int32_t site, int32_t* tile, int32_t* form, double* split_scale);

/* ---------------------------------------------------------------------------
 * Error mitigation by the inverse of the noisy process (Sec. V: the noisy
 * process can be undone with a matrix product operator of its inverse).
 *
 * An mpdo_mpo_t holds rho of a state as the chain of the paper's local
 * density tensors (Eq. (6)),
 *   R_i[(l l'), (p p'), (r r')] = sum_n T_i[l, p, n, r] conj(T_i[l', p', n, r']),
 * whose contraction is rho (Eq. (7)), in complex double on the device.  A
 * channel rho -> sum_j K_j rho K_j^dagger acts on the row-major vector of
 * rho as the superoperator S = sum_j K_j (x) conj(K_j); on q sites it acts
 * on the pair indices (p_1 p_1' .. p_q p_q').  The inverse of a channel is
 * the matrix inverse of its S (a linear map, not completely positive), the
 * inverse of a gate U is U^dagger.  Mitigating the output of a noisy circuit
 * N_L U_L .. N_1 U_1 with a noise model N^ applies N^_L^-1, U_L^-1, ..,
 * N^_2^-1, U_2^-1, N^_1^-1 and then U_2 .. U_L (unwinding the circuit, then
 * replaying it without noise).  After the map rho is linear in the tensors
 * and may be non-positive; the two-site maps split the contracted pair again
 * by an SVD (the Gram matrix of its smaller side and the library's
 * eigensolver) with the rule: smallest rank whose dropped squared singular
 * values are <= cutoff times their total, at most d_max.
 *
 * Limits: one MPO per call sequence on the stream of the state it was made
 * from (the caller's; destroy the MPO before that stream); bonds of the
 * source state <= 32 (MPO bonds <= 1024); a two-site map needs one of its
 * two outer bonds <= 256; gates and channels on q <= 2 adjacent sites.
 * ------------------------------------------------------------------------- */
typedef struct mpdo_mpo_s* mpdo_mpo_t;

/* rho of state h (its queued gates applied first) as an MPO; d_max in
 * [1, 256], cutoff in [0, 1).  Allocates through h's allocator. */
mpdo_status mpdo_mpo_from_state(mpdo_t h, int32_t d_max, double cutoff, mpdo_mpo_t* out);
mpdo_status mpdo_mpo_destroy(mpdo_mpo_t m);
/* The gate U (host, 2^q x 2^q complex, row-major, interleaved re/im) on
 * sites site .. site + q - 1, or its inverse U^dagger when inverse != 0.
 * U is not checked for unitarity. */
mpdo_status mpdo_mpo_apply_gate(mpdo_mpo_t m, int32_t site, int32_t q, const double* U, int32_t inverse);
/* The channel ch (q <= 2, on sites site .. site + q - 1), or the inverse of
 * its superoperator when inverse != 0 (MPDO_ENOTCONV if it is singular:
 * a pivot below 1e-13 of its largest entry). */
mpdo_status mpdo_mpo_apply_channel(mpdo_mpo_t m, int32_t site, mpdo_chan_t ch, int32_t inverse);
/* out[2k], out[2k+1] = Tr(O_k rho) for nops product operators
 * O_k = (x)_i ops[k][i] (ops: host, nops x n x 2 x 2 complex), unnormalised
 * (divide by the value for identities for a normalised expectation). */
mpdo_status mpdo_mpo_expect(mpdo_mpo_t m, const double* ops, int32_t nops, double* out);
/* bonds: n - 1 ints; discarded: summed dropped fraction of the splits. */
mpdo_status mpdo_mpo_dims(mpdo_mpo_t m, int32_t* bonds, double* discarded);
/* rho (host, 2^n x 2^n complex, row-major), n <= 12. */
mpdo_status mpdo_mpo_to_dense(mpdo_mpo_t m, double* rho);

/* ---------------------------------------------------------------------------
 * Surrogate network: a multilayer perceptron trained on MPDO-generated
 * (parameters, noise) -> observables data.  Widths d_0 .. d_L; hidden
 * layers z_l = W_l h_{l-1} + b_l, h_l = GELU(z_l) = z Phi(z) (exact erf
 * form); output y = W_L h_{L-1} + b_L; loss = mean over batch and outputs of
 * (y - t)^2.  Operands of every matrix product (inputs, activations, weights,
 * gradients with respect to z) are bfloat16 (round to nearest even), the
 * products accumulate in FP32 on the matrix cores; biases, pre-activations,
 * gradients, master weights and Adam moments are FP32.
 * Parameters are packed as W_1 (d_1 x d_0, row-major), b_1, W_2, b_2, ...
 * All x / t / y / gradient buffers are device pointers (FP32, row-major,
 * one sample per row) and the work is ordered on the network's stream.
 * ------------------------------------------------------------------------- */
typedef struct mpdo_mlp_s* mpdo_mlp_t;

/* widths: nlayers + 1 ints in [1, 8192]; max_batch in [1, 2^20] sizes the
 * activation buffers.  Parameters start at zero. */
mpdo_status mpdo_mlp_create(const int32_t* widths, int32_t nlayers, int32_t max_batch, void* hip_stream,
                            mpdo_mlp_t* out);
mpdo_status mpdo_mlp_destroy(mpdo_mlp_t h);
mpdo_status mpdo_mlp_info(mpdo_mlp_t h, int64_t* nparams);
/* host FP32 arrays of nparams; set also resets the Adam state. */
mpdo_status mpdo_mlp_set_params(mpdo_mlp_t h, const float* host);
mpdo_status mpdo_mlp_get_params(mpdo_mlp_t h, float* host);
/* y_dev (batch x d_L) = network(x_dev (batch x d_0)). */
mpdo_status mpdo_mlp_forward(mpdo_mlp_t h, const float* x_dev, int32_t batch, float* y_dev);
/* Forward into y_dev, then back-propagate either the MSE loss against
 * targets t_dev, or a given output cotangent gy_dev (exactly one of the two
 * non-NULL).  Parameter gradients are kept for mpdo_mlp_adam and copied to
 * grad_dev (nparams) if non-NULL; the input gradient goes to dx_dev
 * (batch x d_0) if non-NULL; *loss (if non-NULL) receives the MSE (0 with
 * gy_dev) and makes the call synchronous. */
mpdo_status mpdo_mlp_backward(mpdo_mlp_t h, const float* x_dev, const float* t_dev, const float* gy_dev,
                              int32_t batch, float* y_dev, float* grad_dev, float* dx_dev, float* loss);
/* One Adam step (bias-corrected) with the gradients of the last backward. */
mpdo_status mpdo_mlp_adam(mpdo_mlp_t h, float lr, float beta1, float beta2, float eps);
/* `steps` training steps in one call (no host synchronisation unless loss
 * is non-NULL): each draws `batch` rows (in [1, max_batch]) uniformly with
 * replacement from the nrows-row dataset x_dev (nrows x d_0) / t_dev
 * (nrows x d_L), takes the MSE gradient as mpdo_mlp_backward and one Adam
 * step (beta1 0.9, beta2 0.999, eps 1e-8; the step count continues that of
 * mpdo_mlp_adam).  Row b of step s (from 0) is dataset row
 * SplitMix64(seed)_k mod nrows with k = s batch + b + 1, where the k-th
 * output of SplitMix64 seeded with `seed` is its finalizer applied to
 * seed + k 0x9E3779B97F4A7C15.  Learning rate lr, or with cosine != 0
 * lr (1 + cos(pi s / steps)) / 2.  *loss (if non-NULL) receives the last
 * step's MSE and makes the call synchronous. */
mpdo_status mpdo_mlp_fit(mpdo_mlp_t h, const float* x_dev, const float* t_dev, int64_t nrows, int32_t batch,
                         int32_t steps, float lr, int32_t cosine, uint64_t seed, float* loss);
/* Gradient ascent on the network's input: from the input row x0_dev (d_0
 * floats, device), `steps` Adam steps (bias-corrected) on the first nfree
 * entries (the rest are held) along the gradient of output out_index,
 * x += lr mhat / (sqrt(vhat) + eps); the row after step s goes to
 * xs_dev + s d_0 (steps x d_0 floats, device).  The Adam moments and step
 * count are kept in the handle between calls; reset != 0 zeroes them first.
 * Parameter gradients are not touched. */
mpdo_status mpdo_mlp_ascend(mpdo_mlp_t h, const float* x0_dev, int32_t nfree, int32_t out_index, int32_t steps,
                            float lr, float beta1, float beta2, float eps, int32_t reset, float* xs_dev);

#ifdef __cplusplus
}
#endif
#endif /* MPDO_H */
