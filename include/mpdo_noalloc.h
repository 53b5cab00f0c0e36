/*
 * libmpdo -- allocation-free entry point (C ABI), declared apart from
 * mpdo.h.  Conventions as in mpdo.h.
 */
#ifndef MPDO_NOALLOC_H
#define MPDO_NOALLOC_H

#include "mpdo.h"

#ifdef __cplusplus
extern "C" {
#endif

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid it): the conversion of
 * mpdo_channel_from_chi with device inputs and outputs, allocating nothing.
 * Its scratch (Choi matrix, eigensolver work) is a 512 KiB array in the
 * library's device image, one per device, held until the process ends; every
 * call on a device shares it, so calls that overlap on one device (two
 * streams, two threads) race: order them.  Every step is a kernel on
 * `hip_stream` (NULL = default stream); the call returns without waiting.
 *   chi_dev: device, 4^q x 4^q complex (interleaved, row-major), Hermitian
 *     (not checked: the host form checks it);
 *   kraus_dev: device, room for 4^q operators of 2^q x 2^q complex; the kept
 *     operators K_i = sqrt(eta_i) unvec(psi_i) (eigenvalues descending,
 *     weight eta_i / sum eta >= eps, as mpdo_channel_from_chi) are written
 *     first;
 *   info_dev: device, 4 doubles: kept count, max |sum K^dag K - I| of the
 *     unpruned set (above 1e-8: not trace preserving), the smallest Choi
 *     eigenvalue, the Choi rank.
 * EINVAL for null pointers, q outside 1..3 or eps outside [0, 1) (a q that
 * would need more scratch than the array holds is rejected the same way). */
mpdo_status mpdo_kraus_from_chi_noalloc(const double* chi_dev, int32_t q, double eps,
                                        double* kraus_dev, double* info_dev, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* MPDO_NOALLOC_H */
