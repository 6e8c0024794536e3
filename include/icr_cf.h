/*
 * icr_cf.h - C ABI of the correlated-field model on an n x n periodic grid and the
 * Fisher metric of a Poisson likelihood, the operator NIFTy.re benchmarks (section
 * "Performance of NIFTy.re compared to NIFTy": apply M_p = F_p + 1 to random input,
 * with F_p = J^T N^-1 J the Fisher metric at position p; the model is the correlated
 * field of section "Gaussian Processes", s = FT(sqrt(P) xi)).
 *
 * The field is real: FT is the 2-D Hartley transform normalised to be its own inverse,
 *   T x = (Re - Im)(FFT2 x) / n,
 * and sqrt(P) is a fixed amplitude spectrum A(k) = a (1 + (|k| l)^2)^(-slope/4) over the
 * integer harmonic numbers |k| (the shorter way round the periodic grid) with
 * A(0) = zero_mode. The Poisson rate is lambda(xi) = exp(m + T(A xi)), so
 *   M_p v = v + A T(lambda(p) T(A v)).
 * All buffers are FP32 device arrays of n x n elements (row-major, 16-byte aligned),
 * caller-owned; one sample per call; calls are asynchronous on hip_stream and allocate
 * nothing (except icr_cf_create, which allocates A and the FFT twiddles). Status codes
 * as in icr.h.
 */
#ifndef ICR_CF_H
#define ICR_CF_H

#include <stdint.h>

#include "icr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct icr_cf_plan icr_cf_plan;  /* opaque; owns the device amplitude spectrum */

/* n a power of two in [32, 4096]; amplitude a > 0, zero_mode >= 0, length l >= 0,
 * slope and offset_mean m finite. Synchronous. */
icr_status icr_cf_create(int32_t n, double amplitude, double zero_mode, double length, double slope,
                         double offset_mean, void* hip_stream, icr_cf_plan** out_plan);
/* Device workspace for the calls below: 4 n^2 bytes (one real grid, in the transforms'
 * column-blocked order). */
icr_status icr_cf_workspace_bytes(const icr_cf_plan* plan, int64_t* bytes);
/* Copy A (FP32, n x n) to host memory. Synchronous. */
icr_status icr_cf_copy_amplitude(const icr_cf_plan* plan, float* amp);
/* y = T x. */
icr_status icr_cf_transform(const icr_cf_plan* plan, const float* x, float* y, void* workspace,
                            void* hip_stream);
/* Building M_p at position p: lambda = exp(m + T(A p)). */
icr_status icr_cf_rate(const icr_cf_plan* plan, const float* position, float* lambda, void* workspace,
                       void* hip_stream);
/* out = M_p v = v + A T(lambda T(A v)); v and out must differ. */
icr_status icr_cf_metric_apply(const icr_cf_plan* plan, const float* lambda, const float* v, float* out,
                               void* workspace, void* hip_stream);
/* Free the plan (NULL is a no-op). */
icr_status icr_cf_destroy(icr_cf_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* ICR_CF_H */
