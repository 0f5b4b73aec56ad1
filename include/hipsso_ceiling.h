/*
 * Measured hardware ceilings for the roofline of the hipsso kernels (libhipsso.so).
 *
 * The block-Jacobi PCG iteration (the dominant stage of the analysis) moves about 5 bytes per
 * flop, so it is bounded by HBM bandwidth; the element kernels are FP64 arithmetic.  These entry
 * points run kernels of the library's own on the given stream and return the mean duration of
 * one launch over `reps` back-to-back launches (after one untimed launch), timed with HIP events:
 *
 *   hipsso_ceiling_read: a streaming read of n doubles at src (device; n even), per-workgroup
 *     sums written to partials (device, at least 8192 doubles);  bytes = 8 n.
 *   hipsso_ceiling_copy: dst = src for n doubles (device, n even, non-overlapping);
 *     bytes = 16 n (read + write).
 *   hipsso_ceiling_fma: `workgroups` workgroups of 256 lanes, each lane 8 independent FP64 FMA
 *     chains of `iters` steps; flops = 16 * 256 * workgroups * iters.  out: device, at least
 *     `workgroups` doubles (not written for the inputs used).
 *
 * us_per_launch (host) receives the mean launch duration in microseconds.  Returns 0, -1 for a
 * bad argument (null pointer, n odd or not positive, reps < 1), -3 for a failed HIP call.
 */
#ifndef HIPSSO_CEILING_H
#define HIPSSO_CEILING_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

int hipsso_ceiling_read(const double* src, int64_t n, double* partials, int reps,
                        hipStream_t stream, double* us_per_launch);
int hipsso_ceiling_copy(const double* src, double* dst, int64_t n, int reps, hipStream_t stream,
                        double* us_per_launch);
int hipsso_ceiling_fma(double* out, int workgroups, int iters, int reps, hipStream_t stream,
                       double* us_per_launch);

#ifdef __cplusplus
}
#endif
#endif /* HIPSSO_CEILING_H */
