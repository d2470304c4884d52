/* Vector-ALU instruction-rate calibration (measurement only; libscvt_calib.so).
 *
 * Not part of the solver: it backs the roofline denominators that bench.py
 * reports for the quadrature kernel (FP64 and FP32 FMA issue rates) and
 * prices the special functions the quadrature points use.  Each measured
 * kind is one instruction in four independent dependency chains per thread,
 * 8192 wavefronts (every SIMD of the device busy).
 */
#ifndef SCVT_CALIB_H
#define SCVT_CALIB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Number of instruction kinds scvt_calib_valu measures (14). */
int scvt_calib_count(void);

/* ns: host array of scvt_calib_count() doubles, owned by the caller; on
 * return ns[k] is the time per wave-instruction per SIMD in nanoseconds
 * (best of `reps` launches after 40 untimed ones that bring the clocks up;
 * SIMDs counted as 4 per compute unit of the current device).  Kinds in order: f64 fma, f64 mul, f64 rsq, f64 rcp,
 * f64 ldexp, f64 rndne, f64 max, f32 fma, f32 rsq, f32 rcp, f32 exp,
 * u32 add, f64 rsq + 3 f64 fma, f32 rsq + 3 f64 fma (the last two: mean per
 * instruction of the mix).  Runs on the current device's default stream and
 * allocates (and frees) a 4 MiB output buffer.  Returns 0, or -1 on any HIP
 * error. */
int scvt_calib_valu(double* ns, int reps);

/* Checking only: the device values of the solver's refined special
 * functions, whose error bounds the host build cannot test.  x: host array
 * of n doubles; out: host array of n x 9 doubles, owned by the caller; row i
 * receives rsq_pos, rcp_fast, sqrt_fast, rcp_nr, sqrt_nr, rsq_near1 of x[i]
 * (FP64) and the FP32 hardware reciprocal square root, reciprocal and 2^x
 * of (float)x[i], as the kernels evaluate them.  Allocates and frees its own
 * device buffers on the current device.  Returns 0, or -1 on a HIP error or
 * n < 0. */
int scvt_calib_math(int64_t n, const double* x, double* out);

#ifdef __cplusplus
}
#endif

#endif
