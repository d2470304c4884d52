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

#ifdef __cplusplus
}
#endif

#endif
