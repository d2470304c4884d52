// Instruction-rate calibration of the vector ALU (measurement only; not part
// of the solver): every thread runs four independent dependency chains of
// one instruction, 8192 waves keep every SIMD busy, and the time per
// wave-instruction per SIMD is reported.  It confirms the roofline
// denominators (FP64 and FP32 FMA rates) and prices the special functions
// (rsqrt, reciprocal, exp) that the quadrature's points use.
//
// Built into libscvt_calib.so; called by `bench.py --valu-rates`.  It also
// evaluates the solver's refined special functions on the device
// (scvt_calib_math), whose error bounds the host build cannot check: there
// they are exact divisions and square roots.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cellgeom.h"

namespace {

constexpr int kOps = 14;
constexpr int kBlocks = 256 * 8, kThreads = 256, kIters = 2000, kUnroll = 8;

#define SCVT_CH(op) op(a0); op(a1); op(a2); op(a3);
#define SCVT_F64FMA(x) asm volatile("v_fma_f64 %0, %0, %1, %2" : "+v"(x) : "v"(c1), "v"(c2))
#define SCVT_F64MUL(x) asm volatile("v_mul_f64 %0, %0, %1" : "+v"(x) : "v"(c1))
#define SCVT_F64RSQ(x) asm volatile("v_rsq_f64 %0, %0" : "+v"(x))
#define SCVT_F64RCP(x) asm volatile("v_rcp_f64 %0, %0" : "+v"(x))
#define SCVT_F64LDX(x) asm volatile("v_ldexp_f64 %0, %0, %1" : "+v"(x) : "v"(ie))
#define SCVT_F64RND(x) asm volatile("v_rndne_f64 %0, %0" : "+v"(x))
#define SCVT_F64MAX(x) asm volatile("v_max_f64 %0, %0, %1" : "+v"(x) : "v"(c1))
#define SCVT_F32FMA(x) asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(x) : "v"(f1), "v"(f2))
#define SCVT_F32RSQ(x) asm volatile("v_rsq_f32 %0, %0" : "+v"(x))
#define SCVT_F32RCP(x) asm volatile("v_rcp_f32 %0, %0" : "+v"(x))
#define SCVT_F32EXP(x) asm volatile("v_exp_f32 %0, %0" : "+v"(x))
#define SCVT_U32ADD(x) asm volatile("v_add_u32 %0, %0, %1" : "+v"(x) : "v"(iu))

template <int K>
__global__ __launch_bounds__(kThreads) void k_rate(double* out, int iters) {
  const double c1 = 0.999999, c2 = 1e-9;
  const float f1 = 0.999999f, f2 = 1e-9f;
  const int ie = 0;
  const uint32_t iu = 3;
  double a0 = 1.0 + threadIdx.x * 1e-6, a1 = a0 + 0.1, a2 = a0 + 0.2, a3 = a0 + 0.3;
  float b0 = (float)a0, b1 = (float)a1, b2 = (float)a2, b3 = (float)a3;
  uint32_t u0 = threadIdx.x, u1 = u0 + 1, u2 = u0 + 2, u3 = u0 + 3;
  for (int i = 0; i < iters; i++) {
#pragma unroll
    for (int u = 0; u < kUnroll; u++) {
      if (K == 0) { SCVT_CH(SCVT_F64FMA) }
      if (K == 1) { SCVT_CH(SCVT_F64MUL) }
      if (K == 2) { SCVT_CH(SCVT_F64RSQ) }
      if (K == 3) { SCVT_CH(SCVT_F64RCP) }
      if (K == 4) { SCVT_CH(SCVT_F64LDX) }
      if (K == 5) { SCVT_CH(SCVT_F64RND) }
      if (K == 6) { SCVT_CH(SCVT_F64MAX) }
      if (K == 7) { SCVT_F32FMA(b0); SCVT_F32FMA(b1); SCVT_F32FMA(b2); SCVT_F32FMA(b3); }
      if (K == 8) { SCVT_F32RSQ(b0); SCVT_F32RSQ(b1); SCVT_F32RSQ(b2); SCVT_F32RSQ(b3); }
      if (K == 9) { SCVT_F32RCP(b0); SCVT_F32RCP(b1); SCVT_F32RCP(b2); SCVT_F32RCP(b3); }
      if (K == 10) { SCVT_F32EXP(b0); SCVT_F32EXP(b1); SCVT_F32EXP(b2); SCVT_F32EXP(b3); }
      if (K == 11) { SCVT_U32ADD(u0); SCVT_U32ADD(u1); SCVT_U32ADD(u2); SCVT_U32ADD(u3); }
      if (K == 12) { SCVT_F64RSQ(a0); SCVT_F64FMA(a1); SCVT_F64FMA(a2); SCVT_F64FMA(a3); }
      if (K == 13) { SCVT_F32RSQ(b0); SCVT_F64FMA(a1); SCVT_F64FMA(a2); SCVT_F64FMA(a3); }
    }
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] =
      a0 + a1 + a2 + a3 + b0 + b1 + b2 + b3 + (double)(u0 + u1 + u2 + u3);
}

hipError_t launch_rate(int k, double* out, hipStream_t s) {
  switch (k) {
#define SCVT_L(K) \
  case K: k_rate<K><<<kBlocks, kThreads, 0, s>>>(out, kIters); break;
    SCVT_L(0) SCVT_L(1) SCVT_L(2) SCVT_L(3) SCVT_L(4) SCVT_L(5) SCVT_L(6)
    SCVT_L(7) SCVT_L(8) SCVT_L(9) SCVT_L(10) SCVT_L(11) SCVT_L(12) SCVT_L(13)
#undef SCVT_L
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// the device values of the refined special functions, one x per thread
constexpr int kMathOut = 9;
__global__ void k_math(const double* x, double* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = x[i];
  double* o = out + i * kMathOut;
  o[0] = scvt::rsq_pos(v);
  o[1] = scvt::rcp_fast(v);
  o[2] = scvt::sqrt_fast(v);
  o[3] = scvt::rcp_nr(v);
  o[4] = scvt::sqrt_nr(v);
  o[5] = scvt::rsq_near1(v);
  o[6] = (double)scvt::rsqf((float)v);
  o[7] = (double)scvt::rcpf((float)v);
  o[8] = (double)scvt::exp2_hw((float)v);
}

}  // namespace

extern "C" {

// out (host, n x 9, caller-owned): for each x[i] (host) the device's
// rsq_pos, rcp_fast, sqrt_fast, rcp_nr, sqrt_nr, rsq_near1 (FP64) and the
// FP32 hardware rsqrt, reciprocal and 2^x of (float)x.  Allocates and frees
// its own device buffers.  Returns 0, or -1 on a HIP error or n < 0.
int scvt_calib_math(int64_t n, const double* x, double* out) {
  if (n < 0) return -1;
  if (n == 0) return 0;
  double *dx = nullptr, *dout = nullptr;
  int rc = 0;
  if (hipMalloc(&dx, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&dout, sizeof(double) * n * kMathOut) != hipSuccess)
    rc = -1;
  if (!rc && hipMemcpy(dx, x, sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess) rc = -1;
  if (!rc) {
    k_math<<<(unsigned)((n + 255) / 256), 256>>>(dx, dout, n);
    if (hipGetLastError() != hipSuccess) rc = -1;
  }
  if (!rc && hipMemcpy(out, dout, sizeof(double) * n * kMathOut, hipMemcpyDeviceToHost) != hipSuccess)
    rc = -1;
  if (dx) hipFree(dx);
  if (dout) hipFree(dout);
  return rc;
}

// Number of measured instruction kinds.
int scvt_calib_count() { return kOps; }

// ns[k] = nanoseconds per wave-instruction per SIMD for kind k (k < count),
// counting the device's SIMDs as 4 per compute unit; best of `reps` timed
// launches after one untimed one (and 40 untimed FMA launches first).  Kinds: 0 f64 fma, 1 f64 mul, 2 f64 rsq,
// 3 f64 rcp, 4 f64 ldexp, 5 f64 rndne, 6 f64 max, 7 f32 fma, 8 f32 rsq,
// 9 f32 rcp, 10 f32 exp, 11 u32 add, 12 f64 rsq + 3 f64 fma (mean),
// 13 f32 rsq + 3 f64 fma (mean).  Returns 0, or -1 on a HIP error.  The
// library allocates and frees its own 4 MiB output buffer.
int scvt_calib_valu(double* ns, int reps) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return -1;
  double* out = nullptr;
  if (hipMalloc(&out, sizeof(double) * kBlocks * kThreads) != hipSuccess) return -1;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = 0;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = -1;
  // clocks up before the first timed kind: about 50 ms of FMAs
  for (int r = 0; r < 40 && !rc; r++)
    if (launch_rate(0, out, nullptr) != hipSuccess) rc = -1;
  const double simds = 4.0 * cus;
  const double winst = (double)kBlocks * kThreads / 64 * kIters * kUnroll * 4 / simds;
  for (int k = 0; k < kOps && !rc; k++) {
    if (launch_rate(k, out, nullptr) != hipSuccess) rc = -1;
    double best = 1e30;
    for (int r = 0; r < (reps > 0 ? reps : 1) && !rc; r++) {
      float ms = 0.f;
      if (hipEventRecord(e0, nullptr) != hipSuccess || launch_rate(k, out, nullptr) != hipSuccess ||
          hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        rc = -1;
      if (ms < best) best = ms;
    }
    ns[k] = best * 1e6 / winst;
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipFree(out);
  return rc;
}

}  // extern "C"
