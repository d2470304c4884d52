// LBFGS two-loop recursion with the Lloyd preconditioner, history push and
// the per-evaluation reductions, as fused streaming passes.  Every grid
// reduction is taken in a fixed order: thread partials over a fixed
// grid-stride, a block tree, then the block partials in block order, summed
// by whoever needs the value (the next pass, or a one-block finalize
// kernel) -- no atomics, the same bits on every run.
//
// Two-loop (section 2.2.2, initial inverse Hessian replaced by diag(h),
// section 3.1) over c stored pairs (oldest j = 0):
//   q = -g;  for j = c-1..0: a_j = r_j s_j.q ; q -= a_j y_j
//   q = h (.) q  (h_i on the three coordinates of generator i)
//   for j = 0..c-1: b = r_j y_j.q ; q += (a_j - b) s_j
// One pass per loop step: the axpy of step k is fused with the dot product
// of step k+1, so the 2c+1 passes each stream q once.
#include "kernels.h"
#include "lbfgs.h"

namespace scvt {

constexpr int kRedBlock = 256;
constexpr int kRedGrid = 512;

__device__ inline double block_sum(double v, double* sh) {
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = kRedBlock / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}
__device__ inline double block_max(double v, double* sh) {
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = kRedBlock / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}
__device__ inline double block_min(double v, double* sh) {
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = kRedBlock / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = fmin(sh[t], sh[t + s]);
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// fixed-order sum of nb partials (stride `stride`, offset `off`)
__device__ inline double sum_partials(const double* p, int nb, int stride, int off, double* sh) {
  double v = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) v += p[b * stride + off];
  return block_sum(v, sh);
}

// ------------------------------------------------------------- two-loop pass
// Flat, contiguous elements with 32-bit indices (3n < 2^31): element k
// belongs to generator k/3, a multiply-high with a 32-bit divisor.
__global__ __launch_bounds__(kRedBlock) void k_lbfgs_pass(PassArgs a) {
  __shared__ double sh[kRedBlock];
  double coef = 0.0;
  if (a.prev_partials) {
    double sum = sum_partials(a.prev_partials, gridDim.x, 1, 0, sh);
    double v = a.prev_sub ? (*a.prev_sub) - (*a.prev_mul) * sum : (*a.prev_mul) * sum;
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.prev_store = v;
    coef = v;
  }
  const double axc = a.ax_sign * coef;
  double part = 0.0;
  const int n3 = (int)a.n3;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n3; k += gridDim.x * blockDim.x) {
    double qk = a.init_neg_g ? -a.g[k] : a.q[k];
    if (a.ax_vec) qk += axc * a.ax_vec[k];
    if (a.scale_h) qk *= a.h[(unsigned)k / 3u];
    a.q[k] = qk;
    part += a.dot_vec[k] * qk;
  }
  double bs = block_sum(part, sh);
  if (threadIdx.x == 0) a.partials[blockIdx.x] = bs;
}

// --------------------------------------------------------------- push pass
// s = Zt - Z, y = gt - g into the ring slot; partials of y.s, y.y, s.s
__global__ __launch_bounds__(kRedBlock) void k_push(PushArgs a) {
  __shared__ double sh[kRedBlock];
  double ys = 0.0, yy = 0.0, ss = 0.0;
  const int n3 = (int)a.n3;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n3; k += gridDim.x * blockDim.x) {
    double s = a.Zt[k] - a.Z[k];
    double y = a.gt[k] - a.g[k];
    a.s[k] = s;
    a.y[k] = y;
    ys += y * s;
    yy += y * y;
    ss += s * s;
  }
  double b0 = block_sum(ys, sh), b1 = block_sum(yy, sh), b2 = block_sum(ss, sh);
  if (threadIdx.x == 0) {
    a.partials[3 * blockIdx.x] = b0;
    a.partials[3 * blockIdx.x + 1] = b1;
    a.partials[3 * blockIdx.x + 2] = b2;
  }
}

// ------------------------------------------------------ evaluation reduce
// Per generator the gradient, preconditioner and Lloyd step from mu (section
// 3.1), then partials of F = sum e_i, max |l_ik|, sum |g_i|^2, min mu_i . z_i
template <class P>
__global__ __launch_bounds__(kRedBlock) void k_eval_reduce(P p) {
  if (p.idle()) return;
  const EvalRedArgs& a = p.args();
  __shared__ double sh[kRedBlock];
  double F = 0.0, lmax = 0.0, gg = 0.0, mzmin = 1e300;
  const int n = (int)a.n;
  for (int i = p.bx() * blockDim.x + threadIdx.x; i < n; i += p.gx() * blockDim.x) {
    const V3 z = V3{a.Z[3 * i], a.Z[3 * i + 1], a.Z[3 * i + 2]};
    const V3 mu = V3{a.mu[3 * i], a.mu[3 * i + 1], a.mu[3 * i + 2]};
    const double e = a.e[i];
    const double mz = dot(mu, z);
    const V3 g = 2.0 * mz * z - 2.0 * mu;
    const V3 l = normalized(mu) - z;
    a.g[3 * i] = g.x;
    a.g[3 * i + 1] = g.y;
    a.g[3 * i + 2] = g.z;
    a.h[i] = 1.0 / (2.0 * mz);
    a.lloyd[3 * i] = l.x;
    a.lloyd[3 * i + 1] = l.y;
    a.lloyd[3 * i + 2] = l.z;
    F += e;
    lmax = fmax(lmax, fmax(fabs(l.x), fmax(fabs(l.y), fabs(l.z))));
    gg += dot(g, g);
    mzmin = fmin(mzmin, mz);
    if (!(e == e) || !(mz == mz)) mzmin = -1.0;  // NaN guard
  }
  double b0 = block_sum(F, sh), b1 = block_max(lmax, sh), b2 = block_sum(gg, sh),
         b3 = block_min(mzmin, sh);
  if (threadIdx.x == 0) {
    a.partials[4 * p.bx()] = b0;
    a.partials[4 * p.bx() + 1] = b1;
    a.partials[4 * p.bx() + 2] = b2;
    a.partials[4 * p.bx() + 3] = b3;
  }
}

template <class P>
__global__ __launch_bounds__(kRedBlock) void k_finalize(P p) {
  if (p.idle()) return;
  const FinalizeArgs& a = p.args();
  __shared__ double sh[kRedBlock];
  for (int v = 0; v < a.nvals; v++) {
    const int op = a.op[v];
    double acc = op == 0 ? 0.0 : (op == 1 ? -1e300 : 1e300);
    for (int b = threadIdx.x; b < a.nblocks; b += blockDim.x) {
      double x = a.partials[b * a.nvals + v];
      acc = op == 0 ? acc + x : (op == 1 ? fmax(acc, x) : fmin(acc, x));
    }
    acc = op == 0 ? block_sum(acc, sh) : (op == 1 ? block_max(acc, sh) : block_min(acc, sh));
    if (threadIdx.x == 0) a.out[v] = acc;
  }
  if (threadIdx.x == 0 && a.r_slot) *a.r_slot = 1.0 / a.out[0];
}

// ------------------------------------------- history passes (kHmax pairs)
constexpr int kHGrid = 1024;
constexpr int kHVals = 4 + 2 * kHmax;  // most values one block reduces

__device__ inline double wave_sum64(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ void hist_fin(const HistFinArgs& a);

// Block partials of K (<= KMAX) per-thread values: a butterfly within each
// wave, then the four waves in order; value v written to out[v * stride]
// (value-major over the grid: out = partials + block, stride = blocks, so
// that the one-block fin reads each value's partials contiguously).
template <int KMAX>
__device__ inline void block_partials(const double* acc, int K, double* out, int stride) {
  __shared__ double sh[4][KMAX];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < KMAX; v++) {
    if (v < K) {
      const double x = wave_sum64(acc[v]);
      if (lane == 0) sh[wave][v] = x;
    }
  }
  __syncthreads();
  for (int v = threadIdx.x; v < K; v += blockDim.x)
    out[(size_t)v * stride] = ((sh[0][v] + sh[1][v]) + sh[2][v]) + sh[3][v];
}

// The streaming passes read VW consecutive elements per thread and step (16-
// byte loads when 3n is even, so that every vector is 16-byte aligned).
template <int VW>
__device__ inline void ld(const double* __restrict__ p, int u, double (&o)[VW]) {
  if constexpr (VW == 2) {
    const double2 t = reinterpret_cast<const double2*>(p)[u];
    o[0] = t.x;
    o[1] = t.y;
  } else {
    o[0] = p[u];
  }
}
// The history vectors s_j, y_j (2M streams of 3n doubles, far beyond the
// caches) are read once per pass: nontemporal loads keep them from pushing
// g, q and h, which the next passes read again, out of the L2 and MALL
// (the LBFGS passes 0.137 -> 0.128 ms per iteration at n = 1,048,576, M = 10).
template <int VW>
__device__ inline void ld_nt(const double* __restrict__ p, int u, double (&o)[VW]) {
  if constexpr (VW == 2) {
    o[0] = __builtin_nontemporal_load(p + 2 * u);
    o[1] = __builtin_nontemporal_load(p + 2 * u + 1);
  } else {
    o[0] = __builtin_nontemporal_load(p + u);
  }
}
template <int VW>
__device__ inline void st(double* __restrict__ p, int u, const double (&o)[VW]) {
  if constexpr (VW == 2) {
    reinterpret_cast<double2*>(p)[u] = make_double2(o[0], o[1]);
  } else {
    p[u] = o[0];
  }
}

template <int VW, class P>
__global__ __launch_bounds__(kRedBlock) void k_push_ext(P p) {
  if (p.idle()) return;
  const PushExtArgs& a = p.args();
  double acc[kHVals];
#pragma unroll
  for (int v = 0; v < kHVals; v++) acc[v] = 0.0;
  const int c = a.c;
  const int nu = (int)(a.n3 / VW);
  for (int u = p.bx() * blockDim.x + threadIdx.x; u < nu; u += p.gx() * blockDim.x) {
    double gt[VW], zt[VW], z[VW], g[VW], s[VW], y[VW];
    ld<VW>(a.gt, u, gt);
    ld<VW>(a.Zt, u, zt);
    ld<VW>(a.Z, u, z);
    ld<VW>(a.g, u, g);
#pragma unroll
    for (int e = 0; e < VW; e++) {
      s[e] = zt[e] - z[e];
      y[e] = gt[e] - g[e];
    }
    st<VW>(a.s, u, s);
    st<VW>(a.y, u, y);
#pragma unroll
    for (int e = 0; e < VW; e++) {
      acc[0] = fma(y[e], s[e], acc[0]);
      acc[1] = fma(y[e], y[e], acc[1]);
      acc[2] = fma(s[e], s[e], acc[2]);
      acc[3] = fma(s[e], gt[e], acc[3]);
    }
#pragma unroll
    for (int j = 0; j < kHmax; j++) {
      if (j < c) {
        double sj[VW];
        ld_nt<VW>(a.S[j], u, sj);
#pragma unroll
        for (int e = 0; e < VW; e++) {
          acc[4 + 2 * j] = fma(sj[e], gt[e], acc[4 + 2 * j]);
          acc[5 + 2 * j] = fma(sj[e], y[e], acc[5 + 2 * j]);
        }
      }
    }
  }
  block_partials<kHVals>(acc, 4 + 2 * c, a.partials + p.bx(), p.gx());
}

// the same sums as k_push_ext forms for s_j . g and s_j . y (same element
// order per thread), so a restored state recomputes them bit for bit
template <int VW>
__global__ __launch_bounds__(kRedBlock) void k_multi_dot(MultiDotArgs a) {
  double acc[kHmax];
#pragma unroll
  for (int v = 0; v < kHmax; v++) acc[v] = 0.0;
  const int c = a.c;
  const int nu = (int)(a.n3 / VW);
  for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < nu; u += gridDim.x * blockDim.x) {
    double v[VW];
    ld<VW>(a.v, u, v);
#pragma unroll
    for (int j = 0; j < kHmax; j++) {
      if (j < c) {
        double aj[VW];
        ld<VW>(a.A[j], u, aj);
#pragma unroll
        for (int e = 0; e < VW; e++) acc[j] = fma(aj[e], v[e], acc[j]);
      }
    }
  }
  block_partials<kHmax>(acc, c, a.partials + blockIdx.x, (int)gridDim.x);
}

// r = h (.) (-g - sum_k a_k y_k), newest pair first as in the backward loop;
// partials of y_j . r
template <int VW, class P>
__global__ __launch_bounds__(kRedBlock) void k_hist_q0(P p) {
  if (p.idle()) return;
  const HistPassArgs& a = p.args();
  const int c = a.c;
  double coef[kHmax], acc[kHmax];
#pragma unroll
  for (int j = 0; j < kHmax; j++) {
    coef[j] = j < c ? a.coef[j] : 0.0;
    acc[j] = 0.0;
  }
  const int nu = (int)(a.n3 / VW);
  for (int u = p.bx() * blockDim.x + threadIdx.x; u < nu; u += p.gx() * blockDim.x) {
    double yv[kHmax][VW];
    double q[VW];
    ld<VW>(a.g, u, q);
#pragma unroll
    for (int e = 0; e < VW; e++) q[e] = -q[e];
#pragma unroll
    for (int j = kHmax - 1; j >= 0; j--) {
      if (j < c) {
        ld_nt<VW>(a.Y[j], u, yv[j]);
#pragma unroll
        for (int e = 0; e < VW; e++) q[e] = fma(-coef[j], yv[j][e], q[e]);
      }
    }
    double r[VW];
#pragma unroll
    for (int e = 0; e < VW; e++) r[e] = a.h[(unsigned)(u * VW + e) / 3u] * q[e];
    st<VW>(a.q, u, r);
#pragma unroll
    for (int j = 0; j < kHmax; j++)
      if (j < c) {
#pragma unroll
        for (int e = 0; e < VW; e++) acc[j] = fma(yv[j][e], r[e], acc[j]);
      }
  }
  if (c > 0) block_partials<kHmax>(acc, c, a.partials + p.bx(), p.gx());
}

// q = r + sum_k c_k s_k, oldest pair first as in the forward loop; partials
// of g . q
template <int VW, class P>
__global__ __launch_bounds__(kRedBlock) void k_hist_dir(P p) {
  if (p.idle()) return;
  const HistPassArgs& a = p.args();
  const int c = a.c;
  double coef[kHmax];
#pragma unroll
  for (int j = 0; j < kHmax; j++) coef[j] = j < c ? a.coef[j] : 0.0;
  double acc[1] = {0.0};
  const int nu = (int)(a.n3 / VW);
  for (int u = p.bx() * blockDim.x + threadIdx.x; u < nu; u += p.gx() * blockDim.x) {
    double q[VW], g[VW];
    ld<VW>(a.qin, u, q);
    ld<VW>(a.g, u, g);
#pragma unroll
    for (int j = 0; j < kHmax; j++)
      if (j < c) {
        double sj[VW];
        ld_nt<VW>(a.S[j], u, sj);
#pragma unroll
        for (int e = 0; e < VW; e++) q[e] = fma(coef[j], sj[e], q[e]);
      }
    st<VW>(a.q, u, q);
#pragma unroll
    for (int e = 0; e < VW; e++) acc[0] = fma(g[e], q[e], acc[0]);
  }
  block_partials<1>(acc, 1, a.partials + p.bx(), p.gx());
}

// One block: sums the block partials of each value in block order (wave w
// takes values w, w+4, ...; lane l blocks l, l+64, ...), then the scalar
// step of the mode.  The recursions read their operands from LDS (staged by
// all threads), so the one thread that runs them waits on no global loads.
__device__ void hist_fin(const HistFinArgs& a) {
  __shared__ double red[kHVals];
  __shared__ double sg[kHmax], rr[kHmax], co[kHmax], gm[kHmax][kHmax];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // block partials of each value: lane l takes blocks l, l + 64, ... (at
  // most kHGrid / 64 of them, loaded together), then a butterfly
  static_assert(kHGrid % 64 == 0, "partials per lane");
  constexpr int kPer = kHGrid / 64;
  for (int v = wave; v < a.nvals; v += 4) {
    double xs[kPer];
#pragma unroll
    for (int k = 0; k < kPer; k++) {
      const int b = lane + 64 * k;
      xs[k] = b < a.nblocks ? a.partials[(size_t)v * a.nblocks + b] : 0.0;
    }
#pragma unroll
    for (int w = kPer / 2; w > 0; w >>= 1)
#pragma unroll
      for (int k = 0; k < w; k++) xs[k] += xs[k + w];
    const double x = wave_sum64(xs[0]);
    if (lane == 0) red[v] = x;
  }
  double* D = a.dscal;
  const int c = a.c;
  if (a.mode == kFinBackward || a.mode == kFinForward) {
    for (int t = threadIdx.x; t < c * c; t += blockDim.x) {
      const int j = t / c, k = t - j * c;
      gm[j][k] = j < k ? a.gram[a.slot[j] * a.stride + a.slot[k]] : 0.0;  // s_j . y_k, j older
    }
    if (threadIdx.x < c) {
      const int sj = a.slot[threadIdx.x];
      sg[threadIdx.x] = D[kSG + sj];
      rr[threadIdx.x] = D[kR + sj];
      co[threadIdx.x] = D[kA + threadIdx.x];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (a.mode == kFinPush) {
      D[kPush] = red[0];
      D[kPush + 1] = red[1];
      D[kPush + 2] = red[2];
      D[kR + a.p] = 1.0 / red[0];
      D[kYY + a.p] = red[1];
      D[kSG + a.p] = red[3];
      for (int j = 0; j < c; j++) {
        D[kSG + a.slot[j]] = red[4 + 2 * j];
        a.gram[a.slot[j] * a.stride + a.p] = red[5 + 2 * j];
      }
    } else if (a.mode == kFinDots) {
      for (int j = 0; j < c; j++) *a.dst[j] = red[j];
    } else if (a.mode == kFinBackward) {
      // a_j = r_j (-s_j.g - sum_{k>j} a_k s_j.y_k), newest first
      for (int j = c - 1; j >= 0; j--) {
        double t = -sg[j];
        for (int k = c - 1; k > j; k--) t = fma(-co[k], gm[j][k], t);
        co[j] = rr[j] * t;
      }
    } else if (a.mode == kFinForward) {
      // c_j = a_j - r_j (y_j.r + sum_{k<j} c_k s_k.y_j), oldest first; co
      // holds a_j and receives c_j
      for (int j = 0; j < c; j++) {
        double t = red[j];
        for (int k = 0; k < j; k++) t = fma(co[k], gm[k][j], t);
        co[j] = co[j] - rr[j] * t;
      }
    } else {
      D[kGQ] = red[0];
    }
  }
  __syncthreads();
  if (threadIdx.x < c) {
    if (a.mode == kFinBackward) D[kA + threadIdx.x] = co[threadIdx.x];
    if (a.mode == kFinForward) D[kCoef + threadIdx.x] = co[threadIdx.x];
  }
}

template <class P>
__global__ __launch_bounds__(kRedBlock) void k_hist_fin(P p) {
  if (!p.idle()) hist_fin(p.args());
}

// several fin steps in one launch, in order (e.g. a push's scalars, then the
// next direction's backward recursion, which reads them)
template <class P>
__global__ __launch_bounds__(kRedBlock) void k_fin_chain(P p) {
  if (p.idle()) return;
  const FinChain& f = p.args();
  for (int k = 0; k < f.n; k++) {
    hist_fin(f.step[k]);
    __syncthreads();
  }
}

int hist_grid(int64_t n3) {
  int64_t b = (n3 + kRedBlock - 1) / kRedBlock;
  if (b > kHGrid) b = kHGrid;
  if (b < 1) b = 1;
  return (int)b;
}
int hist_grid_max() { return kHGrid * kHVals; }

hipError_t launch_push_ext(const PushExtArgs& a, hipStream_t s) {
  const int nb = hist_grid(a.n3);
  if (a.n3 % 2 == 0)
    k_push_ext<2><<<nb, kRedBlock, 0, s>>>(One<PushExtArgs>{a});
  else
    k_push_ext<1><<<nb, kRedBlock, 0, s>>>(One<PushExtArgs>{a});
  return hipGetLastError();
}
hipError_t launch_multi_dot(const MultiDotArgs& a, hipStream_t s) {
  const int nb = hist_grid(a.n3);
  if (a.n3 % 2 == 0)
    k_multi_dot<2><<<nb, kRedBlock, 0, s>>>(a);
  else
    k_multi_dot<1><<<nb, kRedBlock, 0, s>>>(a);
  return hipGetLastError();
}
hipError_t launch_hist_q0(const HistPassArgs& a, hipStream_t s) {
  const int nb = hist_grid(a.n3);
  if (a.n3 % 2 == 0)
    k_hist_q0<2><<<nb, kRedBlock, 0, s>>>(One<HistPassArgs>{a});
  else
    k_hist_q0<1><<<nb, kRedBlock, 0, s>>>(One<HistPassArgs>{a});
  return hipGetLastError();
}
hipError_t launch_hist_dir(const HistPassArgs& a, hipStream_t s) {
  const int nb = hist_grid(a.n3);
  if (a.n3 % 2 == 0)
    k_hist_dir<2><<<nb, kRedBlock, 0, s>>>(One<HistPassArgs>{a});
  else
    k_hist_dir<1><<<nb, kRedBlock, 0, s>>>(One<HistPassArgs>{a});
  return hipGetLastError();
}
hipError_t launch_hist_fin(const HistFinArgs& a, hipStream_t s) {
  k_hist_fin<<<1, kRedBlock, 0, s>>>(One<HistFinArgs>{a});
  return hipGetLastError();
}
hipError_t launch_fin_chain(const FinChain& f, hipStream_t s) {
  k_fin_chain<<<1, kRedBlock, 0, s>>>(One<FinChain>{f});
  return hipGetLastError();
}

int reduce_grid(int64_t count) {
  int64_t b = (count + kRedBlock - 1) / kRedBlock;
  if (b > kRedGrid) b = kRedGrid;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_lbfgs_pass(const PassArgs& a, hipStream_t s) {
  k_lbfgs_pass<<<reduce_grid(a.n3), kRedBlock, 0, s>>>(a);
  return hipGetLastError();
}
hipError_t launch_push(const PushArgs& a, hipStream_t s) {
  k_push<<<reduce_grid(a.n3), kRedBlock, 0, s>>>(a);
  return hipGetLastError();
}
hipError_t launch_eval_reduce(const EvalRedArgs& a, hipStream_t s) {
  k_eval_reduce<<<reduce_grid(a.n), kRedBlock, 0, s>>>(One<EvalRedArgs>{a});
  return hipGetLastError();
}
hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t s) {
  k_finalize<<<1, kRedBlock, 0, s>>>(One<FinalizeArgs>{a});
  return hipGetLastError();
}
int reduce_grid_max() { return kRedGrid; }

// ---- segmented launches (one per kernel for a batch of problems) ----
hipError_t launch_push_ext_many(const Seg<PushExtArgs>& g, int vw, hipStream_t s) {
  if (vw == 2)
    k_push_ext<2><<<dim3(g.maxnb, g.nseg), kRedBlock, 0, s>>>(Many<PushExtArgs>{g.tab, g.nb});
  else
    k_push_ext<1><<<dim3(g.maxnb, g.nseg), kRedBlock, 0, s>>>(Many<PushExtArgs>{g.tab, g.nb});
  return hipGetLastError();
}
hipError_t launch_hist_q0_many(const Seg<HistPassArgs>& g, int vw, hipStream_t s) {
  if (vw == 2)
    k_hist_q0<2><<<dim3(g.maxnb, g.nseg), kRedBlock, 0, s>>>(Many<HistPassArgs>{g.tab, g.nb});
  else
    k_hist_q0<1><<<dim3(g.maxnb, g.nseg), kRedBlock, 0, s>>>(Many<HistPassArgs>{g.tab, g.nb});
  return hipGetLastError();
}
hipError_t launch_hist_dir_many(const Seg<HistPassArgs>& g, int vw, hipStream_t s) {
  if (vw == 2)
    k_hist_dir<2><<<dim3(g.maxnb, g.nseg), kRedBlock, 0, s>>>(Many<HistPassArgs>{g.tab, g.nb});
  else
    k_hist_dir<1><<<dim3(g.maxnb, g.nseg), kRedBlock, 0, s>>>(Many<HistPassArgs>{g.tab, g.nb});
  return hipGetLastError();
}
hipError_t launch_hist_fin_many(const Seg<HistFinArgs>& g, hipStream_t s) {
  k_hist_fin<<<dim3(g.maxnb, g.nseg), kRedBlock, 0, s>>>(Many<HistFinArgs>{g.tab, g.nb});
  return hipGetLastError();
}
hipError_t launch_fin_chain_many(const Seg<FinChain>& g, hipStream_t s) {
  k_fin_chain<<<dim3(g.maxnb, g.nseg), kRedBlock, 0, s>>>(Many<FinChain>{g.tab, g.nb});
  return hipGetLastError();
}
hipError_t launch_eval_reduce_many(const Seg<EvalRedArgs>& g, hipStream_t s) {
  k_eval_reduce<<<dim3(g.maxnb, g.nseg), kRedBlock, 0, s>>>(Many<EvalRedArgs>{g.tab, g.nb});
  return hipGetLastError();
}
hipError_t launch_finalize_many(const Seg<FinalizeArgs>& g, hipStream_t s) {
  k_finalize<<<dim3(g.maxnb, g.nseg), kRedBlock, 0, s>>>(Many<FinalizeArgs>{g.tab, g.nb});
  return hipGetLastError();
}

}  // namespace scvt
