// Geometry, predicates, density and quadrature shared by the HIP kernels.
//
// Everything here is __host__ __device__ so that the same code can be run on
// the host for the library's CPU self-checks; the kernels in cells.hip call it
// from wave-level drivers.
//
// Problem (Yang, Gunzburger & Ju, section 2.1): the spherical Voronoi cell of
// generator z is {x on S^2 : |x - z| < |x - p| for every other generator p}
// (eq. viInS, Euclidean metric).  On the unit sphere the condition for one p is
// the half-space x . (z - p) >= 0 bounded by a great circle (the bisector).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "exp_table.h"
#include "rules.h"

#define SCVT_HD __host__ __device__ inline

namespace scvt {

// ------------------------------------------------------------------ vectors
struct V3 {
  double x, y, z;
};
SCVT_HD V3 mk(double x, double y, double z) { return V3{x, y, z}; }
SCVT_HD V3 operator+(V3 a, V3 b) { return V3{a.x + b.x, a.y + b.y, a.z + b.z}; }
SCVT_HD V3 operator-(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
SCVT_HD V3 operator-(V3 a) { return V3{-a.x, -a.y, -a.z}; }
SCVT_HD V3 operator*(double s, V3 a) { return V3{s * a.x, s * a.y, s * a.z}; }
SCVT_HD double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
SCVT_HD V3 cross(V3 a, V3 b) {
  return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
// a b + c as one three-address FMA (on the device, v_fma_f64 with all
// operands in vector registers: the compiler otherwise ties the addend to
// the result and copies loop-invariant addends on every use)
SCVT_HD double fma3(double a, double b, double c) {
#if defined(__HIP_DEVICE_COMPILE__)
  double d;
  __asm__("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
#else
  return fma(a, b, c);
#endif
}

// keeps x in a vector register from here on: a loop that uses a kernel
// argument as an FMA addend otherwise copies it from its scalar register at
// every iteration
SCVT_HD void pin_v(double& x) {
#if defined(__HIP_DEVICE_COMPILE__)
  __asm__ volatile("" : "+v"(x));
#endif
}

// reciprocal square root: the device's correctly refined rsqrt, 1/sqrt on
// the host build used by the CPU checks
SCVT_HD double rsq(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return ::rsqrt(x);
#else
  return 1.0 / ::sqrt(x);
#endif
}

// 1/sqrt(x) for positive, finite, normal x: the hardware estimate r and one
// second-order correction, r (1 + e/2 + 3e^2/8) with e = 1 - x r^2 (the
// Taylor series of (1 - e)^(-1/2)); no special-value handling.  The host
// build divides.
SCVT_HD double rsq_pos(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double r = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * r, r, 1.0);
  return fma(r * e, fma(e, 0.375, 0.5), r);
#else
  return 1.0 / ::sqrt(x);
#endif
}

// 1/sqrt(x) for x = |p|^2 of a point p of a flat sub-triangle with vertices
// on the sphere (x <= 1): when e = 1 - x (exact) is at most 1e-4 -- leaves
// below ~0.03 rad across, all but very coarse meshes -- the binomial series
// 1 + e/2 + 3e^2/8 + 5e^3/16 (next term below 3e-17), otherwise rsq_pos.
SCVT_HD double rsq_series(double x) {
  const double e = 1.0 - x;
  return fma(e, fma(e, fma3(e, 0.3125, 0.375), 0.5), 1.0);
}
SCVT_HD double rsq_near1(double x) {
  if (fabs(1.0 - x) <= 1e-4) return rsq_series(x);
  return rsq_pos(x);
}
// NEAR1: the caller knows |1 - |p|^2| <= 1e-4 at every point of the leaf, so
// every point takes the series (the same bits as rsq_near1 would give).
template <bool NEAR1>
SCVT_HD double rsq_leaf(double x) {
  if constexpr (NEAR1) return rsq_series(x);
  else return rsq_near1(x);
}

// Whether every quadrature point of a cell of radius R (all its vertices
// within chord R of the generator) is near the sphere in the sense of
// rsq_near1: a point p = sum l_k V_k of a flat triangle with unit corners
// has 1 - |p|^2 = sum_{j<k} l_j l_k |V_j - V_k|^2 <= max |V_j - V_k|^2 / 3,
// and the corners of every leaf lie within 2R of each other, so
// 1 - |p|^2 <= 4 R^2 / 3 (and >= minus a few roundings of the corners' norms).
SCVT_HD bool cell_near1(double R) { return R <= 8e-3; }  // 4 R^2 / 3 <= 8.6e-5

// a / b and sqrt(x) where the geometry needs neither IEEE rounding nor
// special values: the window and grid arithmetic (whose certified radius is
// shrunk by far more than these errors), the Voronoi vertices (every cell
// computes a shared vertex with the same formula, hence the same bits) and
// norms inside error bounds.  The hardware estimates refined to about one
// ulp: the reciprocal by two Newton steps (b normal, nonzero), the square
// root as x rsq_pos(x) (x >= 0; 0 gives 0).  The host build divides and
// calls sqrt.
SCVT_HD double rcp_fast(double b) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(b);
  r = fma(r, fma(-b, r, 1.0), r);
  return fma(r, fma(-b, r, 1.0), r);
#else
  return 1.0 / b;
#endif
}
SCVT_HD double div_fast(double a, double b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return a * rcp_fast(b);
#else
  return a / b;
#endif
}
SCVT_HD double sqrt_fast(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return x * rsq_pos(fmax(x, 1e-300));
#else
  return ::sqrt(x);
#endif
}

// a / |a| with one rounding per operation (no fused multiply-add): the same
// bits as ((x*x + y*y) + z*z), sqrt, divide evaluated anywhere else
SCVT_HD V3 normalized(V3 a) {
#pragma clang fp contract(off)
  double r = sqrt(a.x * a.x + a.y * a.y + a.z * a.z);
  return V3{a.x / r, a.y / r, a.z / r};
}

// unit round-off of binary64
constexpr double kU = 1.1102230246251565e-16;

// ------------------------------------------------------------- predicates
// det(a, b, c) with a first-order forward error bound.  The inputs are
// themselves rounded differences of generator positions (one rounding each);
// the 2x2 products, minor subtractions, outer products and the final sum add
// at most six more roundings relative to the permanent (same expression with
// absolute values).  Nine roundings; the bound uses 16u.
struct Pred {
  double v, err;
};
SCVT_HD Pred det_pred(V3 a, V3 b, V3 c) {
  double m0 = b.y * c.z - b.z * c.y;
  double m1 = b.z * c.x - b.x * c.z;
  double m2 = b.x * c.y - b.y * c.x;
  double p0 = fabs(b.y * c.z) + fabs(b.z * c.y);
  double p1 = fabs(b.z * c.x) + fabs(b.x * c.z);
  double p2 = fabs(b.x * c.y) + fabs(b.y * c.x);
  Pred r;
  r.v = a.x * m0 + a.y * m1 + a.z * m2;
  r.err = 16.0 * kU * (fabs(a.x) * p0 + fabs(a.y) * p1 + fabs(a.z) * p2);
  return r;
}

// Cached cross product d_j x d_b with its minor permanents, so that
// det(d_j, d_b, d_l) = d_l . c costs three multiply-adds per candidate l.
struct CrossCache {
  V3 c, perm;
};
SCVT_HD CrossCache make_cross(V3 a, V3 b) {
  CrossCache k;
  k.c = cross(a, b);
  k.perm = V3{fabs(a.y * b.z) + fabs(a.z * b.y), fabs(a.z * b.x) + fabs(a.x * b.z),
              fabs(a.x * b.y) + fabs(a.y * b.x)};
  return k;
}
SCVT_HD Pred det_cached(const CrossCache& k, V3 l) {
  Pred r;
  r.v = dot(l, k.c);
  r.err = 16.0 * kU * (fabs(l.x) * k.perm.x + fabs(l.y) * k.perm.y + fabs(l.z) * k.perm.z);
  return r;
}

// --------------------------------------------------- circumcentre (vertex)
// Voronoi vertex shared by generators a, b, c: the point of the sphere
// equidistant from all three, on their side.  Computed from the triple in
// increasing index order so that every cell that meets at the vertex gets the
// same bits: normalize((p_b - p_a) x (p_c - p_a)), signed so that v . p_a > 0.
// The cross product is evaluated without fused multiply-adds (one rounding
// per operation, as the plain formula), and the normalisation is the IEEE
// square root of ((w_x^2 + w_y^2) + w_z^2) and three IEEE divisions: the
// vertex is the correctly rounded value of that expression, as anywhere else
// it is evaluated in this order.
SCVT_HD V3 circumcentre(int ia, V3 pa, int ib, V3 pb, int ic, V3 pc) {
#pragma clang fp contract(off)
  if (ia > ib) {
    int t = ia; ia = ib; ib = t;
    V3 s = pa; pa = pb; pb = s;
  }
  if (ib > ic) {
    int t = ib; ib = ic; ic = t;
    V3 s = pb; pb = pc; pc = s;
  }
  if (ia > ib) {
    int t = ia; ia = ib; ib = t;
    V3 s = pa; pa = pb; pb = s;
  }
  const double ux = pb.x - pa.x, uy = pb.y - pa.y, uz = pb.z - pa.z;
  const double vx = pc.x - pa.x, vy = pc.y - pa.y, vz = pc.z - pa.z;
  double wx = uy * vz - uz * vy;
  double wy = uz * vx - ux * vz;
  double wz = ux * vy - uy * vx;
  const double r = sqrt(wx * wx + wy * wy + wz * wz);
  wx = wx / r;
  wy = wy / r;
  wz = wz / r;
  if (wx * pa.x + wy * pa.y + wz * pa.z < 0.0) {
    wx = -wx;
    wy = -wy;
    wz = -wz;
  }
  return V3{wx, wy, wz};
}

// ------------------------------------------ edge of the cell on one bisector
// Candidate set S (positions p_l and differences d_l = p_l - z).  Every
// bisector is the plane through the origin with normal d_l, and the cell is
// the part of the sphere on z's side of all of them, y . d_l <= 0.  The plane
// of candidate j holds the great circle y(t) = m_j + t b_j with m_j = z - c_j
// d_j, c_j = z.d_j / |d_j|^2 (z projected onto the plane) and b_j = z x d_j
// (t increasing counter-clockwise seen from outside the sphere); candidate l
// bounds it by num_l + t sg_l <= 0 with
//   sg_l = b_j . d_l = det(z, d_j, d_l),  num_l = m_j . d_l = z.d_l - c_j d_j.d_l,
// an upper bound t <= -num_l/sg_l when sg_l > 0, a lower bound when sg_l < 0.
// Bound l is tighter than bound a of the same kind when
//   cmp = num_l sg_a - num_a sg_l
// is positive (upper) or negative (lower): the vertex (j, a) violates l, the
// sign of det(d_j, d_a, d_l) (scalars only, so the scan over l keeps two
// numbers per side instead of a cross product).  The edge runs from the
// tightest lower bound `lo` to the tightest upper bound `hi` and exists if
// num_hi sg_lo - num_lo sg_hi > 0.
//
// Certification: with E = max |d_l| over the candidates (nm) and u = 2^-53,
// the computed sg_l, num_l err by at most 96u |d_j||d_l| and 16u E (z.d_l and
// d_j.d_l from rounded differences, c_j's rounding), and are bounded by
// |d_j| E and E (E + |d_j|)/2; a comparison of two bounds then errs by at
// most B = 1.1 (2 (16u E Sb + Nb 96u |d_j| E) + 4u Nb Sb) with Sb, Nb those
// bounds.  A comparison within B, or a line (nearly) parallel to j in the
// chart (|sg_l| within its error), settles nothing by itself: the latter is
// decided at the foot of line j, the former makes the cell degenerate (it
// goes to the sequential clipper).  B / |cmp| is ~u/h for cells of size h.
enum EdgeStatus { kEdgeNone = 0, kEdgeYes = 1, kEdgeUnbounded = 2, kEdgeDegenerate = 3 };
struct EdgeRes {
  int status, lo, hi;
};

struct CandView {  // structure-of-arrays view (LDS on the device)
  const double *px, *py, *pz, *dx, *dy, *dz, *nrm, *zd;  // nrm[l] = |d_l|, zd[l] = z . d_l
  SCVT_HD V3 p(int l) const { return V3{px[l], py[l], pz[l]}; }
  SCVT_HD V3 d(int l) const { return V3{dx[l], dy[l], dz[l]}; }
};

// Error bound for det(a, b, c) of rounded difference vectors: 16u times the
// permanent, whose six terms are each at most |a||b||c|: 96u |a||b||c|.
constexpr double kDetBound = 96.0 * kU;

// nm: the largest |d_l| of the candidate set (at least |d_j|)
SCVT_HD EdgeRes edge_on_bisector(int j, int ns, V3 z, const CandView& S, double nm) {
  const V3 dj = S.d(j), pj = S.p(j);
  const double nj = S.nrm[j];
  const V3 wj = cross(z, dj);
  const double cj = div_fast(S.zd[j], dot(dj, dj));  // ~1 ulp: inside the bound below
  const double ebj = kDetBound * nj;  // |sg_l| error bound / |d_l|
  const double Sb = 1.01 * nj * nm, Nb = 0.5 * nm * (nm + nj) + 16.0 * kU * nm;
  const double B = 1.1 * (2.0 * (16.0 * kU * nm * Sb + Nb * kDetBound * nj * nm) + 4.0 * kU * Nb * Sb);
  // the tightest bounds so far; (-1, 0) stands for none (t = +-inf)
  int lo = -1, hi = -1;
  double nlo = -1.0, slo = 0.0, nhi = -1.0, shi = 0.0;
  bool degenerate = false, none = false;
  for (int l = 0; l < ns; l++) {  // straight-line but for the rare parallel case
    const V3 dl = S.d(l);
    const double sg = dot(dl, wj);
    const double num = fma(-cj, dot(dj, dl), S.zd[l]);
    const bool self = l == j;
    const bool par = !self && fabs(sg) <= ebj * S.nrm[l];
    if (par) {
      // lines (nearly) parallel in the chart: line l either leaves all of
      // line j feasible or none of it; decided at the foot of line j by the
      // sign of d_l . (p_l - p_j)
      const V3 dd = S.p(l) - pj;
      const double t = dot(dl, dd);
      const double te = 16.0 * kU * (fabs(dl.x * dd.x) + fabs(dl.y * dd.y) + fabs(dl.z * dd.z));
      none |= t < -te;
      degenerate |= fabs(t) <= te;
    }
    const bool up = sg > 0.0, use = !self && !par;
    // > 0: l is tighter than the side's current bound
    const double c = up ? fma(num, shi, -nhi * sg) : -fma(num, slo, -nlo * sg);
    degenerate |= use && (up ? hi : lo) >= 0 && fabs(c) <= B;
    const bool th = use && up && c > 0.0, tl = use && !up && c > 0.0;
    hi = th ? l : hi;
    nhi = th ? num : nhi;
    shi = th ? sg : shi;
    lo = tl ? l : lo;
    nlo = tl ? num : nlo;
    slo = tl ? sg : slo;
  }
  if (none) return EdgeRes{kEdgeNone, -1, -1};  // excluded by a parallel line
  if (degenerate) return EdgeRes{kEdgeDegenerate, lo, hi};
  if (lo < 0 || hi < 0) return EdgeRes{kEdgeUnbounded, lo, hi};
  const double x = fma(nhi, slo, -nlo * shi);
  if (fabs(x) <= B) return EdgeRes{kEdgeDegenerate, lo, hi};
  return EdgeRes{x > 0.0 ? kEdgeYes : kEdgeNone, lo, hi};
}

// ------------------------------------------------------------- densities
enum RhoKind { kRhoConst = 0, kRhoTanh = 1, kRhoX3 = 2, kRhoX16 = 3 };
struct RhoPoly;
struct DensityP {
  int32_t kind, geodesic, nbumps, pad;
  double xc[2][3];
  double beta[2], alpha[2], amp[2];
  double gamma, w_lon, w_lat;
  // filled by density_prepare: k2 = -2 / alpha_k, and the base-2 exponent's
  // K = 2N/(alpha_k ln2) and bK = -beta_k K (N = kExpN); for the per-cell
  // polynomial (RhoPoly): Ks = sqrt(2) K, cc = (1 + |x_c|^2)/2,
  // Kt = 2 sqrt(2)/alpha_k, the squared chord radius poly_r2 of a qualifying
  // cell and the least squared distance poly_near2 of its generator from x_c
  double k2[2], K[2], bK[2], Ks[2], cc[2], Kt[2], poly_r2[2], poly_near2[2];
  // the polynomials' tables (device memory, filled at set-up; RhoPoly) and
  // their entries (0: no table, no cell qualifies): in t (poly_*) and in
  // x = d^2/2 (polyx_*)
  const RhoPoly* poly_tab;
  int64_t poly_n;
  const RhoPoly* polyx_tab[2];  // one per bump (chord tanh bumps, one or two)
  int64_t polyx_n;
};

// Per-cell polynomial of a single chord tanh bump, the quadrature's fast
// path.  With t = 2 (d - beta)/alpha and sigma(t) = 1/(1 + e^t) (so that
// rho = gamma + amp sigma), around t0 = t(d(z)) with q = 1 - sigma(t0):
//   sigma(t0 + D) = sigma(t0) / (1 + q (e^D - 1)) = sigma(t0) sum_n b_n D^n,
//   b_0 = 1,  b_n = -q sum_{j=1..n} b_{n-j} / j!
// (the reciprocal's power series).  For s = x + iy with |y| <= r < pi,
// |1 + e^{+-s}| >= sin r (>= 1 where |y| <= pi/2; else >= |sin y|), so
// |sigma(s)| <= min(1, e^{-x}) / sin r.  Cauchy's estimate on the disc of
// radius r about t0 bounds the degree-K truncation at |D| <= tau by
// min(1, e^{r - t0}) (tau/r)^(K+1) / (sin r (1 - tau/r)), and as
// sigma(t) >= min(1, e^{-t})/2 its error relative to sigma (and so to
// rho >= amp sigma) is at most 2 e^{r + tau} (tau/r)^(K+1) / (sin r (1 - tau/r)):
// with K = 9, r = 2.78 and tau <= kPolyTau = 0.05 below 3.5e-16.
// The expansion points are a fixed grid, t* = t(0) + j/256 (the density's
// table of coefficients, one entry per j); the cell takes the entry nearest
// t(d(z)), so |t - t*| <= (2/alpha) |d(p) - d(z)| + 1/512, and as
// |d(p) - d(z)| <= |p - z| (chord distances) a cell whose fan lies within
// chord R of z qualifies when (2/alpha) R + 1/512 <= kPolyTau.
// The chord comes from a dot product, d^2 = 2 (cc - ri p.c) with
// cc = (1 + |c|^2)/2 (|y| = 1 to a rounding): two instructions fewer than
// the difference vector, but its rounding (~2e-16 absolute in d^2/2) moves d
// by ~2e-16/d, so a qualifying cell also keeps every point at least
// kPolyNear from x_c (d(z) >= kPolyNear + R): there the density's relative
// error from it stays below (2/alpha) 1.1e-14.
constexpr int kPolyDeg = 9;
constexpr double kPolyTau = 0.05;
constexpr double kPolyNear = 0.02;
constexpr int kPolyPerT = 256;       // table entries per unit of t
constexpr int64_t kPolyMax = 65536;  // larger tables (alpha < 0.016) are not built
struct RhoPoly {
  double c[kPolyDeg + 1];  // rho = sum_n c_n D^n
  double off;  // in t: D = Kt h + off (= t - t*), h = |y - x_c| / sqrt(2);
               // in x: D = off - r p.x_c (= x - x*, x = |y - x_c|^2 / 2)
  double lim;  // in x: the largest |x - x*| the entry's bound covers
};
// The expansion in x (RhoPolyX): rho(x) = gamma + amp sigma(Kt sqrt(x) + t0)
// with x = d^2/2 is analytic in the disc |x - x*| <= r_x for r_x < x* (the
// square root's branch point at 0); there
// |sqrt(x) - sqrt(x*)| <= sqrt(x*) w / (1 + sqrt(1 - w)), w = r_x / x*, so
// t stays in the strip |Im t| <= r_t = Kt sqrt(x*) w / (1 + sqrt(1 - w)),
// where |sigma| <= min(1, e^{-Re t}) / sin r_t.  As for t, the degree-9
// truncation at |x - x*| <= delta errs relative to rho by at most
//   2 e^{r_t + dt} (delta/r_x)^10 / (sin r_t (1 - delta/r_x)),
// dt = Kt (sqrt(x*) - sqrt(x* - delta)) the largest move of t.  Each table
// entry stores the largest delta with this below 1e-15 (w chosen so that
// r_t <= 2.5, w <= 0.8).  A cell qualifies when
// |x(z) - x*| + R (d(z) + R/2) <= that delta (|x(p) - x(z)| =
// |d(p) - d(z)| (d(p) + d(z))/2 <= R (d(z) + R/2)).  Its points then need
// neither the square root nor the scaling of the t path.
constexpr double kPolyDx = 1e-4;     // the x grid: x* = j kPolyDx, x in [0, 2]
constexpr double kPolyBound = 1e-15;

SCVT_HD DensityP density_prepare(DensityP d) {
  for (int k = 0; k < 2; k++) {
    d.k2[k] = d.alpha[k] > 0.0 ? -2.0 / d.alpha[k] : 0.0;
    d.K[k] = -d.k2[k] * kExpInvLn;
    d.bK[k] = -d.beta[k] * d.K[k];
    d.Ks[k] = d.K[k] * 1.4142135623730951;
    d.cc[k] = 0.5 * (1.0 + d.xc[k][0] * d.xc[k][0] + d.xc[k][1] * d.xc[k][1] +
                     d.xc[k][2] * d.xc[k][2]);
    d.Kt[k] = -d.k2[k] * 1.4142135623730951;
    const double rl = 0.5 * (kPolyTau - 0.5 / kPolyPerT) * d.alpha[k];
    d.poly_r2[k] = d.alpha[k] > 0.0 ? rl * rl : 0.0;
    d.poly_near2[k] = (kPolyNear + rl) * (kPolyNear + rl);
  }
  // t spans [t(0), t(2)] = [-2 beta/alpha, -2 beta/alpha + 4/alpha]; the
  // tables serve chord tanh bumps with alpha in the t table's range: the
  // expansion in t a single bump, the one in x each of one or two bumps
  const bool chord = d.kind == kRhoTanh && !d.geodesic && (d.nbumps == 1 || d.nbumps == 2);
  bool in_range = chord;
  for (int k = 0; k < d.nbumps && k < 2; k++)
    in_range = in_range && d.alpha[k] > 0.0 && 4.0 / d.alpha[k] * kPolyPerT < (double)(kPolyMax - 2);
  d.poly_n = in_range && d.nbumps == 1 ? (int64_t)(4.0 / d.alpha[0] * kPolyPerT) + 2 : 0;
  d.poly_tab = nullptr;
  d.polyx_n = in_range ? (int64_t)(2.0 / kPolyDx) + 2 : 0;
  d.polyx_tab[0] = d.polyx_tab[1] = nullptr;
  return d;
}


// 2^(u/N), N = kExpN = 128, for u <= N * 1009 (callers cap), table-driven
// (Tang's method in base 2): u = N m + j + f with k = rint(u), j = k mod N,
// m = floor(k / N) and f = u - k exact, |f| <= 1/2, so
// 2^(u/N) = 2^m 2^(j/N) exp(x) with x = f ln2/N, |x| <= ln2/256, and
// exp(x) - 1 is the degree-4 Taylor polynomial written in f (truncation
// error below 1.3e-15).  Below u = -1074 N the result underflows to 0 (the
// integer k saturates beyond 2^31, where f = 0 and 2^m is still 0).
// tab: the 2^(j/N) table or a copy of it (in LDS on the device)
SCVT_HD double exp2_n(double u, const double* tab = SCVT_EXP2_TAB) {
  const double k = rint(u);
  const double f = u - k;
#if defined(__HIP_DEVICE_COMPILE__)
  const int ki = (int)k;  // the conversion saturates
#else
  const int ki = (int)fmax(k, -2147483648.0);  // the same, without undefined behaviour
#endif
  const int j = ki & (kExpN - 1);
  const int m = ki >> 7;  // floor(ki / N): arithmetic shift
  static_assert(kExpN == 128, "table size");
  const double p = f * fma3(f, fma3(f, fma3(f, kExpC4, kExpC3), kExpC2), kExpC1);
  const double T = tab[j];
  return ldexp(fma(T, p, T), m);
}
constexpr double kUMax = 128.0 * 1009;

SCVT_HD double chord_to_angle(double ch) {
  double s = 0.5 * ch;
  return 2.0 * asin(s > 1.0 ? 1.0 : s);
}

// Reciprocal for 1 <= x < 2^1010: one Newton step from the hardware
// estimate (relative error at most 2^-23), so within 2^-46 = 1.4e-14; the
// host build divides
SCVT_HD double rcp_nr(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
#else
  return 1.0 / x;
#endif
}

// sqrt(x) for x >= 0 (x = 0 gives 0): x r (1 + e/2) with r the hardware
// estimate of 1/sqrt(max(x, 1e-300)) (relative error at most 2^-23) and
// e = 1 - x r^2; the dropped term 3e^2/8 bounds the error by 2.2e-14.  The
// host build calls sqrt.
SCVT_HD double sqrt_nr(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double r = __builtin_amdgcn_rsq(fmax(x, 1e-300));
  const double xr = x * r;
  return fma(xr * fma(-xr, r, 1.0), 0.5, xr);
#else
  return ::sqrt(x);
#endif
}
// the same for x >= 1e-300 (callers clamp)
SCVT_HD double sqrt_nr_pos(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double r = __builtin_amdgcn_rsq(x);
  const double xr = x * r;
  return fma(xr * fma(-xr, r, 1.0), 0.5, xr);
#else
  return ::sqrt(x);
#endif
}

// Densities of section 4: constant; tanh bumps
//   rho = gamma + sum_k amp_k (tanh((beta_k - d_k)/alpha_k) + 1)/2
// (the printed prefactor 1/(2(1-gamma)) is read as (1-gamma)/2 so that rho
// spans [gamma, 1]); X3 = (1-gamma) z^4 + gamma; X16 with the anisotropic
// distance built from the latitude/longitude-swapped points.
// (tanh(x) + 1)/2 is evaluated as the equal 1/(1 + exp(-2x)), which does not
// cancel where tanh is close to -1 (far from a bump, where rho ~ gamma).
// The bump's logistic 1/(1 + exp(t)), t = 2 (d - beta)/alpha, is evaluated
// in base 2 from u = t N/ln2 = K (d - beta) with K = 2N/(alpha ln2), one
// fused product with bK = -beta K, capped at N 1009 (where the logistic is
// below 2e-304; there is no lower cap: exp(t) underflows to 0 and the
// logistic is 1).
SCVT_HD double logistic(double bK, double K, double d, const double* tab = SCVT_EXP2_TAB) {
  const double u = fmin(fma(d, K, bK), kUMax);
  return rcp_nr(1.0 + exp2_n(u, tab));
}

// Density variants, each compiled separately so that a kernel carries only
// its own code and registers: kind, and for tanh bumps +8 geodesic distance,
// +16 two bumps.
constexpr int kVarGeo = 8, kVarTwo = 16;

template <int KIND>
SCVT_HD double rho_kind(const DensityP& D, V3 y, const double* tab = SCVT_EXP2_TAB) {
  constexpr int base = KIND & 7;
  if (base == kRhoConst) return 1.0;
  if (base == kRhoTanh) {
    constexpr int NB = (KIND & kVarTwo) ? 2 : 1;
    double rho = D.gamma;
#pragma unroll
    for (int k = 0; k < NB; k++) {
      V3 c = V3{D.xc[k][0], D.xc[k][1], D.xc[k][2]};
      V3 t = y - c;
      double d = sqrt_nr(dot(t, t));
      if (KIND & kVarGeo) d = chord_to_angle(d);
      rho = fma3(logistic(D.bK[k], D.K[k], d, tab), D.amp[k], rho);
    }
    return rho;
  }
  if (base == kRhoX3) {
    double z2 = y.z * y.z;
    return (1.0 - D.gamma) * z2 * z2 + D.gamma;
  }
  // X16
  double sz = y.z > 1.0 ? 1.0 : (y.z < -1.0 ? -1.0 : y.z);
  double la = asin(sz), lo = atan2(y.y, y.x);
  double czc = D.xc[0][2] > 1.0 ? 1.0 : (D.xc[0][2] < -1.0 ? -1.0 : D.xc[0][2]);
  double lac = asin(czc), loc = atan2(D.xc[0][1], D.xc[0][0]);
  V3 zic = V3{cos(la) * cos(loc), cos(la) * sin(loc), sin(la)};
  V3 zci = V3{cos(lac) * cos(lo), cos(lac) * sin(lo), sin(lac)};
  V3 t1 = y - zic, t2 = y - zci;
  double d1 = chord_to_angle(sqrt(dot(t1, t1)));
  double d2 = chord_to_angle(sqrt(dot(t2, t2)));
  double d = sqrt(d1 * d1 / (D.w_lon * D.w_lon) + d2 * d2 / (D.w_lat * D.w_lat));
  return fma3(logistic(D.bK[0], D.K[0], d, tab), D.amp[0], D.gamma);
}

// variant index of a density
SCVT_HD int rho_variant(const DensityP& D) {
  if (D.kind != kRhoTanh) return D.kind;
  return kRhoTanh + (D.geodesic ? kVarGeo : 0) + (D.nbumps == 2 ? kVarTwo : 0);
}

// call f.template operator()<V>() with the density's variant as a constant
#define SCVT_RHO_DISPATCH(var, CALL)                      \
  switch (var) {                                           \
    case kRhoConst: CALL(kRhoConst); break;                \
    case kRhoTanh: CALL(kRhoTanh); break;                  \
    case kRhoTanh + kVarGeo: CALL(kRhoTanh + kVarGeo); break; \
    case kRhoTanh + kVarTwo: CALL(kRhoTanh + kVarTwo); break; \
    case kRhoTanh + kVarGeo + kVarTwo: CALL(kRhoTanh + kVarGeo + kVarTwo); break; \
    case kRhoX3: CALL(kRhoX3); break;                      \
    default: CALL(kRhoX16); break;                         \
  }

SCVT_HD double rho_eval(const DensityP& D, V3 y) {
  double r = 0.0;
#define SCVT_RHO_CALL(V) r = rho_kind<V>(D, y)
  SCVT_RHO_DISPATCH(rho_variant(D), SCVT_RHO_CALL)
#undef SCVT_RHO_CALL
  return r;
}

// ------------------------------------------------------------- quadrature
// Triangle rules (rules.h, weights summing to 1): Radon's 7-point degree-5
// rule (the configured one) and the 4- and 9-point conical product rules of
// degrees 3 and 5 (the sizes the paper uses, section 4.1).  The FP32 copies
// serve the mixed-precision points: (l0, l1, l2, w, l0 l1, l0 l2, l1 l2, 0),
// the products formed in FP64 and rounded once.
#define SCVT_RULE_F(T, r)                                                                  \
  {(float)T[r][0], (float)T[r][1], (float)T[r][2], (float)T[r][3], (float)(T[r][0] * T[r][1]), \
   (float)(T[r][0] * T[r][2]), (float)(T[r][1] * T[r][2]), 0.0f}
__device__ constexpr float kRule7f[7][8] = {
    SCVT_RULE_F(kRule7, 0), SCVT_RULE_F(kRule7, 1), SCVT_RULE_F(kRule7, 2),
    SCVT_RULE_F(kRule7, 3), SCVT_RULE_F(kRule7, 4), SCVT_RULE_F(kRule7, 5),
    SCVT_RULE_F(kRule7, 6)};
__device__ constexpr float kRule4f[4][8] = {SCVT_RULE_F(kRule4, 0), SCVT_RULE_F(kRule4, 1),
                                            SCVT_RULE_F(kRule4, 2), SCVT_RULE_F(kRule4, 3)};
__device__ constexpr float kRule9f[9][8] = {
    SCVT_RULE_F(kRule9, 0), SCVT_RULE_F(kRule9, 1), SCVT_RULE_F(kRule9, 2),
    SCVT_RULE_F(kRule9, 3), SCVT_RULE_F(kRule9, 4), SCVT_RULE_F(kRule9, 5),
    SCVT_RULE_F(kRule9, 6), SCVT_RULE_F(kRule9, 7), SCVT_RULE_F(kRule9, 8)};
constexpr float kRule7fHost[7][8] = {
    SCVT_RULE_F(kRule7Host, 0), SCVT_RULE_F(kRule7Host, 1), SCVT_RULE_F(kRule7Host, 2),
    SCVT_RULE_F(kRule7Host, 3), SCVT_RULE_F(kRule7Host, 4), SCVT_RULE_F(kRule7Host, 5),
    SCVT_RULE_F(kRule7Host, 6)};
constexpr float kRule4fHost[4][8] = {SCVT_RULE_F(kRule4Host, 0), SCVT_RULE_F(kRule4Host, 1),
                                     SCVT_RULE_F(kRule4Host, 2), SCVT_RULE_F(kRule4Host, 3)};
constexpr float kRule9fHost[9][8] = {
    SCVT_RULE_F(kRule9Host, 0), SCVT_RULE_F(kRule9Host, 1), SCVT_RULE_F(kRule9Host, 2),
    SCVT_RULE_F(kRule9Host, 3), SCVT_RULE_F(kRule9Host, 4), SCVT_RULE_F(kRule9Host, 5),
    SCVT_RULE_F(kRule9Host, 6), SCVT_RULE_F(kRule9Host, 7), SCVT_RULE_F(kRule9Host, 8)};
#undef SCVT_RULE_F
#if defined(__HIP_DEVICE_COMPILE__)
#define SCVT_RULE_TABLE_F(nq) ((nq) == 4 ? kRule4f : ((nq) == 9 ? kRule9f : kRule7f))
#else
#define SCVT_RULE_TABLE_F(nq) ((nq) == 4 ? kRule4fHost : ((nq) == 9 ? kRule9fHost : kRule7fHost))
#endif
SCVT_HD bool valid_rule(int nq) { return nq == 4 || nq == 7 || nq == 9; }

struct Acc5 {
  double m, mx, my, mz, e;
};

// Radial projection of the flat triangle (A,B,C) onto the sphere has Jacobian
// (n.p)/|p|^3 with n.p constant = det(A,B,C)/(2 area), so
//   int_sph f dsigma = det(A,B,C)/2 * sum_q w_q f(p_q/|p_q|) / |p_q|^3.
// The first moment is accumulated relative to the generator, as int rho (y - z)
// (mu = m z + that, formed once per cell), which takes one product fewer per
// point than int rho y and keeps the sum small.
template <int KIND>
SCVT_HD void quad_tri_k(V3 A, V3 B, V3 C, V3 z, const DensityP& D, Acc5& acc,
                        const double* tab = SCVT_EXP2_TAB, int nq = 7) {
  const double(*R)[4] = SCVT_RULE_TABLE(nq);
  // det(A,B,C) = A . ((B-A) x (C-A)): the differences of nearby unit vectors
  // are exact to a rounding, so small sub-triangles keep full relative
  // accuracy (the plain triple product cancels ~log10(1/size) digits)
  const V3 BA = B - A, CA = C - A;
  const double hd = 0.5 * dot(A, cross(BA, CA));
#pragma unroll 1
  for (int q = 0; q < nq; q++) {
    // p = l0 A + l1 B + l2 C with l0 = 1 - l1 - l2
    const double l1 = R[q][1], l2 = R[q][2];
    const V3 p = V3{fma(l2, CA.x, fma(l1, BA.x, A.x)), fma(l2, CA.y, fma(l1, BA.y, A.y)),
                    fma(l2, CA.z, fma(l1, BA.z, A.z))};
    const double ri = rsq_near1(dot(p, p));
    const V3 y = ri * p;
    const double jac = ri * ri * ri;
    const double wt = hd * R[q][3] * jac * rho_kind<KIND>(D, y, tab);
    const V3 dy = V3{fma(ri, p.x, -z.x), fma(ri, p.y, -z.y), fma(ri, p.z, -z.z)};  // y - z
    acc.m += wt;
    acc.mx = fma(wt, dy.x, acc.mx);
    acc.my = fma(wt, dy.y, acc.my);
    acc.mz = fma(wt, dy.z, acc.mz);
    acc.e = fma(wt, dot(dy, dy), acc.e);
  }
}

// whether the cell of z whose vertices lie within squared chord r2 of z
// takes the polynomial
SCVT_HD bool poly_qualifies(const DensityP& D, V3 z, double r2) {
  const V3 t = z - V3{D.xc[0][0], D.xc[0][1], D.xc[0][2]};
  return D.poly_n > 0 && r2 <= D.poly_r2[0] && dot(t, t) >= D.poly_near2[0];
}

// Table entry j: the polynomial about t* = t(0) + j/256 (single chord tanh
// bump): sigma(t*) from the exponential, then the coefficients b_n of the
// series above scaled by amp sigma(t*), gamma added to the constant term;
// off = -j/64, as t = Kt h + t(0).
SCVT_HD RhoPoly poly_entry(const DensityP& D, int64_t j, const double* tab = SCVT_EXP2_TAB) {
  constexpr double kInvFact[11] = {1.0,          1.0,           0.5,           1.0 / 6.0,
                                  1.0 / 24.0,   1.0 / 120.0,   1.0 / 720.0,   1.0 / 5040.0,
                                  1.0 / 40320., 1.0 / 362880., 1.0 / 3628800.};
  static_assert(kPolyDeg <= 10, "1/j! table");
  const double off = -(double)j / kPolyPerT;  // exact
  const double ts = D.k2[0] * D.beta[0] - off;  // t* = -2 beta/alpha + j/256
  const double s0 = rcp_nr(1.0 + exp2_n(fmin(ts * kExpInvLn, kUMax), tab));
  const double q = 1.0 - s0;
  double b[kPolyDeg + 1];
  b[0] = 1.0;
  for (int n = 1; n <= kPolyDeg; n++) {
    double t = 0.0;
    for (int k = 1; k <= n; k++) t = fma(b[n - k], kInvFact[k], t);
    b[n] = -q * t;
  }
  RhoPoly P;
  const double as = D.amp[0] * s0;
  P.c[0] = as + D.gamma;
  for (int n = 1; n <= kPolyDeg; n++) P.c[n] = as * b[n];
  P.off = off;
  return P;
}

// the table entry of generator z: j nearest (t(d(z)) - t(0)) 256 = Kt h(z) 256
SCVT_HD int64_t poly_index(const DensityP& D, V3 z) {
  const double zc = dot(z, V3{D.xc[0][0], D.xc[0][1], D.xc[0][2]});
  const double h0 = sqrt_nr_pos(fmax(D.cc[0] - zc, 1e-300));
  // clamped in 32-bit integers (both tables hold fewer than 2^31 entries):
  // the bounds stay scalar operands
  const int j = (int)fmin(rint(h0 * (D.Kt[0] * kPolyPerT)), 2e9);
  return min(max(j, 0), (int)D.poly_n - 1);
}

// Table entry j of the expansion in x about x* = j kPolyDx of bump `bump` (gamma
// added to bump 0's constant term; the bound above is relative to the bump's
// own term, so to rho as well): the t-series
// (poly_entry's b_n about t* = t(x*)) composed with the binomial series of
// t(x* + D) - t* = Kt sqrt(x*) sum_{k>=1} binom(1/2, k) (D/x*)^k, both
// truncated at degree 9; lim from the bound above (bisection).
SCVT_HD RhoPoly polyx_entry(const DensityP& D, int64_t j, int bump = 0,
                            const double* tab = SCVT_EXP2_TAB) {
  constexpr int K = kPolyDeg;
  RhoPoly P{};
  const double xs = (double)j * kPolyDx;
  P.off = D.cc[bump] - xs;
  P.lim = 0.0;
  if (j < 1) return P;
  const double ss = sqrt(xs), ks = D.Kt[bump] * ss;
  const double ts = D.k2[bump] * D.beta[bump] + ks;  // t(x*) = Kt sqrt(x*) - 2 beta/alpha
  const double s0 = rcp_nr(1.0 + exp2_n(fmin(ts * kExpInvLn, kUMax), tab));
  const double q = 1.0 - s0;
  double b[K + 1], a[K + 1], pw[K + 1], nw[K + 1], r[K + 1];
  b[0] = 1.0;
  for (int n = 1; n <= K; n++) {
    double t = 0.0, f = 1.0;  // f = 1/k!
    for (int k = 1; k <= n; k++) {
      f /= (double)k;
      t = fma(b[n - k], f, t);
    }
    b[n] = -q * t;
  }
  a[0] = 0.0;
  double bin = 1.0, inv = 1.0;
  for (int k = 1; k <= K; k++) {
    bin *= (0.5 - (double)(k - 1)) / (double)k;
    inv /= xs;
    a[k] = ks * bin * inv;
  }
  for (int m = 0; m <= K; m++) {
    pw[m] = m == 0 ? 1.0 : 0.0;
    r[m] = m == 0 ? b[0] : 0.0;
  }
  for (int n = 1; n <= K; n++) {
    for (int m = 0; m <= K; m++) {
      double t = 0.0;
      for (int i = 1; i <= m; i++) t = fma(a[i], pw[m - i], t);
      nw[m] = t;
    }
    for (int m = 0; m <= K; m++) {
      pw[m] = nw[m];
      r[m] = fma(b[n], pw[m], r[m]);
    }
  }
  const double as = D.amp[bump] * s0;
  for (int m = 0; m <= K; m++) P.c[m] = as * r[m];
  if (bump == 0) P.c[0] += D.gamma;  // two bumps: the first entry carries gamma
  // the bound: w for |Im t| <= 2.5 (at most 0.8), then the largest delta
  const double y = 2.5 / ks;
  const double w = y >= 0.5528 ? 0.8 : 2.0 * y - y * y;
  const double rx = w * xs, rt = ks * w / (1.0 + sqrt(1.0 - w));
  double lo = 0.0, hi = 0.5 * rx;
  for (int it = 0; it < 60; it++) {
    const double dl = 0.5 * (lo + hi), u = dl / rx;
    const double dt = ks * (1.0 - sqrt(1.0 - dl / xs));
    double pu = 1.0;
    for (int k = 0; k <= K; k++) pu *= u;
    const double bound = 2.0 * exp(rt + dt) * pu / (sin(rt) * (1.0 - u));
    if (bound <= kPolyBound) lo = dl; else hi = dl;
  }
  P.lim = 0.98 * lo;
  return P;
}

// bump b's x table entry of generator z, and x(z) = d(z)^2 / 2
SCVT_HD int64_t polyx_index(const DensityP& D, V3 z, double* xz, int b = 0) {
  const double x = fmax(D.cc[b] - dot(z, V3{D.xc[b][0], D.xc[b][1], D.xc[b][2]}), 0.0);
  *xz = x;
  const int j = (int)fmin(rint(x * (1.0 / kPolyDx)), 2e9);
  return min(max(j, 1), (int)D.polyx_n - 1);
}

// whether the fan of z (vertices within chord r of z) lies inside the radius
// of its entry of bump b's x table: |x - x*| <= |x(z) - x*| + r (d(z) + r/2)
SCVT_HD bool polyx_qualifies(const DensityP& D, V3 z, double r, int b) {
  double xz = 0.0;
  const int64_t j = polyx_index(D, z, &xz, b);
  const double dz = sqrt_nr_pos(fmax(2.0 * xz, 1e-300));
  const double delta = fabs(xz - (double)j * kPolyDx) + r * (dz + 0.5 * r);
  return delta <= D.polyx_tab[b][j].lim;
}

// The x table's entry of bump b taken at the cell of z: as x(y) = cc - y.x_c,
// its offset off = cc - x* becomes off - z.x_c = x(z) - x*, and the argument
// at a point y is x(y) - x* = (x(z) - x*) - (y - z).x_c, the cell's part
// formed once.
SCVT_HD RhoPoly polyx_at(const RhoPoly& P, const DensityP& D, V3 z, int b) {
  RhoPoly Q = P;
  Q.off = P.off - dot(z, V3{D.xc[b][0], D.xc[b][1], D.xc[b][2]});
  return Q;
}

// quad_tri_k with rho from the cell's polynomial (single chord tanh bump)
// (X: the expansion in x, its entry taken at the cell by polyx_at; else the
// one in t)
template <bool X, bool NEAR1 = false>
SCVT_HD void quad_tri_poly(V3 A, V3 B, V3 C, V3 z, const DensityP& D, const RhoPoly& P,
                           Acc5& acc, int nq = 7) {
  const double(*R)[4] = SCVT_RULE_TABLE(nq);
  const V3 BA = B - A, CA = C - A;
  const double hd = 0.5 * dot(A, cross(BA, CA));
  const V3 xc = V3{D.xc[0][0], D.xc[0][1], D.xc[0][2]};
#pragma unroll 1
  for (int q = 0; q < nq; q++) {
    const double l1 = R[q][1], l2 = R[q][2];
    const V3 p = V3{fma(l2, CA.x, fma(l1, BA.x, A.x)), fma(l2, CA.y, fma(l1, BA.y, A.y)),
                    fma(l2, CA.z, fma(l1, BA.z, A.z))};
    const double ri = rsq_leaf<NEAR1>(dot(p, p));
    const V3 dy = V3{fma(ri, p.x, -z.x), fma(ri, p.y, -z.y), fma(ri, p.z, -z.z)};  // y - z
    double dl;
    if constexpr (X) {
      dl = fma(-dy.z, xc.z, fma(-dy.y, xc.y, fma(-dy.x, xc.x, P.off)));
    } else {
      const double h = sqrt_nr_pos(fmax(fma(-ri, dot(p, xc), D.cc[0]), 1e-300));
      dl = fma(h, D.Kt[0], P.off);
    }
    double rho = P.c[kPolyDeg];
#pragma unroll
    for (int n = kPolyDeg - 1; n >= 0; n--) rho = fma(rho, dl, P.c[n]);
    const double wt = hd * R[q][3] * (ri * ri * ri) * rho;
    acc.m += wt;
    acc.mx = fma(wt, dy.x, acc.mx);
    acc.my = fma(wt, dy.y, acc.my);
    acc.mz = fma(wt, dy.z, acc.mz);
    acc.e = fma(wt, dot(dy, dy), acc.e);
  }
}

// quad_tri_k for two chord tanh bumps, rho = P0(x_0 - x_0*) + P1(x_1 - x_1*)
// from both bumps' x tables (the fan inside both entries' radii; both
// entries taken at the cell by polyx_at)
template <bool NEAR1 = false>
SCVT_HD void quad_tri_poly2(V3 A, V3 B, V3 C, V3 z, const DensityP& D, const RhoPoly& P0,
                            const RhoPoly& P1, Acc5& acc, int nq = 7) {
  const double(*R)[4] = SCVT_RULE_TABLE(nq);
  const V3 BA = B - A, CA = C - A;
  const double hd = 0.5 * dot(A, cross(BA, CA));
  const V3 x0 = V3{D.xc[0][0], D.xc[0][1], D.xc[0][2]};
  const V3 x1 = V3{D.xc[1][0], D.xc[1][1], D.xc[1][2]};
#pragma unroll 1
  for (int q = 0; q < nq; q++) {
    const double l1 = R[q][1], l2 = R[q][2];
    const V3 p = V3{fma(l2, CA.x, fma(l1, BA.x, A.x)), fma(l2, CA.y, fma(l1, BA.y, A.y)),
                    fma(l2, CA.z, fma(l1, BA.z, A.z))};
    const double ri = rsq_leaf<NEAR1>(dot(p, p));
    const V3 dy = V3{fma(ri, p.x, -z.x), fma(ri, p.y, -z.y), fma(ri, p.z, -z.z)};  // y - z
    const double d0 = fma(-dy.z, x0.z, fma(-dy.y, x0.y, fma(-dy.x, x0.x, P0.off)));
    const double d1 = fma(-dy.z, x1.z, fma(-dy.y, x1.y, fma(-dy.x, x1.x, P1.off)));
    double r0 = P0.c[kPolyDeg], r1 = P1.c[kPolyDeg];
#pragma unroll
    for (int n = kPolyDeg - 1; n >= 0; n--) {
      r0 = fma(r0, d0, P0.c[n]);
      r1 = fma(r1, d1, P1.c[n]);
    }
    const double wt = hd * R[q][3] * (ri * ri * ri) * (r0 + r1);
    acc.m += wt;
    acc.mx = fma(wt, dy.x, acc.mx);
    acc.my = fma(wt, dy.y, acc.my);
    acc.mz = fma(wt, dy.z, acc.mz);
    acc.e = fma(wt, dot(dy, dy), acc.e);
  }
}

SCVT_HD void quad_tri(V3 A, V3 B, V3 C, V3 z, const DensityP& D, Acc5& acc, int nq = 7) {
#define SCVT_QUAD_CALL(V) quad_tri_k<V>(A, B, C, z, D, acc, SCVT_EXP2_TAB, nq)
  SCVT_RHO_DISPATCH(rho_variant(D), SCVT_QUAD_CALL)
#undef SCVT_QUAD_CALL
}

// ------------------------------------------------ mixed-precision quadrature
// The same rule with the point arithmetic in FP32, in a frame local to the
// generator z: every per-point quantity is a small offset from z (or from
// the cell's own value of the density's argument), so FP32 keeps its
// relative precision on the cell scale h instead of on the unit sphere.  The
// subdivision grid, each leaf's Jacobian determinant and the accumulation
// stay FP64; each leaf's 7-point sums are formed in FP32 and scaled into the
// FP64 accumulators (quad_leaf_mixed).  The first moment is accumulated as
// int rho (y - z), and mu = m z + int rho (y - z) is formed in FP64.
struct F3 {
  float x, y, z;
};
SCVT_HD F3 operator+(F3 a, F3 b) { return F3{a.x + b.x, a.y + b.y, a.z + b.z}; }
SCVT_HD F3 operator-(F3 a, F3 b) { return F3{a.x - b.x, a.y - b.y, a.z - b.z}; }
SCVT_HD F3 operator*(float s, F3 a) { return F3{s * a.x, s * a.y, s * a.z}; }
SCVT_HD float dotf(F3 a, F3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
SCVT_HD F3 crossf(F3 a, F3 b) {
  return F3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
SCVT_HD F3 to_f3(V3 v) { return F3{(float)v.x, (float)v.y, (float)v.z}; }

// hardware reciprocal square root and 2^x (about 1 ulp; no special-value or
// denormal handling: arguments are positive and normal, resp. any finite
// value with overflow to inf and underflow to 0 both harmless below)
SCVT_HD float rsqf(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rsqf(x);
#else
  return 1.0f / ::sqrtf(x);
#endif
}
SCVT_HD float exp2_hw(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_exp2f(x);
#else
  return ::exp2f(x);
#endif
}
SCVT_HD float rcpf(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}

// (1 + s)^(-1/2) - 1 for |s| <= 2^-5 by its binomial series to degree 6:
// the first dropped term is below 0.21 |s|^7, i.e. 0.42 |s|^6 <= 4e-10 of
// the result
SCVT_HD float rm1_series(float s) {
  constexpr float c1 = -0.5f, c2 = 0.375f, c3 = -0.3125f, c4 = 0.2734375f, c5 = -0.24609375f,
                  c6 = 0.2255859375f;
  return s * fmaf(s, fmaf(s, fmaf(s, fmaf(s, fmaf(s, c6, c5), c4), c3), c2), c1);
}

struct DensityF {  // FP32 density parameters
  float gamma, w_lon2i, w_lat2i, pad;
  float amp[2], beta[2], k2l[2];  // k2l = -2 log2(e) / alpha
};

SCVT_HD DensityF density_f32(const DensityP& D) {
  DensityF f{};
  f.gamma = (float)D.gamma;
  f.w_lon2i = (float)(1.0 / (D.w_lon * D.w_lon));
  f.w_lat2i = (float)(1.0 / (D.w_lat * D.w_lat));
  for (int k = 0; k < 2; k++) {
    f.amp[k] = (float)D.amp[k];
    f.beta[k] = (float)D.beta[k];
    f.k2l[k] = (float)(D.k2[k] * 1.4426950408889634);
  }
  return f;
}

SCVT_HD float bumpf(float amp, float beta, float k2l, float d) {
  return amp * rcpf(1.0f + exp2_hw((beta - d) * k2l));
}

SCVT_HD float chord_to_anglef(float ch) {
  float s = 0.5f * ch;
  return 2.0f * asinf(s > 1.0f ? 1.0f : s);
}

// zc[k] = z - x_c_k (FP64 difference, rounded); zf = z rounded
template <int KIND>
SCVT_HD float rho_kind_f(const DensityF& D, const F3* zc, F3 zf, F3 dyz, const DensityP& Dd) {
  constexpr int base = KIND & 7;
  if (base == kRhoConst) return 1.0f;
  if (base == kRhoTanh) {
    constexpr int NB = (KIND & kVarTwo) ? 2 : 1;
    float rho = D.gamma;
#pragma unroll
    for (int k = 0; k < NB; k++) {
      F3 t = zc[k] + dyz;
      float t2 = dotf(t, t);
      float d = t2 * rsqf(fmaxf(t2, 1e-30f));  // 0 at t2 = 0
      if (KIND & kVarGeo) d = chord_to_anglef(d);
      rho += bumpf(D.amp[k], D.beta[k], D.k2l[k], d);
    }
    return rho;
  }
  F3 y = zf + dyz;
  if (base == kRhoX3) {
    float z2 = y.z * y.z;
    return (1.0f - D.gamma) * z2 * z2 + D.gamma;
  }
  // X16
  float sz = y.z > 1.0f ? 1.0f : (y.z < -1.0f ? -1.0f : y.z);
  float la = asinf(sz), lo = atan2f(y.y, y.x);
  float czc = (float)Dd.xc[0][2];
  czc = czc > 1.0f ? 1.0f : (czc < -1.0f ? -1.0f : czc);
  float lac = asinf(czc), loc = atan2f((float)Dd.xc[0][1], (float)Dd.xc[0][0]);
  F3 zic = F3{cosf(la) * cosf(loc), cosf(la) * sinf(loc), sinf(la)};
  F3 zci = F3{cosf(lac) * cosf(lo), cosf(lac) * sinf(lo), sinf(lac)};
  F3 t1 = y - zic, t2 = y - zci;
  float d1 = chord_to_anglef(sqrtf(dotf(t1, t1)));
  float d2 = chord_to_anglef(sqrtf(dotf(t2, t2)));
  float d = sqrtf(d1 * d1 * D.w_lon2i + d2 * d2 * D.w_lat2i);
  return bumpf(D.amp[0], D.beta[0], D.k2l[0], d) + D.gamma;
}

// ---- the mixed path's leaf: FP64 leaf, FP32 points ------------------------
// Per cell: z = zf + zl as a pair of floats (so that 2 z.d keeps its
// precision where d is small), and for every chord tanh bump the logistic
// taken apart about the cell's own distance d_z = |z - x_c|:
//   sigma(u_z + du) = sigma_z / (1 + q (2^du - 1)),  q = 1 - sigma_z,
//   du = K2 (d - d_z) = K2 (d^2 - d_z^2) / (d + d_z),
//   d^2 - d_z^2 = 2 (z - x_c).(y - z) + |y - z|^2
// (K2 = 2 log2(e) / alpha, sigma in base 2).  Every per-point quantity is
// then a small offset: in FP32 the bump's argument u = K2 (d - beta) itself
// (|u| up to ~20 at the far side of the sphere) would carry ~1e-6 absolute
// rounding into every point's density, and the distance d (~1) ~6e-8, which
// the factor K2 (~19 at alpha = 0.15) turns into ~1e-6 relative noise in rho
// point to point; as offsets they carry ~6e-8 of |y - z| ~ R.
// With the geodesic distance theta = 2 asin(c/2) of the chord c, the offset
// is taken from sin(asin a - asin b) = (a^2 - b^2) / (a sqrt(1 - b^2) +
// b sqrt(1 - a^2)) with a = c/2, b = c_z/2 (a^2 - b^2 = (c^2 - c_z^2)/4, no
// cancellation): theta - theta_z = 2 asin(X).
// A cell within the FP64 expansion in x = d^2/2 (single chord bump, the
// table entry about x*) takes its first six coefficients in FP32 instead:
// rho = sum_k c_k D^k with D = x(y) - x* = (x(z) - x*) - (y - z).x_c, the
// per-cell part formed in FP64.  Inside the entry's radius (chosen for the
// degree-9 truncation below 1e-15, |D|/r <= ~0.025 of the series' radius r)
// the degree-5 truncation is below ~1e-8 relative, and no special function
// is left at the point.
// The per-cell constants share one array (a cell takes one of the two
// forms), so that the kernel holds one set of registers for them: bump k
// at k[8k..8k+7] = z - x_c (3), amp sigma(d_z), 1 - sigma(d_z), c_z, c_z^2,
// sqrt(1 - c_z^2/4) (geodesic); the expansion in x of bump k at
// k[10k..10k+9] = the six coefficients, x(z) - x*, x_c (3).  Densities other
// than tanh bumps use z - x_c at k[0..2] (and k[8..10]).
struct CellF {
  F3 zf, zl;
  float k[20];
  SCVT_HD F3 v3(int o) const { return F3{k[o], k[o + 1], k[o + 2]}; }
  SCVT_HD void set3(int o, F3 v) {
    k[o] = v.x;
    k[o + 1] = v.y;
    k[o + 2] = v.z;
  }
};

template <int KIND>
SCVT_HD CellF cell_f32(const DensityP& D, V3 z, const double* tab = SCVT_EXP2_TAB) {
  CellF c{};
  c.zf = to_f3(z);
  c.zl = to_f3(z - V3{(double)c.zf.x, (double)c.zf.y, (double)c.zf.z});
  constexpr int NB = (KIND & kVarTwo) ? 2 : 1;
#pragma unroll
  for (int b = 0; b < NB; b++) {
    const V3 t = z - V3{D.xc[b][0], D.xc[b][1], D.xc[b][2]};
    c.set3(8 * b, to_f3(t));
    if ((KIND & 7) == kRhoTanh) {
      const double dz2 = dot(t, t), dz = sqrt(dz2);
      const double sig = logistic(D.bK[b], D.K[b], (KIND & kVarGeo) ? chord_to_angle(dz) : dz, tab);
      c.k[8 * b + 3] = (float)(D.amp[b] * sig);
      c.k[8 * b + 4] = (float)(1.0 - sig);
      c.k[8 * b + 5] = (float)dz;
      c.k[8 * b + 6] = (float)dz2;
      c.k[8 * b + 7] = (float)sqrt(fmax(1.0 - 0.25 * dz2, 0.0));
    }
  }
  return c;
}

// A cell within the FP64 expansion in x = d^2/2 (single chord bump, the
// table entry about x*) takes its first six coefficients in FP32 instead:
// rho = sum_k c_k D^k with D = x(y) - x* = (x(z) - x*) - (y - z).x_c, the
// per-cell part formed in FP64.  Inside the entry's radius (chosen for the
// degree-9 truncation below 1e-15, |D|/r <= ~0.025 of the series' radius r)
// the degree-5 truncation is below ~1e-8 relative, and no special function
// is left at the point.
// the expansions in x of the first nb bumps (entries P[0..nb-1], taken at
// the cell by polyx_at)
SCVT_HD CellF cell_f32_poly(const DensityP& D, const RhoPoly* P, int nb, V3 z) {
  CellF c{};
  c.zf = to_f3(z);
  c.zl = to_f3(z - V3{(double)c.zf.x, (double)c.zf.y, (double)c.zf.z});
  for (int b = 0; b < nb; b++) {
    const V3 xc = V3{D.xc[b][0], D.xc[b][1], D.xc[b][2]};
    for (int k = 0; k < 6; k++) c.k[10 * b + k] = (float)P[b].c[k];
    c.k[10 * b + 6] = (float)P[b].off;  // x(z) - x*: the entry taken at the cell (polyx_at)
    c.set3(10 * b + 7, to_f3(xc));
  }
  return c;
}

// rho at y = z + dyz (|dyz|^2 = dyz2): tanh bumps in the split form above,
// every other density directly
template <int KIND>
SCVT_HD float rho_cell_f(const DensityF& D, const CellF& c, F3 dyz, float dyz2,
                         const DensityP& Dd) {
  if ((KIND & 7) == kRhoTanh) {
    constexpr int NB = (KIND & kVarTwo) ? 2 : 1;
    float rho = D.gamma;
#pragma unroll
    for (int b = 0; b < NB; b++) {
      const float* kb = c.k + 8 * b;
      const float dd2 = fmaf(2.0f, dotf(c.v3(8 * b), dyz), dyz2);  // c^2 - c_z^2
      const float t2 = fmaxf(kb[6] + dd2, 1e-30f);
      const float ch = t2 * rsqf(t2);  // c
      float dd;                        // d - d_z
      if (KIND & kVarGeo) {
        const float u = fmaxf(fmaf(-0.25f, t2, 1.0f), 1e-30f);
        const float den = fmaxf(0.5f * fmaf(ch, kb[7], kb[5] * (u * rsqf(u))), 1e-30f);
        const float X = 0.25f * dd2 * rcpf(den);  // sin((theta - theta_z)/2)
        const float X2 = X * X;
        // asin X by its series to X^5 (next term below 3e-10 of X for
        // |X| <= 2^-4), else the library's
        const float as = fabsf(X) <= 0.0625f ? X * fmaf(X2, fmaf(X2, 0.075f, 0.16666667f), 1.0f)
                                             : asinf(X);
        dd = 2.0f * as;
      } else {
        dd = dd2 * rcpf(fmaxf(ch + kb[5], 1e-30f));  // (c^2 - c_z^2) / (c + c_z)
      }
      const float du = -D.k2l[b] * dd;
      rho = fmaf(kb[3], rcpf(fmaf(kb[4], exp2_hw(du) - 1.0f, 1.0f)), rho);
    }
    return rho;
  }
  const F3 zc[2] = {c.v3(0), c.v3(8)};
  return rho_kind_f<KIND>(D, zc, c.zf, dyz, Dd);
}

// One leaf (A, B, C on the sphere, FP64) of a cell of z in the mixed
// precision: the leaf's Jacobian determinant in FP64 (its rounding in FP32
// would be a per-leaf relative error of ~1e-7, and the cell boundary's
// corners rounded to FP32 would move the cell's edges by ~6e-8 R), the
// points in FP32 offsets d = p - z from the rounded corner offsets.  For a
// point p = sum l_k V_k of a flat triangle with unit corners,
//   s = |p|^2 - 1 = -(l0 l1 |V0 - V1|^2 + l0 l2 |V0 - V2|^2 + l1 l2 |V1 - V2|^2)
// (no cancellation: from the leaf's edge lengths, |s| <= max edge^2 / 3),
// r - 1 = (1 + s)^(-1/2) - 1 from its binomial series (two terms when the
// leaf bounds |s| by 2^-16: the rest is below 1e-15 absolute; six up to
// 2^-5; else the hardware rsqrt), y - z = d + (r - 1)(z + d) and the
// Jacobian r^3 = 1 + 3(r - 1) + 3(r - 1)^2 (+ (r - 1)^3 beyond two terms)
// (no "1 +" rounded away at any point); the 7 weighted points summed in
// FP32 and scaled by the FP64 determinant into the FP64 accumulators.
// Accumulates m, int rho (y - z) (mx, my, mz) and e.
template <int KIND, int XP = 0>
SCVT_HD void quad_leaf_mixed(V3 A, V3 B, V3 C, V3 z, const CellF& cf, const DensityF& D,
                             const DensityP& Dd, Acc5& acc, int nq = 7) {
  const float(*R)[8] = SCVT_RULE_TABLE_F(nq);
  const V3 BA = B - A, CA = C - A;
  const double hd = 0.5 * dot(A, cross(BA, CA));
  const F3 dA = to_f3(A - z), dBA = to_f3(BA), dCA = to_f3(CA);
  const F3 dCB = dCA - dBA;
  const float eAB = dotf(dBA, dBA), eAC = dotf(dCA, dCA), eBC = dotf(dCB, dCB);
  const float smax = fmaxf(eAB, fmaxf(eAC, eBC)) * (1.0f / 3.0f);
  const int form = smax <= 0x1p-16f ? 0 : (smax <= 0x1p-5f ? 1 : 2);  // uniform over the leaf
  float sm = 0.f, sx = 0.f, sy = 0.f, sz = 0.f, se = 0.f;
  // point q of the rule with r - 1 and the Jacobian's r^3 - 1 given
  auto point = [&](const float* Rq, float rm1, float jm1) {
    const float l1 = Rq[1], l2 = Rq[2];
    const F3 d = F3{fmaf(l2, dCA.x, fmaf(l1, dBA.x, dA.x)), fmaf(l2, dCA.y, fmaf(l1, dBA.y, dA.y)),
                    fmaf(l2, dCA.z, fmaf(l1, dBA.z, dA.z))};
    const F3 p = cf.zf + d;
    const F3 dyz = F3{fmaf(rm1, p.x, d.x), fmaf(rm1, p.y, d.y), fmaf(rm1, p.z, d.z)};
    const float dyz2 = dotf(dyz, dyz);
    float rho;
    if (XP > 0) {  // the expansions in x of XP bumps
#pragma unroll
      for (int b = 0; b < XP; b++) {
        const float* kb = cf.k + 10 * b;
        const float Dx = fmaf(-dyz.z, kb[9], fmaf(-dyz.y, kb[8], fmaf(-dyz.x, kb[7], kb[6])));
        float rb = kb[5];
#pragma unroll
        for (int k = 4; k >= 0; k--) rb = fmaf(rb, Dx, kb[k]);
        rho = b == 0 ? rb : rho + rb;
      }
    } else {
      rho = rho_cell_f<KIND>(D, cf, dyz, dyz2, Dd);
    }
    const float b = Rq[3] * rho;
    const float wt = fmaf(b, jm1, b);
    sm += wt;
    sx = fmaf(wt, dyz.x, sx);
    sy = fmaf(wt, dyz.y, sy);
    sz = fmaf(wt, dyz.z, sz);
    se = fmaf(wt, dyz2, se);
  };
  // s at point q (no cancellation: the leaf's squared edge lengths)
  auto sq = [&](const float* Rq) { return -fmaf(Rq[6], eBC, fmaf(Rq[5], eAC, Rq[4] * eAB)); };
  // one loop per form: the common one (every leaf of a cell at n >~ 10^4)
  // runs without a branch per point
  auto tiny = [&](const float* Rq) {  // tiny leaves: two terms
    const float s = sq(Rq);
    const float rm1 = s * fmaf(s, 0.375f, -0.5f);
    point(Rq, rm1, rm1 * fmaf(rm1, 3.0f, 3.0f));
  };
  // the polynomial points and the single bump's direct ones with the rule's
  // constants as immediates (unrolled, the other densities run out of
  // registers)
  if ((XP > 0 || KIND == kRhoTanh) && form == 0 && nq == 7) {
    const float(*R7)[8] = SCVT_RULE_TABLE_F(7);
#pragma unroll
    for (int q = 0; q < 7; q++) tiny(R7[q]);
  } else if (form == 0) {
#pragma unroll 1
    for (int q = 0; q < nq; q++) tiny(R[q]);
  } else {
#pragma unroll 1
    for (int q = 0; q < nq; q++) {
      const float s = sq(R[q]);
      float rm1;
      if (form == 1) {
        rm1 = rm1_series(s);
      } else {
        const float r = rsqf(1.0f + s);
        rm1 = -s * r * r * rcpf(1.0f + r);
      }
      point(R[q], rm1, rm1 * fmaf(rm1, rm1 + 3.0f, 3.0f));
    }
  }
  acc.m = fma(hd, (double)sm, acc.m);
  acc.mx = fma(hd, (double)sx, acc.mx);
  acc.my = fma(hd, (double)sy, acc.my);
  acc.mz = fma(hd, (double)sz, acc.mz);
  acc.e = fma(hd, (double)se, acc.e);
}

// a / |a| through the reciprocal square root (quadrature only; the shared
// vertices use the correctly rounded `normalized`)
SCVT_HD V3 normalized_fast(V3 a) { return rsq_pos(dot(a, a)) * a; }

// Leaf `s` (base-4 digits, most significant first) of `levels` geodesic
// midpoint subdivisions of (A,B,C): children (A,ab,ca), (ab,B,bc), (ca,bc,C),
// (ab,bc,ca), midpoints normalize(a+b).
SCVT_HD void subtriangle(V3& A, V3& B, V3& C, int s, int levels) {
  for (int lv = levels - 1; lv >= 0; lv--) {
    int k = (s >> (2 * lv)) & 3;
    V3 ab = normalized_fast(A + B), bc = normalized_fast(B + C), ca = normalized_fast(C + A);
    if (k == 0) {
      B = ab; C = ca;
    } else if (k == 1) {
      A = ab; C = bc;
    } else if (k == 2) {
      A = ca; B = bc;
    } else {
      A = ab; B = bc; C = ca;
    }
  }
}

// Two levels of that subdivision share their points: the 16 leaves of a
// triangle use the 15 points of a triangular grid with barycentric numerators
// (i, j, k), i + j + k = 4, for (A, B, C), numbered lexicographically in
// (i, j) (A = 14, B = 4, C = 0).  The 3 level-1 midpoints and then the 9
// level-2 midpoints are normalize(P + Q) of two grid points, the same sums
// subtriangle() forms, so the leaves are the same bits.
// kGrid2Task[t] = {point, P, Q}: t < 3 level 1, then level 2.
__host__ __device__ constexpr int8_t kGrid2Task[12][3] = {
    {11, 14, 4}, {2, 4, 0},  {9, 0, 14},                                    // level 1
    {13, 14, 11}, {10, 11, 9}, {12, 9, 14}, {8, 11, 4}, {3, 4, 2}, {7, 2, 11},  // level 2
    {6, 9, 2},   {1, 2, 0},  {5, 0, 9}};
// kGrid2Leaf[s] = grid points of leaf s in subtriangle()'s vertex order
__host__ __device__ constexpr int8_t kGrid2Leaf[16][3] = {
    {14, 13, 12}, {13, 11, 10}, {12, 10, 9}, {13, 10, 12}, {11, 8, 7}, {8, 4, 3},
    {7, 3, 2},    {8, 3, 7},    {9, 6, 5},   {6, 2, 1},    {5, 1, 0},  {6, 1, 5},
    {11, 7, 10},  {7, 2, 6},    {10, 6, 9},  {7, 6, 10}};
// the same tables packed four bits per entry (lane-indexed without memory)
constexpr uint64_t grid2_pack(const int8_t (*t)[3], int n, int col) {
  uint64_t v = 0;
  for (int k = 0; k < n; k++) v |= (uint64_t)t[k][col] << (4 * k);
  return v;
}
constexpr uint64_t kG2TaskPt = grid2_pack(kGrid2Task, 12, 0);
constexpr uint64_t kG2TaskP = grid2_pack(kGrid2Task, 12, 1);
constexpr uint64_t kG2TaskQ = grid2_pack(kGrid2Task, 12, 2);
constexpr uint64_t kG2LeafA = grid2_pack(kGrid2Leaf, 16, 0);
constexpr uint64_t kG2LeafB = grid2_pack(kGrid2Leaf, 16, 1);
constexpr uint64_t kG2LeafC = grid2_pack(kGrid2Leaf, 16, 2);
SCVT_HD int nib(uint64_t v, int k) { return (int)((v >> (4 * k)) & 15); }

// sequential form (host checks): the 15 grid points of (A, B, C)
SCVT_HD void grid2_points(V3 A, V3 B, V3 C, V3* P) {
  P[14] = A;
  P[4] = B;
  P[0] = C;
  for (int t = 0; t < 12; t++)
    P[nib(kG2TaskPt, t)] = normalized_fast(P[nib(kG2TaskP, t)] + P[nib(kG2TaskQ, t)]);
}

// ------------------------------------------------------------ cube-map grid
// Each face f = 2k + (sign<0) of the cube [-1,1]^3 carries a gnomonic grid:
// a point p with depth n = +-p_k > 0 has face coordinates u = p_k+1 / n,
// v = p_k+2 / n, and cells of side du in (u, v).  G cells span the face
// proper ([-1,1]), B more on each side hold copies ("ghosts") of generators
// of the neighbouring faces (|u|,|v| up to U = 1 + B du), so that a search
// window around any generator stays on its own face.  Lines u = const are
// great circles through the face's v axis, so every bound below is algebraic.
struct GridP {
  int G, B, W;
  int pad;
  double du, inv_du, U;  // cell side, its inverse, extent of the extended grid
  int64_t ncells;        // 6 W^2
};

SCVT_HD int home_face(V3 p) {
  double ax = fabs(p.x), ay = fabs(p.y), az = fabs(p.z);
  if (ax >= ay && ax >= az) return p.x >= 0.0 ? 0 : 1;
  if (ay >= az) return p.y >= 0.0 ? 2 : 3;
  return p.z >= 0.0 ? 4 : 5;
}

// depth along the face normal and the two in-face coordinates (unscaled)
SCVT_HD void face_local(V3 p, int f, double& n, double& u, double& v) {
  int k = f >> 1;
  double s = (f & 1) ? -1.0 : 1.0;
  double c[3] = {p.x, p.y, p.z};
  n = s * c[k];
  u = c[(k + 1) % 3];
  v = c[(k + 2) % 3];
}

SCVT_HD int64_t cell_of(const GridP& g, int f, int ia, int ib) {
  return (int64_t)f * g.W * g.W + (int64_t)ib * g.W + ia;
}

// cell of p on face f, or -1 if p is outside that face's extended grid
SCVT_HD int64_t cell_on_face(const GridP& g, V3 p, int f) {
  double n, u, v;
  face_local(p, f, n, u, v);
  if (!(n > 0.0)) return -1;
  const double ni = rcp_fast(n);
  double fa = floor((u * ni + g.U) * g.inv_du), fb = floor((v * ni + g.U) * g.inv_du);
  if (fa < 0.0 || fb < 0.0 || fa >= (double)g.W || fb >= (double)g.W) return -1;
  return cell_of(g, f, (int)fa, (int)fb);
}

// A rectangle of cells on face f and the chord radius D around z inside
// which every generator of the sphere is stored in the rectangle.
struct Window {
  int f, ia_lo, ia_hi, ib_lo, ib_hi;
  double D;
};

// Bounds c_lo <= c_z <= c_hi on one face coordinate (c = w/n) such that the
// planes c = c_lo, c = c_hi are at angular distance >= theta from z, where
// sin(theta) = st: z sits at angle phi_z = atan(c_z) about the other face
// axis, at radius rho = sqrt(n^2 + w^2) from it, so the planes must be at
// phi_z -+ delta with sin(delta) = st / rho; tan(phi_z -+ delta) in closed form.
// FP32: the bounds only choose the window's columns (the radius the window
// certifies is computed from the columns taken, below).
SCVT_HD void coord_bounds(float cz, float rho, float st, float& lo, float& hi) {
  const float s = st * rcpf(rho);
  if (!(s < 1.0f)) {
    lo = -1e30f;
    hi = 1e30f;
    return;
  }
  const float t = s * rsqf(fmaxf(1.0f - s * s, 1e-30f));  // tan(delta)
  const float dl = fmaf(cz, t, 1.0f), dh = fmaf(-cz, t, 1.0f);
  lo = dl > 0.0f ? (cz - t) * rcpf(dl) : -1e30f;
  hi = dh > 0.0f ? (cz + t) * rcpf(dh) : 1e30f;
}

// A lower bound on the sine of the angular distance from z (depth n,
// coordinate w) to the plane c = cc through the face's other axis, signed
// positive on z's side (sgn): the offset in FP64, 1/sqrt(1 + cc^2) from the
// FP32 estimate (within a few 1e-7) lowered by 4e-6.
SCVT_HD double plane_sine(double n, double w, double cc, double sgn) {
  const float q = (float)fma(cc, cc, 1.0);
  return sgn * (w - cc * n) * (double)(rsqf(q) * (1.0f - 4e-6f));
}

// Window around z (face f = home face) that covers the chord radius rt
// (clamped to the grid and to at most maxw cells a side), and the radius D
// that the window actually chosen certifies: every generator within chord D
// of z is stored in its cells.  D is the least sine of the angular distance
// from z to a window side or to the face's horizon (points behind the face
// are not in its grid): a chord is never shorter than the sine of its angle,
// 2 sin(a/2) >= sin a.  The columns are chosen in FP32, widened by 1% of a
// cell so that the window covers rt despite the rounding; z's own cell is
// found in FP64 as the binning finds it.
SCVT_HD Window make_window(const GridP& g, V3 z, int f, double rt, int maxw) {
  double n, u, v;
  face_local(z, f, n, u, v);
  const double ni = rcp_fast(n);
  const double uz = u * ni, vz = v * ni;
  int ca = (int)floor((uz + g.U) * g.inv_du), cb = (int)floor((vz + g.U) * g.inv_du);
  ca = ca < 0 ? 0 : (ca >= g.W ? g.W - 1 : ca);
  cb = cb < 0 ? 0 : (cb >= g.W ? g.W - 1 : cb);
  const float r = rt > 2.0 ? 2.0f : (float)rt;
  const float q = fmaxf(1.0f - 0.25f * r * r, 1e-30f);
  float st = r * q * rsqf(q);                 // sin of the angular radius
  if (rt >= 1.4142135623730951) st = 1.0f;   // beyond 90 degrees: everything
  const float nf = (float)n, uf = (float)u, vf = (float)v;
  const float nif = rcpf(nf);
  float ulo, uhi, vlo, vhi;
  const float ru = fmaf(nf, nf, uf * uf), rv = fmaf(nf, nf, vf * vf);
  coord_bounds(uf * nif, ru * rsqf(ru), st, ulo, uhi);
  coord_bounds(vf * nif, rv * rsqf(rv), st, vlo, vhi);
  const int half_max = (maxw - 1) / 2;
  const float sc = (float)g.inv_du, of = (float)(g.U * g.inv_du);
  auto col = [&](float c, int centre, int dir) {
    const float x = floorf(fmaf(c, sc, of) + (float)dir * 0.01f);
    const float lim = (float)(centre + dir * half_max);
    if (dir < 0) return x < lim ? (int)lim : (int)x;
    return x > lim ? (int)lim : (int)x;
  };
  int ia_lo = col(ulo, ca, -1), ia_hi = col(uhi, ca, 1);
  int ib_lo = col(vlo, cb, -1), ib_hi = col(vhi, cb, 1);
  if (ia_lo < 0) ia_lo = 0;
  if (ib_lo < 0) ib_lo = 0;
  if (ia_hi > g.W - 1) ia_hi = g.W - 1;
  if (ib_hi > g.W - 1) ib_hi = g.W - 1;
  if (ia_lo > ca) ia_lo = ca;
  if (ia_hi < ca) ia_hi = ca;
  if (ib_lo > cb) ib_lo = cb;
  if (ib_hi < cb) ib_hi = cb;
  const double a0 = -g.U + ia_lo * g.du, a1 = -g.U + (ia_hi + 1) * g.du;
  const double b0 = -g.U + ib_lo * g.du, b1 = -g.U + (ib_hi + 1) * g.du;
  double sm = n;
  sm = fmin(sm, plane_sine(n, u, a0, 1.0));
  sm = fmin(sm, plane_sine(n, u, a1, -1.0));
  sm = fmin(sm, plane_sine(n, v, b0, 1.0));
  sm = fmin(sm, plane_sine(n, v, b1, -1.0));
  Window w;
  w.f = f;
  w.ia_lo = ia_lo;
  w.ia_hi = ia_hi;
  w.ib_lo = ib_lo;
  w.ib_hi = ib_hi;
  // shrunk to cover points binned across a side by rounding
  w.D = sm > 0.0 ? fmax(fmin(sm, 1.0) * (1.0 - 1e-10) - 1e-14, 0.0) : 0.0;
  return w;
}

// ---------------------------------------------- sequential spherical clipper
// Fallback construction of one cell: Sutherland-Hodgman clipping of a convex
// spherical polygon by the half-spaces x . (z - p) >= 0, in any order.  The
// first candidate's hemisphere is the starting polygon (four vertices on its
// circle); edges longer than 90 degrees get a midpoint on their own circle so
// that every arc stays below 180 degrees.  Each polygon slot holds a vertex
// and the generator whose bisector carries the outgoing edge; a vertex is a
// Voronoi vertex where consecutive edges change generator.  Works for any
// cell the sphere allows (also cells beyond a hemisphere, small n).
constexpr int kClipMax = 64;
struct ClipPoly {
  double P[2][kClipMax][3];   // vertices
  double EP[2][kClipMax][3];  // position of the outgoing edge's generator
  int32_t ec[2][kClipMax];    // id of that generator
  int32_t K[2];
  int32_t cur, err, degen, pad;
  double R;  // bound on |x - z| over the polygon (2 when unknown)
};

SCVT_HD V3 cp_get(const double (*A)[3], int k) { return V3{A[k][0], A[k][1], A[k][2]}; }
SCVT_HD void cp_set(double (*A)[3], int k, V3 v) {
  A[k][0] = v.x;
  A[k][1] = v.y;
  A[k][2] = v.z;
}

SCVT_HD void clip_reset(ClipPoly& C) {
  C.cur = 0;
  C.K[0] = C.K[1] = 0;
  C.err = C.degen = 0;
  C.R = 2.0;
}

// bound: max vertex distance if the polygon lies in z's open hemisphere (then
// the farthest point is a vertex: along an arc inside that hemisphere x.z is
// concave), else 2
SCVT_HD void clip_update_R(ClipPoly& C, V3 z) {
  const int b = C.cur, K = C.K[b];
  double r2 = 0.0;
  bool hemi = K > 0;
  for (int k = 0; k < K; k++) {
    V3 P = cp_get(C.P[b], k);
    if (!(dot(P, z) > 0.0)) hemi = false;
    V3 d = P - z;
    r2 = fmax(r2, dot(d, d));
  }
  C.R = hemi ? sqrt(r2) : 2.0;
}

SCVT_HD void clip_init(ClipPoly& C, V3 z, int j, V3 pj) {
  V3 N = normalized(z - pj);
  V3 ax = fabs(N.x) < 0.6 ? V3{1, 0, 0} : (fabs(N.y) < 0.6 ? V3{0, 1, 0} : V3{0, 0, 1});
  V3 u1 = normalized(cross(N, ax));
  V3 u2 = normalized(cross(N, u1));
  C.cur = 0;
  C.K[0] = 4;
  V3 v[4] = {u1, u2, -u1, -u2};
  for (int k = 0; k < 4; k++) {
    cp_set(C.P[0], k, v[k]);
    cp_set(C.EP[0], k, pj);
    C.ec[0][k] = j;
  }
}

SCVT_HD void clip_by(ClipPoly& C, V3 z, int m, V3 pm) {
  const int b = C.cur, nb = 1 - b, K = C.K[b];
  for (int k = 0; k < K; k++)
    if (C.ec[b][k] == m) return;  // already an edge of the polygon
  const V3 N = z - pm;
  double s[kClipMax];
  bool any_out = false;
  for (int k = 0; k < K; k++) {
    V3 P = cp_get(C.P[b], k);
    s[k] = dot(P, N);
    double err = 8.0 * kU * (fabs(P.x * N.x) + fabs(P.y * N.y) + fabs(P.z * N.z));
    if (fabs(s[k]) <= err) C.degen = 1;
    if (s[k] < 0.0) any_out = true;
  }
  if (!any_out) return;
  int c = 0;
  for (int k = 0; k < K; k++) {
    if (c > kClipMax - 2) {
      C.err = 1;
      break;
    }
    int k1 = (k + 1) % K;
    V3 P = cp_get(C.P[b], k), Q = cp_get(C.P[b], k1);
    bool inP = s[k] >= 0.0, inQ = s[k1] >= 0.0;
    if (inP) {
      cp_set(C.P[nb], c, P);
      cp_set(C.EP[nb], c, cp_get(C.EP[b], k));
      C.ec[nb][c++] = C.ec[b][k];
    }
    if (inP != inQ) {
      V3 X = normalized(fabs(s[k1]) * P + fabs(s[k]) * Q);
      cp_set(C.P[nb], c, X);
      if (inP) {  // leaving: the new edge runs along m
        cp_set(C.EP[nb], c, pm);
        C.ec[nb][c++] = m;
      } else {    // entering: continue along the old edge
        cp_set(C.EP[nb], c, cp_get(C.EP[b], k));
        C.ec[nb][c++] = C.ec[b][k];
      }
    }
  }
  // midpoints of arcs longer than 90 degrees, rotated along the arc's circle
  int c2 = 0;
  for (int k = 0; k < c; k++) {
    if (c2 > kClipMax - 2) {
      C.err = 1;
      break;
    }
    V3 P = cp_get(C.P[nb], k), Q = cp_get(C.P[nb], (k + 1) % c);
    V3 EPk = cp_get(C.EP[nb], k);
    int e = C.ec[nb][k];
    cp_set(C.P[b], c2, P);
    cp_set(C.EP[b], c2, EPk);
    C.ec[b][c2++] = e;
    if (dot(P, Q) < 0.0) {
      V3 Nh = normalized(z - EPk);
      V3 T = normalized(cross(Nh, P));
      double th = atan2(dot(Q, T), dot(Q, P));
      if (th < 0.0) th += 6.283185307179586;
      V3 Mid = normalized(cos(0.5 * th) * P + sin(0.5 * th) * T);
      cp_set(C.P[b], c2, Mid);
      cp_set(C.EP[b], c2, EPk);
      C.ec[b][c2++] = e;
    }
  }
  C.cur = b;
  C.K[b] = c2;
}

// offer generator j at pj (j != own index) to the clipper
SCVT_HD void clip_offer(ClipPoly& C, V3 z, int j, V3 pj) {
  if (C.K[C.cur] == 0) {
    clip_init(C, z, j, pj);
  } else {
    clip_by(C, z, j, pj);
  }
  clip_update_R(C, z);
}

// Finish: real vertices in counter-clockwise order, each recomputed as the
// canonical circumcentre of (own, incoming, outgoing generator) on the side
// of the clipped vertex; edges k (v_k -> v_k+1 on the bisector with
// enbr[k]) written sorted by neighbour index.  Returns the edge count (0 and
// err set when the polygon is not a proper cell); C.R becomes the circumradius.
template <class Pos>
SCVT_HD int clip_finish(ClipPoly& C, int self, V3 z, const Pos& pos, int32_t* enbr, double* v0,
                        double* v1, int vmax) {
  const int b = C.cur, K = C.K[b], ob = 1 - b;
  int nreal = 0;
  for (int k = 0; k < K; k++) {
    int ein = C.ec[b][(k + K - 1) % K], eout = C.ec[b][k];
    if (ein == eout) continue;
    if (nreal >= kClipMax) {
      C.err = 1;
      break;
    }
    V3 X = cp_get(C.P[b], k);
    V3 v = circumcentre(self, z, ein, pos(ein), eout, pos(eout));
    if (dot(v, X) < 0.0) v = -v;
    cp_set(C.P[ob], nreal, v);
    C.ec[ob][nreal] = eout;
    nreal++;
  }
  if (nreal < 3 || nreal > vmax) C.err = 1;
  const int E = C.err ? 0 : nreal;
  double r2 = 0.0;
  for (int k = 0; k < E; k++) {
    int nbk = C.ec[ob][k];
    V3 p0 = cp_get(C.P[ob], k), p1 = cp_get(C.P[ob], (k + 1) % E);
    V3 d0 = p0 - z;
    r2 = fmax(r2, dot(d0, d0));
    V3 dd = p1 - p0;
    if (dot(dd, dd) == 0.0) C.degen = 1;
    int r = k;
    while (r > 0 && enbr[r - 1] > nbk) {
      enbr[r] = enbr[r - 1];
      for (int c = 0; c < 3; c++) {
        v0[3 * r + c] = v0[3 * (r - 1) + c];
        v1[3 * r + c] = v1[3 * (r - 1) + c];
      }
      r--;
    }
    enbr[r] = nbk;
    v0[3 * r] = p0.x; v0[3 * r + 1] = p0.y; v0[3 * r + 2] = p0.z;
    v1[3 * r] = p1.x; v1[3 * r + 1] = p1.y; v1[3 * r + 2] = p1.z;
  }
  C.R = sqrt(r2);
  return E;
}

}  // namespace scvt
