/*
 * SCVT oracle -- plain FP64 CPU reference for the cell integrals.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the HIP library.
 *
 * What it computes (Yang, Gunzburger & Ju, "Fast spherical centroidal Voronoi
 * mesh generation", section 2.1):
 *   mass        m_i  = int_{V_i} rho dsigma                 (mass centroid eq.)
 *   first moment mu_i = int_{V_i} y rho dsigma               (the paper's c_i,
 *                                                             section 3.1)
 *   energy      e_i  = int_{V_i} |y - z_i|^2 rho dsigma      (CCVT energy)
 * over the spherical Voronoi cell V_i of generator z_i (eq. viInS).
 *
 * The paper does not name the quadrature used for the configurations timed
 * here, so the rule is the documented reading:
 *   - cell i is split into fan triangles (z_i, v_k, v_k+1) over its cyclically
 *     ordered Voronoi vertices (same exact integral as the paper's
 *     six-sub-triangle split of each Delaunay triangle, section 3.2.2);
 *   - each fan triangle is split `levels` times into 4 by geodesic midpoints
 *     normalize(a+b);
 *   - on each spherical sub-triangle (A,B,C) the flat triangle is mapped onto
 *     the sphere by radial projection, whose exact Jacobian gives
 *       int_sph f dsigma = 1/2 det(A,B,C) * sum_q w_q f(p_q/|p_q|) / |p_q|^3,
 *     p_q = sum of barycentric weights times (A,B,C);
 *   - the planar rule is Radon's 7-point degree-5 rule (Stroud T2:5-1) by
 *     default, or a rule passed in (oracle_rule: barycentric points and
 *     weights summing to one), e.g. the conical product rules of 4 and 9
 *     points built by oracle/rules.py.
 *
 * Densities (section 4): constant; the tanh bump family with the prefactor
 * read as (1-gamma)/2 (the printed 1/(2(1-gamma)) cannot give a density whose
 * range is [gamma, 1]); a sum of such bumps; X3 = (1-gamma) z^4 + gamma.
 *
 * Everything is double precision; build with -ffp-contract=off so that no
 * fused multiply-add changes the rounding the reader sees in the source.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define ORACLE_RHO_CONST 0
#define ORACLE_RHO_TANH 1 /* sum of up to two tanh bumps over a floor gamma */
#define ORACLE_RHO_X3 2
#define ORACLE_RHO_X16 3 /* anisotropic-distance tanh bump */

typedef struct {
  int32_t kind;
  int32_t geodesic; /* 1: d = geodesic angle, 0: d = chord |y - x_c| */
  int32_t nbumps;   /* 1 or 2 for ORACLE_RHO_TANH */
  int32_t pad;
  double xc[2][3];
  double beta[2];
  double alpha[2];
  double amp[2]; /* bump heights: rho = gamma + sum_k amp_k (tanh(.)+1)/2 */
  double gamma;
  double w_lon, w_lat; /* X16 widths */
} oracle_density;

/* ---------------------------------------------------------------- rule --- */

/* Radon's 7-point rule of degree 5 on a triangle in barycentric form; the
 * weights are normalised to sum to one (multiply by the triangle's area). */
void oracle_rule7(double lam[21], double w[7]) {
  const double r15 = sqrt(15.0);
  const double a1 = (6.0 - r15) / 21.0, a2 = (6.0 + r15) / 21.0;
  const double w1 = (155.0 - r15) / 1200.0, w2 = (155.0 + r15) / 1200.0;
  double pts[7][3] = {{1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0},
                      {1.0 - 2.0 * a1, a1, a1},
                      {a1, 1.0 - 2.0 * a1, a1},
                      {a1, a1, 1.0 - 2.0 * a1},
                      {1.0 - 2.0 * a2, a2, a2},
                      {a2, 1.0 - 2.0 * a2, a2},
                      {a2, a2, 1.0 - 2.0 * a2}};
  double ww[7] = {9.0 / 40.0, w1, w1, w1, w2, w2, w2};
  for (int q = 0; q < 7; q++) {
    for (int k = 0; k < 3; k++) lam[3 * q + k] = pts[q][k];
    w[q] = ww[q];
  }
}

/* A triangle rule: nq points (barycentric lam[3q..3q+2]) and weights w[q]
 * summing to one.  NULL means Radon's rule. */
typedef struct {
  int32_t nq;
  int32_t pad;
  double lam[3 * 16];
  double w[16];
} oracle_rule;

/* ------------------------------------------------------------- density --- */

static double dot3(const double *a, const double *b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static double chord(const double *y, const double *c) {
  double d0 = y[0] - c[0], d1 = y[1] - c[1], d2 = y[2] - c[2];
  return sqrt(d0 * d0 + d1 * d1 + d2 * d2);
}

/* geodesic angle between two unit vectors from their chord length */
static double chord_to_angle(double ch) {
  double s = ch / 2.0;
  if (s > 1.0) s = 1.0;
  return 2.0 * asin(s);
}

static double lat_of(const double *y) {
  double s = y[2];
  if (s > 1.0) s = 1.0;
  if (s < -1.0) s = -1.0;
  return asin(s);
}

static double lon_of(const double *y) { return atan2(y[1], y[0]); }

static void from_latlon(double lat, double lon, double *out) {
  out[0] = cos(lat) * cos(lon);
  out[1] = cos(lat) * sin(lon);
  out[2] = sin(lat);
}

/* (tanh(x) + 1) / 2 of the section-4 bump, in the equal form 1/(1 + e^{-2x}):
 * tanh(x) + 1 cancels to a few digits where the bump is far below 1, and the
 * density's floor gamma can be as small as 64^-4 (X64), so the tanh form
 * would carry errors of ~1e-9 relative into rho there. */
static double half_tanh_plus_one(double x) { return 1.0 / (1.0 + exp(-2.0 * x)); }

double oracle_rho(const oracle_density *D, const double *y) {
  switch (D->kind) {
    case ORACLE_RHO_CONST:
      return 1.0;
    case ORACLE_RHO_TANH: {
      double rho = D->gamma;
      for (int k = 0; k < D->nbumps; k++) {
        double d = chord(y, D->xc[k]);
        if (D->geodesic) d = chord_to_angle(d);
        rho += D->amp[k] * half_tanh_plus_one((D->beta[k] - d) / D->alpha[k]);
      }
      return rho;
    }
    case ORACLE_RHO_X3: {
      double z2 = y[2] * y[2];
      return (1.0 - D->gamma) * z2 * z2 + D->gamma;
    }
    case ORACLE_RHO_X16: {
      /* z_ic: latitude of y, longitude of x_c; z_ci: latitude of x_c,
       * longitude of y; both distances geodesic (section 4). */
      double la = lat_of(y), lo = lon_of(y);
      double lac = lat_of(D->xc[0]), loc = lon_of(D->xc[0]);
      double zic[3], zci[3];
      from_latlon(la, loc, zic);
      from_latlon(lac, lo, zci);
      double d1 = chord_to_angle(chord(y, zic));
      double d2 = chord_to_angle(chord(y, zci));
      double d = sqrt(d1 * d1 / (D->w_lon * D->w_lon) + d2 * d2 / (D->w_lat * D->w_lat));
      return D->amp[0] * half_tanh_plus_one((D->beta[0] - d) / D->alpha[0]) + D->gamma;
    }
  }
  return NAN;
}

/* ------------------------------------------------------- spherical tri --- */

typedef struct {
  double m, mu[3], e;
} acc5;

static void normalize3(double *v) {
  double r = sqrt(dot3(v, v));
  v[0] /= r;
  v[1] /= r;
  v[2] /= r;
}

static void midpoint(const double *a, const double *b, double *out) {
  out[0] = a[0] + b[0];
  out[1] = a[1] + b[1];
  out[2] = a[2] + b[2];
  normalize3(out);
}

static double det3(const double *a, const double *b, const double *c) {
  return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
         a[2] * (b[0] * c[1] - b[1] * c[0]);
}

/* Integrate rho, y rho and |y - z|^2 rho over the spherical triangle (A,B,C)
 * with the radial-projection rule (no subdivision). */
static void tri_rule(const oracle_density *D, const oracle_rule *R, const double *z,
                     const double *A, const double *B, const double *C, acc5 *acc) {
  double lam7[21], w7[7];
  oracle_rule7(lam7, w7);
  const int nq = R ? R->nq : 7;
  const double *lam = R ? R->lam : lam7;
  const double *w = R ? R->w : w7;
  /* det(A,B,C) = det(A, B-A, C-A): the same value, computed from the
   * differences of the nearby vertices so that small sub-triangles do not
   * lose digits to cancellation */
  double u[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
  double v[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
  double half_det = 0.5 * det3(A, u, v);
  for (int q = 0; q < nq; q++) {
    double p[3];
    for (int k = 0; k < 3; k++)
      p[k] = lam[3 * q + 0] * A[k] + lam[3 * q + 1] * B[k] + lam[3 * q + 2] * C[k];
    double r = sqrt(dot3(p, p));
    double y[3] = {p[0] / r, p[1] / r, p[2] / r};
    double jac = 1.0 / (r * r * r);
    double rho = oracle_rho(D, y);
    double wt = half_det * w[q] * jac * rho;
    double dy[3] = {y[0] - z[0], y[1] - z[1], y[2] - z[2]};
    acc->m += wt;
    acc->mu[0] += wt * y[0];
    acc->mu[1] += wt * y[1];
    acc->mu[2] += wt * y[2];
    acc->e += wt * dot3(dy, dy);
  }
}

/* Split (A,B,C) into four by geodesic midpoints `levels` times, then apply
 * the rule on every leaf. */
static void tri_subdivide(const oracle_density *D, const oracle_rule *R, const double *z,
                          const double *A, const double *B, const double *C, int levels,
                          acc5 *acc) {
  if (levels == 0) {
    tri_rule(D, R, z, A, B, C, acc);
    return;
  }
  double ab[3], bc[3], ca[3];
  midpoint(A, B, ab);
  midpoint(B, C, bc);
  midpoint(C, A, ca);
  tri_subdivide(D, R, z, A, ab, ca, levels - 1, acc);
  tri_subdivide(D, R, z, ab, B, bc, levels - 1, acc);
  tri_subdivide(D, R, z, ca, bc, C, levels - 1, acc);
  tri_subdivide(D, R, z, ab, bc, ca, levels - 1, acc);
}

/* One spherical triangle, exposed for the closed-form tests.
 * out[0]=mass, out[1..3]=moment, out[4]=energy about z. */
void oracle_triangle_integrals(const oracle_density *D, const double *z, const double *A,
                               const double *B, const double *C, int levels,
                               const oracle_rule *R, double *out) {
  acc5 acc = {0.0, {0.0, 0.0, 0.0}, 0.0};
  tri_subdivide(D, R, z, A, B, C, levels, &acc);
  out[0] = acc.m;
  out[1] = acc.mu[0];
  out[2] = acc.mu[1];
  out[3] = acc.mu[2];
  out[4] = acc.e;
}

/* ------------------------------------------------------------ all cells --- */

/* Cells are given in CSR form: the Voronoi vertices of cell i are
 * V[ptr[i]..ptr[i+1]) (each 3 doubles), ordered counter-clockwise seen from
 * outside the sphere.  Output per cell: mass m[i], moment mu[3i..3i+2],
 * energy e[i].  Returns 0. */
int oracle_cell_integrals(int64_t n, const double *Z, const int64_t *ptr, const double *V,
                          const oracle_density *D, int levels, const oracle_rule *R, double *m,
                          double *mu, double *e) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; i++) {
    const double *z = Z + 3 * i;
    acc5 acc = {0.0, {0.0, 0.0, 0.0}, 0.0};
    int64_t b = ptr[i], deg = ptr[i + 1] - ptr[i];
    for (int64_t k = 0; k < deg; k++) {
      const double *v0 = V + 3 * (b + k);
      const double *v1 = V + 3 * (b + (k + 1) % deg);
      tri_subdivide(D, R, z, z, v0, v1, levels, &acc);
    }
    m[i] = acc.m;
    mu[3 * i + 0] = acc.mu[0];
    mu[3 * i + 1] = acc.mu[1];
    mu[3 * i + 2] = acc.mu[2];
    e[i] = acc.e;
  }
  return 0;
}

/* Density at many points (for tests). */
void oracle_rho_many(const oracle_density *D, int64_t npts, const double *Y, double *out) {
  for (int64_t k = 0; k < npts; k++) out[k] = oracle_rho(D, Y + 3 * k);
}

/* Threads the integrals use from now on (the benchmark's single-thread
 * baseline); values below 1 are ignored. */
void oracle_set_num_threads(int t) {
#ifdef _OPENMP
  extern void omp_set_num_threads(int);
  if (t >= 1) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/* Number of OpenMP threads the integrals use (reported by the benchmark). */
int oracle_num_threads(void) {
  int t = 1;
#pragma omp parallel
  {
#pragma omp single
    {
#ifdef _OPENMP
      extern int omp_get_num_threads(void);
      t = omp_get_num_threads();
#endif
    }
  }
  return t;
}
