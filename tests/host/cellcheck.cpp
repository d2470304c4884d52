// Host build of the HIP path's geometry code (csrc/cellgeom.h) for the CPU
// tests: runs the per-bisector edge construction the kernels run per lane,
// the sequential fallback clipper, the window certificate and the cell
// quadrature on the host, so that their logic is checked against the oracle
// without a GPU.  Compiled by tests/test_hostcheck.py with hipcc.
#include <stdint.h>
#include <string.h>

#include <vector>

#include "cellgeom.h"

using namespace scvt;

extern "C" {

// Certified-path construction for every generator with all generators
// within chord radius rad[i] as candidates (emulates the wave: one loop
// iteration per lane).  Outputs per cell: status (0 ok certified, 1
// degenerate, 2 unbounded, 3 not certified, 4 too many candidates), deg,
// nbr[i*32+k] sorted ascending, verts[(i*32+k)*6 + 0..5] edge endpoints.
// At most `cap` candidates (<= 64) are kept; on overflow Rout[i] holds the
// number of generators inside the radius.
int hc_cells(int64_t n, const double* Z, const double* rad, int32_t* status, int32_t* deg,
             int32_t* nbr, double* verts, double* Rout, int cap) {
  if (cap < 1 || cap > 64) return -1;
  std::vector<double> px(64), py(64), pz(64), dx(64), dy(64), dz(64), nr(64), zd(64);
  std::vector<int> idx(64);
  for (int64_t i = 0; i < n; i++) {
    V3 z = V3{Z[3 * i], Z[3 * i + 1], Z[3 * i + 2]};
    int ns = 0, total = 0;
    for (int64_t j = 0; j < n; j++) {
      if (j == i) continue;
      V3 p = V3{Z[3 * j], Z[3 * j + 1], Z[3 * j + 2]};
      V3 d = p - z;
      if (dot(d, d) < rad[i] * rad[i]) {
        if (total++ >= cap) continue;
        px[ns] = p.x; py[ns] = p.y; pz[ns] = p.z;
        dx[ns] = d.x; dy[ns] = d.y; dz[ns] = d.z;
        nr[ns] = sqrt(dot(d, d));
        zd[ns] = dot(z, d);
        idx[ns] = (int)j;
        ns++;
      }
    }
    deg[i] = 0;
    for (int k = 0; k < 32; k++) nbr[i * 32 + k] = -1;
    if (total > cap) {
      status[i] = 4;
      Rout[i] = (double)total;
      continue;
    }
    CandView S = {px.data(), py.data(), pz.data(), dx.data(), dy.data(), dz.data(), nr.data(),
                  zd.data()};
    double nm = 0.0;
    for (int l = 0; l < ns; l++) nm = fmax(nm, nr[l]);
    std::vector<EdgeRes> er(ns);
    int st = 0;
    for (int l = 0; l < ns; l++) {
      er[l] = edge_on_bisector(l, ns, z, S, nm);
      if (er[l].status == kEdgeDegenerate) st = 1;
      if (er[l].status == kEdgeUnbounded && st == 0) st = 2;
    }
    if (ns < 3 && st == 0) st = 2;
    if (st) {
      status[i] = st;
      continue;
    }
    double r2 = 0.0;
    int E = 0;
    std::vector<int> en;
    std::vector<V3> a0, a1;
    for (int l = 0; l < ns; l++) {
      if (er[l].status != kEdgeYes) continue;
      V3 vlo = circumcentre((int)i, z, idx[l], S.p(l), idx[er[l].lo], S.p(er[l].lo));
      V3 vhi = circumcentre((int)i, z, idx[l], S.p(l), idx[er[l].hi], S.p(er[l].hi));
      V3 q0 = vlo - z, q1 = vhi - z;
      r2 = fmax(r2, fmax(dot(q0, q0), dot(q1, q1)));
      en.push_back(idx[l]);
      a0.push_back(vlo);
      a1.push_back(vhi);
      E++;
    }
    Rout[i] = sqrt(r2);
    if (!(4.0 * r2 * (1.0 + 1e-12) <= rad[i] * rad[i]) || E < 3 || E > 32) {
      status[i] = 3;
      continue;
    }
    status[i] = 0;
    deg[i] = E;
    for (int k = 0; k < E; k++) {
      int rank = 0;
      for (int t = 0; t < E; t++) rank += en[t] < en[k];
      nbr[i * 32 + rank] = en[k];
      double* v = verts + (i * 32 + rank) * 6;
      v[0] = a0[k].x; v[1] = a0[k].y; v[2] = a0[k].z;
      v[3] = a1[k].x; v[4] = a1[k].y; v[5] = a1[k].z;
    }
  }
  return 0;
}

// Fallback clipper for cell i over all generators in index order.
int hc_clip(int64_t n, const double* Z, int64_t i, int32_t* deg, int32_t* nbr, double* verts,
            int32_t* flags, double* Rout) {
  static ClipPoly C;
  clip_reset(C);
  V3 z = V3{Z[3 * i], Z[3 * i + 1], Z[3 * i + 2]};
  for (int64_t j = 0; j < n; j++) {
    if (j == i) continue;
    V3 p = V3{Z[3 * j], Z[3 * j + 1], Z[3 * j + 2]};
    V3 d = p - z;
    if (dot(d, d) < 4.0 * C.R * C.R * (1.0 + 1e-9) + 1e-300) clip_offer(C, z, (int)j, p);
  }
  int32_t en[32];
  double v0[96], v1[96];
  auto pos = [&](int j) { return V3{Z[3 * j], Z[3 * j + 1], Z[3 * j + 2]}; };
  int E = clip_finish(C, (int)i, z, pos, en, v0, v1, 32);
  *deg = E;
  *flags = (C.err ? 4 : 0) | (C.degen ? 2 : 0);
  *Rout = C.R;
  for (int k = 0; k < 32; k++) nbr[k] = k < E ? en[k] : -1;
  for (int k = 0; k < E; k++)
    for (int c = 0; c < 3; c++) {
      verts[6 * k + c] = v0[3 * k + c];
      verts[6 * k + 3 + c] = v1[3 * k + c];
    }
  return 0;
}

// Cell integrals from fan edges (z, v0[k], v1[k]), k < E, as the kernels do.
int hc_quad(const double* z3, int E, const double* verts, const DensityP* D, int levels,
            int nq, double* out5) {
  Acc5 acc = {0, 0, 0, 0, 0};
  DensityP Dp = density_prepare(*D);
  V3 z = V3{z3[0], z3[1], z3[2]};
  const int per = 1 << (2 * levels);
  for (int t = 0; t < E * per; t++) {
    int e = t >> (2 * levels), s = t & (per - 1);
    V3 A = z, B = V3{verts[6 * e], verts[6 * e + 1], verts[6 * e + 2]},
       C = V3{verts[6 * e + 3], verts[6 * e + 4], verts[6 * e + 5]};
    subtriangle(A, B, C, s, levels);
    quad_tri(A, B, C, z, Dp, acc, nq);
  }
  out5[0] = acc.m;  // mu = m z + int rho (y - z), as the kernels' epilogue
  out5[1] = acc.m * z.x + acc.mx;
  out5[2] = acc.m * z.y + acc.my;
  out5[3] = acc.m * z.z + acc.mz;
  out5[4] = acc.e;
  return 0;
}

// Cell integrals through the per-cell density polynomial (single chord tanh
// bump) as the FP64 kernel takes them: the expansion in x if the cell
// qualifies for it (returns 2), else the one in t if it qualifies for that
// (returns 1); returns 0 (nothing computed) otherwise.  force: 1 only t, 2
// only x (0: the kernel's choice).
int hc_quad_poly(const double* z3, int E, const double* verts, const DensityP* D, int levels,
                 int nq, double* out5, int force) {
  Acc5 acc = {0, 0, 0, 0, 0};
  DensityP Dp = density_prepare(*D);
  if (Dp.kind != kRhoTanh || Dp.geodesic || Dp.polyx_n == 0) return 0;
  const int nb = Dp.nbumps;
  V3 z = V3{z3[0], z3[1], z3[2]};
  double r2 = 0.0;
  for (int e = 0; e < E; e++)
    for (int c = 0; c < 2; c++) {
      const V3 v = V3{verts[6 * e + 3 * c], verts[6 * e + 3 * c + 1], verts[6 * e + 3 * c + 2]} - z;
      r2 = fmax(r2, dot(v, v));
    }
  const double r = sqrt(r2);
  // the x entries of every bump, and whether the fan lies inside each radius
  RhoPoly PX[2];
  bool xq = true;
  for (int b = 0; b < nb; b++) {
    double xz = 0.0;
    const int64_t jx = polyx_index(Dp, z, &xz, b);
    PX[b] = polyx_entry(Dp, jx, b);
    const double delta = fabs(xz - (double)jx * kPolyDx) + r * (sqrt(2.0 * xz) + 0.5 * r);
    xq = xq && delta <= PX[b].lim;
  }
  const bool tq = nb == 1 && poly_qualifies(Dp, z, r2);
  int mode = 0;
  if (force == 2) mode = xq ? 2 : 0;
  else if (force == 1) mode = tq ? 1 : 0;
  else mode = xq ? 2 : (tq ? 1 : 0);
  if (mode == 0) return 0;
  if (mode == 2)  // the x entries taken at the cell, as the kernel takes them
    for (int b = 0; b < nb; b++) PX[b] = polyx_at(PX[b], Dp, z, b);
  const RhoPoly P = mode == 2 ? PX[0] : poly_entry(Dp, poly_index(Dp, z));
  const int per = 1 << (2 * levels);
  for (int t = 0; t < E * per; t++) {
    int e = t >> (2 * levels), s = t & (per - 1);
    V3 A = z, B = V3{verts[6 * e], verts[6 * e + 1], verts[6 * e + 2]},
       C = V3{verts[6 * e + 3], verts[6 * e + 4], verts[6 * e + 5]};
    subtriangle(A, B, C, s, levels);
    if (mode == 2 && nb == 2)
      quad_tri_poly2(A, B, C, z, Dp, PX[0], PX[1], acc, nq);
    else if (mode == 2)
      quad_tri_poly<true>(A, B, C, z, Dp, P, acc, nq);
    else
      quad_tri_poly<false>(A, B, C, z, Dp, P, acc, nq);
  }
  out5[0] = acc.m;  // mu = m z + int rho (y - z)
  out5[1] = acc.m * z.x + acc.mx;
  out5[2] = acc.m * z.y + acc.my;
  out5[3] = acc.m * z.z + acc.mz;
  out5[4] = acc.e;
  return mode;
}

// Mixed-precision cell integrals through the FP32 copies of the expansions
// in x (one or two chord tanh bumps), as the mixed kernel takes a qualifying
// cell; returns 0 (nothing computed) if the fan is not inside every entry's
// radius.
int hc_quad_mixed_poly(const double* z3, int E, const double* verts, const DensityP* D,
                       int levels, int nq, double* out5) {
  Acc5 acc = {0, 0, 0, 0, 0};
  DensityP Dp = density_prepare(*D);
  if (Dp.kind != kRhoTanh || Dp.geodesic || Dp.polyx_n == 0) return 0;
  const int nb = Dp.nbumps;
  const V3 z = V3{z3[0], z3[1], z3[2]};
  double r2 = 0.0;
  for (int e = 0; e < E; e++)
    for (int c = 0; c < 2; c++) {
      const V3 v = V3{verts[6 * e + 3 * c], verts[6 * e + 3 * c + 1], verts[6 * e + 3 * c + 2]} - z;
      r2 = fmax(r2, dot(v, v));
    }
  const double r = sqrt(r2);
  RhoPoly PX[2];
  for (int b = 0; b < nb; b++) {
    double xz = 0.0;
    const int64_t jx = polyx_index(Dp, z, &xz, b);
    PX[b] = polyx_entry(Dp, jx, b);
    if (fabs(xz - (double)jx * kPolyDx) + r * (sqrt(2.0 * xz) + 0.5 * r) > PX[b].lim) return 0;
    PX[b] = polyx_at(PX[b], Dp, z, b);
  }
  const CellF cf = cell_f32_poly(Dp, PX, nb, z);
  const DensityF Df = density_f32(Dp);
  const int per = 1 << (2 * levels);
  for (int t = 0; t < E * per; t++) {
    int e = t >> (2 * levels), s = t & (per - 1);
    V3 A = z, B = V3{verts[6 * e], verts[6 * e + 1], verts[6 * e + 2]},
       C = V3{verts[6 * e + 3], verts[6 * e + 4], verts[6 * e + 5]};
    subtriangle(A, B, C, s, levels);
    if (nb == 2)
      quad_leaf_mixed<kRhoTanh + kVarTwo, 2>(A, B, C, z, cf, Df, Dp, acc, nq);
    else
      quad_leaf_mixed<kRhoTanh, 1>(A, B, C, z, cf, Df, Dp, acc, nq);
  }
  out5[0] = acc.m;  // mu = m z + int rho (y - z)
  out5[1] = acc.m * z.x + acc.mx;
  out5[2] = acc.m * z.y + acc.my;
  out5[3] = acc.m * z.z + acc.mz;
  out5[4] = acc.e;
  return 1;
}

// rho at the unit points y (n x 3) from the polynomial table's entry of
// generator z (mode 0: in t, 1: in x), and from the exact evaluation; lim
// receives the x entry's radius
int hc_rho_poly(const double* z3, const DensityP* D, int64_t n, const double* y, double* poly,
                double* exact, int mode, double* lim) {
  DensityP Dp = density_prepare(*D);
  V3 z = V3{z3[0], z3[1], z3[2]};
  // two bumps (x only): the sum of both entries' polynomials, lim the smaller radius
  const int nb = mode == 1 ? Dp.nbumps : 1;
  RhoPoly P[2];
  *lim = 1e300;
  for (int b = 0; b < nb; b++) {
    double xz = 0.0;
    P[b] = mode == 1 ? polyx_entry(Dp, polyx_index(Dp, z, &xz, b), b)
                     : poly_entry(Dp, poly_index(Dp, z));
    *lim = fmin(*lim, P[b].lim);
  }
  for (int64_t k = 0; k < n; k++) {
    const V3 p = V3{y[3 * k], y[3 * k + 1], y[3 * k + 2]};
    double sum = 0.0;
    for (int b = 0; b < nb; b++) {
      const double u = fma(-1.0, dot(p, V3{Dp.xc[b][0], Dp.xc[b][1], Dp.xc[b][2]}),
                           mode == 1 ? P[b].off : Dp.cc[0]);
      const double dl = mode == 1 ? u : fma(sqrt_nr_pos(fmax(u, 1e-300)), Dp.Kt[0], P[b].off);
      double r = P[b].c[kPolyDeg];
      for (int j = kPolyDeg - 1; j >= 0; j--) r = fma(r, dl, P[b].c[j]);
      sum += r;
    }
    poly[k] = sum;
    exact[k] = rho_eval(Dp, p);
  }
  return 0;
}

// Mixed-precision cell integrals as the kernel computes them (FP64
// subdivision and leaf determinants, FP32 local-frame points, FP64
// accumulation, mu = m z + ...)
int hc_quad_mixed(const double* z3, int E, const double* verts, const DensityP* D, int levels,
                  int nq, double* out5) {
  Acc5 acc = {0, 0, 0, 0, 0};
  DensityP Dp = density_prepare(*D);
  V3 z = V3{z3[0], z3[1], z3[2]};
  DensityF Df = density_f32(Dp);
  const int per = 1 << (2 * levels);
  const int var = rho_variant(Dp);
  for (int t = 0; t < E * per; t++) {
    int e = t >> (2 * levels), s = t & (per - 1);
    V3 A = z, B = V3{verts[6 * e], verts[6 * e + 1], verts[6 * e + 2]},
       C = V3{verts[6 * e + 3], verts[6 * e + 4], verts[6 * e + 5]};
    subtriangle(A, B, C, s, levels);
#define HC_MIXED(V) quad_leaf_mixed<V>(A, B, C, z, cell_f32<V>(Dp, z), Df, Dp, acc, nq)
    SCVT_RHO_DISPATCH(var, HC_MIXED)
#undef HC_MIXED
  }
  out5[0] = acc.m;
  out5[1] = acc.m * z.x + acc.mx;
  out5[2] = acc.m * z.y + acc.my;
  out5[3] = acc.m * z.z + acc.mz;
  out5[4] = acc.e;
  return 0;
}

// Grid helpers: grid parameters for n, the window for (z, rt), the cell of
// p on face f (-1 outside the face's extended grid).
int hc_grid(int64_t n, int32_t* GBW, double* dd) {
  int G = (int)llround(sqrt((double)n / 12.0));
  if (G < 1) G = 1;
  int B = G / 2;
  if (B > 24) B = 24;
  GBW[0] = G;
  GBW[1] = B;
  GBW[2] = G + 2 * B;
  dd[0] = 2.0 / G;
  dd[1] = G / 2.0;
  dd[2] = 1.0 + B * dd[0];
  return 0;
}

static GridP gp(const int32_t* GBW, const double* dd) {
  GridP g{};
  g.G = GBW[0];
  g.B = GBW[1];
  g.W = GBW[2];
  g.du = dd[0];
  g.inv_du = dd[1];
  g.U = dd[2];
  g.ncells = 6LL * g.W * g.W;
  return g;
}

int hc_window(const int32_t* GBW, const double* dd, const double* z3, double rt, int maxw,
              int32_t* out5, double* D) {
  GridP g = gp(GBW, dd);
  V3 z = V3{z3[0], z3[1], z3[2]};
  int f = home_face(z);
  Window w = make_window(g, z, f, rt, maxw);
  out5[0] = w.f;
  out5[1] = w.ia_lo;
  out5[2] = w.ia_hi;
  out5[3] = w.ib_lo;
  out5[4] = w.ib_hi;
  *D = w.D;
  return 0;
}

int hc_cell_on_face(const int32_t* GBW, const double* dd, int64_t n, const double* P, int f,
                    int64_t* out) {
  GridP g = gp(GBW, dd);
  for (int64_t k = 0; k < n; k++) out[k] = cell_on_face(g, V3{P[3 * k], P[3 * k + 1], P[3 * k + 2]}, f);
  return 0;
}

int hc_home_face(int64_t n, const double* P, int32_t* out) {
  for (int64_t k = 0; k < n; k++) out[k] = home_face(V3{P[3 * k], P[3 * k + 1], P[3 * k + 2]});
  return 0;
}

}  // extern "C"

extern "C" {
// the table-driven exponential of the FP64 density path, 2^(u/128)
int hc_exp(int64_t n, const double* u, double* out) {
  for (int64_t k = 0; k < n; k++) out[k] = exp2_n(u[k]);
  return 0;
}
}

extern "C" {
// leaves of two subdivision levels: recursive (subtriangle) and from the
// shared 15-point grid; out[s * 18 + 0..8] recursive, +9..17 grid
int hc_leaves2(const double* abc, double* out) {
  V3 A = V3{abc[0], abc[1], abc[2]}, B = V3{abc[3], abc[4], abc[5]},
     C = V3{abc[6], abc[7], abc[8]};
  V3 P[15];
  grid2_points(A, B, C, P);
  for (int s = 0; s < 16; s++) {
    V3 a = A, b = B, c = C;
    subtriangle(a, b, c, s, 2);
    V3 g[3] = {P[nib(kG2LeafA, s)], P[nib(kG2LeafB, s)], P[nib(kG2LeafC, s)]};
    V3 r[3] = {a, b, c};
    for (int v = 0; v < 3; v++) {
      out[s * 18 + 3 * v] = r[v].x;
      out[s * 18 + 3 * v + 1] = r[v].y;
      out[s * 18 + 3 * v + 2] = r[v].z;
      out[s * 18 + 9 + 3 * v] = g[v].x;
      out[s * 18 + 9 + 3 * v + 1] = g[v].y;
      out[s * 18 + 9 + 3 * v + 2] = g[v].z;
    }
  }
  return 0;
}
}

