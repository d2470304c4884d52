/*
 * Driver for a sanitizer build of the oracle's C integrals (AddressSanitizer
 * and UndefinedBehaviorSanitizer, host code only): the six cells of the
 * octahedron under every density kind and the 7- and 4-point rules, single
 * triangles at several subdivision levels, and the density at many points.
 * Exit status 0 when every total is finite and the constant density's cells
 * add up to 4 pi; the sanitizers abort on the first error.
 */
#include <math.h>
#include <stdio.h>

#include "../../oracle/scvt_oracle.c"

int main(void) {
  /* generator s e_k: cell vertices (+-1, +-1, +-1)/sqrt(3) with coordinate
   * k equal to s, counter-clockwise seen from outside */
  double Z[18], V[72];
  int64_t ptr[7];
  const double r3 = 1.0 / sqrt(3.0);
  int nv = 0;
  for (int g = 0; g < 6; g++) {
    const int k = g / 2;
    const double s = (g % 2) ? -1.0 : 1.0;
    for (int c = 0; c < 3; c++) Z[3 * g + c] = c == k ? s : 0.0;
    ptr[g] = nv;
    const int a = (k + 1) % 3, b = (k + 2) % 3;
    const double sa[4] = {1, -1, -1, 1}, sb[4] = {1, 1, -1, -1};
    for (int t = 0; t < 4; t++) {
      const int tt = s > 0 ? t : 3 - t;
      double v[3];
      v[k] = s * r3;
      v[a] = sa[tt] * r3;
      v[b] = sb[tt] * r3;
      for (int c = 0; c < 3; c++) V[3 * nv + c] = v[c];
      nv++;
    }
  }
  ptr[6] = nv;
  oracle_density D[4] = {{0}};
  D[0].kind = ORACLE_RHO_CONST;
  D[1].kind = ORACLE_RHO_TANH;
  D[1].nbumps = 2;
  for (int b = 0; b < 2; b++) {
    D[1].xc[b][0] = 0.6;
    D[1].xc[b][1] = b ? -0.8 : 0.8;
    D[1].beta[b] = 0.5;
    D[1].alpha[b] = 0.2;
    D[1].amp[b] = 0.5;
  }
  D[1].gamma = 1e-4;
  D[2].kind = ORACLE_RHO_X3;
  D[2].gamma = 1.0 / 81.0;
  D[3].kind = ORACLE_RHO_X16;
  D[3].xc[0][0] = 1.0;
  D[3].beta[0] = 0.5;
  D[3].alpha[0] = 0.3;
  D[3].amp[0] = 1.0;
  D[3].gamma = 1e-5;
  D[3].w_lon = 0.3;
  D[3].w_lat = 1.2;
  oracle_rule R4 = {0};
  R4.nq = 4;
  const double l4[4][3] = {{0.6, 0.2, 0.2}, {0.2, 0.6, 0.2}, {0.2, 0.2, 0.6}, {1.0 / 3, 1.0 / 3, 1.0 / 3}};
  for (int q = 0; q < 4; q++) {
    for (int c = 0; c < 3; c++) R4.lam[3 * q + c] = l4[q][c];
    R4.w[q] = 0.25;
  }
  double m[6], mu[18], e[6];
  int bad = 0;
  for (int d = 0; d < 4; d++) {
    for (int rule = 0; rule < 2; rule++) {
      for (int lv = 0; lv <= 2; lv++) {
        oracle_cell_integrals(6, Z, ptr, V, &D[d], lv, rule ? &R4 : NULL, m, mu, e);
        double tot = 0.0;
        for (int i = 0; i < 6; i++) {
          if (!isfinite(m[i]) || !isfinite(e[i]) || !(m[i] > 0.0)) bad++;
          tot += m[i];
        }
        if (d == 0 && rule == 0 && lv == 2 && fabs(tot - 4.0 * M_PI) > 1e-5) bad++;  /* 4.3e-6 at L = 2 */
      }
    }
    double Y[30], out[10];
    for (int k = 0; k < 10; k++) {
      const double t = 0.6 * k;
      Y[3 * k] = cos(t) * 0.6;
      Y[3 * k + 1] = sin(t) * 0.6;
      Y[3 * k + 2] = 0.8;
    }
    oracle_rho_many(&D[d], 10, Y, out);
    for (int k = 0; k < 10; k++)
      if (!(out[k] > 0.0)) bad++;
    double tri[5];
    oracle_triangle_integrals(&D[d], Z, Z, Z + 6, Z + 12, 3, NULL, tri);
    if (!isfinite(tri[0])) bad++;
  }
  oracle_set_num_threads(2);
  printf("oracle sanitizer run: %d threads, %d failures\n", oracle_num_threads(), bad);
  return bad ? 1 : 0;
}
