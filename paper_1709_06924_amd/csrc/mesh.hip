// Mesh operations on the cells of the current generators.
//
// Triangle list (the Delaunay triangulation the paper exports at the end of
// its algorithm, section 3.3): the edge of cell i shared with j ends at the
// Voronoi vertex of the triangle (i, j, k), where k is the neighbour across
// the next edge counter-clockwise (the one starting at that vertex).  Each
// triangle is listed once, by its smallest index i, as (i, j, k)
// counter-clockwise seen from outside, ordered by i then j.
// Quality (section 4): cellQ = min / max edge of a cell, triQ =
// (a+b-c)(b+c-a)(c+a-b)/(abc); chord lengths.
//
// Bisection (the optimisation-bisection initialisation of section 3.3, used
// from 2,562 to 655,362 generators in section 4.3): every Delaunay edge
// (i, j) -- a pair of cells sharing a Voronoi edge -- receives the
// normalised midpoint of its generators, so n generators become n + (3n - 6)
// = 4n - 6.  New points are ordered by the edge's smaller index, then the
// larger, so the result does not depend on scheduling.
#include "kernels.h"

namespace scvt {

__global__ void k_refine_count(const int32_t* __restrict__ deg, const int32_t* __restrict__ nbr,
                               int64_t n, int32_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = 0;
  const int d = deg[i];
  for (int k = 0; k < d; k++) c += nbr[i * kVmax + k] > (int32_t)i ? 1 : 0;
  cnt[i] = c;
}

__global__ void k_refine_emit(const double* __restrict__ Z, const int32_t* __restrict__ deg,
                              const int32_t* __restrict__ nbr, const int32_t* __restrict__ off,
                              int64_t n, double* __restrict__ out) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const V3 zi = V3{Z[3 * i], Z[3 * i + 1], Z[3 * i + 2]};
  out[3 * i] = zi.x;
  out[3 * i + 1] = zi.y;
  out[3 * i + 2] = zi.z;
  int64_t o = n + off[i];
  const int d = deg[i];
  for (int k = 0; k < d; k++) {  // neighbours are stored in increasing index order
    const int64_t j = nbr[i * kVmax + k];
    if (j <= i) continue;
    const V3 m = normalized(zi + V3{Z[3 * j], Z[3 * j + 1], Z[3 * j + 2]});
    out[3 * o] = m.x;
    out[3 * o + 1] = m.y;
    out[3 * o + 2] = m.z;
    o++;
  }
}

// the neighbour across the edge of cell i that starts where edge k ends
__device__ inline int next_neighbour(const double* __restrict__ edges,
                                     const int32_t* __restrict__ nbr, int64_t i, int d, int k) {
  const double* ek = edges + (i * kVmax + k) * 6;
  const V3 v1 = V3{ek[3], ek[4], ek[5]};
  int best = 0;
  double bd = 1e300;
  for (int t = 0; t < d; t++) {  // the shared vertex is computed from the same triple: equal
    const double* et = edges + (i * kVmax + t) * 6;
    const V3 dv = V3{et[0], et[1], et[2]} - v1;
    const double dd = dot(dv, dv);
    if (dd < bd) {
      bd = dd;
      best = t;
    }
  }
  return nbr[i * kVmax + best];
}

__global__ void k_tri_list(const int32_t* __restrict__ deg, const int32_t* __restrict__ nbr,
                           const double* __restrict__ edges, int64_t n,
                           const int32_t* __restrict__ off, int32_t* __restrict__ cnt,
                           int32_t* __restrict__ tri) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int d = deg[i];
  int c = 0;
  for (int k = 0; k < d; k++) {
    const int32_t j = nbr[i * kVmax + k];
    if (j <= (int32_t)i) continue;
    const int32_t kk = next_neighbour(edges, nbr, i, d, k);
    if (kk <= (int32_t)i) continue;
    if (tri) {
      const int64_t o = off[i] + c;
      tri[3 * o] = (int32_t)i;
      tri[3 * o + 1] = j;
      tri[3 * o + 2] = kk;
    }
    c++;
  }
  if (cnt) cnt[i] = c;
}

__global__ void k_cell_quality(const int32_t* __restrict__ deg, const double* __restrict__ edges,
                               int64_t n, double* __restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int d = deg[i];
  double lo = 1e300, hi = 0.0;
  for (int k = 0; k < d; k++) {
    const double* e = edges + (i * kVmax + k) * 6;
    const V3 dv = V3{e[3] - e[0], e[4] - e[1], e[5] - e[2]};
    const double l = sqrt(dot(dv, dv));
    lo = fmin(lo, l);
    hi = fmax(hi, l);
  }
  q[i] = d > 0 ? lo / hi : 0.0;
}

__global__ void k_tri_quality(const double* __restrict__ Z, const int32_t* __restrict__ tri,
                              int64_t ntri, double* __restrict__ q) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntri) return;
  const int64_t i0 = tri[3 * t], i1 = tri[3 * t + 1], i2 = tri[3 * t + 2];
  const V3 A = V3{Z[3 * i0], Z[3 * i0 + 1], Z[3 * i0 + 2]};
  const V3 B = V3{Z[3 * i1], Z[3 * i1 + 1], Z[3 * i1 + 2]};
  const V3 C = V3{Z[3 * i2], Z[3 * i2 + 1], Z[3 * i2 + 2]};
  const V3 ea = C - B, eb = A - C, ec = B - A;
  const double a = sqrt(dot(ea, ea)), b = sqrt(dot(eb, eb)), c = sqrt(dot(ec, ec));
  q[t] = (a + b - c) * (b + c - a) * (c + a - b) / (a * b * c);
}

hipError_t launch_tri_list(const int32_t* deg, const int32_t* nbr, const double* edges, int64_t n,
                           const int32_t* off, int32_t* cnt, int32_t* tri, hipStream_t s) {
  k_tri_list<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(deg, nbr, edges, n, off, cnt, tri);
  return hipGetLastError();
}
hipError_t launch_cell_quality(const int32_t* deg, const double* edges, int64_t n, double* q,
                               hipStream_t s) {
  k_cell_quality<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(deg, edges, n, q);
  return hipGetLastError();
}
hipError_t launch_tri_quality(const double* Z, const int32_t* tri, int64_t ntri, double* q,
                              hipStream_t s) {
  if (ntri <= 0) return hipSuccess;
  k_tri_quality<<<(unsigned)((ntri + 255) / 256), 256, 0, s>>>(Z, tri, ntri, q);
  return hipGetLastError();
}

hipError_t launch_refine_count(const int32_t* deg, const int32_t* nbr, int64_t n, int32_t* cnt,
                               hipStream_t s) {
  k_refine_count<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(deg, nbr, n, cnt);
  return hipGetLastError();
}

hipError_t launch_refine_emit(const double* Z, const int32_t* deg, const int32_t* nbr,
                              const int32_t* off, int64_t n, double* out, hipStream_t s) {
  k_refine_emit<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(Z, deg, nbr, off, n, out);
  return hipGetLastError();
}

}  // namespace scvt
