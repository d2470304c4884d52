// Cube-map bucketing of the generators (counting sort by cell).
//
// count:   every generator adds itself to its home cell and to the ghost
//          border of each neighbouring face whose extended grid holds it;
// scan:    exclusive prefix sums of the counts (three-kernel block scan);
// scatter: positions are taken by decrementing the counts back to zero, so
//          the counts are ready for the next evaluation without a memset.
// Both passes take the generators in the previous build's order (by home
// cell) and aggregate per block (see k_grid_count).
#include "kernels.h"

namespace scvt {

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t count) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; t < count; t += (int64_t)gridDim.x * blockDim.x) p[t] = v;
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  k_fill_i32<<<(unsigned)blocks, 256, 0, s>>>(p, v, count);
  return hipGetLastError();
}

__global__ void k_fill_gamma(double* p, int64_t count, const double* dscal, int r_at, int yy_at) {
  const double g = r_at < 0 ? 1.0 : 1.0 / (dscal[r_at] * dscal[yy_at]);
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; t < count; t += (int64_t)gridDim.x * blockDim.x) p[t] = g;
}

hipError_t launch_fill_gamma(double* p, int64_t count, const double* dscal, int r_at, int yy_at,
                             hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_fill_gamma<<<(unsigned)blocks, 256, 0, s>>>(p, count, dscal, r_at, yy_at);
  return hipGetLastError();
}

// trial point: Zt = normalize(Z + alpha q) (q == nullptr: normalize Z)
template <class P>
__global__ void k_normalize_trial(P p) {
#pragma clang fp contract(off)
  if (p.idle()) return;
  const NormArgs& a = p.args();
  const double* __restrict__ Z = a.Z;
  const double* __restrict__ q = a.q;
  double* __restrict__ Zt = a.Zt;
  const double alpha = a.alpha;
  int64_t i = (int64_t)p.bx() * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  V3 z = V3{Z[3 * i], Z[3 * i + 1], Z[3 * i + 2]};
  // z + alpha q with one rounding per operation, then z / |z|
  if (q) z = z + alpha * V3{q[3 * i], q[3 * i + 1], q[3 * i + 2]};
  V3 w = normalized(z);
  Zt[3 * i] = w.x;
  Zt[3 * i + 1] = w.y;
  Zt[3 * i + 2] = w.z;
}

int normalize_grid(int64_t n) { return (int)((n + 255) / 256); }

hipError_t launch_normalize_trial(const double* Z, const double* q, double alpha, double* Zt,
                                  int64_t n, hipStream_t s) {
  const NormArgs a = {Z, q, alpha, Zt, n};
  k_normalize_trial<<<(unsigned)normalize_grid(n), 256, 0, s>>>(One<NormArgs>{a});
  return hipGetLastError();
}

hipError_t launch_normalize_trial_many(const Seg<NormArgs>& g, hipStream_t s) {
  k_normalize_trial<<<dim3(g.maxnb, g.nseg), 256, 0, s>>>(Many<NormArgs>{g.tab, g.nb});
  return hipGetLastError();
}

// the four faces sharing an edge with face f (all but f and its opposite)
__device__ inline void side_faces(int f, int out[4]) {
  int k = f >> 1, c = 0;
  for (int g = 0; g < 6; g++)
    if ((g >> 1) != k) out[c++] = g;
}

// Generators are taken in the previous build's cell order, so a block's
// 256 generators fall into few grid cells (dense regions hold tens of
// generators per cell).  Each block counts its cells in a small LDS hash
// table and adds one device-scope atomic per distinct cell instead of one
// per generator; the scatter reserves one contiguous range per (block, cell)
// the same way and places its entries by LDS ranks.
constexpr int kBucketBlock = 256;
constexpr int kHashSize = 1024;  // > 3 cells x 256 generators: probing ends

struct BucketLds {
  int32_t key[kHashSize];
  int32_t ntot[kHashSize], nhome[kHashSize];
  int32_t btot[kHashSize], bhome[kHashSize];  // reserved range starts (scatter)
};

__device__ inline int hash_slot(BucketLds& L, int32_t c) {
  uint32_t h = ((uint32_t)c * 2654435761u) >> 22;  // 10 bits
  for (;;) {
    const int32_t k = atomicCAS(&L.key[h], -1, c);
    if (k == -1 || k == c) return (int)h;
    h = (h + 1) & (kHashSize - 1);
  }
}

__device__ inline void bucket_init(BucketLds& L) {
  for (int s = threadIdx.x; s < kHashSize; s += blockDim.x) {
    L.key[s] = -1;
    L.ntot[s] = 0;
    L.nhome[s] = 0;
  }
  __syncthreads();
}

// home cell and up to two ghost cells of generator i (cell3 row)
__device__ inline void generator_cells(const double* __restrict__ Z, int64_t i, const GridP& g,
                                       int32_t out[3]) {
  V3 p = V3{Z[3 * i], Z[3 * i + 1], Z[3 * i + 2]};
  int f = home_face(p);
  int64_t c = cell_on_face(g, p, f);
  // a point always lies inside its home face (|u|,|v| <= 1); guard the
  // index anyway against rounding at the face edge
  if (c < 0) {
    double nn, u, v;
    face_local(p, f, nn, u, v);
    const double ni = rcp_fast(nn);
    double fa = floor((u * ni + g.U) * g.inv_du);
    double fb = floor((v * ni + g.U) * g.inv_du);
    int ia = fa < 0.0 ? 0 : (fa > g.W - 1 ? g.W - 1 : (int)fa);
    int ib = fb < 0.0 ? 0 : (fb > g.W - 1 ? g.W - 1 : (int)fb);
    c = cell_of(g, f, ia, ib);
  }
  out[0] = (int32_t)c;
  int k = 1;
  int sf[4];
  side_faces(f, sf);
  for (int t = 0; t < 4 && g.B > 0; t++) {
    int64_t cg = cell_on_face(g, p, sf[t]);
    if (cg >= 0 && k < 3) out[k++] = (int32_t)cg;
  }
  for (; k < 3; k++) out[k] = -1;
}

// a cell's two counts as one 64-bit word (entries in the low half, home
// entries in the high half; neither exceeds 2^31, so no carry or borrow
// crosses the halves)
__device__ inline unsigned long long pack2(int32_t tot, int32_t home) {
  return (unsigned long long)(uint32_t)tot | ((unsigned long long)(uint32_t)home << 32);
}

template <class P>
__global__ __launch_bounds__(kBucketBlock) void k_grid_count(P p) {
  if (p.idle()) return;
  const GridBuildArgs& a = p.args();
  const double* __restrict__ Z = a.Z;
  const int64_t n = a.n;
  const GridP& g = a.gb.g;
  const int32_t* __restrict__ order_prev = a.gb.order_prev;
  unsigned long long* __restrict__ cnt2 = reinterpret_cast<unsigned long long*>(a.gb.cnt2);
  int32_t* __restrict__ cell3 = a.gb.cell3;
  int32_t* __restrict__ clear = a.clear;
  __shared__ BucketLds L;
  if (clear && p.bx() == 0 && threadIdx.x < 8) clear[threadIdx.x] = 0;
  bucket_init(L);
  const int64_t t = (int64_t)p.bx() * blockDim.x + threadIdx.x;
  if (t < n) {
    const int64_t i = order_prev[t];
    int32_t c[3];
    generator_cells(Z, i, g, c);
    for (int k = 0; k < 3; k++) {
      cell3[3 * t + k] = c[k];  // by position: the scatter reads it back coalesced
      if (c[k] < 0) continue;
      const int s = hash_slot(L, c[k]);
      atomicAdd(&L.ntot[s], 1);
      if (k == 0) atomicAdd(&L.nhome[s], 1);
    }
  }
  __syncthreads();
  for (int s = threadIdx.x; s < kHashSize; s += blockDim.x) {
    const int32_t c = L.key[s];
    if (c < 0) continue;
    atomicAdd(&cnt2[c], pack2(L.ntot[s], L.nhome[s]));
  }
}

// ---- exclusive scan of two int arrays of length m (m+1 outputs) ----
constexpr int kScanItems = 8;
constexpr int kScanBlock = 256;
constexpr int kScanTile = kScanItems * kScanBlock;

__device__ inline int block_exclusive_scan(int v, int* sh, int& total) {
  // Hillis-Steele in shared memory over 256 threads
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    int add = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  total = sh[kScanBlock - 1];
  int excl = sh[t] - v;
  __syncthreads();
  return excl;
}

// pass 1: per-tile sums of both arrays
template <class P>
__global__ void k_scan_tiles(P p) {
  if (p.idle()) return;
  const ScanArgs& A = p.args();
  const int32_t* __restrict__ a = A.a;
  const int32_t* __restrict__ b = A.b;
  const int64_t m = A.m;
  int32_t* __restrict__ sums = A.sums;
  __shared__ int sh[kScanBlock];
  int64_t base = (int64_t)p.bx() * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int sa = 0, sb = 0;
  const int64_t st = A.stride;
  for (int k = 0; k < kScanItems; k++) {
    int64_t t = base + k;
    if (t < m) {
      sa += a[t * st];
      sb += b[t * st];
    }
  }
  int tot;
  block_exclusive_scan(sa, sh, tot);
  if (threadIdx.x == 0) sums[2 * p.bx()] = tot;
  block_exclusive_scan(sb, sh, tot);
  if (threadIdx.x == 0) sums[2 * p.bx() + 1] = tot;
}

// pass 2: exclusive scan of the tile sums by one block (loops over chunks)
template <class P>
__global__ void k_scan_sums(P p) {
  if (p.idle()) return;
  int32_t* sums = p.args().sums;
  const int64_t ntiles = p.args().ntiles;
  __shared__ int sh[kScanBlock];
  int carry_a = 0, carry_b = 0;
  for (int64_t c0 = 0; c0 < ntiles; c0 += kScanBlock) {
    int64_t t = c0 + threadIdx.x;
    int va = t < ntiles ? sums[2 * t] : 0;
    int vb = t < ntiles ? sums[2 * t + 1] : 0;
    int ta, tb;
    int ea = block_exclusive_scan(va, sh, ta);
    int eb = block_exclusive_scan(vb, sh, tb);
    if (t < ntiles) {
      sums[2 * t] = ea + carry_a;
      sums[2 * t + 1] = eb + carry_b;
    }
    carry_a += ta;
    carry_b += tb;
  }
}

// pass 3: scan inside each tile, add the tile offset; element m gets the total
template <class P>
__global__ void k_scan_apply(P p) {
  if (p.idle()) return;
  const ScanArgs& A = p.args();
  const int32_t* __restrict__ a = A.a;
  const int32_t* __restrict__ b = A.b;
  const int64_t m = A.m;
  const int32_t* __restrict__ sums = A.sums;
  int32_t* __restrict__ oa = A.oa;
  int32_t* __restrict__ ob = A.ob;
  __shared__ int sh[kScanBlock];
  int64_t base = (int64_t)p.bx() * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int va[kScanItems], vb[kScanItems];
  int sa = 0, sb = 0;
  const int64_t st = A.stride;
  for (int k = 0; k < kScanItems; k++) {
    int64_t t = base + k;
    va[k] = t < m ? a[t * st] : 0;
    vb[k] = t < m ? b[t * st] : 0;
    sa += va[k];
    sb += vb[k];
  }
  int tot;
  int ea = block_exclusive_scan(sa, sh, tot) + sums[2 * p.bx()];
  int eb = block_exclusive_scan(sb, sh, tot) + sums[2 * p.bx() + 1];
  for (int k = 0; k < kScanItems; k++) {
    int64_t t = base + k;
    if (t <= m) {
      oa[t] = ea;
      ob[t] = eb;
    }
    ea += va[k];
    eb += vb[k];
  }
}

template <class P>
__global__ __launch_bounds__(kBucketBlock) void k_grid_scatter(P p) {
  if (p.idle()) return;
  const GridBuildArgs& a = p.args();
  const double* __restrict__ Z = a.Z;
  const int64_t n = a.n;
  const int32_t* __restrict__ order_prev = a.gb.order_prev;
  const int32_t* __restrict__ cell3 = a.gb.cell3;
  const int32_t* __restrict__ start_tot = a.gb.start_tot;
  const int32_t* __restrict__ start_home = a.gb.start_home;
  unsigned long long* cnt2 = reinterpret_cast<unsigned long long*>(a.gb.cnt2);
  Entry* __restrict__ entries = a.gb.entries;
  const int64_t cap = a.gb.cap_entries;
  int32_t* __restrict__ order = a.gb.order;
  int32_t* overflow = a.gb.overflow;
  __shared__ BucketLds L;
  bucket_init(L);
  const int64_t t = (int64_t)p.bx() * blockDim.x + threadIdx.x;
  const bool valid = t < n;
  const int64_t i = valid ? order_prev[t] : 0;
  int32_t c[3] = {-1, -1, -1};
  int slot[3] = {0, 0, 0};
  if (valid) {
    for (int k = 0; k < 3; k++) {
      c[k] = cell3[3 * t + k];
      if (c[k] >= 0) slot[k] = hash_slot(L, c[k]);
    }
    for (int k = 0; k < 3; k++) {
      if (c[k] < 0) continue;
      atomicAdd(&L.ntot[slot[k]], 1);
      if (k == 0) atomicAdd(&L.nhome[slot[k]], 1);
    }
  }
  __syncthreads();
  // reserve this block's range in every cell: the counts run down to zero
  // over all blocks (ready for the next build)
  for (int s = threadIdx.x; s < kHashSize; s += blockDim.x) {
    const int32_t cs = L.key[s];
    if (cs < 0) continue;
    const unsigned long long v = pack2(L.ntot[s], L.nhome[s]);
    const unsigned long long old = atomicAdd(&cnt2[cs], 0ull - v);  // both counts down at once
    L.btot[s] = (int32_t)(uint32_t)old - L.ntot[s];
    L.bhome[s] = (int32_t)(uint32_t)(old >> 32) - L.nhome[s];
    L.ntot[s] = 0;  // reused as the in-block rank counters
    L.nhome[s] = 0;
  }
  __syncthreads();
  if (!valid) return;
  Entry en;
  en.x = Z[3 * i];
  en.y = Z[3 * i + 1];
  en.z = Z[3 * i + 2];
  en.idx = (int32_t)i;
  en.pad = 0;
  for (int k = 0; k < 3; k++) {
    if (c[k] < 0) continue;
    const int s = slot[k];
    const int32_t pos = start_tot[c[k]] + L.btot[s] + atomicAdd(&L.ntot[s], 1);
    if (pos < cap) {
      entries[pos] = en;
    } else {
      atomicOr(overflow, 1);
    }
    if (k == 0) order[start_home[c[k]] + L.bhome[s] + atomicAdd(&L.nhome[s], 1)] = (int32_t)i;
  }
}

__global__ void k_iota(int32_t* p, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = (int32_t)t;
}

hipError_t launch_iota(int32_t* p, int64_t n, hipStream_t s) {
  k_iota<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
  return hipGetLastError();
}

__global__ void k_centroid(const double* __restrict__ mu, const double* __restrict__ m,
                           double* __restrict__ out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < 3; k++) out[3 * i + k] = mu[3 * i + k] / m[i];
}

hipError_t launch_centroid(const double* mu, const double* m, double* out, int64_t n,
                           hipStream_t s) {
  k_centroid<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(mu, m, out, n);
  return hipGetLastError();
}

int64_t scan_tiles(int64_t m) { return (m + 1 + kScanTile - 1) / kScanTile; }

hipError_t launch_scan_pair(const int32_t* a, const int32_t* b, int64_t m, int32_t* tmp,
                            int32_t* oa, int32_t* ob, hipStream_t s) {
  const int64_t ntiles = scan_tiles(m);
  const ScanArgs sa = {a, b, m, tmp, oa, ob, ntiles, 1};
  k_scan_tiles<<<(unsigned)ntiles, kScanBlock, 0, s>>>(One<ScanArgs>{sa});
  k_scan_sums<<<1, kScanBlock, 0, s>>>(One<ScanArgs>{sa});
  k_scan_apply<<<(unsigned)ntiles, kScanBlock, 0, s>>>(One<ScanArgs>{sa});
  return hipGetLastError();
}

int64_t scan_tmp_ints(int64_t m) { return 2 * ((m + 1 + kScanTile - 1) / kScanTile + 1); }

int bucket_grid(int64_t n) { return (int)((n + kBucketBlock - 1) / kBucketBlock); }

ScanArgs grid_scan_args(const GridBufs& gb) {
  const int64_t m = gb.g.ncells;
  return ScanArgs{gb.cnt2, gb.cnt2 + 1, m, gb.scan_tmp, gb.start_tot, gb.start_home,
                  scan_tiles(m), 2};
}

hipError_t launch_grid_build(const double* Z, int64_t n, GridBufs& gb, int32_t* clear,
                             hipStream_t s) {
  const GridBuildArgs a = {Z, n, gb, clear};
  const ScanArgs sa = grid_scan_args(gb);
  const unsigned nb = (unsigned)bucket_grid(n);
  k_grid_count<<<nb, kBucketBlock, 0, s>>>(One<GridBuildArgs>{a});
  k_scan_tiles<<<(unsigned)sa.ntiles, kScanBlock, 0, s>>>(One<ScanArgs>{sa});
  k_scan_sums<<<1, kScanBlock, 0, s>>>(One<ScanArgs>{sa});
  k_scan_apply<<<(unsigned)sa.ntiles, kScanBlock, 0, s>>>(One<ScanArgs>{sa});
  k_grid_scatter<<<nb, kBucketBlock, 0, s>>>(One<GridBuildArgs>{a});
  return hipGetLastError();
}

hipError_t launch_grid_build_many(const Seg<GridBuildArgs>& g, const Seg<ScanArgs>& tiles,
                                  const Seg<ScanArgs>& one, hipStream_t s) {
  k_grid_count<<<dim3(g.maxnb, g.nseg), kBucketBlock, 0, s>>>(Many<GridBuildArgs>{g.tab, g.nb});
  k_scan_tiles<<<dim3(tiles.maxnb, tiles.nseg), kScanBlock, 0, s>>>(
      Many<ScanArgs>{tiles.tab, tiles.nb});
  k_scan_sums<<<dim3(one.maxnb, one.nseg), kScanBlock, 0, s>>>(Many<ScanArgs>{one.tab, one.nb});
  k_scan_apply<<<dim3(tiles.maxnb, tiles.nseg), kScanBlock, 0, s>>>(
      Many<ScanArgs>{tiles.tab, tiles.nb});
  k_grid_scatter<<<dim3(g.maxnb, g.nseg), kBucketBlock, 0, s>>>(Many<GridBuildArgs>{g.tab, g.nb});
  return hipGetLastError();
}

}  // namespace scvt
