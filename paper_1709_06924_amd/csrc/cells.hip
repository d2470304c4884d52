// Voronoi cell construction, cell quadrature and per-cell epilogue.
//
// k_cells_geom: a group of 8 lanes per generator z (eight per wavefront),
// in cube-map order (neighbouring groups share cached grid data), blocks
// dealt to the XCDs in chunks of neighbouring cells.
//   A. candidates: every generator within chord radius rc of z, read from a
//      rectangle of grid cells whose certified radius D >= rc (at most 16);
//   B. each lane takes two candidates j and computes the edge of the cell on
//      the bisector of (z, p_j) against all other candidates
//      (edge_on_bisector);
//   C. certificate: the cell's circumradius R obeys 2R <= rc, so no
//      generator outside the candidate set can cut the cell (a point p can
//      only cut if |p - z| < 2R); otherwise the radius grows and A-C repeat.
//   The edges (vertex pairs, ordered by neighbour index) go to the cell's
//   slot in HBM.  Cells that cannot be certified with 16 candidates go to
//   the list passes k_cells_tier (32, then 64 candidates, one per lane);
//   what those cannot certify, or meets a predicate within its error bound,
//   goes to a list for
// k_fallback: a sequential half-space clipper run by lane 0 (no size limit:
//   any cell the sphere allows), writing the same slot.
// k_quad: one cell per half-wave, cells sorted by degree within a block:
//   fan triangles (z, v_lo, v_hi), each split into 4^levels geodesic
//   sub-triangles with the triangle rule, one (edge, sub-triangle) item per
//   lane; m, mu, e per cell (g, h and the Lloyd step of section 3.1 follow
//   in the evaluation's reduction pass).
#include "kernels.h"

namespace scvt {

// ------------------------------------------------------------- wave tools
__device__ inline int lane_id() { return threadIdx.x & 63; }
__device__ inline int mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ inline double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ inline int wave_sum_i(int v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Logical block for a physical one: consecutive physical blocks go to
// different XCDs (8 of them, round robin), so give each XCD whole chunks of
// kXcdChunk consecutive logical blocks (neighbouring cells share their
// windows' grid data in its L2), dealt out in turn: chunk c to XCD c mod 8.
// Contiguous eighths would leave the XCD holding a dense region (whose
// windows hold more generators) the last to finish.  The grid is padded to
// a multiple of 8 kXcdChunk blocks, so the map is a bijection; logical
// blocks past the end have no work.
constexpr int64_t kXcdChunk = 16;
__device__ inline int64_t xcd_block(int64_t b) {
  const int64_t x = b % 8, k = b / 8;
  return ((k / kXcdChunk) * 8 + x) * kXcdChunk + k % kXcdChunk;
}

// ------------------------------------------------------------- edge slots
// Edge k of cell i (ordered by neighbour index): vertices v0 -> v1,
// counter-clockwise seen from outside, at edges[(i * kVmax + k) * 6 ...].
__device__ inline void store_edge(const EvalOut& o, int64_t i, int k, V3 v0, V3 v1, int nbr,
                                  int keep) {
  double* e = o.edges + (i * kVmax + k) * 6;
  e[0] = v0.x;
  e[1] = v0.y;
  e[2] = v0.z;
  e[3] = v1.x;
  e[4] = v1.y;
  e[5] = v1.z;
  if (keep) o.cell_nbr[i * kVmax + k] = nbr;
}

// ---------------------------------------------------------- certified path
// A cell is built by a group of GS lanes holding at most CAP candidates
// (CAP / GS per lane) from a window of at most ROWS x ROWS grid cells.
// Once the generators are spread evenly a cell has 6-8 candidates, so the
// main kernel uses groups of 8 lanes (eight cells per wave, 16 candidates);
// cells that need more go through two list passes, 16 lanes / 32
// candidates, then a whole wave / 64 candidates, and only what those cannot
// certify to the fallback clipper.
template <int GS, int CAP, int ROWS>
struct CandLds {
  double px[CAP], py[CAP], pz[CAP], dx[CAP], dy[CAP], dz[CAP], nrm[CAP], zd[CAP];
  int32_t idx[CAP];
  int32_t rowoff[ROWS + 1];
  int32_t rowstart[ROWS];
};

template <int GS>
__device__ inline double group_max(double v) {
  for (int off = GS / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}
template <int GS>
__device__ inline int group_scan_incl(int v, int gl) {
  for (int off = 1; off < GS; off <<= 1) {
    int t = __shfl_up(v, off, GS);
    if (gl >= off) v += t;
  }
  return v;
}

// Lanes of one group: gl = lane within the group, gid = group within the
// wave, gm = the group's lanes as a wave mask.
struct GroupPos {
  int gl, gid;
  uint64_t gm;
};
template <int GS>
__device__ inline GroupPos group_pos() {
  const int ln = lane_id();
  GroupPos g;
  g.gl = ln & (GS - 1);
  g.gid = ln / GS;
  g.gm = GS == 64 ? ~0ull : (((1ull << GS) - 1) << (GS * g.gid));
  return g;
}

// Gather every generator p != z with |p - z| < rc from window w into the
// group's candidate arrays; returns the count (> CAP means overflow).  All
// lanes of the wave take part; groups with active == false gather nothing.
template <int GS, int CAP, int ROWS>
__device__ int gather(const CellArgs& a, CandLds<GS, CAP, ROWS>& L, const Window& w, int64_t i, V3 z,
                      double rc2, bool active, const GroupPos& G) {
  const GridP& g = a.grid.g;
  const int nrows = active ? w.ib_hi - w.ib_lo + 1 : 0;
  wave_sync();  // earlier reads of the candidate arrays are done
  int base = 0;
  for (int r0 = 0;; r0 += GS) {
    if (!__ballot(r0 < nrows)) break;
    const int r = r0 + G.gl;
    const bool in = r < nrows;
    int cnt = 0, st = 0;
    if (in) {
      int64_t c0 = cell_of(g, w.f, w.ia_lo, w.ib_lo + r);
      int64_t c1 = cell_of(g, w.f, w.ia_hi, w.ib_lo + r) + 1;
      st = a.grid.start_tot[c0];
      cnt = a.grid.start_tot[c1] - st;
    }
    const int incl = group_scan_incl<GS>(cnt, G.gl);
    if (in) {
      L.rowoff[r] = base + incl - cnt;
      L.rowstart[r] = st;
    }
    base += __shfl(incl, G.gid * GS + GS - 1, 64);
  }
  const int T = base;
  wave_sync();
  int kept = 0;
  for (int t0 = 0;; t0 += GS) {
    if (!__ballot(t0 < T)) break;
    const int t = t0 + G.gl;
    bool keep = false;
    Entry en;
    V3 d;
    if (t < T) {
      int lo = 0, hi = nrows - 1;  // the last row whose offset is <= t
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L.rowoff[mid] <= t) lo = mid;
        else hi = mid - 1;
      }
      en = a.grid.entries[L.rowstart[lo] + (t - L.rowoff[lo])];
      d = V3{en.x - z.x, en.y - z.y, en.z - z.z};
      keep = en.idx != (int32_t)i && dot(d, d) < rc2;
      if (en.idx != (int32_t)i && d.x == 0.0 && d.y == 0.0 && d.z == 0.0) {
        atomicAdd(&a.ctr->n_duplicate, 1);
        keep = false;
      }
    }
    const uint64_t m = __ballot(keep) & G.gm;
    const int slot = kept + mbcnt(m);
    if (keep && slot < CAP) {
      L.px[slot] = en.x;
      L.py[slot] = en.y;
      L.pz[slot] = en.z;
      L.dx[slot] = d.x;
      L.dy[slot] = d.y;
      L.dz[slot] = d.z;
      L.nrm[slot] = sqrt_fast(dot(d, d));
      L.zd[slot] = dot(z, d);
      L.idx[slot] = en.idx;
    }
    kept += __popcll(m);
  }
  wave_sync();
  return kept;
}

enum CellOutcome { kCellOk = 0, kCellDegenerate = 1, kCellOpen = 2 };

// Build and certify cell i (all lanes of the wave call this together; a
// group with valid == false only keeps step).  Search radius: grow to
// min(2.1 R, 1.6 r) after an uncertified attempt and to 1.6 r after an
// unbounded one; on overflow shrink toward 3/4 CAP candidates, unless that
// is no larger than a radius already found too small (the cell needs more
// than CAP candidates).  Writes the edges, deg, R and flags of a certified
// cell and returns the outcome.
template <int GS, int CAP, int ROWS>
__device__ int build_cell(const CellArgs& a, CandLds<GS, CAP, ROWS>& L, bool valid, int64_t i,
                          const GroupPos& G) {
  constexpr int PER = CAP / GS;
  static_assert(PER * GS == CAP && PER >= 1 && PER <= 2, "one or two candidates per lane");
  const V3 z = valid ? V3{a.Z[3 * i], a.Z[3 * i + 1], a.Z[3 * i + 2]} : V3{0.0, 0.0, 1.0};
  const int f = home_face(z);
  const CandView S = {L.px, L.py, L.pz, L.dx, L.dy, L.dz, L.nrm, L.zd};
  const double Rg = valid ? a.out.R[i] : 0.0;
  double rt = Rg > 0.0 ? 2.3 * Rg : a.r_default;
  double r_small = 0.0;  // largest radius found too small
  double rc_over = 0.0;  // last radius that held more than CAP candidates
  bool active = valid;
  int outcome = kCellOpen, E = 0;
  double R = 0.0;
  for (int attempt = 0; attempt < 8; attempt++) {
    if (!__ballot(active)) break;
    const Window w = make_window(a.grid.g, z, f, rt, ROWS);
    const double rc = rt < w.D ? rt : w.D;
    const int ns = gather<GS, CAP, ROWS>(a, L, w, i, z, rc * rc, active, G);
    bool go = active;
    // the configured cap (a test knob) can only lower the pass's own
    const int cap = a.kmax > 0 && a.kmax < CAP ? a.kmax : CAP;
    if (go && ns > cap) {
      rc_over = rc;
      rt = rc * sqrt_fast(0.75 * cap / (double)ns);
      if (rt <= r_small) active = false;
      go = false;
    }
    EdgeRes er[PER];
    bool anydeg = false, anyunb = false;
    double nm = 0.0;  // the largest |d_l| of the cell's candidates
    for (int k = 0; k < PER; k++) {
      const int j = G.gl + k * GS;
      if (go && j < ns) nm = fmax(nm, L.nrm[j]);
    }
    nm = group_max<GS>(nm);
    for (int k = 0; k < PER; k++) {
      const int j = G.gl + k * GS;
      er[k] = EdgeRes{kEdgeNone, -1, -1};
      if (go && j < ns) er[k] = edge_on_bisector(j, ns, z, S, nm);
      anydeg |= er[k].status == kEdgeDegenerate;
      anyunb |= er[k].status == kEdgeUnbounded;
    }
    if (go && (__ballot(anydeg) & G.gm)) {
      outcome = kCellDegenerate;
      active = false;
      go = false;
    }
    if (go && ((__ballot(anyunb) & G.gm) || ns < 3)) {
      if (rc < rt) active = false;  // the window cannot grow
      r_small = fmax(r_small, rc);
      rt = 1.6 * rc;
      go = false;
    }
    uint64_t em[PER];
    V3 vlo[PER], vhi[PER];
    bool has[PER];
    double r2 = 0.0;
    int En = 0;
    // every vertex once per cell: edge j ends at (j, hi) and starts at
    // (j, lo), the end of edge lo (the same sorted triple, so the same bits)
    for (int k = 0; k < PER; k++) {
      const int j = G.gl + k * GS;
      has[k] = go && er[k].status == kEdgeYes;
      em[k] = __ballot(has[k]) & G.gm;
      En += __popcll(em[k]);
      vhi[k] = V3{0.0, 0.0, 0.0};
      if (has[k]) {
        vhi[k] = circumcentre((int)i, z, L.idx[j], S.p(j), L.idx[er[k].hi], S.p(er[k].hi));
        const V3 q1 = vhi[k] - z;
        r2 = fmax(r2, dot(q1, q1));
      }
    }
    wave_sync();  // the candidates' differences and norms are read no more
    for (int k = 0; k < PER; k++) {
      const int j = G.gl + k * GS;
      if (go && j < ns) {  // edge ends by candidate, and whose end it is
        L.dx[j] = vhi[k].x;
        L.dy[j] = vhi[k].y;
        L.dz[j] = vhi[k].z;
        L.nrm[j] = has[k] ? (double)er[k].hi : -1.0;
      }
    }
    wave_sync();
    bool broken = false;
    for (int k = 0; k < PER; k++) {
      const int j = G.gl + k * GS;
      vlo[k] = V3{0.0, 0.0, 0.0};
      if (has[k]) {
        const int lo = er[k].lo;
        vlo[k] = V3{L.dx[lo], L.dy[lo], L.dz[lo]};
        broken |= L.nrm[lo] != (double)j;  // certified predicates make this impossible
      }
    }
    if (go && (__ballot(broken) & G.gm)) {
      outcome = kCellDegenerate;
      active = false;
      go = false;
    }
    r2 = group_max<GS>(r2);
    bool store = false;
    if (go) {
      R = sqrt(r2);  // as the fallback clipper's, so that R does not depend on the path
      if (4.0 * r2 * (1.0 + 1e-12) <= rc * rc && En >= 3 && En <= kVmax) {
        outcome = kCellOk;
        active = false;
        E = En;
        store = true;
      } else if (rc < rt && 2.0 * R >= w.D) {
        active = false;  // window-limited
      } else {
        // R of an incomplete candidate set overestimates the cell: grow by
        // at most 1.6x per attempt (about 2.5x the candidates)
        r_small = fmax(r_small, rc);
        rt = fmin(2.1 * R, 1.6 * rt);
      }
    }
    if (store) {
      // rank edges by neighbour index (deterministic summation order)
      for (int k = 0; k < PER; k++) {
        const int j = G.gl + k * GS;
        if (!(er[k].status == kEdgeYes)) continue;
        const int me = L.idx[j];
        int rank = 0;
        for (int kk = 0; kk < PER; kk++) {
          uint64_t mm = em[kk] >> (GS == 64 ? 0 : GS * G.gid);
          while (mm) {
            const int t = __builtin_ctzll(mm);
            mm &= mm - 1;
            rank += L.idx[t + kk * GS] < me ? 1 : 0;
          }
        }
        store_edge(a.out, i, rank, vlo[k], vhi[k], me, a.keep_cells);
      }
    }
  }
  // a cell handed on starts the next pass where this one stopped: at the
  // radius that held too many candidates, else at the next one to try
  if (valid && outcome == kCellOpen && G.gl == 0)
    a.out.R[i] = (rc_over > r_small ? rc_over : rt) * (1.0 / 2.3);
  if (valid && outcome == kCellOk) {
    if (G.gl == 0) {
      a.out.deg[i] = E;
      a.out.R[i] = R;
      a.out.flags[i] = 0;
    }
    // the lane recounted from the exec mask's bits below it: reading
    // threadIdx.x again here would keep it live through the whole build
    if (a.keep_cells)
      for (int k = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)) & (GS - 1);
           k < kVmax; k += GS)
        if (k >= E) a.out.cell_nbr[i * kVmax + k] = -1;
  }
  return outcome;
}

__device__ inline void to_list(int32_t* list, int32_t* count, int64_t i) {
  const int k = atomicAdd(count, 1);
  list[k] = (int32_t)i;
}

// where a cell goes when a pass could not certify it: degenerate ones to
// the fallback clipper, the others to the next pass (or the fallback)
__device__ inline void hand_on(const CellArgs& a, int64_t i, int oc, int next_tier) {
  a.out.deg[i] = 0;
  if (oc == kCellDegenerate) atomicAdd(&a.ctr->n_degenerate, 1);
  if (oc == kCellDegenerate || next_tier < 0)
    to_list(a.fb_list, &a.ctr->fb_count, i);
  else
    to_list(a.tier_list[next_tier], &a.ctr->tier_count[next_tier], i);
}

// Main certified pass: eight cells per wave in cube-map order.
template <class P>
__global__ __launch_bounds__(256, 4) void k_cells_geom(P p) {
  if (p.idle()) return;
  const CellArgs& a = p.args();
  constexpr int GS = 8, GPW = 64 / GS;
  __shared__ CandLds<GS, 16, 15> lds[4 * GPW];
  const GroupPos G = group_pos<GS>();
  const int wv = threadIdx.x >> 6;
  const int64_t pos = (xcd_block(p.bx()) * 4 + wv) * GPW + G.gid;
  const bool valid = pos < a.n;
  if (!__ballot(valid)) return;
  const int64_t i = valid ? a.grid.order[pos] : 0;
  const int oc = build_cell(a, lds[wv * GPW + G.gid], valid, i, G);
  if (valid && G.gl == 0 && oc != kCellOk) hand_on(a, i, oc, 0);
}

// List passes: the cells of tier list T, GS lanes each; what stays open
// goes to list T + 1 (or, after the last pass, to the fallback).
template <int T, int GS, int CAP, int ROWS, class P>
__global__ __launch_bounds__(256, 2) void k_cells_tier(P p) {
  if (p.idle()) return;
  const CellArgs& a = p.args();
  constexpr int GPW = 64 / GS;
  __shared__ CandLds<GS, CAP, ROWS> lds[4 * GPW];
  const GroupPos G = group_pos<GS>();
  const int wv = threadIdx.x >> 6;
  const int count = a.ctr->tier_count[T];
  const int stride = p.gx() * 4 * GPW;
  for (int base = (p.bx() * 4 + wv) * GPW; base < count; base += stride) {
    const int w = base + G.gid;
    const bool valid = w < count;
    const int64_t i = valid ? a.tier_list[T][w] : 0;
    const int oc = build_cell(a, lds[wv * GPW + G.gid], valid, i, G);
    if (valid && G.gl == 0 && oc != kCellOk) hand_on(a, i, oc, T + 1 < kTiers ? T + 1 : -1);
  }
}

// ------------------------------------------------------------ fallback path
struct FbLds {
  ClipPoly poly;
  int32_t brute;
  int32_t enbr[kVmax];
  double v0[kVmax][3], v1[kVmax][3];
};

__device__ inline V3 genpos(const double* Z, int j) { return V3{Z[3 * j], Z[3 * j + 1], Z[3 * j + 2]}; }

// Whole wave: offer the generators of `count` candidates (given by a
// callable index -> generator id) to the clipper; lanes prefilter by the
// polygon bound |p - z| < 2R, lane 0 clips by the survivors in lane order.
template <class Src>
__device__ void fb_offer(FbLds& F, const double* Z, V3 z, int64_t self, int64_t count,
                         const Src& src, int32_t* ctr_dup) {
  const int ln = lane_id();
  for (int64_t t0 = 0; t0 < count; t0 += 64) {
    int64_t t = t0 + ln;
    int j = -1;
    bool cand = false;
    if (t < count) {
      j = src(t);
      if (j != (int)self) {
        V3 d = genpos(Z, j) - z;
        double R = F.poly.R;
        cand = dot(d, d) < 4.0 * R * R * (1.0 + 1e-9) + 1e-300;
        if (d.x == 0.0 && d.y == 0.0 && d.z == 0.0) {
          atomicAdd(&ctr_dup[0], 1);  // duplicate generator
          cand = false;
        }
      }
    }
    uint64_t m = __ballot(cand);
    while (m) {
      int k = __builtin_ctzll(m);
      m &= m - 1;
      int jk = __shfl(j, k, 64);
      if (ln == 0) clip_offer(F.poly, z, jk, genpos(Z, jk));
      wave_sync();
    }
  }
}

template <class P>
__global__ __launch_bounds__(64) void k_fallback(P p) {
  if (p.idle()) return;
  const CellArgs& a = p.args();
  __shared__ FbLds F;
  const int ln = lane_id();
  const int count = a.ctr->fb_count;
  for (int64_t w = p.bx(); w < count; w += p.gx()) {
    const int64_t i = a.fb_list[w];
    const V3 z = V3{a.Z[3 * i], a.Z[3 * i + 1], a.Z[3 * i + 2]};
    if (ln == 0) {
      clip_reset(F.poly);
      F.brute = 0;
    }
    wave_sync();
    bool done = false;
    const GridP& g = a.grid.g;
    if (a.n > 256 && g.B > 0) {
      // nearby first: growing windows of the grid
      const int f = home_face(z);
      double rt = a.out.R[i] > 0.0 ? 2.3 * a.out.R[i] : a.r_default;
      for (int it = 0; it < 6 && !done; it++) {
        Window win = make_window(g, z, f, rt, kWinMax);
        const int nrows = win.ib_hi - win.ib_lo + 1;
        for (int r = 0; r < nrows; r++) {
          int64_t c0 = cell_of(g, f, win.ia_lo, win.ib_lo + r);
          int64_t c1 = cell_of(g, f, win.ia_hi, win.ib_lo + r) + 1;
          const int32_t st = a.grid.start_tot[c0], en = a.grid.start_tot[c1];
          const Entry* E = a.grid.entries;
          fb_offer(F, a.Z, z, i, en - st, [&](int64_t t) { return (int)E[st + t].idx; },
                   &a.ctr->n_duplicate);
        }
        wave_sync();
        if (F.poly.K[F.poly.cur] > 0 && 2.0 * F.poly.R * (1.0 + 1e-12) <= win.D) done = true;
        double grow = 2.0 * F.poly.R * 1.05;
        if (!done && win.D <= rt * 0.999 && grow > win.D) break;  // window cannot grow
        rt = fmax(2.0 * rt, grow);
      }
    }
    if (!done) {
      if (ln == 0) F.brute = 1;
      wave_sync();
      fb_offer(F, a.Z, z, i, a.n, [](int64_t t) { return (int)t; }, &a.ctr->n_duplicate);
    }
    wave_sync();
    // real vertices (where consecutive edges change circle), canonical
    // positions, edges sorted by neighbour index
    if (ln == 0) {
      int E = clip_finish(F.poly, (int)i, z, [&](int j) { return genpos(a.Z, j); }, F.enbr,
                          &F.v0[0][0], &F.v1[0][0], kVmax);
      F.poly.K[0] = E;  // reuse as the edge count
    }
    wave_sync();
    const int E = F.poly.K[0];
    if (ln < E)
      store_edge(a.out, i, ln, V3{F.v0[ln][0], F.v0[ln][1], F.v0[ln][2]},
                 V3{F.v1[ln][0], F.v1[ln][1], F.v1[ln][2]}, F.enbr[ln], a.keep_cells);
    else if (a.keep_cells && ln < kVmax)
      a.out.cell_nbr[i * kVmax + ln] = -1;
    if (ln == 0) {
      a.out.deg[i] = E;
      a.out.R[i] = F.poly.R;
      a.out.flags[i] = kFlagFallback | (F.poly.degen ? kFlagDegenerate : 0) |
                       (F.poly.err ? kFlagError : 0) | (F.brute ? kFlagBrute : 0);
      atomicAdd(&a.ctr->n_fallback, 1);
      if (F.poly.err) atomicAdd(&a.ctr->n_error, 1);
      if (F.brute) atomicAdd(&a.ctr->n_brute, 1);
      if (F.poly.degen) atomicAdd(&a.ctr->n_degenerate, 1);
    }
    wave_sync();
  }
}

// -------------------------------------------------------------- quadrature
// 64 cells per block of four waves.  The block first sorts its cells by
// degree (counting sort in LDS); each wave then takes eight pairs of
// neighbours in that order, one cell per half-wave, so that the two cells of
// a pair mostly have the same degree and finish in the same round.  A
// half-wave covers its cell's (edge, sub-triangle) items 32 at a time, adds
// each into one accumulator per lane, and sums its 32 lanes in a fixed
// butterfly order: a cell's result depends neither on its partner nor on
// the sort nor on the schedule.  MIXED: FP32 points in the generator's local
// frame (quad_leaf_mixed), FP64 subdivision grid, leaf determinants,
// accumulation and epilogue.  Writes m, mu, e of the cell (g, h and the Lloyd step follow in
// k_eval_reduce).
template <bool MIXED>
__device__ inline void cell_epilogue(const EvalOut& o, int64_t i, V3 z, Acc5 acc) {
  const V3 mu = acc.m * z + V3{acc.mx, acc.my, acc.mz};  // first moment from int rho (y - z)
  o.m[i] = acc.m;
  o.e[i] = acc.e;
  o.mu[3 * i] = mu.x;
  o.mu[3 * i + 1] = mu.y;
  o.mu[3 * i + 2] = mu.z;
}

// sum over each half-wave (lanes 0-31 and 32-63 separately)
__device__ inline double half_sum(double v) {
  for (int off = 16; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// (the direct path keeps the per-point test of the series: a second copy of
// its loop for cells near the sphere measured slower, 0.255 -> 0.285 ms at
// n = 163,842, where many cells take it)
template <int KIND, bool MIXED>
__device__ inline void quad_item(const CellArgs& a, V3 A, V3 B, V3 C, V3 z, const CellF& cf,
                                 const DensityF& Df, const double* tab, Acc5& acc) {
  if (MIXED)
    quad_leaf_mixed<KIND>(A, B, C, z, cf, Df, a.rho, acc, a.quad_rule);
  else
    quad_tri_k<KIND>(A, B, C, z, a.rho, acc, tab, a.quad_rule);
}

// Two subdivision levels (the configured rule): the 32 lanes of a half-wave
// build the 15-point grids of all the cell's edges (up to kGridEdges at a
// time) together in LDS -- the corners, then the 3 level-1 midpoints of
// every edge, then its 9 level-2 ones, one point per lane and pass -- and
// each leaf's lane reads its three points, instead of every lane repeating
// both subdivision levels.  Whole-cell passes keep the lanes busy: a
// degree-6 cell takes four short passes, not three per pair of edges.
constexpr int kGridEdges = 7;  // edges whose grids a half-wave holds at once
struct QuadLds {
  double p[2][kGridEdges][15][3];  // per wave: the two cells' edge grids
};
constexpr int kQuadCells = 64;  // cells per block: eight pairs per wave

template <int KIND, bool MIXED, class P>
__global__ __launch_bounds__(256, 4) void k_quad(P p) {
  if (p.idle()) return;
  const CellArgs& a = p.args();
  __shared__ QuadLds lds[4];
  __shared__ double tab[kExpN];  // the exponential's 2^(j/N) table
  // FP64 single chord tanh bump: cells whose fan lies within the density
  // polynomial's radius take it (RhoPoly); they are sorted ahead of the
  // others so that the two halves of a wave mostly take the same path
  // (MIXED: the expansion in x only, as FP32 coefficients)
  constexpr bool POLY = KIND == kRhoTanh;
  // two chord tanh bumps: the expansion in x of each (both or nothing)
  constexpr bool POLY2 = KIND == kRhoTanh + kVarTwo;
  constexpr bool XPOLY = POLY || POLY2;
  constexpr int kBins = (XPOLY ? 3 : 1) * (kVmax + 1);
  __shared__ int bin[kBins];
  __shared__ int list[kQuadCells];
  const int tid = threadIdx.x;
  const EvalOut& o = a.out;
  const int64_t base = (int64_t)p.bx() * kQuadCells;
  const int ncell = a.n - base < kQuadCells ? (int)(a.n - base) : kQuadCells;
  if (tid < kExpN) tab[tid] = kExp2Tab[tid];
  if (tid < kBins) bin[tid] = 0;
  __syncthreads();
  // sort key of each cell: degree, and for POLY which density path it takes
  // -- the polynomial in x, else the one in t, else the direct evaluation --
  // from the farthest vertex's distance (the geometry passes leave it, or a
  // bound on it, in R; a relative 1e-9 covers its rounding)
  int key = 0, dm = 0;
  const bool lead = tid < ncell;
  if (lead) {
    const int64_t i = base + tid;
    dm = min(max(o.deg[i], 0), kVmax);
    key = dm;
    if (XPOLY) {
      const V3 z = V3{a.Z[3 * i], a.Z[3 * i + 1], a.Z[3 * i + 2]};
      const double r = o.R[i] * (1.0 + 1e-9);
      bool xmode = false;
      if (a.rho.polyx_n > 0) {
        xmode = polyx_qualifies(a.rho, z, r, 0);
        if (POLY2) xmode = xmode && polyx_qualifies(a.rho, z, r, 1);
      }
      key = xmode ? dm
                  : (POLY && !MIXED && poly_qualifies(a.rho, z, r * r) ? kVmax + 1 + dm
                                                                       : 2 * (kVmax + 1) + dm);
    }
  }
  if (lead) atomicAdd(&bin[key], 1);
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int b = 0; b < kBins; b++) {
      const int c = bin[b];
      bin[b] = run;
      run += c;
    }
  }
  __syncthreads();
  // entries: the cell's place in the block, +256 if it takes a polynomial,
  // +512 if that is the one in x, its degree from bit 10 on
  if (lead) {
    const int cls = XPOLY ? key / (kVmax + 1) : 2;
    list[atomicAdd(&bin[key], 1)] = tid + (cls < 2 ? 256 : 0) + (cls == 0 ? 512 : 0) + (dm << 10);
  }
  __syncthreads();

  const int ln = lane_id(), w = tid >> 6, hl = ln & 31;
  const int lv = a.levels, per = 1 << (2 * lv);
  CellArgs ar = a;  // FP64 density constants held in vector registers
  if (!MIXED && !POLY2) {  // (two bumps: the registers hold both expansions instead)
    pin_v(ar.rho.gamma);
    for (int k = 0; k < 2; k++) {
      pin_v(ar.rho.K[k]);
      pin_v(ar.rho.bK[k]);
      pin_v(ar.rho.amp[k]);
    }
  }
  DensityF Df{};
  if (MIXED) Df = density_f32(a.rho);
  double(*G)[15][3] = lds[w].p[ln >> 5];  // this half's cell grids
  const int s = ln & 15;
  for (int pr = 0; pr < kQuadCells / 8; pr++) {
    const int slot = (pr * 4 + w) * 2 + (ln >> 5);
    const bool has = slot < ncell;
    const int ent = has ? list[slot] : 0;
    const int64_t i = base + (ent & 255);
    const int d = ent >> 10;
    const V3 z = V3{a.Z[3 * i], a.Z[3 * i + 1], a.Z[3 * i + 2]};
    const double* eb = o.edges + i * (kVmax * 6);  // the cell's edge slots
    const int items = d * per;  // this half's (edge, sub-triangle) items
    const int both = max(items, __shfl_xor(items, 32, 64));
    if (both == 0) continue;  // wave-uniform
    Acc5 acc = {0.0, 0.0, 0.0, 0.0, 0.0};
    // (the mixed path and two bumps have no expansion in t: their cells
    // take x or nothing)
    const bool xmode = XPOLY && (ent & 512);
    const bool use_poly = XPOLY && (MIXED || POLY2 ? xmode : (ent & 256));
    RhoPoly rp[POLY2 ? 2 : 1] = {};
    if (use_poly) {
      double xz;
      rp[0] = xmode ? ar.rho.polyx_tab[0][polyx_index(ar.rho, z, &xz, 0)]
                    : ar.rho.poly_tab[poly_index(ar.rho, z)];
      if (POLY2) rp[POLY2 ? 1 : 0] = ar.rho.polyx_tab[1][polyx_index(ar.rho, z, &xz, 1)];
      if (xmode) {
        rp[0] = polyx_at(rp[0], ar.rho, z, 0);
        if (POLY2) rp[POLY2 ? 1 : 0] = polyx_at(rp[POLY2 ? 1 : 0], ar.rho, z, 1);
      }
    }
    // every point of the cell near the sphere: the FP64 paths skip the
    // per-point test of the reciprocal square root's series (same bits)
    const bool near1 = !MIXED && has && cell_near1(o.R[i]);
    CellF cf{};
    if (MIXED) cf = xmode ? cell_f32_poly(ar.rho, rp, POLY2 ? 2 : 1, z) : cell_f32<KIND>(ar.rho, z, tab);
    if (lv == 2) {
      // the whole cell's grids (up to kGridEdges edges at a time), then its
      // leaves (FP64 grid points on both paths)
      const int dboth = max(d, __shfl_xor(d, 32, 64));
      for (int e0 = 0; e0 < dboth; e0 += kGridEdges) {
        const int ne = min(max(d - e0, 0), kGridEdges);
        const int neb = max(ne, __shfl_xor(ne, 32, 64));
        // corners: v_lo (4) and v_hi (0) of each edge, then z (14); the edge
        // slots are read once, so their loads are marked streaming and do
        // not push the density tables out of the L2
        if (hl < 3 * ne) {
          const bool vert = hl < 2 * ne;
          const int e = vert ? hl >> 1 : hl - 2 * ne, k = vert ? ((hl & 1) ? 0 : 4) : 14;
          const double* ed = eb + (e0 + e) * 6 + ((hl & 1) ? 3 : 0);
          const V3 X = vert ? V3{__builtin_nontemporal_load(ed), __builtin_nontemporal_load(ed + 1),
                                    __builtin_nontemporal_load(ed + 2)} : z;
          G[e][k][0] = X.x;
          G[e][k][1] = X.y;
          G[e][k][2] = X.z;
        }
        wave_sync();
        // level-1 midpoints (3 per edge), then level-2 (9 per edge)
        for (int level = 0; level < 2; level++) {
          const int per_e = level == 0 ? 3 : 9;
          for (int q0 = 0; q0 < per_e * neb; q0 += 32) {
            const unsigned q = (unsigned)(q0 + hl);
            if ((int)q < per_e * ne) {
              const int e = (int)(q / (unsigned)per_e);
              const int task = (int)q - per_e * e + (level == 0 ? 0 : 3);
              const int kp = nib(kG2TaskP, task), kq = nib(kG2TaskQ, task), km = nib(kG2TaskPt, task);
              const V3 m = normalized_fast(V3{G[e][kp][0], G[e][kp][1], G[e][kp][2]} +
                                           V3{G[e][kq][0], G[e][kq][1], G[e][kq][2]});
              G[e][km][0] = m.x;
              G[e][km][1] = m.y;
              G[e][km][2] = m.z;
            }
          }
          wave_sync();
        }
        for (int t0 = 0; t0 < 16 * neb; t0 += 32) {  // two edges' leaves per half and round
          const int t = t0 + hl;
          if (t < 16 * ne) {
            const int e = t >> 4;
            const int ka = nib(kG2LeafA, s), kb = nib(kG2LeafB, s), kc = nib(kG2LeafC, s);
            const V3 A = V3{G[e][ka][0], G[e][ka][1], G[e][ka][2]};
            const V3 B = V3{G[e][kb][0], G[e][kb][1], G[e][kb][2]};
            const V3 C = V3{G[e][kc][0], G[e][kc][1], G[e][kc][2]};
            if (MIXED && xmode) {
              quad_leaf_mixed<KIND, POLY2 ? 2 : 1>(A, B, C, z, cf, Df, ar.rho, acc, ar.quad_rule);
            } else if (POLY2 && xmode) {
              if (near1)
                quad_tri_poly2<true>(A, B, C, z, ar.rho, rp[0], rp[POLY2 ? 1 : 0], acc, ar.quad_rule);
              else
                quad_tri_poly2<false>(A, B, C, z, ar.rho, rp[0], rp[POLY2 ? 1 : 0], acc, ar.quad_rule);
            } else if (POLY && xmode) {
              if (near1)
                quad_tri_poly<true, true>(A, B, C, z, ar.rho, rp[0], acc, ar.quad_rule);
              else
                quad_tri_poly<true, false>(A, B, C, z, ar.rho, rp[0], acc, ar.quad_rule);
            } else if (POLY && use_poly) {
              quad_tri_poly<false>(A, B, C, z, ar.rho, rp[0], acc, ar.quad_rule);
            } else {
              quad_item<KIND, MIXED>(ar, A, B, C, z, cf, Df, tab, acc);
            }
          }
        }
        wave_sync();  // the next chunk or cell rewrites the grids
      }
    } else {
      for (int t = hl; t < items; t += 32) {
        const int e = t >> (2 * lv), sub = t & (per - 1);
        const double* ed = eb + e * 6;
        V3 A = z;
        V3 B = V3{ed[0], ed[1], ed[2]};
        V3 C = V3{ed[3], ed[4], ed[5]};
        subtriangle(A, B, C, sub, lv);
        if (MIXED && xmode)
          quad_leaf_mixed<KIND, POLY2 ? 2 : 1>(A, B, C, z, cf, Df, ar.rho, acc, ar.quad_rule);
        else if (POLY2 && xmode)
          quad_tri_poly2(A, B, C, z, ar.rho, rp[0], rp[POLY2 ? 1 : 0], acc, ar.quad_rule);
        else if (POLY && xmode)
          quad_tri_poly<true>(A, B, C, z, ar.rho, rp[0], acc, ar.quad_rule);
        else if (POLY && use_poly)
          quad_tri_poly<false>(A, B, C, z, ar.rho, rp[0], acc, ar.quad_rule);
        else
          quad_item<KIND, MIXED>(ar, A, B, C, z, cf, Df, tab, acc);
      }
    }
    const Acc5 tot = {half_sum(acc.m), half_sum(acc.mx), half_sum(acc.my), half_sum(acc.mz),
                      half_sum(acc.e)};
    if (hl == 0 && has) cell_epilogue<MIXED>(o, i, z, tot);
  }
}

// small problems: every cell goes through the fallback clipper
template <class P>
__global__ void k_fb_all(P p) {
  if (p.idle()) return;
  const CellArgs& a = p.args();
  int64_t i = (int64_t)p.bx() * blockDim.x + threadIdx.x;
  if (i < a.n) a.fb_list[i] = (int32_t)i;
  if (i == 0) a.ctr->fb_count = (int32_t)a.n;
}

// grid sizes of the cell kernels for a problem (the segmented launches use
// the same ones per problem)
int cells_main_grid(int64_t n) {
  const int64_t nb = (n + 31) / 32;  // eight cells per wave, four waves per block
  const int64_t pad = 8 * kXcdChunk;
  return (int)((nb + pad - 1) / pad * pad);
}
// list lengths are only known on the device: fixed grids, large enough for
// a long list (a random start hands on a few percent of the cells) to run
// at several waves per SIMD; idle blocks exit at once.  The second list
// holds what the first could not certify: far shorter
int cells_tier_grid(int64_t n, int tier) {
  const int64_t nb = (n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048;
  return (int)(tier == 0 ? nb : (nb < 512 ? nb : 512));
}
// one cell per block; after the certified passes the list is short
int cells_fallback_grid(int64_t n, int all) {
  const int64_t cap = all ? 8192 : 1024;
  return (int)(n < cap ? n : cap);
}
int fb_all_grid(int64_t n) { return (int)((n + 255) / 256); }
int quad_grid(int64_t n) { return (int)((n + kQuadCells - 1) / kQuadCells); }

hipError_t launch_cells_main(const CellArgs& a, hipStream_t s) {
  k_cells_geom<<<(unsigned)cells_main_grid(a.n), 256, 0, s>>>(One<CellArgs>{a});
  return hipGetLastError();
}

hipError_t launch_cells_tiers(const CellArgs& a, hipStream_t s) {
  k_cells_tier<0, 32, 32, 31><<<(unsigned)cells_tier_grid(a.n, 0), 256, 0, s>>>(One<CellArgs>{a});
  k_cells_tier<1, 64, 64, kWinMax><<<(unsigned)cells_tier_grid(a.n, 1), 256, 0, s>>>(One<CellArgs>{a});
  return hipGetLastError();
}

hipError_t launch_cells_fallback(const CellArgs& a, int all, hipStream_t s) {
  if (all) k_fb_all<<<(unsigned)fb_all_grid(a.n), 256, 0, s>>>(One<CellArgs>{a});
  k_fallback<<<(unsigned)cells_fallback_grid(a.n, all), 64, 0, s>>>(One<CellArgs>{a});
  return hipGetLastError();
}

// segmented: main pass, list passes and fallback of a batch (tabs[k]: the
// batch's table of kernel k's grids, all on one args table)
hipError_t launch_cells_many(const CellArgs* tab, const int32_t* nb_main, int max_main,
                             const int32_t* nb_t0, int max_t0, const int32_t* nb_t1, int max_t1,
                             const int32_t* nb_all, int max_all, const int32_t* nb_fb, int max_fb,
                             int nseg, hipStream_t s) {
  if (max_main > 0)
    k_cells_geom<<<dim3(max_main, nseg), 256, 0, s>>>(Many<CellArgs>{tab, nb_main});
  if (max_t0 > 0)
    k_cells_tier<0, 32, 32, 31><<<dim3(max_t0, nseg), 256, 0, s>>>(Many<CellArgs>{tab, nb_t0});
  if (max_t1 > 0)
    k_cells_tier<1, 64, 64, kWinMax><<<dim3(max_t1, nseg), 256, 0, s>>>(Many<CellArgs>{tab, nb_t1});
  if (max_all > 0) k_fb_all<<<dim3(max_all, nseg), 256, 0, s>>>(Many<CellArgs>{tab, nb_all});
  k_fallback<<<dim3(max_fb, nseg), 64, 0, s>>>(Many<CellArgs>{tab, nb_fb});
  return hipGetLastError();
}

// the density polynomials' tables (single chord tanh bump): entry j per
// thread, of the expansion in t (X = false) or in x
// the tables' entries, one per thread (x tables: blockIdx.y = bump)
template <bool X>
__global__ void k_poly_table(DensityP D, RhoPoly* out, RhoPoly* out2) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = (int)blockIdx.y;
  if (j < (X ? D.polyx_n : D.poly_n))
    (b ? out2 : out)[j] = X ? polyx_entry(D, j, b, kExp2Tab) : poly_entry(D, j, kExp2Tab);
}

hipError_t launch_poly_table(const DensityP& D, RhoPoly* out, RhoPoly* outx0, RhoPoly* outx1,
                             hipStream_t s) {
  if (D.poly_n > 0)
    k_poly_table<false><<<(unsigned)((D.poly_n + 255) / 256), 256, 0, s>>>(D, out, out);
  if (D.polyx_n > 0) {
    const dim3 g((unsigned)((D.polyx_n + 255) / 256), D.nbumps == 2 ? 2 : 1);
    k_poly_table<true><<<g, 256, 0, s>>>(D, outx0, outx1);
  }
  return hipGetLastError();
}

hipError_t launch_quad(const CellArgs& a, hipStream_t s) {
  const unsigned nb = (unsigned)quad_grid(a.n);
#define SCVT_LAUNCH_QUAD(V)                                  \
  do {                                                       \
    if (a.mixed)                                             \
      k_quad<V, true><<<nb, 256, 0, s>>>(One<CellArgs>{a});  \
    else                                                     \
      k_quad<V, false><<<nb, 256, 0, s>>>(One<CellArgs>{a}); \
  } while (0)
  SCVT_RHO_DISPATCH(rho_variant(a.rho), SCVT_LAUNCH_QUAD)
#undef SCVT_LAUNCH_QUAD
  return hipGetLastError();
}

// segmented: every problem of the batch has density variant `var` and
// precision `mixed`
hipError_t launch_quad_many(const Seg<CellArgs>& g, int var, int mixed, hipStream_t s) {
  const dim3 grid(g.maxnb, g.nseg);
#define SCVT_LAUNCH_QUAD_MANY(V)                                          \
  do {                                                                    \
    if (mixed)                                                            \
      k_quad<V, true><<<grid, 256, 0, s>>>(Many<CellArgs>{g.tab, g.nb});  \
    else                                                                  \
      k_quad<V, false><<<grid, 256, 0, s>>>(Many<CellArgs>{g.tab, g.nb}); \
  } while (0)
  SCVT_RHO_DISPATCH(var, SCVT_LAUNCH_QUAD_MANY)
#undef SCVT_LAUNCH_QUAD_MANY
  return hipGetLastError();
}

}  // namespace scvt
