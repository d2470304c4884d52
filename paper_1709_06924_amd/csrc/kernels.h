// Internal declarations shared by the kernel files and the host engine.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cellgeom.h"

namespace scvt {

// Where a kernel takes its arguments and block numbers from.  One: one
// problem per launch, the arguments by value.  Many: one launch for a batch
// of problems (the serving loop's segmented launches): blockIdx.y picks the
// problem, whose arguments and own grid size sit in device tables; blocks
// beyond that problem's grid exit at once.  A kernel body sees the same
// arguments and block numbers either way, so a problem's results do not
// depend on the batch it runs in.
template <class A>
struct One {
  A a;
  __device__ const A& args() const { return a; }
  __device__ int bx() const { return (int)blockIdx.x; }
  __device__ int gx() const { return (int)gridDim.x; }
  __device__ bool idle() const { return false; }
};
template <class A>
struct Many {
  const A* tab;       // per problem
  const int32_t* nb;  // each problem's own grid size
  __device__ const A& args() const { return tab[blockIdx.y]; }
  __device__ int bx() const { return (int)blockIdx.x; }
  __device__ int gx() const { return nb[blockIdx.y]; }
  __device__ bool idle() const { return (int)blockIdx.x >= nb[blockIdx.y]; }
};

// A segmented launch's device tables: nseg problems, the largest grid maxnb.
template <class A>
struct Seg {
  const A* tab;
  const int32_t* nb;
  int nseg, maxnb;
};

constexpr int kVmax = 32;          // max Voronoi edges per cell kept in debug output
constexpr int kWinMax = 63;        // max window side in cells
constexpr int kFbPolyMax = 64;     // polygon capacity of the fallback clipper

// sorted grid entry: a generator (or a ghost copy of it) in one cell
struct Entry {
  double x, y, z;
  int32_t idx;
  int32_t pad;
};

// per-cell status bits
enum CellFlags : uint8_t {
  kFlagFallback = 1,    // built by the sequential fallback
  kFlagDegenerate = 2,  // a predicate was within its error bound
  kFlagError = 4,       // the fallback could not build the cell
  kFlagBrute = 8,       // the fallback scanned every generator
};

struct EvalOut {  // per-generator results of one evaluation
  double *m, *mu, *e, *g, *h, *lloyd;  // mu, g, lloyd are n x 3
  double* R;                           // circumradius of the cell (next search radius)
  uint8_t* flags;
  int32_t* deg;
  double* edges;      // n x kVmax x 6: edge k of cell i, v0 -> v1
  int32_t* cell_nbr;  // n x kVmax neighbour ids (only with keep_cells)
};

struct GridBufs {
  GridP g;
  // per cell the pair (entries, home entries), one 64-bit word (total in the
  // low half), so that a block adds or takes both counts with one atomic;
  // ncells (+1) pairs
  int32_t* cnt2;
  int32_t* start_tot;  // ncells + 1 (exclusive scan)
  int32_t* start_home; // ncells + 1
  int32_t* cell3;      // n x 3 cells (home, ghosts, -1) of the generator at each position of order_prev
  Entry* entries;      // capacity cap_entries
  int32_t* order;      // n: generators sorted by home cell
  int32_t* order_prev; // n: the previous build's order (input of the next build)
  int64_t cap_entries;
  int32_t* scan_tmp;   // block sums for the scan
  int32_t* overflow;   // 1 int: set when entries exceed capacity
};

struct Counters {  // device-side counters of one evaluation
  int32_t fb_count;
  int32_t n_fallback, n_degenerate, n_error, n_brute;
  int32_t n_duplicate;    // duplicate generators seen
  int32_t tier_count[2];  // cells handed to the list passes of the certified path
};
constexpr int kTiers = 2;

struct CellArgs {
  int64_t n;
  const double* Z;  // n x 3 (unit rows)
  GridBufs grid;
  DensityP rho;
  int levels;
  int keep_cells;
  int mixed;
  int quad_rule;  // points of the triangle rule: 7 (default), 4 or 9
  EvalOut out;
  int32_t* fb_list;    // n: cells for the fallback clipper
  int32_t* tier_list[2];  // n each: cells for the list passes of the certified path
  Counters* ctr;
  double r_default;  // initial search radius when no previous one is known
  int kmax;          // > 0: at most kmax candidates per cell in the certified passes
};

// arguments of the trial normalisation, the grid build and the scans
struct NormArgs {
  const double* Z;
  const double* q;  // null: normalise Z itself
  double alpha;
  double* Zt;
  int64_t n;
};
struct GridBuildArgs {
  const double* Z;
  int64_t n;
  GridBufs gb;
  int32_t* clear;  // 8 ints zeroed by the first kernel, or null
};
struct ScanArgs {  // exclusive scans of a and b (m entries) into oa, ob
  const int32_t *a, *b;  // entry t at a[t * stride], b[t * stride]
  int64_t m;
  int32_t* sums;  // tile sums (scratch)
  int32_t *oa, *ob;
  int64_t ntiles;
  int stride;
};
int normalize_grid(int64_t n);
int bucket_grid(int64_t n);
int64_t scan_tiles(int64_t m);
ScanArgs grid_scan_args(const GridBufs& gb);

// ---- launch wrappers (return hipError_t) ----
hipError_t launch_normalize_trial(const double* Z, const double* q, double alpha, double* Zt,
                                  int64_t n, hipStream_t s);
// builds the buckets of Z; then gb.order holds the new order (the caller
// swaps order and order_prev before the next build)
// (clear: 8 ints zeroed by the first kernel, e.g. the evaluation's counters)
hipError_t launch_grid_build(const double* Z, int64_t n, GridBufs& gb, int32_t* clear,
                             hipStream_t s);
hipError_t launch_iota(int32_t* p, int64_t n, hipStream_t s);
// exclusive scans of a[0..m) and b[0..m) into oa, ob (m+1 entries each; the
// last holds the total); tmp holds scan_tmp_ints(m) ints
hipError_t launch_scan_pair(const int32_t* a, const int32_t* b, int64_t m, int32_t* tmp,
                            int32_t* oa, int32_t* ob, hipStream_t s);
int64_t scan_tmp_ints(int64_t m);
// bisection (n -> n + #edges): cnt[i] = neighbours of i with a larger index
hipError_t launch_refine_count(const int32_t* deg, const int32_t* nbr, int64_t n, int32_t* cnt,
                               hipStream_t s);
// out[0..n) = Z, then normalize(z_i + z_j) for every edge i < j, by i then j,
// at n + off[i] + t
// triangle list: cnt[i] (if cnt) = triangles listed by cell i; with tri,
// they are written at off[i] (3 ints each)
hipError_t launch_tri_list(const int32_t* deg, const int32_t* nbr, const double* edges, int64_t n,
                           const int32_t* off, int32_t* cnt, int32_t* tri, hipStream_t s);
hipError_t launch_cell_quality(const int32_t* deg, const double* edges, int64_t n, double* q,
                               hipStream_t s);
hipError_t launch_tri_quality(const double* Z, const int32_t* tri, int64_t ntri, double* q,
                              hipStream_t s);
hipError_t launch_refine_emit(const double* Z, const int32_t* deg, const int32_t* nbr,
                              const int32_t* off, int64_t n, double* out, hipStream_t s);
hipError_t launch_cells_main(const CellArgs& a, hipStream_t s);
hipError_t launch_cells_tiers(const CellArgs& a, hipStream_t s);
hipError_t launch_cells_fallback(const CellArgs& a, int all, hipStream_t s);
hipError_t launch_poly_table(const DensityP& D, RhoPoly* out, RhoPoly* outx0, RhoPoly* outx1,
                             hipStream_t s);
hipError_t launch_quad(const CellArgs& a, hipStream_t s);
hipError_t launch_centroid(const double* mu, const double* m, double* out, int64_t n,
                           hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t s);
// p[0..count) = gamma = 1 / (dscal[r_at] * dscal[yy_at]) (y.s / y.y of a stored
// pair), or 1 when r_at < 0
hipError_t launch_fill_gamma(double* p, int64_t count, const double* dscal, int r_at, int yy_at,
                             hipStream_t s);

// ---- segmented launches: the same kernels over a batch of problems ----
// grid sizes of a single problem's launches (a batch uses them per problem)
int cells_main_grid(int64_t n);
int cells_tier_grid(int64_t n, int tier);
int cells_fallback_grid(int64_t n, int all);
int fb_all_grid(int64_t n);
int quad_grid(int64_t n);
hipError_t launch_normalize_trial_many(const Seg<NormArgs>& g, hipStream_t s);
// grid build: count and scatter over g, the scans' tiles over `tiles`, one
// block per problem over `one` (the same ScanArgs table)
hipError_t launch_grid_build_many(const Seg<GridBuildArgs>& g, const Seg<ScanArgs>& tiles,
                                  const Seg<ScanArgs>& one, hipStream_t s);
// main pass, the two list passes, the small problems' full lists (max_all 0:
// none) and the fallback clipper, each with its own per-problem grid sizes
hipError_t launch_cells_many(const CellArgs* tab, const int32_t* nb_main, int max_main,
                             const int32_t* nb_t0, int max_t0, const int32_t* nb_t1, int max_t1,
                             const int32_t* nb_all, int max_all, const int32_t* nb_fb, int max_fb,
                             int nseg, hipStream_t s);
// every problem of the batch with density variant var and precision mixed
hipError_t launch_quad_many(const Seg<CellArgs>& g, int var, int mixed, hipStream_t s);

}  // namespace scvt
