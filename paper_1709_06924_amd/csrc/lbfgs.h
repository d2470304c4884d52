// Arguments of the streaming LBFGS / reduction kernels (lbfgs.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scvt {

// One two-loop pass: optionally finish the previous pass's dot product
// (sum of its block partials in fixed order; value = prev_sub - prev_mul*sum
// or prev_mul*sum, stored to prev_store), then
//   q = (init_neg_g ? -g : q) + ax_sign * coef * ax_vec;  q *= h if scale_h
// with coef = that finished value, and write this pass's partials of
// dot_vec . q.
struct PassArgs {
  int64_t n3;
  double* q;
  const double* g;
  const double* h;        // per generator
  int init_neg_g;
  int scale_h;
  const double* ax_vec;   // null: no axpy
  double ax_sign;
  const double* prev_partials;  // null: no previous scalar
  const double* prev_mul;       // device scalar (r_j)
  const double* prev_sub;       // device scalar (a_j) or null
  double* prev_store;           // where the finished scalar is kept
  const double* dot_vec;
  double* partials;             // this pass's block partials
};

// Sum/max/min of per-block partials (nvals interleaved values per block) in
// fixed order; op[v] = 0 sum, 1 max, 2 min.  If r_slot is set, it receives
// 1/out[0].
struct FinalizeArgs {
  const double* partials;
  int nblocks, nvals;
  int op[4];
  double* out;
  double* r_slot;
};

struct PushArgs {
  int64_t n3;
  const double *Z, *Zt, *g, *gt;
  double *s, *y;
  double* partials;  // ys, yy, ss per block
};

struct EvalRedArgs {
  int64_t n;
  const double *e, *lloyd, *g, *mu, *Z;
  double* partials;  // F, max|l|, sum|g|^2, min mu.z per block
};

hipError_t launch_lbfgs_pass(const PassArgs& a, hipStream_t s);
hipError_t launch_push(const PushArgs& a, hipStream_t s);
hipError_t launch_eval_reduce(const EvalRedArgs& a, hipStream_t s);
hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t s);
int reduce_grid(int64_t count);  // blocks the streaming kernels use for count items
int reduce_grid_max();

}  // namespace scvt
