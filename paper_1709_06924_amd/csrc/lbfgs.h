// Arguments of the streaming LBFGS / reduction kernels (lbfgs.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scvt {

struct PassArgs {
  int64_t n3;
  double* q;
  const double* g;
  const double* h;        // per generator
  int init_neg_g;         // q = -g before the axpy
  int scale_h;            // q = h (.) q after the axpy
  const double* ax_vec;   // q += ax_sign * (*ax_coef) * ax_vec (null: none)
  const double* ax_coef;  // device scalar
  double ax_sign;
  const double* dot_vec;  // result dot = dot_vec . q (after the update)
  const double* mul;      // device scalar or null: r = mul * dot
  const double* sub_from; // device scalar or null: out = sub_from - r
  double* out;            // device scalar
  double* partials;       // >= grid size
  unsigned* ticket;       // zero-initialised counter
};

struct PushArgs {
  int64_t n3;
  const double *Z, *Zt, *g, *gt;
  double *s, *y;
  double* out;     // ys, yy, ss
  double* r_slot;  // 1 / ys
  double* partials;
  unsigned* ticket;
};

struct EvalRedArgs {
  int64_t n;
  const double *e, *lloyd, *g, *mu, *Z;
  double* out;  // F, max|l|, sum|g|^2, min mu.z
  double* partials;
  unsigned* ticket;
};

hipError_t launch_lbfgs_pass(const PassArgs& a, hipStream_t s);
hipError_t launch_push(const PushArgs& a, hipStream_t s);
hipError_t launch_eval_reduce(const EvalRedArgs& a, hipStream_t s);
int reduce_grid_max();

}  // namespace scvt
