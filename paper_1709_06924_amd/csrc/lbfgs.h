// Arguments of the streaming LBFGS / reduction kernels (lbfgs.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

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

// per generator: g = 2 (mu.z) z - 2 mu, h = 1 / (2 mu.z), l = mu/|mu| - z
// (section 3.1), written; partials of F, max |l|, sum |g|^2, min mu.z
struct EvalRedArgs {
  int64_t n;
  const double *e, *mu, *Z;
  double *g, *h, *lloyd;
  double* partials;  // F, max|l|, sum|g|^2, min mu.z per block
};

// ---- two-loop through the history's inner products (up to kHmax pairs) ----
// The backward loop's a_j = r_j s_j.q_{j+1} with q_{j+1} = -g - sum_{k>j} a_k y_k
// equals r_j (-s_j.g - sum_{k>j} a_k s_j.y_k), and the forward loop's
// b_j = r_j y_j.(r + sum_{k<j} c_k s_k) equals r_j (y_j.r + sum_{k<j} c_k s_k.y_j)
// with r = h (.) q_0.  With s_j.g (from the push of the previous iteration) and
// the products s_j.y_k, j older than k (kept as pairs arrive), the two
// recursions are scalar work; the vectors are streamed twice:
//   q0 pass:  r = h (.) (-g - sum_k a_k y_k), partials of y_j.r
//   dir pass: q = r + sum_k c_k s_k, partials of g.q
constexpr int kHmax = 16;

// device scalar layout (doubles, in the handle's scalar buffer)
enum : int {
  kA = 0,       // a_j by ring position
  kCoef = 64,   // c_j = a_j - b_j by ring position
  kR = 128,     // r = 1 / y.s by slot
  kGQ = 200,    // g . q
  kPush = 201,  // y.s, y.y, s.s of the last push
  kEval = 204,  // F, max |l|, sum |g|^2, min mu.z
  kCtr = 208,   // the evaluation's Counters (32 bytes)
  kSG = 256,    // s.g by slot (g at the current point)
  kYY = 320,    // y.y by slot (plain LBFGS scaling)
  kNScal = 384
};

enum : int { kFinPush = 0, kFinDots = 1, kFinBackward = 2, kFinForward = 3, kFinGQ = 4 };
struct HistFinArgs {
  int mode;
  const double* partials;
  int nblocks, nvals;
  int c;
  int slot[kHmax];  // ring slots, oldest first
  int p;            // push: slot of the new pair
  int stride;       // row stride of the s.y table (the handle's slot count)
  double* dscal;
  double* gram;     // s_j.y_k at [slot_j * stride + slot_k]
  double* dst[kHmax];
};

// Up to two fin steps run in order by one launch.
struct FinChain {
  int n;
  HistFinArgs step[2];
};

struct HistPassArgs {
  int64_t n3;
  int c;  // stored pairs, ring order (oldest first)
  const double* S[kHmax];
  const double* Y[kHmax];
  const double* g;
  const double* h;     // per generator
  const double* qin;   // dir pass: r
  double* q;           // output
  const double* coef;  // a_j (q0 pass) or c_j (dir pass), ring order
  double* partials;
};

// s = Zt - Z, y = gt - g into the new slot; per block: y.s, y.y, s.s,
// s.gt, then s_j.gt and s_j.y for the c stored pairs.
struct PushExtArgs {
  int64_t n3;
  const double *Z, *Zt, *g, *gt;
  double *s, *y;
  int c;
  const double* S[kHmax];
  double* partials;
};

// per block: A_j . v for j < c
struct MultiDotArgs {
  int64_t n3;
  int c;
  const double* A[kHmax];
  const double* v;
  double* partials;
};



hipError_t launch_push_ext(const PushExtArgs& a, hipStream_t s);
hipError_t launch_multi_dot(const MultiDotArgs& a, hipStream_t s);
hipError_t launch_hist_q0(const HistPassArgs& a, hipStream_t s);
hipError_t launch_fin_chain(const FinChain& f, hipStream_t s);
hipError_t launch_hist_dir(const HistPassArgs& a, hipStream_t s);
hipError_t launch_hist_fin(const HistFinArgs& a, hipStream_t s);
int hist_grid(int64_t n3);  // blocks of the history passes
int hist_grid_max();

hipError_t launch_lbfgs_pass(const PassArgs& a, hipStream_t s);
hipError_t launch_push(const PushArgs& a, hipStream_t s);
hipError_t launch_eval_reduce(const EvalRedArgs& a, hipStream_t s);
hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t s);
int reduce_grid(int64_t count);  // blocks the streaming kernels use for count items
int reduce_grid_max();

// segmented launches: the same kernels over a batch of problems (vw: 2 when
// the problems' 3n is even, as the single launch chooses)
hipError_t launch_push_ext_many(const Seg<PushExtArgs>& g, int vw, hipStream_t s);
hipError_t launch_hist_q0_many(const Seg<HistPassArgs>& g, int vw, hipStream_t s);
hipError_t launch_hist_dir_many(const Seg<HistPassArgs>& g, int vw, hipStream_t s);
hipError_t launch_hist_fin_many(const Seg<HistFinArgs>& g, hipStream_t s);
hipError_t launch_fin_chain_many(const Seg<FinChain>& g, hipStream_t s);
hipError_t launch_eval_reduce_many(const Seg<EvalRedArgs>& g, hipStream_t s);
hipError_t launch_finalize_many(const Seg<FinalizeArgs>& g, hipStream_t s);

}  // namespace scvt
