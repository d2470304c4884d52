// Host engine behind the C ABI: device state, the evaluation pipeline and
// the P-LBFGS state machine (two-loop direction, descent check, Armijo line
// search with projection, history ring).
#include <hip/hip_runtime.h>
#include <math.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "../../include/scvt.h"
#include "engine_batch.h"
#include "kernels.h"
#include "lbfgs.h"
#include "round.h"

using namespace scvt;

namespace {

struct EvalSet {
  double *m = nullptr, *mu = nullptr, *e = nullptr, *g = nullptr, *h = nullptr,
         *lloyd = nullptr;
  uint8_t* flags = nullptr;
  int32_t* deg = nullptr;
  int32_t* cell_nbr = nullptr;
  double* edges = nullptr;
};

struct Timer {
  double ms = 0.0;
  int64_t launches = 0;
};

constexpr int kTimers = 7;
constexpr int kStateMagic = 0x53435654;  // "SCVT"

}  // namespace

struct scvt_handle {
  scvt_config cfg;
  int64_t n = 0;
  int M = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  DensityP rho{};
  GridBufs grid{};
  double *Z = nullptr, *Zt = nullptr, *q = nullptr, *R = nullptr;
  EvalSet cur, trial;
  // history slots: M + 2 of 3n each -- the M stored pairs, a pair whose
  // curvature test is pending, and the slot the next trial's early push
  // writes (never one that undoing the pending pair would restore)
  int nslots = 0;
  double *S = nullptr, *Y = nullptr;
  double* dscal = nullptr;            // device scalars
  double* partials = nullptr;
  double* gram = nullptr;   // s_j . y_k (j older than k) by slot, nslots^2
  double* hgam = nullptr;   // plain LBFGS: gamma_n on every generator
  double* hpart = nullptr;  // block partials of the history passes
  int32_t* fb_list = nullptr;
  int32_t* tier_list[2] = {nullptr, nullptr};
  Counters* ctr = nullptr;
  double* pinned = nullptr;  // host-pinned mirror of scalars
  // the trial's push (s, y and their products) launched behind its
  // evaluation, ahead of the host's acceptance test (push_pair reuses it
  // when the history it was launched for is still the history)
  bool pre_valid = false;
  int pre_slot = -1;
  std::vector<int> pre_ring;
  hipEvent_t ev_copy = nullptr;
  std::vector<void*> allocs;
  // ring: slots ordered oldest -> newest
  std::vector<int> ring;
  std::vector<int> free_slots;
  // current state
  double F = 0, step_inf = 0, gnorm2 = 0, min_mz = 0, alpha = 0;
  int64_t iter = 0, n_evals = 0, n_fb = 0, n_deg = 0, n_lloyd_fallback = 0, n_wide[2] = {0, 0};
  // the last SCVT_RECORD_RING per-iteration records (the initial
  // evaluation's and one after every iteration), a ring once full
  std::vector<scvt_info> records;
  int64_t rec_total = 0;
  // evaluation results of the last trial
  double tF = 0, tstep = 0, tg2 = 0, tmz = 0;
  int64_t tfb = 0, tdeg = 0, twide[2] = {0, 0};
  bool timing = false;      // all kernel timers
  bool timing_quad = false;  // the quadrature kernel's timer (also set by timing)
  Timer timers[kTimers];
  hipEvent_t ev[9] = {};
  int main_path = 1;
  double r_default = 0;
  double* shared_edges = nullptr;
  bool dry_run = false;
  size_t dry_bytes = 0;
  double ls_noise = 0.0;
  // the last pushed pair joined the history on the assumption that it
  // passes the curvature test; decided at the next host sync (resolve_push)
  bool push_pending = false;
  std::vector<int> ring_prev, free_prev;
  bool dir_timer_pending = false;  // direction timer events awaiting a sync
  // a_j of the backward recursion for the current history already computed
  // (by the last push's chained fin steps)
  bool backward_ready = false;
  // ---- batched (serving) mode: device memory from a caller's arena, the
  // pinned scalars and stream from the server, launches recorded into a
  // round instead of issued (rec), and the P-LBFGS iteration as a state
  // machine advanced once per round
  bool batched = false;
  char* arena = nullptr;
  size_t arena_bytes = 0, arena_used = 0;
  Round* rec = nullptr;
  int bstate = 0, bk = 0;
  double balpha = 1.0, bgq = 0.0;
  int64_t bmax_iter = 0;
  double btol = 0.0;
};

namespace {

// host-pinned scalar mirror: [0] g.q, [1..3] y.s, y.y, s.s of the last push,
// [4..7] F, max |l|, sum |g|^2, min mu.z of the last evaluation (one copy of
// the adjacent device scalars), [8..] the counters
constexpr int kPinGQ = 0, kPinPush = 1, kPinEval = 4, kPinCtr = 8;
static_assert(kPush == kGQ + 1 && kEval == kPush + 3 && kCtr == kGQ + kPinCtr,
              "adjacent device scalars");
static_assert(sizeof(Counters) <= 4 * sizeof(double) && kCtr + 4 <= kSG, "counters' slot");
constexpr int kPinWords = kPinCtr + 4;  // doubles of one evaluation's copy

// partial-sum buffers, in units of reduce_grid_max() doubles
enum : int { kPartPass = 0, kPartPush = 2, kPartEval = 5, kPartTotal = 9 };

int hip_err(hipError_t e) { return e == hipSuccess ? SCVT_OK : SCVT_E_HIP; }

// a roctx range over a scope (visible to rocprofv3 --marker-trace; the
// calls cost a few nanoseconds when no tool is attached)
struct Range {
  explicit Range(const char* what) { roctxRangePushA(what); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

void fill_info(scvt_handle* h, scvt_info* info, int status);

// the state after an evaluation or iteration, into the record ring
void record(scvt_handle* h) {
  scvt_info r;
  fill_info(h, &r, SCVT_OK);
  if ((int64_t)h->records.size() < SCVT_RECORD_RING)
    h->records.push_back(r);
  else
    h->records[(size_t)(h->rec_total % SCVT_RECORD_RING)] = r;
  h->rec_total++;
}
#define HIPCK(x)                          \
  do {                                    \
    hipError_t _e = (x);                  \
    if (_e != hipSuccess) return SCVT_E_HIP; \
  } while (0)

template <class T>
int dalloc(scvt_handle* h, T** p, size_t count) {
  void* v = nullptr;
  if (count == 0) count = 1;
  if (h->dry_run) {  // footprint only: count the bytes, allocate nothing
    h->dry_bytes += (count * sizeof(T) + 255) / 256 * 256;
    *p = (T*)(uintptr_t)256;
    return SCVT_OK;
  }
  if (h->arena) {  // the caller's memory, laid out as the dry run counts it
    const size_t bytes = (count * sizeof(T) + 255) / 256 * 256;
    if (h->arena_used + bytes > h->arena_bytes) return SCVT_E_OOM;
    *p = (T*)(h->arena + h->arena_used);
    h->arena_used += bytes;
    return SCVT_OK;
  }
  if (hipMalloc(&v, count * sizeof(T)) != hipSuccess) return SCVT_E_OOM;
  h->allocs.push_back(v);
  *p = (T*)v;
  return SCVT_OK;
}
#define ALLOC(p, cnt)                    \
  do {                                   \
    int _r = dalloc(h, &(p), (size_t)(cnt)); \
    if (_r) return _r;                   \
  } while (0)

int alloc_set(scvt_handle* h, EvalSet& s) {
  const int64_t n = h->n;
  ALLOC(s.m, n);
  ALLOC(s.mu, 3 * n);
  ALLOC(s.e, n);
  ALLOC(s.g, 3 * n);
  ALLOC(s.h, n);
  ALLOC(s.lloyd, 3 * n);
  ALLOC(s.flags, n);
  ALLOC(s.deg, n);
  // edge slots: per set when the cells are kept for scvt_get_cells, else one
  // buffer shared by both sets (it only lives through one evaluation)
  if (h->cfg.keep_cells) {
    ALLOC(s.cell_nbr, n * kVmax);
    ALLOC(s.edges, n * kVmax * 6);
  } else {
    if (!h->shared_edges) ALLOC(h->shared_edges, n * kVmax * 6);
    s.edges = h->shared_edges;
  }
  return SCVT_OK;
}

GridP make_grid(int64_t n) {
  GridP g{};
  int G = (int)llround(sqrt((double)n / 12.0));
  if (G < 1) G = 1;
  int B = G / 2;  // ghost border up to U = 2 (about 63 degrees off the face axis)
  if (B > 24) B = 24;
  g.G = G;
  g.B = B;
  g.W = G + 2 * B;
  g.du = 2.0 / G;
  g.inv_du = G / 2.0;
  g.U = 1.0 + B * g.du;
  g.ncells = 6LL * g.W * g.W;
  return g;
}

DensityP to_dev(const scvt_density& d) {
  DensityP r{};
  r.kind = d.kind;
  r.geodesic = d.geodesic;
  r.nbumps = d.nbumps;
  for (int k = 0; k < 2; k++) {
    for (int c = 0; c < 3; c++) r.xc[k][c] = d.xc[k][c];
    r.beta[k] = d.beta[k];
    r.alpha[k] = d.alpha[k];
    r.amp[k] = d.amp[k];
  }
  r.gamma = d.gamma;
  r.w_lon = d.w_lon;
  r.w_lat = d.w_lat;
  return density_prepare(r);
}

int validate(const scvt_config* c) {
  if (!c || c->n < 4 || c->n > (int64_t)1 << 28) return SCVT_E_INVALID;  // 3n < 2^31
  // M + 2 history slots index the per-slot scalars (64 entries each)
  static_assert(kYY + 62 <= kNScal && kR + 62 <= kGQ && kSG + 62 <= kYY, "slot scalars");
  if (c->m_hist < 0 || c->m_hist > 60) return SCVT_E_INVALID;
  if (c->method < SCVT_METHOD_PLBFGS || c->method > SCVT_METHOD_LBFGS) return SCVT_E_INVALID;
  if (c->precision != SCVT_FP64 && c->precision != SCVT_MIXED) return SCVT_E_INVALID;
  if (c->quad_levels < 0 || c->quad_levels > 3) return SCVT_E_INVALID;
  if (c->quad_rule != 4 && c->quad_rule != 7 && c->quad_rule != 9) return SCVT_E_INVALID;
  if (c->ls_max_evals < 1 || !(c->ls_c1 > 0.0 && c->ls_c1 < 1.0)) return SCVT_E_INVALID;
  if (!(c->curv_eps >= 0.0)) return SCVT_E_INVALID;
  if (c->k_max < 0) return SCVT_E_INVALID;
  const scvt_density& d = c->rho;
  if (d.kind < 0 || d.kind > 3) return SCVT_E_INVALID;
  if (d.kind == SCVT_RHO_TANH) {
    if (d.nbumps < 1 || d.nbumps > 2) return SCVT_E_INVALID;
    for (int k = 0; k < d.nbumps; k++)
      if (!(d.alpha[k] > 0.0)) return SCVT_E_INVALID;
  }
  if (d.kind == SCVT_RHO_X16 && !(d.alpha[0] > 0.0 && d.w_lon > 0.0 && d.w_lat > 0.0))
    return SCVT_E_INVALID;
  if (d.kind != SCVT_RHO_CONST && !(d.gamma > 0.0)) return SCVT_E_INVALID;
  return SCVT_OK;
}

CellArgs cell_args(scvt_handle* h, const double* Zsrc, EvalSet& s) {
  CellArgs a{};
  a.n = h->n;
  a.Z = Zsrc;
  a.grid = h->grid;
  a.rho = h->rho;
  a.levels = h->cfg.quad_levels;
  a.keep_cells = h->cfg.keep_cells;
  a.mixed = h->cfg.precision == SCVT_MIXED;
  a.quad_rule = h->cfg.quad_rule;
  a.out.m = s.m;
  a.out.mu = s.mu;
  a.out.e = s.e;
  a.out.g = s.g;
  a.out.h = s.h;
  a.out.lloyd = s.lloyd;
  a.out.R = h->R;
  a.out.flags = s.flags;
  a.out.deg = s.deg;
  a.out.cell_nbr = s.cell_nbr;
  a.out.edges = s.edges;
  a.fb_list = h->fb_list;
  a.tier_list[0] = h->tier_list[0];
  a.tier_list[1] = h->tier_list[1];
  a.ctr = h->ctr;
  a.r_default = h->r_default;
  a.kmax = h->cfg.k_max;
  return a;
}

void timer_add(scvt_handle* h, int k, hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) == hipSuccess) {
    h->timers[k].ms += ms;
    h->timers[k].launches += 1;
  }
}

int launch_push_pre(scvt_handle* h);

// Launches of the iteration's steps: issued on the handle's stream, or, in
// batched mode, recorded into the round (the same arguments).
int vw_of(int64_t n3) { return n3 % 2 == 0 ? 2 : 1; }
hipError_t L_hist_fin(scvt_handle* h, const HistFinArgs& f) {
  if (!h->rec) return launch_hist_fin(f, h->stream);
  if (f.mode == kFinBackward) h->rec->fin_back.push_back(f);
  else if (f.mode == kFinForward) h->rec->fin_fwd.push_back(f);
  else if (f.mode == kFinGQ) h->rec->fin_gq.push_back(f);
  else return hipErrorInvalidValue;  // no other step runs in a round
  return hipSuccess;
}
hipError_t L_hist_q0(scvt_handle* h, const HistPassArgs& p) {
  if (!h->rec) return launch_hist_q0(p, h->stream);
  h->rec->q0[vw_of(p.n3) - 1].push_back(p);
  return hipSuccess;
}
hipError_t L_hist_dir(scvt_handle* h, const HistPassArgs& p) {
  if (!h->rec) return launch_hist_dir(p, h->stream);
  h->rec->dir[vw_of(p.n3) - 1].push_back(p);
  return hipSuccess;
}
hipError_t L_push_ext(scvt_handle* h, const PushExtArgs& p) {
  if (!h->rec) return launch_push_ext(p, h->stream);
  h->rec->push_ext[vw_of(p.n3) - 1].push_back(p);
  return hipSuccess;
}
hipError_t L_fin_chain(scvt_handle* h, const FinChain& f) {
  if (!h->rec) return launch_fin_chain(f, h->stream);
  h->rec->fin_chain.push_back(f);
  return hipSuccess;
}
hipError_t L_normalize(scvt_handle* h, const double* Z, const double* q, double alpha, double* Zt) {
  if (!h->rec) return launch_normalize_trial(Z, q, alpha, Zt, h->n, h->stream);
  h->rec->norm.push_back(NormArgs{Z, q, alpha, Zt, h->n});
  return hipSuccess;
}

// per generator g, h, l and the block partials of the evaluation's scalars;
// then their fixed-order finish into the device scalars
EvalRedArgs eval_red_args(scvt_handle* h, const double* Zsrc, EvalSet& s) {
  EvalRedArgs r{};
  r.n = h->n;
  r.e = s.e;
  r.mu = s.mu;
  r.Z = Zsrc;
  r.g = s.g;
  r.h = s.h;
  r.lloyd = s.lloyd;
  r.partials = h->partials + kPartEval * reduce_grid_max();
  return r;
}
FinalizeArgs eval_fin_args(scvt_handle* h, const EvalRedArgs& r) {
  FinalizeArgs fa{};
  fa.partials = r.partials;
  fa.nblocks = reduce_grid(h->n);
  fa.nvals = 4;
  fa.op[0] = 0;
  fa.op[1] = 1;
  fa.op[2] = 0;
  fa.op[3] = 2;
  fa.out = h->dscal + kEval;
  return fa;
}
int evaluate_complete(scvt_handle* h);

// An evaluation at Zsrc into set s recorded into the handle's round (batched
// mode): the same launches as evaluate(), and the same scalars gathered into
// the pinned mirror at the round's end (evaluate_complete then reads them).
int record_evaluation(scvt_handle* h, const double* Zsrc, EvalSet& s) {
  Round* R = h->rec;
  std::swap(h->grid.order, h->grid.order_prev);  // last build's order drives this one
  R->grid.push_back(GridBuildArgs{Zsrc, h->n, h->grid, (int32_t*)h->ctr});  // also clears ctr
  const CellArgs a = cell_args(h, Zsrc, s);
  (h->main_path ? R->cells : R->cells_all).push_back(a);
  R->quad[{rho_variant(a.rho), a.mixed}].push_back(a);
  const EvalRedArgs r = eval_red_args(h, Zsrc, s);
  R->reduce.push_back(r);
  R->fin.push_back(eval_fin_args(h, r));
  R->out.push_back(Round::Out{h->dscal + kGQ, kPinWords, h->pinned + kPinGQ});
  h->pre_valid = false;
  return SCVT_OK;
}

// Evaluate at Zsrc into set s: grid, cells, reductions; one host sync.
// prepush (a trial of the P-LBFGS loop): the push of the trial as the next
// pair is launched behind the evaluation, and the host waits for the
// scalars' copy only, so the push runs while the host decides.
int evaluate(scvt_handle* h, const double* Zsrc, EvalSet& s, bool prepush = false) {
  Range range("scvt evaluation");  // the launches and the wait for their scalars
  hipStream_t st = h->stream;
  const bool tm = h->timing, tq = h->timing_quad;
  if (tm) HIPCK(hipEventRecord(h->ev[0], st));
  std::swap(h->grid.order, h->grid.order_prev);  // last build's order drives this one
  HIPCK(launch_grid_build(Zsrc, h->n, h->grid, (int32_t*)h->ctr, st));  // also clears ctr
  if (tm) HIPCK(hipEventRecord(h->ev[1], st));
  CellArgs a = cell_args(h, Zsrc, s);
  if (h->main_path) HIPCK(launch_cells_main(a, st));
  if (tm) HIPCK(hipEventRecord(h->ev[8], st));
  if (h->main_path) HIPCK(launch_cells_tiers(a, st));
  if (tm) HIPCK(hipEventRecord(h->ev[2], st));
  HIPCK(launch_cells_fallback(a, h->main_path ? 0 : 1, st));
  if (tq) HIPCK(hipEventRecord(h->ev[3], st));
  HIPCK(launch_quad(a, st));
  if (tq) HIPCK(hipEventRecord(h->ev[7], st));
  const EvalRedArgs r = eval_red_args(h, Zsrc, s);
  HIPCK(launch_eval_reduce(r, st));
  HIPCK(launch_finalize(eval_fin_args(h, r), st));
  if (tm) HIPCK(hipEventRecord(h->ev[4], st));
  // one copy brings g.q, the last push's curvature scalars, this
  // evaluation's scalars and its counters (adjacent device scalars)
  HIPCK(hipMemcpyAsync(h->pinned + kPinGQ, h->dscal + kGQ, kPinWords * sizeof(double),
                       hipMemcpyDeviceToHost, st));
  h->pre_valid = false;
  if (prepush && h->M > 0 && h->M <= kHmax) {
    HIPCK(hipEventRecord(h->ev_copy, st));
    const int rp = launch_push_pre(h);
    if (rp) return rp;
    HIPCK(hipEventSynchronize(h->ev_copy));
  } else {
    HIPCK(hipStreamSynchronize(st));
  }
  if (h->dir_timer_pending) {
    timer_add(h, 3, h->ev[5], h->ev[6]);
    h->dir_timer_pending = false;
  }
  if (tm) {
    if (h->main_path) timer_add(h, 0, h->ev[1], h->ev[8]);
    if (h->main_path) timer_add(h, 6, h->ev[8], h->ev[2]);
    timer_add(h, 1, h->ev[2], h->ev[3]);
    timer_add(h, 2, h->ev[0], h->ev[1]);
    timer_add(h, 4, h->ev[0], h->ev[4]);
  }
  if (tq) timer_add(h, 5, h->ev[3], h->ev[7]);
  return evaluate_complete(h);
}

// the evaluation's scalars, once they are in the pinned mirror
int evaluate_complete(scvt_handle* h) {
  Counters c;
  memcpy(&c, h->pinned + kPinCtr, sizeof(Counters));
  h->tF = h->pinned[kPinEval];
  h->tstep = h->pinned[kPinEval + 1];
  h->tg2 = h->pinned[kPinEval + 2];
  h->tmz = h->pinned[kPinEval + 3];
  h->tfb = c.n_fallback;
  h->tdeg = c.n_degenerate;
  h->twide[0] = c.tier_count[0];
  h->twide[1] = c.tier_count[1];
  if (c.n_duplicate > 0) return SCVT_E_DEGENERATE;
  if (c.n_error > 0) return SCVT_E_CERT;
  if (!(h->tF == h->tF) || !(h->tmz > 0.0)) return SCVT_E_NUMERIC;
  return SCVT_OK;
}

// Cells of Zsrc with their neighbour lists written to nbr (n x kVmax, the
// neighbours of a cell in increasing index order); uses the trial set's
// buffers, so the current evaluation is left as it is.
int geometry_with_neighbours(scvt_handle* h, const double* Zsrc, int32_t* nbr) {
  hipStream_t st = h->stream;
  std::swap(h->grid.order, h->grid.order_prev);  // last build's order drives this one
  HIPCK(launch_grid_build(Zsrc, h->n, h->grid, (int32_t*)h->ctr, st));  // also clears ctr
  CellArgs a = cell_args(h, Zsrc, h->trial);
  a.keep_cells = 1;
  a.out.cell_nbr = nbr;
  if (h->main_path) {
    HIPCK(launch_cells_main(a, st));
    HIPCK(launch_cells_tiers(a, st));
  }
  HIPCK(launch_cells_fallback(a, h->main_path ? 0 : 1, st));
  HIPCK(hipMemcpyAsync(h->pinned + kPinCtr, h->ctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  Counters c;
  memcpy(&c, h->pinned + kPinCtr, sizeof(Counters));
  if (c.n_duplicate > 0) return SCVT_E_DEGENERATE;
  if (c.n_error > 0) return SCVT_E_CERT;
  return SCVT_OK;
}

// device buffers of one call, freed on every return path
struct TempBufs {
  std::vector<void*> p;
  template <class T>
  T* get(size_t count) {
    void* v = nullptr;
    if (hipMalloc(&v, (count ? count : 1) * sizeof(T)) != hipSuccess) return nullptr;
    p.push_back(v);
    return (T*)v;
  }
  ~TempBufs() {
    for (void* v : p) hipFree(v);
  }
};

void swap_sets(scvt_handle* h) {
  EvalSet t = h->cur;
  h->cur = h->trial;
  h->trial = t;
  double* z = h->Z;
  h->Z = h->Zt;
  h->Zt = z;
}

void adopt_trial_scalars(scvt_handle* h) {
  h->F = h->tF;
  h->step_inf = h->tstep;
  h->gnorm2 = h->tg2;
  h->min_mz = h->tmz;
  h->n_fb = h->tfb;
  h->n_deg = h->tdeg;
  h->n_wide[0] = h->twide[0];
  h->n_wide[1] = h->twide[1];
}

// g . q of the direction just launched: into *gq after a host sync, or, with
// gq == nullptr, left on the device for the next evaluation's sync to bring
// (the direction timer is taken then too)
int finish_direction(scvt_handle* h, double* gq) {
  if (!gq) {
    h->dir_timer_pending = h->timing;
    return SCVT_OK;
  }
  HIPCK(hipMemcpyAsync(h->pinned + kPinGQ, h->dscal + kGQ, sizeof(double), hipMemcpyDeviceToHost,
                       h->stream));
  HIPCK(hipStreamSynchronize(h->stream));
  if (h->timing) timer_add(h, 3, h->ev[5], h->ev[6]);
  h->dir_timer_pending = false;
  *gq = h->pinned[kPinGQ];
  return SCVT_OK;
}

// P-LBFGS direction into h->q; g . q as finish_direction.
//
// Up to kHmax pairs: the two recursions run on the history's inner products
// (s_j.g from the last push, s_j.y_k kept as pairs arrive), so the vectors
// are streamed twice (q0 pass, direction pass), see lbfgs.h.
int direction_fused(scvt_handle* h, const double* hv, double* gq) {
  hipStream_t st = h->stream;
  const int64_t n3 = 3 * h->n;
  double* D = h->dscal;
  const int c = (int)h->ring.size();
  if (h->timing) HIPCK(hipEventRecord(h->ev[5], st));
  HistFinArgs f{};
  f.partials = h->hpart;
  f.nblocks = hist_grid(n3);
  f.c = c;
  f.stride = h->nslots;
  f.dscal = D;
  f.gram = h->gram;
  HistPassArgs p{};
  p.n3 = n3;
  p.c = c;
  p.g = h->cur.g;
  p.h = hv;
  p.partials = h->hpart;
  for (int j = 0; j < c; j++) {
    f.slot[j] = h->ring[j];
    p.S[j] = h->S + (size_t)h->ring[j] * n3;
    p.Y[j] = h->Y + (size_t)h->ring[j] * n3;
  }
  if (c > 0 && !h->backward_ready) {
    f.mode = kFinBackward;
    f.nvals = 0;
    HIPCK(L_hist_fin(h, f));
  }
  h->backward_ready = false;
  p.coef = D + kA;
  p.q = h->q;
  HIPCK(L_hist_q0(h, p));
  if (c > 0) {
    f.mode = kFinForward;
    f.nvals = c;
    HIPCK(L_hist_fin(h, f));
  }
  p.coef = D + kCoef;
  p.qin = h->q;
  p.q = h->q;
  HIPCK(L_hist_dir(h, p));
  f.mode = kFinGQ;
  f.nvals = 1;
  HIPCK(L_hist_fin(h, f));
  if (h->timing) HIPCK(hipEventRecord(h->ev[6], st));
  return finish_direction(h, gq);
}

// s_j . g for the stored pairs and s_j . y_k (j older than k), recomputed
// from the vectors (after a restored state); the same kernels' sums as the
// pushes that produced them, so the values are the same bits.
int hist_rebuild(scvt_handle* h) {
  const int c = (int)h->ring.size();
  if (h->M > kHmax || c == 0) return SCVT_OK;
  hipStream_t st = h->stream;
  const int64_t n3 = 3 * h->n;
  const int stride = h->nslots;
  auto S = [&](int j) { return h->S + (size_t)h->ring[j] * n3; };
  for (int k = 0; k <= c; k++) {  // k = c: against g; else against y_k
    const int cnt = k == c ? c : k;
    if (cnt == 0) continue;
    MultiDotArgs m{};
    m.n3 = n3;
    m.c = cnt;
    m.v = k == c ? h->cur.g : h->Y + (size_t)h->ring[k] * n3;
    m.partials = h->hpart;
    HistFinArgs f{};
    f.mode = kFinDots;
    f.partials = h->hpart;
    f.nblocks = hist_grid(n3);
    f.nvals = cnt;
    f.c = cnt;
    for (int j = 0; j < cnt; j++) {
      m.A[j] = S(j);
      f.dst[j] = k == c ? h->dscal + kSG + h->ring[j] : h->gram + h->ring[j] * stride + h->ring[k];
    }
    HIPCK(launch_multi_dot(m, st));
    HIPCK(launch_hist_fin(f, st));
  }
  HIPCK(hipStreamSynchronize(st));
  return SCVT_OK;
}

// y.y of every stored pair (plain LBFGS scaling) after a restored state
int yy_rebuild(scvt_handle* h) {
  const int64_t n3 = 3 * h->n;
  for (int slot : h->ring) {
    MultiDotArgs m{};
    m.n3 = n3;
    m.c = 1;
    m.A[0] = h->Y + (size_t)slot * n3;
    m.v = m.A[0];
    m.partials = h->hpart;
    HistFinArgs f{};
    f.mode = kFinDots;
    f.partials = h->hpart;
    f.nblocks = hist_grid(n3);
    f.nvals = 1;
    f.c = 1;
    f.dst[0] = h->dscal + kYY + slot;
    HIPCK(launch_multi_dot(m, h->stream));
    HIPCK(launch_hist_fin(f, h->stream));
  }
  HIPCK(hipStreamSynchronize(h->stream));
  return SCVT_OK;
}

// More than kHmax pairs: the two-loop as 2c+1 streaming passes; each pass
// finishes the previous pass's dot product from its block partials (no
// separate reduction launch), see lbfgs.hip.
int direction_passes(scvt_handle* h, const double* hv, double* gq) {
  hipStream_t st = h->stream;
  const int64_t n3 = 3 * h->n;
  double* D = h->dscal;
  const int c = (int)h->ring.size();
  auto S = [&](int j) { return h->S + (size_t)h->ring[j] * n3; };
  auto Y = [&](int j) { return h->Y + (size_t)h->ring[j] * n3; };
  auto R = [&](int j) { return D + kR + h->ring[j]; };
  double* pb[2] = {h->partials, h->partials + reduce_grid_max()};
  int cur = 0;
  if (h->timing) HIPCK(hipEventRecord(h->ev[5], st));
  PassArgs base{};
  base.n3 = n3;
  base.q = h->q;
  base.g = h->cur.g;
  base.h = hv;
  auto run = [&](PassArgs p) -> hipError_t {
    p.partials = pb[1 - cur];
    hipError_t e = launch_lbfgs_pass(p, st);
    cur = 1 - cur;
    return e;
  };
  if (c == 0) {
    PassArgs p = base;
    p.init_neg_g = 1;
    p.scale_h = 1;
    p.dot_vec = h->cur.g;
    HIPCK(run(p));
  } else {
    // backward loop, newest to oldest: a_j = r_j s_j.q ; q -= a_j y_j
    PassArgs b = base;
    b.init_neg_g = 1;
    b.dot_vec = S(c - 1);
    HIPCK(run(b));
    for (int j = c - 2; j >= 0; j--) {
      PassArgs m = base;
      m.prev_partials = pb[cur];
      m.prev_mul = R(j + 1);
      m.prev_store = D + kA + (j + 1);
      m.ax_vec = Y(j + 1);
      m.ax_sign = -1.0;
      m.dot_vec = S(j);
      HIPCK(run(m));
    }
    // turn-around: finish a_0, q -= a_0 y_0, apply diag(h), dot y_0.q
    PassArgs t = base;
    t.prev_partials = pb[cur];
    t.prev_mul = R(0);
    t.prev_store = D + kA;
    t.ax_vec = Y(0);
    t.ax_sign = -1.0;
    t.scale_h = 1;
    t.dot_vec = Y(0);
    HIPCK(run(t));
    // forward loop, oldest to newest: coef_j = a_j - r_j y_j.q ; q += coef_j s_j
    for (int j = 1; j <= c; j++) {
      PassArgs f = base;
      f.prev_partials = pb[cur];
      f.prev_mul = R(j - 1);
      f.prev_sub = D + kA + (j - 1);
      f.prev_store = D + kCoef + (j - 1);
      f.ax_vec = S(j - 1);
      f.ax_sign = 1.0;
      f.dot_vec = j < c ? Y(j) : h->cur.g;
      HIPCK(run(f));
    }
  }
  FinalizeArgs fa{};
  fa.partials = pb[cur];
  fa.nblocks = reduce_grid(n3);
  fa.nvals = 1;
  fa.out = D + kGQ;
  HIPCK(launch_finalize(fa, st));
  if (h->timing) HIPCK(hipEventRecord(h->ev[6], st));
  return finish_direction(h, gq);
}

// The initial inverse Hessian's diagonal: the Lloyd preconditioner h, or for
// plain LBFGS gamma_n = y.s / y.y of the newest stored pair (1 without one).
const double* initial_diag(scvt_handle* h) {
  if (h->cfg.method != SCVT_METHOD_LBFGS) return h->cur.h;
  const int newest = h->ring.empty() ? -1 : h->ring.back();
  if (launch_fill_gamma(h->hgam, h->n, h->dscal, newest < 0 ? -1 : kR + newest,
                        newest < 0 ? -1 : kYY + newest, h->stream) != hipSuccess)
    return nullptr;
  return h->hgam;
}

int direction(scvt_handle* h, double* gq) {
  Range range("scvt direction");
  const double* hv = initial_diag(h);
  if (!hv) return SCVT_E_HIP;
  return h->M <= kHmax ? direction_fused(h, hv, gq) : direction_passes(h, hv, gq);
}

// direction with no history and the Lloyd preconditioner: q = -h (.) g, the
// Lloyd step (z - h g = mu / (mu . z))
int lloyd_direction(scvt_handle* h, double* gq) {
  return h->M <= kHmax ? direction_fused(h, h->cur.h, gq) : direction_passes(h, h->cur.h, gq);
}

// Relative rise of F the Lloyd fallback may show and still count as a
// decrease: the evaluation's rounding (1e-13 relative in FP64; the mixed
// path's FP32 noise allowance when larger)
double lloyd_allowance(const scvt_handle* h) { return h->ls_noise > 1e-13 ? h->ls_noise : 1e-13; }

// Armijo's sufficient decrease for the trial just evaluated at step alpha
bool armijo(const scvt_handle* h, double alpha, double gq) {
  return h->tF <= h->F + h->cfg.ls_c1 * alpha * gq + h->ls_noise * fabs(h->F);
}

// Armijo backtracking along q from the current point, from the k0-th
// evaluation on (alpha = 2^-k0); on success the trial set holds the
// accepted evaluation.
int line_search(scvt_handle* h, double gq, int k0, bool* accepted, double* alpha_out) {
  double alpha = ldexp(1.0, -k0);
  *accepted = false;
  for (int k = k0; k < h->cfg.ls_max_evals; k++) {
    HIPCK(launch_normalize_trial(h->Z, h->q, alpha, h->Zt, h->n, h->stream));
    int rc = evaluate(h, h->Zt, h->trial, true);
    h->n_evals++;
    if (rc < 0) return rc;
    if (armijo(h, alpha, gq)) {
      *accepted = true;
      *alpha_out = alpha;
      return SCVT_OK;
    }
    alpha *= 0.5;
  }
  return SCVT_OK;
}

// s = Zt - Z and y = g_t - g of the trial into the history's next free
// slot, with y.s, |y|^2, |s|^2 and s_j . g_t, s_j . y for the stored pairs
// (block partials; fused history path)
hipError_t launch_push_ext_now(scvt_handle* h, int slot) {
  const int64_t n3 = 3 * h->n;
  PushExtArgs p{};
  p.n3 = n3;
  p.Z = h->Z;
  p.Zt = h->Zt;
  p.g = h->cur.g;
  p.gt = h->trial.g;
  p.s = h->S + (size_t)slot * n3;
  p.y = h->Y + (size_t)slot * n3;
  p.c = (int)h->ring.size();
  p.partials = h->hpart;
  for (int j = 0; j < p.c; j++) p.S[j] = h->S + (size_t)h->ring[j] * n3;
  return L_push_ext(h, p);
}

// the trial's push, ahead of its acceptance (a rejected trial's slot stays
// free and its partials are overwritten).  While the last pair's curvature
// test is pending, the slot must not be one the history held before that
// push: undoing the push restores that history, vectors included.
int launch_push_pre(scvt_handle* h) {
  int slot = -1;
  for (int k = (int)h->free_slots.size() - 1; k >= 0 && slot < 0; k--) {
    const int c = h->free_slots[k];
    bool held = false;
    if (h->push_pending)
      for (int r : h->ring_prev) held = held || r == c;
    if (!held) slot = c;
  }
  if (slot < 0) return SCVT_OK;  // no such slot: push_pair launches the push
  HIPCK(launch_push_ext_now(h, slot));
  h->pre_valid = true;
  h->pre_slot = slot;
  h->pre_ring = h->ring;
  return SCVT_OK;
}

int push_pair(scvt_handle* h) {
  if (h->M == 0) return SCVT_OK;
  // the slot of the push launched behind the trial's evaluation, if it was
  // launched for this history; else any free slot
  int slot_pos = (int)h->free_slots.size() - 1;
  if (h->pre_valid && h->pre_ring == h->ring)
    for (int k = 0; k < (int)h->free_slots.size(); k++)
      if (h->free_slots[k] == h->pre_slot) slot_pos = k;
  const int slot = h->free_slots[slot_pos];
  const int64_t n3 = 3 * h->n;
  // the history the pair joins (decided at the next host sync, resolve_push)
  std::vector<int> ring_next = h->ring;
  ring_next.push_back(slot);
  if ((int)ring_next.size() > h->M) ring_next.erase(ring_next.begin());
  if (h->M <= kHmax) {
    // also s_j . g_new and s_j . y_new for the stored pairs (next direction)
    const int c = (int)h->ring.size();
    HistFinArgs f{};
    f.mode = kFinPush;
    f.partials = h->hpart;
    f.nblocks = hist_grid(n3);
    f.nvals = 4 + 2 * c;
    f.c = c;
    f.p = slot;
    f.stride = h->nslots;
    f.dscal = h->dscal;
    f.gram = h->gram;
    for (int j = 0; j < c; j++) f.slot[j] = h->ring[j];
    // one launch: the push's scalars (also y.y into the slot's kYY entry),
    // then the next direction's backward recursion over the history with
    // the pair
    FinChain fc{};
    fc.n = 2;
    fc.step[0] = f;
    fc.step[1] = f;
    fc.step[1].mode = kFinBackward;
    fc.step[1].nvals = 0;
    fc.step[1].c = (int)ring_next.size();
    for (int j = 0; j < fc.step[1].c; j++) fc.step[1].slot[j] = ring_next[j];
    // the push launched behind the trial's evaluation serves if the history
    // is still the one it was launched for
    if (!(h->pre_valid && h->pre_slot == slot && h->pre_ring == h->ring))
      HIPCK(launch_push_ext_now(h, slot));
    h->pre_valid = false;
    HIPCK(L_fin_chain(h, fc));
    h->backward_ready = true;
  } else {
    PushArgs p{};
    p.n3 = n3;
    p.Z = h->Z;
    p.Zt = h->Zt;
    p.g = h->cur.g;
    p.gt = h->trial.g;
    p.s = h->S + (size_t)slot * n3;
    p.y = h->Y + (size_t)slot * n3;
    p.partials = h->partials + kPartPush * reduce_grid_max();
    HIPCK(launch_push(p, h->stream));
    FinalizeArgs fa{};
    fa.partials = p.partials;
    fa.nblocks = reduce_grid(n3);
    fa.nvals = 3;
    fa.out = h->dscal + kPush;
    fa.r_slot = h->dscal + kR + slot;
    HIPCK(launch_finalize(fa, h->stream));
    HIPCK(hipMemcpyAsync(h->dscal + kYY + slot, h->dscal + kPush + 1, sizeof(double),
                         hipMemcpyDeviceToDevice, h->stream));
  }
  // The pair joins the history now; the curvature test (section 2.2.2: a
  // pair enters only with y.s > 0) is taken at the next host sync, and
  // resolve_push restores the history if it fails.
  h->ring_prev = h->ring;
  h->free_prev = h->free_slots;
  h->free_slots.erase(h->free_slots.begin() + slot_pos);
  h->ring.push_back(slot);
  if ((int)h->ring.size() > h->M) {
    h->free_slots.push_back(h->ring.front());
    h->ring.erase(h->ring.begin());
  }
  h->push_pending = true;
  return SCVT_OK;
}

// Decides the pending push: y.s > curv_eps |y| |s| keeps the pair, anything
// else restores the history as it was before the push (*undone).  synced:
// the caller's last host sync already brought the scalars.
int resolve_push(scvt_handle* h, bool synced, bool* undone) {
  if (undone) *undone = false;
  if (!h->push_pending) return SCVT_OK;
  if (!synced) {
    HIPCK(hipMemcpyAsync(h->pinned + kPinPush, h->dscal + kPush, 3 * sizeof(double),
                         hipMemcpyDeviceToHost, h->stream));
    HIPCK(hipStreamSynchronize(h->stream));
  }
  h->push_pending = false;
  const double ys = h->pinned[kPinPush], yy = h->pinned[kPinPush + 1], ss = h->pinned[kPinPush + 2];
  if (!(ys > h->cfg.curv_eps * sqrt(yy * ss))) {
    h->ring = h->ring_prev;
    h->free_slots = h->free_prev;
    h->backward_ready = false;
    if (undone) *undone = true;
  }
  return SCVT_OK;
}

// every entry point other than the iteration loops starts from a decided
// history
int settle(scvt_handle* h) { return resolve_push(h, false, nullptr); }

void clear_history(scvt_handle* h) {
  h->backward_ready = false;
  for (int s : h->ring) h->free_slots.push_back(s);
  h->ring.clear();
}

int lloyd_step(scvt_handle* h) {
  int rc = lloyd_direction(h, nullptr);
  if (rc) return rc;
  HIPCK(launch_normalize_trial(h->Z, h->q, 1.0, h->Zt, h->n, h->stream));
  rc = evaluate(h, h->Zt, h->trial);
  h->n_evals++;
  if (rc < 0) return rc;
  swap_sets(h);
  adopt_trial_scalars(h);
  h->alpha = 1.0;
  h->iter++;
  record(h);
  return SCVT_OK;
}

// One P-LBFGS (or plain LBFGS) iteration.  The first trial (alpha = 1) is
// launched right behind the direction, so that one host sync -- the
// evaluation's -- brings g.q, the trial's energy and the curvature scalars
// of the previous push; the speculative parts (the previous pair's place in
// the history, a direction that turns out not to descend) are redone in the
// rare case they were wrong, and not counted as evaluations.
int quasi_newton_step(scvt_handle* h) {
  int rc;
  for (;;) {
    rc = direction(h, nullptr);
    if (rc) return rc;
    HIPCK(launch_normalize_trial(h->Z, h->q, 1.0, h->Zt, h->n, h->stream));
    rc = evaluate(h, h->Zt, h->trial, true);
    if (rc == SCVT_E_HIP) return rc;  // no scalars arrived
    bool undone = false;
    const int rc2 = resolve_push(h, true, &undone);
    if (rc2) return rc2;
    if (!undone) break;  // else: the direction used a pair the history does not hold
  }
  if (rc < 0) return rc;
  double gq = h->pinned[kPinGQ];
  bool ok = false;
  double alpha = 1.0;
  if (!(gq < 0.0)) {
    // not a descent direction: back to the Lloyd direction (no history)
    clear_history(h);
    rc = direction(h, &gq);
    if (rc) return rc;
    rc = line_search(h, gq, 0, &ok, &alpha);
  } else {
    h->n_evals++;
    ok = armijo(h, 1.0, gq);
    if (!ok) rc = line_search(h, gq, 1, &ok, &alpha);
  }
  if (rc) return rc;
  if (!ok) {
    // No sufficient decrease along the direction within ls_max_evals
    // evaluations -- near convergence the energy differences fall below the
    // evaluation's rounding (the mixed path's FP32 quadrature above all).
    // Take the Lloyd step (alpha = 1 along -h g, i.e. z <- mu/|mu|), which
    // decreases F without a line search (section 2.2.1), and restart the
    // history from there.
    clear_history(h);
    rc = lloyd_direction(h, nullptr);
    if (rc) return rc;
    HIPCK(launch_normalize_trial(h->Z, h->q, 1.0, h->Zt, h->n, h->stream));
    rc = evaluate(h, h->Zt, h->trial, true);
    h->n_evals++;
    if (rc < 0) return rc;
    // Lloyd's step lowers the exact energy (section 2.2.1); if the evaluated
    // energy rose beyond its rounding allowance (the quadrature of very
    // large cells can do that), stop here: the generators stay where they
    // are, with the history cleared
    if (!(h->tF <= h->F + lloyd_allowance(h) * fabs(h->F))) return SCVT_E_LINESEARCH;
    alpha = 1.0;
    h->n_lloyd_fallback++;
  }
  rc = push_pair(h);
  if (rc) return rc;
  swap_sets(h);
  adopt_trial_scalars(h);
  h->alpha = alpha;
  h->iter++;
  record(h);
  return SCVT_OK;
}

// lazy: leave the last push's curvature test to the next iteration's sync
// (the solve loops); otherwise decide it before returning
int do_step(scvt_handle* h, bool lazy) {
  int rc = h->cfg.method == SCVT_METHOD_LLOYD ? lloyd_step(h) : quasi_newton_step(h);
  if (!rc && !lazy) rc = settle(h);
  return rc;
}

void fill_info(scvt_handle* h, scvt_info* info, int status) {
  if (!info) return;
  info->iter = h->iter;
  info->n_evals = h->n_evals;
  info->F = h->F;
  info->grad_norm2 = sqrt(h->gnorm2);
  info->step_inf = h->step_inf;
  info->alpha = h->alpha;
  info->n_fallback = h->n_fb;
  info->n_degenerate = h->n_deg;
  info->status = status;
  info->hist_len = (int32_t)h->ring.size();
  info->n_lloyd_fallback = h->n_lloyd_fallback;
  info->n_wide[0] = h->n_wide[0];
  info->n_wide[1] = h->n_wide[1];
}

void destroy(scvt_handle* h) {
  if (!h) return;
  if (h->stream) hipStreamSynchronize(h->stream);
  for (void* p : h->allocs) hipFree(p);
  if (h->pinned && !h->batched) hipHostFree(h->pinned);
  for (auto& e : h->ev)
    if (e) hipEventDestroy(e);
  if (h->ev_copy) hipEventDestroy(h->ev_copy);
  if (h->own_stream && h->stream) hipStreamDestroy(h->stream);
  delete h;
}

int alloc_device_state(scvt_handle* h) {
  const int64_t n = h->n;
  const int M = h->M;
  h->grid.g = make_grid(n);
  const int64_t nc = h->grid.g.ncells;
  ALLOC(h->Z, 3 * n);
  ALLOC(h->Zt, 3 * n);
  ALLOC(h->q, 3 * n);
  ALLOC(h->R, n);
  int rc = alloc_set(h, h->cur);
  if (rc) return rc;
  rc = alloc_set(h, h->trial);
  if (rc) return rc;
  h->nslots = M > 0 ? M + 2 : 0;
  if (M > 0) {
    ALLOC(h->S, (size_t)h->nslots * 3 * n);
    ALLOC(h->Y, (size_t)h->nslots * 3 * n);
  }
  ALLOC(h->dscal, kNScal);
  h->ctr = reinterpret_cast<Counters*>(h->dscal + kCtr);
  ALLOC(h->partials, kPartTotal * reduce_grid_max());
  ALLOC(h->gram, (size_t)h->nslots * h->nslots);
  if (h->cfg.method == SCVT_METHOD_LBFGS) ALLOC(h->hgam, n);
  ALLOC(h->hpart, hist_grid_max());
  ALLOC(h->fb_list, n);
  ALLOC(h->tier_list[0], n);
  ALLOC(h->tier_list[1], n);
  ALLOC(h->grid.cnt2, 2 * (nc + 1));
  ALLOC(h->grid.start_tot, nc + 1);
  ALLOC(h->grid.start_home, nc + 1);
  ALLOC(h->grid.cell3, 3 * n);
  h->grid.cap_entries = 3 * n;
  ALLOC(h->grid.entries, 3 * n);
  ALLOC(h->grid.order, n);
  ALLOC(h->grid.order_prev, n);
  ALLOC(h->grid.scan_tmp, 2 * ((nc + 1) / 2048 + 2));
  ALLOC(h->grid.overflow, 1);
  if (h->rho.poly_n > 0) {
    RhoPoly* t = nullptr;
    ALLOC(t, h->rho.poly_n);
    h->rho.poly_tab = t;
  }
  for (int b = 0; h->rho.polyx_n > 0 && b < (h->rho.nbumps == 2 ? 2 : 1); b++) {
    RhoPoly* t = nullptr;
    ALLOC(t, h->rho.polyx_n);
    h->rho.polyx_tab[b] = t;
  }
  return SCVT_OK;
}

int init_device_state(scvt_handle* h) {
  int rc = alloc_device_state(h);
  if (rc) return rc;
  const int64_t n = h->n;
  const int M = h->M;
  const int64_t nc = h->grid.g.ncells;
  if (!h->batched) {  // batched: the server's pinned scalars, no events (no timing)
    static_assert(64 * sizeof(double) == kBatchPinnedBytes, "pinned scalars");
    if (hipHostMalloc((void**)&h->pinned, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess)
      return SCVT_E_OOM;
    if (hipEventCreateWithFlags(&h->ev_copy, hipEventDisableTiming) != hipSuccess) return SCVT_E_HIP;
    // timing only, read after a stream synchronisation: no system-scope fence
    // (which writes back and invalidates caches at every record)
    for (auto& e : h->ev)
      if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return SCVT_E_HIP;
  }
  hipStream_t st = h->stream;
  HIPCK(launch_fill_i32(h->grid.cnt2, 0, 2 * (nc + 1), st));
  HIPCK(launch_fill_i32(h->grid.overflow, 0, 1, st));
  HIPCK(launch_iota(h->grid.order, n, st));  // first build: generator order
  HIPCK(launch_fill_i32((int32_t*)h->R, 0, 2 * n, st));
  HIPCK(launch_fill_i32((int32_t*)h->dscal, 0, 2 * kNScal, st));
  HIPCK(launch_fill_i32((int32_t*)h->q, 0, 6 * n, st));
  HIPCK(launch_poly_table(h->rho, const_cast<RhoPoly*>(h->rho.poly_tab),
                          const_cast<RhoPoly*>(h->rho.polyx_tab[0]),
                          const_cast<RhoPoly*>(h->rho.polyx_tab[1]), st));
  for (int s = h->nslots - 1; s >= 0; s--) h->free_slots.push_back(s);
  h->main_path = n > 256 ? 1 : 0;
  h->r_default = 2.0 * sqrt(4.0 * 3.141592653589793 / (double)n);
  return SCVT_OK;
}

}  // namespace

// ============================================================ batched mode
// The P-LBFGS iteration of quasi_newton_step (with scvt_solve's late
// curvature decision) as a state machine: each state records the launches
// of one evaluation (and what precedes it) into a round, and batch_finish
// takes the decision quasi_newton_step takes after that evaluation's host
// sync.  The evaluations, their order and their results are those of
// scvt_solve (the trial's early push aside, which only moves work earlier).
namespace scvt {

enum BatchState : int {
  kBEval0 = 0,  // the initial evaluation
  kBIter,       // direction and the first trial (alpha = 1)
  kBRestart,    // not a descent direction: history cleared, Lloyd direction, alpha = 1
  kBSearch,     // backtracking: trial at balpha
  kBLloyd,      // no sufficient decrease: the Lloyd step
  kBDone
};

int batch_create(const scvt_config* cfg, const double* z0, void* arena, size_t arena_bytes,
                 double* pinned, void* stream, int64_t max_iter, double tol, scvt_handle** out) {
  if (!out || !z0 || !arena || !pinned || !stream) return SCVT_E_INVALID;
  *out = nullptr;
  int rc = validate(cfg);
  if (rc) return rc;
  if (cfg->method != SCVT_METHOD_PLBFGS || cfg->m_hist > kHmax) return SCVT_E_INVALID;
  const int64_t n = cfg->n;
  for (int64_t k = 0; k < 3 * n; k++)
    if (!isfinite(z0[k])) return SCVT_E_INVALID;
  for (int64_t i = 0; i < n; i++)
    if (z0[3 * i] == 0.0 && z0[3 * i + 1] == 0.0 && z0[3 * i + 2] == 0.0) return SCVT_E_DEGENERATE;
  scvt_handle* h = new (std::nothrow) scvt_handle();
  if (!h) return SCVT_E_OOM;
  h->cfg = *cfg;
  h->cfg.hip_stream = stream;
  h->n = n;
  h->M = cfg->m_hist;
  h->rho = to_dev(cfg->rho);
  h->ls_noise = cfg->ls_noise >= 0.0 ? cfg->ls_noise : (cfg->precision == SCVT_MIXED ? 1e-8 : 0.0);
  h->stream = (hipStream_t)stream;
  h->batched = true;
  h->arena = (char*)arena;
  h->arena_bytes = arena_bytes;
  h->pinned = pinned;
  h->bmax_iter = max_iter;
  h->btol = tol;
  h->bstate = kBEval0;
  rc = init_device_state(h);
  if (!rc)
    rc = hip_err(hipMemcpyAsync(h->Zt, z0, 3 * n * sizeof(double), hipMemcpyHostToDevice, h->stream));
  if (rc) {
    destroy(h);
    return rc;
  }
  *out = h;
  return SCVT_OK;
}

int batch_plan(scvt_handle* h, Round& r) {
  h->rec = &r;
  int rc = SCVT_OK;
  switch (h->bstate) {
    case kBEval0:  // rows normalised to the sphere, then evaluated
      rc = hip_err(L_normalize(h, h->Zt, nullptr, 0.0, h->Z));
      if (!rc) rc = record_evaluation(h, h->Z, h->cur);
      break;
    case kBIter:
    case kBRestart:
    case kBLloyd:  // (the history is already cleared for the last two)
      rc = direction(h, nullptr);
      if (!rc) rc = hip_err(L_normalize(h, h->Z, h->q, 1.0, h->Zt));
      if (!rc) rc = record_evaluation(h, h->Zt, h->trial);
      break;
    case kBSearch:
      rc = hip_err(L_normalize(h, h->Z, h->q, h->balpha, h->Zt));
      if (!rc) rc = record_evaluation(h, h->Zt, h->trial);
      break;
    default:
      rc = SCVT_E_INVALID;
  }
  h->rec = nullptr;
  return rc;
}

namespace {

// the solve's status once an iterate is adopted: SCVT_PENDING to go on
int batch_status(scvt_handle* h) {
  if (h->step_inf < h->btol) return SCVT_OK;
  if (h->iter >= h->bmax_iter) return SCVT_NOT_CONVERGED;
  return SCVT_PENDING;
}

// the trial is the next iterate (quasi_newton_step's tail): the history push
// goes into the next round unless the solve stops here
int batch_accept(scvt_handle* h, double alpha, Round& next) {
  const bool last = h->tstep < h->btol || h->iter + 1 >= h->bmax_iter;
  if (!last) {
    h->rec = &next;
    const int rc = push_pair(h);
    h->rec = nullptr;
    if (rc) return rc;
  }
  swap_sets(h);
  adopt_trial_scalars(h);
  h->alpha = alpha;
  h->iter++;
  record(h);
  h->bstate = kBIter;
  return batch_status(h);
}

// Armijo failed at the k-th trial of the line search along the direction
int batch_backtrack(scvt_handle* h, int k) {
  if (k + 1 < h->cfg.ls_max_evals) {
    h->bk = k + 1;
    h->balpha = ldexp(1.0, -(k + 1));
    h->bstate = kBSearch;
  } else {
    clear_history(h);
    h->bstate = kBLloyd;
  }
  return SCVT_PENDING;
}

}  // namespace

int batch_finish(scvt_handle* h, Round& next) {
  const int st = h->bstate;
  int rc = evaluate_complete(h);
  if (rc < 0) {
    h->bstate = kBDone;
    return rc;
  }
  switch (st) {
    case kBEval0:
      h->n_evals = 1;
      adopt_trial_scalars(h);
      record(h);
      h->bstate = kBIter;
      return batch_status(h);
    case kBIter: {
      bool undone = false;
      rc = resolve_push(h, true, &undone);
      if (rc) return rc;
      if (undone) return SCVT_PENDING;  // the direction used a pair the history does not hold
      const double gq = h->pinned[kPinGQ];
      if (!(gq < 0.0)) {  // not a descent direction: back to the Lloyd direction
        clear_history(h);
        h->bstate = kBRestart;
        return SCVT_PENDING;
      }
      h->n_evals++;
      h->bgq = gq;
      if (armijo(h, 1.0, gq)) return batch_accept(h, 1.0, next);
      return batch_backtrack(h, 0);
    }
    case kBRestart: {  // the first trial of the line search along the Lloyd direction
      h->bgq = h->pinned[kPinGQ];
      h->n_evals++;
      if (armijo(h, 1.0, h->bgq)) return batch_accept(h, 1.0, next);
      return batch_backtrack(h, 0);
    }
    case kBSearch:
      h->n_evals++;
      if (armijo(h, h->balpha, h->bgq)) return batch_accept(h, h->balpha, next);
      return batch_backtrack(h, h->bk);
    case kBLloyd:
      h->n_evals++;
      if (!(h->tF <= h->F + lloyd_allowance(h) * fabs(h->F))) {
        h->bstate = kBDone;
        return SCVT_E_LINESEARCH;
      }
      h->n_lloyd_fallback++;
      return batch_accept(h, 1.0, next);
    default:
      return SCVT_E_INVALID;
  }
}

void batch_info(scvt_handle* h, scvt_info* info, int status) { fill_info(h, info, status); }

void batch_destroy(scvt_handle* h) { destroy(h); }

}  // namespace scvt

// =============================================================== C ABI ====
extern "C" {

int scvt_footprint(const scvt_config* cfg, size_t* bytes) try {
  if (!bytes) return SCVT_E_INVALID;
  int rc = validate(cfg);
  if (rc) return rc;
  scvt_handle* h = new (std::nothrow) scvt_handle();
  if (!h) return SCVT_E_OOM;
  h->cfg = *cfg;
  h->n = cfg->n;
  h->M = cfg->m_hist;
  h->rho = to_dev(cfg->rho);
  h->dry_run = true;
  rc = alloc_device_state(h);
  *bytes = h->dry_bytes;
  delete h;
  return rc;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

int scvt_config_init(scvt_config* c, int64_t n) try {
  if (!c) return SCVT_E_INVALID;
  memset(c, 0, sizeof(*c));
  c->n = n;
  c->m_hist = 7;
  c->precision = SCVT_FP64;
  c->rho.kind = SCVT_RHO_CONST;
  c->rho.nbumps = 0;
  c->rho.w_lon = 1.0;
  c->rho.w_lat = 1.0;
  c->quad_levels = 2;
  c->quad_rule = 7;
  c->ls_max_evals = 10;
  c->ls_c1 = 1e-4;
  c->curv_eps = 1e-10;
  c->ls_noise = -1.0;
  c->keep_cells = 0;
  c->hip_stream = nullptr;
  return SCVT_OK;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

int scvt_create(const scvt_config* cfg, const double* z0, int z0_on_device, scvt_handle** out) try {
  if (!out) return SCVT_E_INVALID;
  *out = nullptr;
  int rc = validate(cfg);
  if (rc) return rc;
  if (!z0) return SCVT_E_INVALID;
  const int64_t n = cfg->n;
  if (!z0_on_device) {
    for (int64_t k = 0; k < 3 * n; k++)
      if (!isfinite(z0[k])) return SCVT_E_INVALID;
    for (int64_t i = 0; i < n; i++)
      if (z0[3 * i] == 0.0 && z0[3 * i + 1] == 0.0 && z0[3 * i + 2] == 0.0)
        return SCVT_E_DEGENERATE;
  }
  scvt_handle* h = new (std::nothrow) scvt_handle();
  if (!h) return SCVT_E_OOM;
  h->cfg = *cfg;
  h->n = n;
  h->M = cfg->m_hist;
  h->rho = to_dev(cfg->rho);
  h->ls_noise = cfg->ls_noise >= 0.0 ? cfg->ls_noise : (cfg->precision == SCVT_MIXED ? 1e-8 : 0.0);
  if (cfg->hip_stream) {
    h->stream = (hipStream_t)cfg->hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
      delete h;
      return SCVT_E_HIP;
    }
    h->own_stream = true;
  }
  rc = init_device_state(h);
  if (!rc) {
    hipError_t e = hipMemcpyAsync(h->Zt, z0, 3 * n * sizeof(double),
                                  z0_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                  h->stream);
    if (e == hipSuccess) e = launch_normalize_trial(h->Zt, nullptr, 0.0, h->Z, n, h->stream);
    rc = hip_err(e);
  }
  if (!rc) {
    rc = evaluate(h, h->Z, h->cur);
    h->n_evals = 1;
    if (!rc) {
      adopt_trial_scalars(h);
      record(h);
    }
  }
  if (rc) {
    destroy(h);
    return rc;
  }
  *out = h;
  return SCVT_OK;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

int scvt_get_records(scvt_handle* h, int64_t max, scvt_info* out, int64_t* count) try {
  if (!h || max < 0 || (max > 0 && !out)) return SCVT_E_INVALID;
  const int64_t kept = (int64_t)h->records.size();
  const int64_t m = max < kept ? max : kept;
  // the last m records, oldest first: record k of the run sits at k mod ring
  for (int64_t t = 0; t < m; t++) {
    const int64_t k = h->rec_total - m + t;
    out[t] = h->records[(size_t)(k % SCVT_RECORD_RING)];
  }
  if (count) *count = m;
  return SCVT_OK;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

int scvt_step(scvt_handle* h, scvt_info* info) try {
  if (!h) return SCVT_E_INVALID;
  Range range("scvt_step");
  int rc = settle(h);
  if (!rc) rc = do_step(h, false);
  fill_info(h, info, rc);
  return rc;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

int scvt_solve(scvt_handle* h, int64_t max_iter, double tol, scvt_info* info) try {
  if (!h) return SCVT_E_INVALID;
  Range range("scvt_solve");
  int rc = SCVT_OK;
  while (!(h->step_inf < tol) && h->iter < max_iter) {
    rc = do_step(h, true);
    if (rc) break;
  }
  const int rs = settle(h);
  if (!rc) rc = rs;
  if (!rc && !(h->step_inf < tol)) rc = SCVT_NOT_CONVERGED;
  fill_info(h, info, rc);
  return rc;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

int scvt_solve_rel(scvt_handle* h, int64_t max_iter, double step_tol, double grad_rel_tol,
                   double f_rel_tol, scvt_info* info) try {
  if (!h) return SCVT_E_INVALID;
  Range range("scvt_solve_rel");
  const bool qn = h->cfg.method != SCVT_METHOD_LLOYD;
  int rc = SCVT_OK;
  bool done = false;
  double F_prev = h->F;
  bool have_prev = false;
  for (;;) {
    if (step_tol > 0.0 && h->step_inf < step_tol) done = true;
    if (qn && grad_rel_tol > 0.0 && sqrt(h->gnorm2) / h->F <= grad_rel_tol) done = true;
    if (qn && f_rel_tol > 0.0 && have_prev && fabs(F_prev - h->F) / F_prev < f_rel_tol)
      done = true;
    if (done || h->iter >= max_iter) break;
    F_prev = h->F;
    have_prev = true;
    rc = do_step(h, true);
    if (rc) break;
  }
  const int rs = settle(h);
  if (!rc) rc = rs;
  if (!rc && !done) rc = SCVT_NOT_CONVERGED;
  fill_info(h, info, rc);
  return rc;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

int scvt_energy(scvt_handle* h, double* F, double* mass, double* centroid, double* e_cell,
                int on_dev) try {
  if (!h) return SCVT_E_INVALID;
  const int64_t n = h->n;
  const hipMemcpyKind k = on_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (F) *F = h->F;
  if (mass) HIPCK(hipMemcpyAsync(mass, h->cur.m, n * sizeof(double), k, h->stream));
  if (e_cell) HIPCK(hipMemcpyAsync(e_cell, h->cur.e, n * sizeof(double), k, h->stream));
  if (centroid) {
    if (on_dev) {
      HIPCK(launch_centroid(h->cur.mu, h->cur.m, centroid, n, h->stream));
    } else {
      HIPCK(launch_centroid(h->cur.mu, h->cur.m, h->q, n, h->stream));
      HIPCK(hipMemcpyAsync(centroid, h->q, 3 * n * sizeof(double), k, h->stream));
    }
  }
  HIPCK(hipStreamSynchronize(h->stream));
  return SCVT_OK;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

int scvt_get_generators(scvt_handle* h, double* z, int on_dev) try {
  if (!h || !z) return SCVT_E_INVALID;
  HIPCK(hipMemcpyAsync(z, h->Z, 3 * h->n * sizeof(double),
                       on_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->stream));
  HIPCK(hipStreamSynchronize(h->stream));
  return SCVT_OK;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

int scvt_get_vectors(scvt_handle* h, int which, double* out, int on_dev) try {
  if (!h || !out) return SCVT_E_INVALID;
  const int64_t n = h->n;
  const double* src = nullptr;
  int64_t cnt = 3 * n;
  switch (which) {
    case 0: src = h->cur.g; break;
    case 1: src = h->cur.h; cnt = n; break;
    case 2: src = h->cur.lloyd; break;
    case 3: src = h->cur.mu; break;
    case 4: src = h->q; break;
    case 5: src = h->R; cnt = n; break;
    default: return SCVT_E_INVALID;
  }
  HIPCK(hipMemcpyAsync(out, src, cnt * sizeof(double),
                       on_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->stream));
  HIPCK(hipStreamSynchronize(h->stream));
  return SCVT_OK;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

int scvt_direction(scvt_handle* h, double* out, int on_dev, double* gq) try {
  if (!h) return SCVT_E_INVALID;
  double v = 0.0;
  int rc = settle(h);
  if (!rc) rc = direction(h, &v);
  if (rc) return rc;
  if (gq) *gq = v;
  if (out) return scvt_get_vectors(h, 4, out, on_dev);
  return SCVT_OK;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

int scvt_num_generators(scvt_handle* h, int64_t* n) try {
  if (!h || !n) return SCVT_E_INVALID;
  *n = h->n;
  return SCVT_OK;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

int scvt_refine(scvt_handle* h, double* z_out, int on_device, int64_t* n_out) try {
  if (!h || !n_out) return SCVT_E_INVALID;
  const int64_t n = h->n;
  hipStream_t st = h->stream;
  TempBufs t;
  int32_t* nbr = t.get<int32_t>((size_t)n * kVmax);
  int32_t* cnt = t.get<int32_t>(n);
  int32_t* off = t.get<int32_t>(n + 1);
  int32_t* junk = t.get<int32_t>(n + 1);
  int32_t* tmp = t.get<int32_t>(scan_tmp_ints(n));
  if (!nbr || !cnt || !off || !junk || !tmp) return SCVT_E_OOM;
  int rc = geometry_with_neighbours(h, h->Z, nbr);
  if (rc) return rc;
  HIPCK(launch_refine_count(h->trial.deg, nbr, n, cnt, st));
  HIPCK(launch_scan_pair(cnt, cnt, n, tmp, off, junk, st));
  int32_t edges = 0;
  HIPCK(hipMemcpyAsync(&edges, off + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  const int64_t m = n + edges;
  *n_out = m;
  if (!z_out) return SCVT_OK;
  double* dst = z_out;
  if (!on_device) {
    dst = t.get<double>((size_t)3 * m);
    if (!dst) return SCVT_E_OOM;
  }
  HIPCK(launch_refine_emit(h->Z, h->trial.deg, nbr, off, n, dst, st));
  if (!on_device)
    HIPCK(hipMemcpyAsync(z_out, dst, 3 * m * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  return SCVT_OK;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

}  // extern "C"

// ---- refinement without allocation ----------------------------------------
// scvt_refine's temporary buffers (neighbour lists, per-cell edge counts and
// their scan) live in one static device array per GPU, sized for
// SCVT_REFINE_NOALLOC_MAX_N generators.  Host code never passes the array's
// name to a kernel or a copy: it stands for a device symbol, whose address
// on each device comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[(size_t)96 << 20];

namespace {

struct NoAllocLayout {
  size_t nbr, cnt, off, junk, tmp, bytes;  // byte offsets, total
};

constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }

NoAllocLayout noalloc_layout(int64_t n) {
  NoAllocLayout L{};
  size_t o = 0;
  L.nbr = o;
  o += align256((size_t)n * kVmax * sizeof(int32_t));
  L.cnt = o;
  o += align256((size_t)n * sizeof(int32_t));
  L.off = o;
  o += align256((size_t)(n + 1) * sizeof(int32_t));
  L.junk = o;
  o += align256((size_t)(n + 1) * sizeof(int32_t));
  L.tmp = o;
  o += align256((size_t)scan_tmp_ints(n) * sizeof(int32_t));
  L.bytes = o;
  return L;
}

constexpr size_t kNoAllocScratchBytes = sizeof(scratch);
constexpr int kNoAllocMaxDevices = 64;

std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocMaxDevices] = {};

// the current device's copy of the scratch array (looked up once per device)
int scratch_ptr(void** out) {
  int dev = -1;
  HIPCK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocMaxDevices) return SCVT_E_INVALID;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return SCVT_E_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SCVT_OK;
}

}  // namespace

extern "C" {

int scvt_refine_noalloc(scvt_handle* h, double* z_out, int64_t* n_out) try {
  if (!h || !n_out) return SCVT_E_INVALID;
  const int64_t n = h->n;
  if (n > SCVT_REFINE_NOALLOC_MAX_N) return SCVT_E_OOM;
  const NoAllocLayout L = noalloc_layout(n);
  if (L.bytes > kNoAllocScratchBytes) return SCVT_E_OOM;
  void* base = nullptr;
  int rc = scratch_ptr(&base);
  if (rc) return rc;
  unsigned char* b = (unsigned char*)base;
  int32_t* nbr = (int32_t*)(b + L.nbr);
  int32_t* cnt = (int32_t*)(b + L.cnt);
  int32_t* off = (int32_t*)(b + L.off);
  int32_t* junk = (int32_t*)(b + L.junk);
  int32_t* tmp = (int32_t*)(b + L.tmp);
  hipStream_t st = h->stream;
  // every scratch word read below is written first in this call (neighbour
  // lists and counts per cell, the scan's tiles), so nothing is cleared
  rc = geometry_with_neighbours(h, h->Z, nbr);
  if (rc) return rc;
  HIPCK(launch_refine_count(h->trial.deg, nbr, n, cnt, st));
  HIPCK(launch_scan_pair(cnt, cnt, n, tmp, off, junk, st));
  int32_t* edges = (int32_t*)(h->pinned + kPinWords);  // the handle's pinned words
  HIPCK(hipMemcpyAsync(edges, off + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  const int64_t m = n + *edges;
  *n_out = m;
  if (!z_out) return SCVT_OK;
  HIPCK(launch_refine_emit(h->Z, h->trial.deg, nbr, off, n, z_out, st));
  HIPCK(hipStreamSynchronize(st));
  return SCVT_OK;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

int scvt_mesh(scvt_handle* h, int32_t* tri, int64_t* ntri, double* cell_q, double* tri_q) try {
  if (!h || !ntri) return SCVT_E_INVALID;
  const int64_t n = h->n;
  hipStream_t st = h->stream;
  TempBufs t;
  int32_t* nbr = t.get<int32_t>((size_t)n * kVmax);
  int32_t* cnt = t.get<int32_t>(n);
  int32_t* off = t.get<int32_t>(n + 1);
  int32_t* junk = t.get<int32_t>(n + 1);
  int32_t* tmp = t.get<int32_t>(scan_tmp_ints(n));
  if (!nbr || !cnt || !off || !junk || !tmp) return SCVT_E_OOM;
  int rc = geometry_with_neighbours(h, h->Z, nbr);
  if (rc) return rc;
  const double* edges = h->trial.edges;
  HIPCK(launch_tri_list(h->trial.deg, nbr, edges, n, nullptr, cnt, nullptr, st));
  HIPCK(launch_scan_pair(cnt, cnt, n, tmp, off, junk, st));
  int32_t total = 0;
  HIPCK(hipMemcpyAsync(&total, off + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  *ntri = total;
  if (cell_q) {
    double* cq = t.get<double>(n);
    if (!cq) return SCVT_E_OOM;
    HIPCK(launch_cell_quality(h->trial.deg, edges, n, cq, st));
    HIPCK(hipMemcpyAsync(cell_q, cq, n * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  if (tri || tri_q) {
    int32_t* td = t.get<int32_t>((size_t)3 * total);
    if (!td) return SCVT_E_OOM;
    HIPCK(launch_tri_list(h->trial.deg, nbr, edges, n, off, nullptr, td, st));
    if (tri) HIPCK(hipMemcpyAsync(tri, td, 3 * total * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (tri_q) {
      double* tq = t.get<double>(total);
      if (!tq) return SCVT_E_OOM;
      HIPCK(launch_tri_quality(h->Z, td, total, tq, st));
      HIPCK(hipMemcpyAsync(tri_q, tq, total * sizeof(double), hipMemcpyDeviceToHost, st));
    }
  }
  HIPCK(hipStreamSynchronize(st));
  return SCVT_OK;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

int scvt_multilevel(const scvt_config* cfg0, const double* z0, int z0_on_device, int levels,
                    int64_t max_iter, double tol, scvt_info* infos, scvt_handle** out) try {
  if (!cfg0 || !z0 || !out || levels < 0 || max_iter < 0) return SCVT_E_INVALID;
  *out = nullptr;
  scvt_handle* h = nullptr;
  int rc = scvt_create(cfg0, z0, z0_on_device, &h);
  if (rc) return rc;
  rc = scvt_solve(h, max_iter, tol, infos ? &infos[0] : nullptr);
  for (int l = 1; l <= levels && rc >= 0; l++) {
    int64_t m = 0;
    rc = scvt_refine(h, nullptr, 1, &m);
    if (rc) break;
    if (m > ((int64_t)1 << 28)) {
      rc = SCVT_E_INVALID;
      break;
    }
    double* z = nullptr;
    if (hipMalloc(&z, 3 * m * sizeof(double)) != hipSuccess) {
      rc = SCVT_E_OOM;
      break;
    }
    rc = scvt_refine(h, z, 1, &m);
    scvt_handle* h2 = nullptr;
    if (!rc) {
      scvt_config cfg = h->cfg;
      cfg.n = m;
      cfg.hip_stream = h->own_stream ? nullptr : h->stream;
      rc = scvt_create(&cfg, z, 1, &h2);  // synchronises before it returns
    }
    hipFree(z);
    if (rc) break;
    destroy(h);
    h = h2;
    rc = scvt_solve(h, max_iter, tol, infos ? &infos[l] : nullptr);
  }
  if (rc < 0) {
    destroy(h);
    return rc;
  }
  *out = h;
  return rc;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

int scvt_get_cells(scvt_handle* h, int32_t max_deg, int32_t* nbr, int32_t* deg, double* verts,
                   uint8_t* flags) try {
  if (!h || max_deg != kVmax) return SCVT_E_INVALID;
  const int64_t n = h->n;
  hipStream_t st = h->stream;
  if ((nbr || verts) && !h->cfg.keep_cells) return SCVT_E_INVALID;
  if (nbr)
    HIPCK(hipMemcpyAsync(nbr, h->cur.cell_nbr, n * kVmax * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  if (verts)
    HIPCK(hipMemcpyAsync(verts, h->cur.edges, n * kVmax * 6 * sizeof(double),
                         hipMemcpyDeviceToHost, st));
  if (deg) HIPCK(hipMemcpyAsync(deg, h->cur.deg, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  if (flags) HIPCK(hipMemcpyAsync(flags, h->cur.flags, n, hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  return SCVT_OK;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

// state blob: int64 header[8] = {magic, n, M, ring size, iter, n_evals, 0, 0},
// double alpha, then Z (3n), then per ring entry oldest first: r, s (3n), y (3n)
int scvt_get_state(scvt_handle* h, void* buf, size_t* bytes) try {
  if (!h || !bytes) return SCVT_E_INVALID;
  const int rs = settle(h);
  if (rs) return rs;
  const int64_t n3 = 3 * h->n;
  const size_t c = h->ring.size();
  const size_t need = 8 * sizeof(int64_t) + sizeof(double) + n3 * sizeof(double) +
                      c * (sizeof(double) + 2 * n3 * sizeof(double));
  if (!buf) {
    *bytes = need;
    return SCVT_OK;
  }
  if (*bytes < need) return SCVT_E_INVALID;
  char* p = (char*)buf;
  int64_t hdr[8] = {kStateMagic, h->n, h->M, (int64_t)c, h->iter, h->n_evals, 0, 0};
  memcpy(p, hdr, sizeof(hdr));
  p += sizeof(hdr);
  memcpy(p, &h->alpha, sizeof(double));
  p += sizeof(double);
  hipStream_t st = h->stream;
  HIPCK(hipMemcpyAsync(p, h->Z, n3 * sizeof(double), hipMemcpyDeviceToHost, st));
  p += n3 * sizeof(double);
  std::vector<double> rr(c);
  for (size_t j = 0; j < c; j++) {
    int slot = h->ring[j];
    HIPCK(hipMemcpyAsync(&rr[j], h->dscal + kR + slot, sizeof(double), hipMemcpyDeviceToHost, st));
  }
  HIPCK(hipStreamSynchronize(st));
  for (size_t j = 0; j < c; j++) {
    int slot = h->ring[j];
    memcpy(p, &rr[j], sizeof(double));
    p += sizeof(double);
    HIPCK(hipMemcpy(p, h->S + (size_t)slot * n3, n3 * sizeof(double), hipMemcpyDeviceToHost));
    p += n3 * sizeof(double);
    HIPCK(hipMemcpy(p, h->Y + (size_t)slot * n3, n3 * sizeof(double), hipMemcpyDeviceToHost));
    p += n3 * sizeof(double);
  }
  *bytes = need;
  return SCVT_OK;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

int scvt_set_state(scvt_handle* h, const void* buf, size_t bytes) try {
  if (!h || !buf || bytes < 8 * sizeof(int64_t) + sizeof(double)) return SCVT_E_INVALID;
  const char* p = (const char*)buf;
  int64_t hdr[8];
  memcpy(hdr, p, sizeof(hdr));
  p += sizeof(hdr);
  const int64_t n3 = 3 * h->n;
  const int64_t c = hdr[3];
  if (hdr[0] != kStateMagic || hdr[1] != h->n || hdr[2] != h->M || c < 0 || c > h->M)
    return SCVT_E_INVALID;
  const size_t need = 8 * sizeof(int64_t) + sizeof(double) + n3 * sizeof(double) +
                      c * (sizeof(double) + 2 * n3 * sizeof(double));
  if (bytes < need) return SCVT_E_INVALID;
  double alpha;
  memcpy(&alpha, p, sizeof(double));
  p += sizeof(double);
  hipStream_t st = h->stream;
  HIPCK(hipStreamSynchronize(st));
  h->push_pending = false;  // the restored history replaces it
  HIPCK(hipMemcpy(h->Z, p, n3 * sizeof(double), hipMemcpyHostToDevice));
  p += n3 * sizeof(double);
  clear_history(h);
  for (int64_t j = 0; j < c; j++) {
    int slot = h->free_slots.back();
    h->free_slots.pop_back();
    double r;
    memcpy(&r, p, sizeof(double));
    p += sizeof(double);
    HIPCK(hipMemcpy(h->dscal + kR + slot, &r, sizeof(double), hipMemcpyHostToDevice));
    HIPCK(hipMemcpy(h->S + (size_t)slot * n3, p, n3 * sizeof(double), hipMemcpyHostToDevice));
    p += n3 * sizeof(double);
    HIPCK(hipMemcpy(h->Y + (size_t)slot * n3, p, n3 * sizeof(double), hipMemcpyHostToDevice));
    p += n3 * sizeof(double);
    h->ring.push_back(slot);
  }
  h->iter = hdr[4];
  h->n_evals = hdr[5];
  h->alpha = alpha;
  int rc = evaluate(h, h->Z, h->cur);
  if (!rc) adopt_trial_scalars(h);
  if (!rc) rc = hist_rebuild(h);
  if (!rc && h->cfg.method == SCVT_METHOD_LBFGS) rc = yy_rebuild(h);
  return rc;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

int scvt_set_timing(scvt_handle* h, int enable) try {
  if (!h) return SCVT_E_INVALID;
  h->timing = enable == 1;
  h->timing_quad = enable == 1 || enable == 2;
  for (auto& t : h->timers) t = Timer{};
  return SCVT_OK;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

int scvt_kernel_time(scvt_handle* h, int kernel, double* total_ms, int64_t* launches) try {
  if (!h || kernel < 0 || kernel >= kTimers) return SCVT_E_INVALID;
  if (total_ms) *total_ms = h->timers[kernel].ms;
  if (launches) *launches = h->timers[kernel].launches;
  return SCVT_OK;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

void scvt_destroy(scvt_handle* h) { destroy(h); }

const char* scvt_strerror(int code) {
  switch (code) {
    case SCVT_OK: return "ok";
    case SCVT_NOT_CONVERGED: return "not converged (iteration cap reached)";
    case SCVT_PENDING: return "pending";
    case SCVT_E_INVALID: return "invalid argument";
    case SCVT_E_OOM: return "out of device memory";
    case SCVT_E_DEGENERATE: return "degenerate generators (duplicate or zero)";
    case SCVT_E_CERT: return "a Voronoi cell could not be built";
    case SCVT_E_LINESEARCH: return "line search failed after reset";
    case SCVT_E_NUMERIC: return "numeric failure (NaN or mu.z <= 0)";
    case SCVT_E_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

}  // extern "C"
