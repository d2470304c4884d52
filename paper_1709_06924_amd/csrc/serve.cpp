// Serving engine: continuous batching of SCVT solves with segmented launches.
//
// Requests (generators, density, tolerance, iteration cap) are submitted at
// any time.  Admission: a request enters when one of max_slots slots is free
// and its exact device footprint (scvt_footprint) fits in a free range of
// the server's arena -- one device allocation of hbm_budget bytes made at
// creation -- first come, first served; a request larger than the budget is
// rejected at submission.  An admitted request's generators, cells and LBFGS
// history live in its arena range until it finishes; nothing is allocated
// or freed per request.
//
// One driver thread runs rounds: every admitted request records the
// launches of its next evaluation (direction passes, trial point, grid,
// cells, quadrature, reductions) into the round, and the round issues one
// launch per kernel for all of them (blockIdx.y = request, round.h), gathers
// every request's scalars with one copy and synchronises once.  Then each
// request takes its own decision (Armijo test, history update, stopping
// test) and the next round begins, with newly admitted requests joining and
// finished ones leaving at round boundaries: continuous batching at the
// granularity of one evaluation.  A request's blocks compute exactly what
// its own single launches would, so its result does not depend on the mix.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/scvt.h"
#include "arena.h"
#include "engine_batch.h"
#include "round.h"

using namespace scvt;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

enum ReqState { kWaiting = 0, kRunning = 1, kDone = 2, kFailed = 3 };

struct Request {
  int64_t id = 0;
  scvt_config cfg{};
  std::vector<double> z0, z;
  double tol = 0.0;
  int64_t max_iter = 0;
  size_t footprint = 0;
  int state = kWaiting;
  int rc = 0;
  scvt_info info{};
  double t_submit = 0, t_start = 0, t_done = 0;
  // while admitted (driver thread only)
  size_t off = 0;     // arena range
  int slot = -1;      // pinned scalars
  scvt_handle* h = nullptr;
};

constexpr size_t kRoundTableBytes = (size_t)4 << 20;  // argument tables of one round
constexpr int kScalarsPerRequest = 16;                // gathered doubles per request and round

}  // namespace

struct scvt_server {
  size_t budget = 0, used = 0;
  int max_slots = 1;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int64_t next_id = 1;
  bool stop = false;
  bool dead = false;  // the driver thread ended on a failed host allocation
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::map<int64_t, Request*> reqs;
  std::vector<Request*> active;  // admitted (driver thread; membership under mu)
  int running = 0;
  Arena arena;
  char* arena_base = nullptr;
  double* pinned = nullptr;  // kBatchPinnedBytes per slot
  std::vector<int> free_slots;
  RoundBuffers rb;
  std::thread driver;
};

namespace {

void finish_request(scvt_server* s, Request* r, int rc) {
  if (r->h) {
    batch_info(r->h, &r->info, rc);
    if (rc >= 0) {
      r->z.assign(3 * (size_t)r->cfg.n, 0.0);
      const int rc2 = scvt_get_generators(r->h, r->z.data(), 0);
      if (rc2) rc = rc2;
    }
    batch_destroy(r->h);
    r->h = nullptr;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  r->rc = rc;
  r->info.status = rc;
  r->state = rc >= 0 ? kDone : kFailed;
  r->t_done = now_s();
  r->z0.clear();
  r->z0.shrink_to_fit();
  s->arena.give(r->off, r->footprint);
  s->used -= r->footprint;
  s->free_slots.push_back(r->slot);
  s->running--;
  s->cv.notify_all();
}

// admit waiting requests in order while a slot and an arena range are free
// (called with mu held); returns the admitted ones
std::vector<Request*> admit(scvt_server* s) {
  std::vector<Request*> in;
  while (!s->queue.empty() && !s->free_slots.empty()) {
    Request* r = s->queue.front();
    size_t off = 0;
    if (!s->arena.take(r->footprint, &off)) break;  // first come, first served
    s->queue.pop_front();
    r->off = off;
    r->slot = s->free_slots.back();
    s->free_slots.pop_back();
    s->used += r->footprint;
    s->running++;
    r->state = kRunning;
    r->t_start = now_s();
    in.push_back(r);
  }
  return in;
}

void driver_loop(scvt_server* s) {
  hipSetDevice(s->device);
  Round round, next;  // next: launches one round leaves for the following one
  for (;;) {
    std::vector<Request*> in;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait(lk, [&] {
        return s->stop || !s->active.empty() || (!s->queue.empty() && !s->free_slots.empty());
      });
      if (s->stop && s->active.empty()) return;
      if (!s->stop) in = admit(s);
    }
    for (Request* r : in) {
      const int rc = batch_create(&r->cfg, r->z0.data(), s->arena_base + r->off, r->footprint,
                                  s->pinned + (size_t)r->slot * (kBatchPinnedBytes / sizeof(double)),
                                  s->stream, r->max_iter, r->tol, &r->h);
      if (rc) {
        if (r->h) batch_destroy(r->h);
        r->h = nullptr;
        finish_request(s, r, rc);
      } else {
        std::lock_guard<std::mutex> lk(s->mu);
        s->active.push_back(r);
      }
    }
    if (s->active.empty()) continue;
    // one round: the history pushes the last one left, then every admitted
    // request's next evaluation
    std::swap(round, next);
    next.clear();
    std::vector<int> plan_rc(s->active.size(), SCVT_OK);
    for (size_t k = 0; k < s->active.size(); k++) plan_rc[k] = batch_plan(s->active[k]->h, round);
    roctxRangePushA("scvt serving round");  // planning is host work; this is the round itself
    const hipError_t e = round_run(round, s->rb, s->stream);
    roctxRangePop();
    round.clear();
    std::vector<Request*> keep, done;
    std::vector<int> codes;
    for (size_t k = 0; k < s->active.size(); k++) {
      Request* r = s->active[k];
      const int rc = e != hipSuccess ? SCVT_E_HIP : (plan_rc[k] ? plan_rc[k] : batch_finish(r->h, next));
      if (rc == SCVT_PENDING) {
        keep.push_back(r);
      } else {
        done.push_back(r);
        codes.push_back(rc);
      }
    }
    // (a request records launches for the next round only when it goes on:
    // its last iteration pushes no pair)
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->active = keep;
    }
    for (size_t k = 0; k < done.size(); k++) finish_request(s, done[k], codes[k]);
  }
}

// The driver thread: a failed host allocation ends it, and every request
// still admitted or waiting then fails with SCVT_E_OOM (as do later
// submissions) instead of the exception ending the process.
void driver(scvt_server* s) {
  try {
    driver_loop(s);
  } catch (...) {
    std::lock_guard<std::mutex> lk(s->mu);
    for (Request* r : s->active) {
      if (r->h) batch_destroy(r->h);
      r->h = nullptr;
      r->rc = r->info.status = SCVT_E_OOM;
      r->state = kFailed;
    }
    for (Request* r : s->queue) {
      r->rc = r->info.status = SCVT_E_OOM;
      r->state = kFailed;
    }
    s->active.clear();
    s->queue.clear();
    s->dead = true;
    s->cv.notify_all();
  }
}

void free_server(scvt_server* s) {
  if (s->rb.dev) hipFree(s->rb.dev);
  if (s->rb.host) hipHostFree(s->rb.host);
  if (s->rb.dscal) hipFree(s->rb.dscal);
  if (s->rb.hscal) hipHostFree(s->rb.hscal);
  if (s->pinned) hipHostFree(s->pinned);
  if (s->arena_base) hipFree(s->arena_base);
  if (s->own_stream && s->stream) hipStreamDestroy(s->stream);
  delete s;
}

}  // namespace

extern "C" {

int scvt_server_create(size_t hbm_budget, int max_slots, void* stream, scvt_server** out) try {
  if (!out || max_slots < 1 || max_slots > 64 || hbm_budget < 256) return SCVT_E_INVALID;
  *out = nullptr;
  scvt_server* s = new (std::nothrow) scvt_server();
  if (!s) return SCVT_E_OOM;
  s->budget = hbm_budget / 256 * 256;
  s->max_slots = max_slots;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return SCVT_E_HIP;
  }
  int rc = SCVT_OK;
  if (stream) {
    s->stream = (hipStream_t)stream;
  } else if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) == hipSuccess) {
    s->own_stream = true;
  } else {
    rc = SCVT_E_HIP;
  }
  // everything the server will ever use, allocated here
  if (!rc && hipMalloc((void**)&s->arena_base, s->budget) != hipSuccess) rc = SCVT_E_OOM;
  if (!rc && hipHostMalloc((void**)&s->pinned, max_slots * kBatchPinnedBytes, hipHostMallocDefault) !=
                 hipSuccess)
    rc = SCVT_E_OOM;
  s->rb.bytes = kRoundTableBytes;
  s->rb.max_scal = max_slots * kScalarsPerRequest;
  if (!rc && hipMalloc(&s->rb.dev, s->rb.bytes) != hipSuccess) rc = SCVT_E_OOM;
  if (!rc && hipHostMalloc(&s->rb.host, s->rb.bytes, hipHostMallocDefault) != hipSuccess)
    rc = SCVT_E_OOM;
  if (!rc && hipMalloc((void**)&s->rb.dscal, s->rb.max_scal * sizeof(double)) != hipSuccess)
    rc = SCVT_E_OOM;
  if (!rc && hipHostMalloc((void**)&s->rb.hscal, s->rb.max_scal * sizeof(double),
                           hipHostMallocDefault) != hipSuccess)
    rc = SCVT_E_OOM;
  if (rc) {
    free_server(s);
    return rc;
  }
  s->arena.free[0] = s->budget;
  for (int k = max_slots - 1; k >= 0; k--) s->free_slots.push_back(k);
  try {
    s->driver = std::thread(driver, s);
  } catch (...) {
    free_server(s);
    return SCVT_E_OOM;
  }
  *out = s;
  return SCVT_OK;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

int scvt_server_submit(scvt_server* s, const scvt_config* cfg, const double* z0, double tol,
                       int64_t max_iter, int64_t* req_id) try {
  if (!s || !cfg || !z0 || !req_id || cfg->n < 4 || max_iter < 0) return SCVT_E_INVALID;
  if (cfg->method != SCVT_METHOD_PLBFGS || cfg->m_hist > 16) return SCVT_E_INVALID;
  scvt_config c = *cfg;
  c.keep_cells = 0;
  size_t fp = 0;
  int rc = scvt_footprint(&c, &fp);
  if (rc) return rc;
  if (fp > s->budget) return SCVT_E_OOM;
  Request* r = new (std::nothrow) Request();
  if (!r) return SCVT_E_OOM;
  try {
    r->z0.assign(z0, z0 + 3 * cfg->n);
  } catch (...) {
    delete r;
    return SCVT_E_OOM;
  }
  r->cfg = c;
  r->tol = tol;
  r->max_iter = max_iter;
  r->footprint = fp;
  r->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->dead) {
      delete r;
      return SCVT_E_OOM;
    }
    r->id = s->next_id++;
    try {
      s->reqs[r->id] = r;
      s->queue.push_back(r);
    } catch (...) {
      s->reqs.erase(r->id);
      delete r;
      return SCVT_E_OOM;
    }
  }
  s->cv.notify_all();
  *req_id = r->id;
  return SCVT_OK;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

int scvt_server_poll(scvt_server* s, int64_t req_id, double* z_out, scvt_info* info,
                     double* times) try {
  if (!s) return SCVT_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(req_id);
  if (it == s->reqs.end()) return SCVT_E_INVALID;
  Request* r = it->second;
  if (r->state == kWaiting || r->state == kRunning) return SCVT_PENDING;
  if (info) *info = r->info;
  if (times) {
    times[0] = r->t_submit;
    times[1] = r->t_start;
    times[2] = r->t_done;
  }
  if (z_out && r->state == kDone) memcpy(z_out, r->z.data(), r->z.size() * sizeof(double));
  return r->rc;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

int scvt_server_release(scvt_server* s, int64_t req_id) try {
  if (!s) return SCVT_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(req_id);
  if (it == s->reqs.end()) return SCVT_E_INVALID;
  Request* r = it->second;
  if (r->state == kWaiting || r->state == kRunning) return SCVT_PENDING;
  delete r;
  s->reqs.erase(it);
  return SCVT_OK;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

int scvt_server_stats(scvt_server* s, int64_t* waiting, int64_t* running, size_t* bytes_used) try {
  if (!s) return SCVT_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  if (waiting) *waiting = (int64_t)s->queue.size();
  if (running) *running = s->running;
  if (bytes_used) *bytes_used = s->used;
  return SCVT_OK;
} catch (...) {  // host allocation (no exception leaves the C ABI)
  return SCVT_E_OOM;
}

void scvt_server_destroy(scvt_server* s) try {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    // waiting requests are dropped; running ones finish first
    for (Request* r : s->queue) r->state = kFailed;
    s->queue.clear();
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->driver.joinable()) s->driver.join();
  hipStreamSynchronize(s->stream);
  for (auto& kv : s->reqs) delete kv.second;
  free_server(s);
} catch (...) {
}

}  // extern "C"
