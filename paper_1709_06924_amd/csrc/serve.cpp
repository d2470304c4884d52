// Serving engine: a persistent request loop over the solver.
//
// Requests (generators, density, tolerance, iteration cap) are submitted at
// any time.  Admission: a request enters when a slot is free and its device
// footprint fits in what the budget has left (first come, first served; a
// request larger than the whole budget is rejected at submission).  Every
// admitted request gets its own HIP stream and handle -- generators, cells
// and LBFGS history stay resident in HBM until it finishes -- and is driven
// by one of the server's host threads, so the kernels of all admitted
// requests are in flight together on the device.  Finished requests release
// their slot and memory at once and the next waiting request is admitted:
// continuous batching at iteration granularity.  All kernels are
// deterministic, so a request's result does not depend on what else runs.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/scvt.h"

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
};

}  // namespace

struct scvt_server {
  size_t budget = 0, used = 0;
  int max_slots = 1, running = 0;
  int device = 0;
  int64_t next_id = 1;
  bool stop = false;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::map<int64_t, Request*> reqs;
  std::vector<std::thread> workers;
};

namespace {

void run_request(scvt_server* s, Request* r) {
  hipSetDevice(s->device);
  hipStream_t st = nullptr;
  int rc = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess ? SCVT_OK : SCVT_E_HIP;
  scvt_handle* h = nullptr;
  if (!rc) {
    r->cfg.hip_stream = st;
    rc = scvt_create(&r->cfg, r->z0.data(), 0, &h);
  }
  if (!rc) {
    rc = scvt_solve(h, r->max_iter, r->tol, &r->info);
    if (rc >= 0) {
      r->z.assign(r->z0.size(), 0.0);
      int rc2 = scvt_get_generators(h, r->z.data(), 0);
      if (rc2) rc = rc2;
    }
  }
  if (h) scvt_destroy(h);
  if (st) hipStreamDestroy(st);
  std::lock_guard<std::mutex> lk(s->mu);
  r->rc = rc;
  r->info.status = rc;
  r->state = rc >= 0 ? kDone : kFailed;
  r->t_done = now_s();
  r->z0.clear();
  r->z0.shrink_to_fit();
  s->used -= r->footprint;
  s->running--;
  s->cv.notify_all();
}

void worker(scvt_server* s) {
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait(lk, [&] {
        if (s->stop) return true;
        if (s->queue.empty() || s->running >= s->max_slots) return false;
        return s->used + s->queue.front()->footprint <= s->budget;
      });
      if (s->stop) return;
      r = s->queue.front();
      s->queue.pop_front();
      s->used += r->footprint;
      s->running++;
      r->state = kRunning;
      r->t_start = now_s();
    }
    run_request(s, r);
  }
}

}  // namespace

extern "C" {

int scvt_server_create(size_t hbm_budget, int max_slots, scvt_server** out) {
  if (!out || max_slots < 1 || max_slots > 64 || hbm_budget == 0) return SCVT_E_INVALID;
  *out = nullptr;
  scvt_server* s = new (std::nothrow) scvt_server();
  if (!s) return SCVT_E_OOM;
  s->budget = hbm_budget;
  s->max_slots = max_slots;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return SCVT_E_HIP;
  }
  try {
    for (int k = 0; k < max_slots; k++) s->workers.emplace_back(worker, s);
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv.notify_all();
    for (auto& t : s->workers) t.join();
    delete s;
    return SCVT_E_OOM;
  }
  *out = s;
  return SCVT_OK;
}

int scvt_server_submit(scvt_server* s, const scvt_config* cfg, const double* z0, double tol,
                       int64_t max_iter, int64_t* req_id) {
  if (!s || !cfg || !z0 || !req_id || cfg->n < 4 || max_iter < 0) return SCVT_E_INVALID;
  size_t fp = 0;
  int rc = scvt_footprint(cfg, &fp);
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
  r->cfg = *cfg;
  r->cfg.keep_cells = 0;
  r->tol = tol;
  r->max_iter = max_iter;
  r->footprint = fp;
  r->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->id = s->next_id++;
    s->reqs[r->id] = r;
    s->queue.push_back(r);
  }
  s->cv.notify_all();
  *req_id = r->id;
  return SCVT_OK;
}

int scvt_server_poll(scvt_server* s, int64_t req_id, double* z_out, scvt_info* info,
                     double* times) {
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
  if (z_out && r->state == kDone)
    for (size_t k = 0; k < r->z.size(); k++) z_out[k] = r->z[k];
  return r->rc;
}

int scvt_server_release(scvt_server* s, int64_t req_id) {
  if (!s) return SCVT_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(req_id);
  if (it == s->reqs.end()) return SCVT_E_INVALID;
  Request* r = it->second;
  if (r->state == kWaiting || r->state == kRunning) return SCVT_PENDING;
  delete r;
  s->reqs.erase(it);
  return SCVT_OK;
}

int scvt_server_stats(scvt_server* s, int64_t* waiting, int64_t* running, size_t* bytes_used) {
  if (!s) return SCVT_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  if (waiting) *waiting = (int64_t)s->queue.size();
  if (running) *running = s->running;
  if (bytes_used) *bytes_used = s->used;
  return SCVT_OK;
}

void scvt_server_destroy(scvt_server* s) {
  if (!s) return;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    // waiting requests are dropped; running ones finish first
    for (Request* r : s->queue) r->state = kFailed;
    s->queue.clear();
    s->cv.wait(lk, [&] { return s->running == 0; });
    s->stop = true;
  }
  s->cv.notify_all();
  for (auto& t : s->workers) t.join();
  for (auto& kv : s->reqs) delete kv.second;
  delete s;
}

}  // extern "C"
