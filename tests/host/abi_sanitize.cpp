// The library's host code (engine.cpp, serve.cpp) under AddressSanitizer and
// UndefinedBehaviorSanitizer: this program, linked with sanitized host
// objects of the library and its unchanged GPU kernels, drives every entry
// point of include/scvt.h on small problems -- solves in both precisions and
// with every optimiser, state round trips, the record ring's wrap, cells,
// mesh and refinement, the multilevel driver, argument errors -- and a
// server with more requests than slots, polled and released from this thread
// while its driver thread runs rounds.  It checks return codes and a few
// invariants; the sanitizers check the memory and arithmetic of the host
// code.  Exit status 0 when every check held.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <thread>
#include <vector>

#include "../../include/scvt.h"

static int g_fail = 0;
#define CHECK(cond)                                                              \
  do {                                                                           \
    if (!(cond)) {                                                               \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond);         \
      g_fail = 1;                                                                \
    }                                                                            \
  } while (0)

// n points on the unit sphere from a seeded 64-bit LCG (Marsaglia's method)
static std::vector<double> points(int64_t n, uint64_t seed) {
  std::vector<double> z(3 * n);
  uint64_t s = seed * 6364136223846793005ull + 1442695040888963407ull;
  auto u = [&]() {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(s >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
  };
  for (int64_t i = 0; i < n; i++) {
    double a, b, q;
    do {
      a = u();
      b = u();
      q = a * a + b * b;
    } while (q >= 1.0 || q == 0.0);
    const double r = 2.0 * sqrt(1.0 - q);
    z[3 * i] = a * r;
    z[3 * i + 1] = b * r;
    z[3 * i + 2] = 1.0 - 2.0 * q;
  }
  return z;
}

static scvt_density tanh_bump(double scale) {
  scvt_density d;
  memset(&d, 0, sizeof(d));
  d.kind = SCVT_RHO_TANH;
  d.nbumps = 1;
  d.xc[0][0] = 0.0;
  d.xc[0][1] = 0.8660254037844387;
  d.xc[0][2] = 0.5;
  d.beta[0] = 0.3490658503988659;
  d.alpha[0] = 0.15;
  d.gamma = 1.0 / (scale * scale * scale * scale);
  d.amp[0] = 1.0 - d.gamma;
  d.w_lon = d.w_lat = 1.0;
  return d;
}

static void one_handle(int64_t n, int precision, int method, const scvt_density& rho, int keep) {
  scvt_config c;
  CHECK(scvt_config_init(&c, n) == SCVT_OK);
  c.m_hist = 5;
  c.precision = precision;
  c.method = method;
  c.rho = rho;
  c.keep_cells = keep;
  const std::vector<double> z0 = points(n, (uint64_t)n + 17 * method + 3 * precision);
  scvt_handle* h = nullptr;
  CHECK(scvt_create(&c, z0.data(), 0, &h) == SCVT_OK);
  if (!h) return;
  scvt_info info;
  CHECK(scvt_step(h, &info) == SCVT_OK);
  const int rc = scvt_solve(h, 12, 1e-14, &info);
  CHECK(rc == SCVT_OK || rc == SCVT_NOT_CONVERGED);
  CHECK(info.iter == 12);  // max_iter counts from the start
  std::vector<double> m(n), cen(3 * n), e(n), z(3 * n), v(3 * n);
  double F = 0.0;
  CHECK(scvt_energy(h, &F, m.data(), cen.data(), e.data(), 0) == SCVT_OK);
  double msum = 0.0;
  for (double x : m) msum += x;
  CHECK(F > 0.0 && msum > 0.0);
  CHECK(scvt_get_generators(h, z.data(), 0) == SCVT_OK);
  for (int w = 0; w <= 5; w++) CHECK(scvt_get_vectors(h, w, v.data(), 0) == SCVT_OK);
  double gq = 0.0;
  if (method != SCVT_METHOD_LLOYD) CHECK(scvt_direction(h, v.data(), 0, &gq) == SCVT_OK);
  // the record ring: the initial evaluation and one record per iteration
  std::vector<scvt_info> rec(64);
  int64_t cnt = -1;
  CHECK(scvt_get_records(h, 64, rec.data(), &cnt) == SCVT_OK);
  CHECK(cnt == 13 && rec[12].iter == 12);
  CHECK(scvt_get_records(h, 0, nullptr, &cnt) == SCVT_OK && cnt == 0);
  CHECK(scvt_get_records(h, 3, nullptr, &cnt) == SCVT_E_INVALID);
  // state round trip
  size_t bytes = 0;
  CHECK(scvt_get_state(h, nullptr, &bytes) == SCVT_OK && bytes > 0);
  std::vector<char> st(bytes);
  CHECK(scvt_get_state(h, st.data(), &bytes) == SCVT_OK);
  CHECK(scvt_set_state(h, st.data(), bytes) == SCVT_OK);
  CHECK(scvt_set_state(h, st.data(), bytes / 2) != SCVT_OK);
  // timers
  CHECK(scvt_set_timing(h, 1) == SCVT_OK);
  CHECK(scvt_step(h, &info) == SCVT_OK);
  double ms = 0.0;
  int64_t launches = 0;
  for (int k = 0; k <= 6; k++) CHECK(scvt_kernel_time(h, k, &ms, &launches) == SCVT_OK);
  CHECK(scvt_set_timing(h, 0) == SCVT_OK);
  if (keep) {
    std::vector<int32_t> nbr(32 * n), deg(n);
    std::vector<double> verts(32 * 6 * n);
    std::vector<uint8_t> flags(n);
    CHECK(scvt_get_cells(h, 32, nbr.data(), deg.data(), verts.data(), flags.data()) == SCVT_OK);
    int64_t dsum = 0;
    for (int32_t d : deg) dsum += d;
    CHECK(dsum == 6 * n - 12);
    int64_t ntri = 0;
    CHECK(scvt_mesh(h, nullptr, &ntri, nullptr, nullptr) == SCVT_OK && ntri == 2 * n - 4);
    std::vector<int32_t> tri(3 * ntri);
    std::vector<double> cq(n), tq(ntri);
    CHECK(scvt_mesh(h, tri.data(), &ntri, cq.data(), tq.data()) == SCVT_OK);
    int64_t nr = 0;
    CHECK(scvt_refine(h, nullptr, 0, &nr) == SCVT_OK && nr == 4 * n - 6);
    std::vector<double> zr(3 * nr);
    CHECK(scvt_refine(h, zr.data(), 0, &nr) == SCVT_OK);
  }
  int64_t nn = 0;
  CHECK(scvt_num_generators(h, &nn) == SCVT_OK && nn == n);
  scvt_destroy(h);
}

static void ring_wrap() {
  // more iterations than the record ring holds (Lloyd: cheap, no history)
  const int64_t n = 642;
  scvt_config c;
  scvt_config_init(&c, n);
  c.method = SCVT_METHOD_LLOYD;
  c.m_hist = 0;
  const std::vector<double> z0 = points(n, 5);
  scvt_handle* h = nullptr;
  CHECK(scvt_create(&c, z0.data(), 0, &h) == SCVT_OK);
  if (!h) return;
  scvt_info info;
  const int64_t iters = SCVT_RECORD_RING + 37;
  const int rc = scvt_solve(h, iters, 0.0, &info);
  CHECK(rc == SCVT_NOT_CONVERGED || rc == SCVT_OK);
  std::vector<scvt_info> rec(SCVT_RECORD_RING + 5);
  int64_t cnt = 0;
  CHECK(scvt_get_records(h, SCVT_RECORD_RING + 5, rec.data(), &cnt) == SCVT_OK);
  CHECK(cnt == SCVT_RECORD_RING);
  CHECK(rec[cnt - 1].iter == info.iter && rec[0].iter == info.iter - SCVT_RECORD_RING + 1);
  scvt_destroy(h);
}

static void argument_errors() {
  scvt_config c;
  scvt_config_init(&c, 3);
  scvt_handle* h = nullptr;
  const std::vector<double> z0 = points(100, 9);
  CHECK(scvt_create(&c, z0.data(), 0, &h) == SCVT_E_INVALID && h == nullptr);
  CHECK(scvt_create(nullptr, z0.data(), 0, &h) == SCVT_E_INVALID);
  scvt_config_init(&c, 100);
  CHECK(scvt_create(&c, nullptr, 0, &h) == SCVT_E_INVALID);
  std::vector<double> dup(z0);
  for (int k = 0; k < 3; k++) dup[3 + k] = dup[k];
  const int rc = scvt_create(&c, dup.data(), 0, &h);
  CHECK(rc == SCVT_E_DEGENERATE);
  if (rc == SCVT_OK) scvt_destroy(h);
  CHECK(scvt_step(nullptr, nullptr) == SCVT_E_INVALID);
  size_t fp = 0;
  scvt_config_init(&c, 1 << 20);
  CHECK(scvt_footprint(&c, &fp) == SCVT_OK && fp > 0);
  for (int code = -7; code <= 2; code++) CHECK(scvt_strerror(code) != nullptr);
  scvt_destroy(nullptr);
}

static void multilevel() {
  scvt_config c;
  scvt_config_init(&c, 642);
  const std::vector<double> z0 = points(642, 11);
  scvt_info infos[3];
  scvt_handle* h = nullptr;
  const int rc = scvt_multilevel(&c, z0.data(), 0, 2, 15, 1e-14, infos, &h);
  CHECK(rc == SCVT_OK || rc == SCVT_NOT_CONVERGED);
  int64_t n = 0;
  if (h) {
    CHECK(scvt_num_generators(h, &n) == SCVT_OK && n == 16 * 642 - 30);
    scvt_destroy(h);
  }
}

static void serving() {
  scvt_server* s = nullptr;
  CHECK(scvt_server_create((size_t)2 << 30, 3, nullptr, &s) == SCVT_OK);
  if (!s) return;
  const int64_t sizes[8] = {642, 2562, 1000, 5000, 10242, 3000, 642, 8000};
  std::vector<int64_t> ids;
  for (int r = 0; r < 8; r++) {
    scvt_config c;
    scvt_config_init(&c, sizes[r]);
    c.m_hist = 5 + r % 3;
    c.precision = r % 2 ? SCVT_MIXED : SCVT_FP64;
    if (r % 3 == 1) c.rho = tanh_bump(4.0);
    const std::vector<double> z0 = points(sizes[r], 100 + r);
    int64_t id = -1;
    CHECK(scvt_server_submit(s, &c, z0.data(), 1e-14, 25, &id) == SCVT_OK);
    ids.push_back(id);
  }
  // rejected at submission: over the whole budget, another method
  {
    scvt_config c;
    scvt_config_init(&c, 1 << 24);
    const std::vector<double> z0 = points(16, 1);
    int64_t id = -1;
    CHECK(scvt_server_submit(s, &c, z0.data(), 1e-8, 10, &id) == SCVT_E_INVALID ||
          scvt_server_submit(s, &c, z0.data(), 1e-8, 10, &id) == SCVT_E_OOM);
    scvt_config_init(&c, 642);
    c.method = SCVT_METHOD_LLOYD;
    const std::vector<double> z1 = points(642, 2);
    CHECK(scvt_server_submit(s, &c, z1.data(), 1e-8, 10, &id) == SCVT_E_INVALID);
  }
  int done = 0;
  std::vector<bool> fin(ids.size(), false);
  for (int spin = 0; spin < 6000 && done < (int)ids.size(); spin++) {
    for (size_t k = 0; k < ids.size(); k++) {
      if (fin[k]) continue;
      std::vector<double> z(3 * sizes[k]);
      scvt_info info;
      double times[3];
      const int rc = scvt_server_poll(s, ids[k], z.data(), &info, times);
      if (rc == SCVT_PENDING) continue;
      CHECK(rc == SCVT_OK || rc == SCVT_NOT_CONVERGED);
      CHECK(info.iter == 25 || rc == SCVT_OK);
      CHECK(times[0] <= times[1] && times[1] <= times[2]);
      CHECK(scvt_server_release(s, ids[k]) == SCVT_OK);
      CHECK(scvt_server_poll(s, ids[k], nullptr, nullptr, nullptr) == SCVT_E_INVALID);
      fin[k] = true;
      done++;
    }
    int64_t waiting = 0, running = 0;
    size_t used = 0;
    CHECK(scvt_server_stats(s, &waiting, &running, &used) == SCVT_OK);
    CHECK(running <= 3);
    if (done < (int)ids.size()) std::this_thread::sleep_for(std::chrono::milliseconds(5));
  }
  CHECK(done == (int)ids.size());
  // destroy with requests still queued and running
  for (int r = 0; r < 5; r++) {
    scvt_config c;
    scvt_config_init(&c, 2562);
    const std::vector<double> z0 = points(2562, 200 + r);
    int64_t id = -1;
    CHECK(scvt_server_submit(s, &c, z0.data(), 1e-14, 200, &id) == SCVT_OK);
  }
  scvt_server_destroy(s);
}

int main() {
  argument_errors();
  fprintf(stderr, "step: handles\n");
  const scvt_density rho1 = [] {
    scvt_density d;
    memset(&d, 0, sizeof(d));
    d.kind = SCVT_RHO_CONST;
    d.w_lon = d.w_lat = 1.0;
    return d;
  }();
  one_handle(642, SCVT_FP64, SCVT_METHOD_PLBFGS, rho1, 1);
  one_handle(10242, SCVT_FP64, SCVT_METHOD_PLBFGS, tanh_bump(4.0), 1);
  one_handle(10242, SCVT_MIXED, SCVT_METHOD_PLBFGS, tanh_bump(4.0), 0);
  one_handle(2562, SCVT_FP64, SCVT_METHOD_LBFGS, rho1, 0);
  one_handle(2562, SCVT_FP64, SCVT_METHOD_LLOYD, tanh_bump(2.0), 1);
  fprintf(stderr, "step: record ring\n");
  ring_wrap();
  fprintf(stderr, "step: multilevel\n");
  multilevel();
  fprintf(stderr, "step: serving\n");
  serving();
  fprintf(stderr, g_fail ? "abi_sanitize: FAILED\n" : "abi_sanitize: all checks held\n");
  return g_fail;
}
