// Randomised check of the serving arena's first-fit ranges (arena.h)
// against a byte-map model, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_hostcheck.py.
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "arena.h"

namespace {

int failures = 0;
#define CHECK(c)                                                    \
  do {                                                              \
    if (!(c)) {                                                     \
      printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);            \
      failures++;                                                   \
    }                                                               \
  } while (0)

struct Taken {
  size_t off, bytes;
};

// free ranges are disjoint, non-adjacent, inside [0, total), and cover
// exactly the bytes the model marks free
void check_invariants(const scvt::Arena& A, const std::vector<char>& used, size_t unit) {
  size_t prev_end = 0;
  bool first = true;
  std::vector<char> fr(used.size(), 0);
  for (const auto& kv : A.free) {
    CHECK(kv.second > 0);
    CHECK(kv.first % unit == 0 && kv.second % unit == 0);
    if (!first) CHECK(kv.first > prev_end);  // no overlap and no adjacency
    first = false;
    prev_end = kv.first + kv.second;
    CHECK(prev_end <= used.size() * unit);
    for (size_t u = kv.first / unit; u < prev_end / unit && u < fr.size(); u++) fr[u] = 1;
  }
  for (size_t u = 0; u < used.size(); u++) CHECK(fr[u] == !used[u]);
}

// the lowest offset of a free run of at least `units` in the model
long first_fit(const std::vector<char>& used, size_t units) {
  size_t run = 0;
  for (size_t u = 0; u < used.size(); u++) {
    run = used[u] ? 0 : run + 1;
    if (run >= units) return (long)(u + 1 - units);
  }
  return -1;
}

}  // namespace

int main() {
  const size_t unit = 256;
  for (int seed = 0; seed < 20; seed++) {
    std::mt19937_64 rng(seed);
    const size_t units = 64 + rng() % 512;
    scvt::Arena A;
    A.give(0, units * unit);
    std::vector<char> used(units, 0);
    std::vector<Taken> live;
    for (int step = 0; step < 4000; step++) {
      const bool do_take = live.empty() || (rng() % 100) < 55;
      if (do_take) {
        const size_t want = 1 + rng() % (units / 4 + 1);
        size_t off = 12345;
        const long expect = first_fit(used, want);
        const bool ok = A.take(want * unit, &off);
        CHECK(ok == (expect >= 0));
        if (ok) {
          CHECK(off == (size_t)expect * unit);
          for (size_t u = off / unit; u < off / unit + want; u++) {
            CHECK(!used[u]);
            used[u] = 1;
          }
          live.push_back({off, want * unit});
        }
      } else {
        const size_t k = rng() % live.size();
        const Taken t = live[k];
        live[k] = live.back();
        live.pop_back();
        A.give(t.off, t.bytes);
        for (size_t u = t.off / unit; u < (t.off + t.bytes) / unit; u++) used[u] = 0;
      }
      check_invariants(A, used, unit);
    }
    for (const Taken& t : live) A.give(t.off, t.bytes);
    // everything back: one range, the whole arena
    CHECK(A.free.size() == 1 && A.free.begin()->first == 0 &&
          A.free.begin()->second == units * unit);
  }
  // an exact fit leaves no empty range; a zero-byte give changes nothing
  scvt::Arena B;
  B.give(0, 1024);
  size_t off = 0;
  CHECK(B.take(1024, &off) && off == 0 && B.free.empty());
  B.give(0, 0);
  CHECK(B.free.empty());
  CHECK(!B.take(256, &off));
  printf("%d failures\n", failures);
  return failures ? 1 : 0;
}
