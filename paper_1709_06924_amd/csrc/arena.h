// First-fit ranges of the serving arena: one device allocation made when
// the server is created, handed out to admitted requests as byte ranges and
// taken back (coalesced with free neighbours) when they finish.  Host code
// only; offsets and sizes are bytes (the caller keeps them 256-byte aligned).
#pragma once
#include <stddef.h>

#include <iterator>
#include <map>

namespace scvt {

struct Arena {
  std::map<size_t, size_t> free;  // offset -> size, no two ranges adjacent

  // The lowest free range of at least `bytes`: its start in *off, the rest
  // of the range stays free.  False (and nothing changed) if none fits.
  bool take(size_t bytes, size_t* off) {
    for (auto it = free.begin(); it != free.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, at = it->first + bytes;
      free.erase(it);
      if (rest) free[at] = rest;
      return true;
    }
    return false;
  }

  // Return [off, off + bytes) (a range take() handed out), merged with the
  // free ranges it touches.
  void give(size_t off, size_t bytes) {
    if (bytes == 0) return;
    auto it = free.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free.erase(nx);
    }
    if (it != free.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free.erase(it);
      }
    }
  }
};

}  // namespace scvt
