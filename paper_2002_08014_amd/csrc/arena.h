// First-fit allocator of ranges of one device arena: host bookkeeping only (no
// HIP calls), shared by the serving layer and its host test.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace lp {

// Free ranges of [0, size) by offset, disjoint, and merged with their
// neighbours on release.  take() returns the lowest free range that holds
// `bytes`; give() returns a range taken before.
struct Arena {
  char* base = nullptr;
  size_t size = 0;
  std::map<size_t, size_t> free_ranges;   // offset -> length
  bool take(size_t bytes, size_t* off) {
    for (auto it = free_ranges.begin(); it != free_ranges.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, at = it->first + bytes;
      free_ranges.erase(it);
      if (rest > 0) free_ranges.emplace(at, rest);
      return true;
    }
    return false;
  }
  void give(size_t off, size_t bytes) {
    auto it = free_ranges.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_ranges.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_ranges.erase(nx);
    }
    if (it != free_ranges.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_ranges.erase(it);
      }
    }
  }
};


}  // namespace lp
