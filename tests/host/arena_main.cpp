// Drives lp::Arena (paper_2002_08014_amd/csrc/arena.h) from stdin for the host
// test: first line "size"; then "t bytes" (take: prints the offset or -1) and
// "g offset bytes" (give); "f" prints the free ranges as "offset length" pairs.
#include <cstdio>
#include <iostream>
#include <string>

#include "../../paper_2002_08014_amd/csrc/arena.h"

int main() {
  lp::Arena a;
  std::cin >> a.size;
  a.free_ranges.emplace(0, a.size);
  std::string op;
  while (std::cin >> op) {
    if (op == "t") {
      size_t b, off = 0;
      std::cin >> b;
      if (a.take(b, &off)) std::printf("%zu\n", off);
      else std::printf("-1\n");
    } else if (op == "g") {
      size_t off, b;
      std::cin >> off >> b;
      a.give(off, b);
    } else if (op == "f") {
      for (const auto& r : a.free_ranges) std::printf("%zu %zu ", r.first, r.second);
      std::printf("\n");
    }
  }
  return 0;
}
