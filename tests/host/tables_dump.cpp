// Test harness (host only): builds the oct tables of a hierarchy read from a binary
// file and prints them as text, so that a test can compare them with tables derived
// independently.  Input: int32 n_levels, then per level int32 level, int64 n_oct,
// int32[n_oct][3] oct coordinates (the first level is the base).  Output: per level
// "level n_oct n_leaf" and the lines ijk, nbr, cnb, parent, child; or "ERR level reason".
#include <cstdio>
#include <vector>

#include "tables.h"

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t n_levels = 0;
  if (std::fread(&n_levels, 4, 1, f) != 1) return 2;
  std::vector<amrfld::LevelTables> lev(n_levels);
  for (int k = 0; k < n_levels; ++k) {
    int32_t level = 0;
    int64_t n_oct = 0;
    if (std::fread(&level, 4, 1, f) != 1 || std::fread(&n_oct, 8, 1, f) != 1) return 2;
    std::vector<int32_t> ijk(3 * n_oct);
    if (n_oct > 0 && std::fread(ijk.data(), 4, ijk.size(), f) != ijk.size()) return 2;
    const std::string why =
        amrfld::build_level_tables(level, k == 0, n_oct, ijk.data(), k == 0 ? nullptr : &lev[k - 1], &lev[k]);
    if (!why.empty()) {
      std::printf("ERR %d %s\n", level, why.c_str());
      return 0;
    }
  }
  std::fclose(f);
  auto line = [](const std::vector<int32_t>& v) {
    for (size_t i = 0; i < v.size(); ++i) std::printf(i ? " %d" : "%d", v[i]);
    std::printf("\n");
  };
  for (const auto& t : lev) {
    std::printf("%d %lld %lld\n", t.level, static_cast<long long>(t.n_oct), static_cast<long long>(t.n_leaf));
    line(t.ijk);
    line(t.nbr);
    line(t.cnb);
    line(t.parent);
    line(t.child);
  }
  return 0;
}
