// Host-side oct tables of one AMR level: Morton order, same-level neighbour
// octs, parent cells and coarse neighbour cells (the oct tree of Fig. 1).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace amrfld {

// Directions: d = 2 * axis + side; side 0 is the minus face, side 1 the plus face.
constexpr int kDirs = 6;

struct LevelTables {
  int level = -1;
  int64_t n_oct = 0;
  std::vector<int32_t> ijk;     // [n_oct][3] oct coordinates, Morton-sorted
  std::vector<uint64_t> key;    // [n_oct] Morton keys, ascending
  std::vector<int32_t> nbr;     // [n_oct][6] same-level neighbour oct, -1 if none
  std::vector<int32_t> cnb;     // [n_oct][6] coarse neighbour slot (level-1) when nbr = -1 inside the box, else -1
  std::vector<int32_t> parent;  // [n_oct] parent slot at level-1 (-1 on the base level)
  std::vector<int32_t> child;   // [8 n_oct] child oct at level+1 or -1
  int64_t n_leaf = 0;

  int64_t n_slots() const { return 8 * n_oct; }
  // Oct index of coordinates (I,J,K) at this level, or -1.
  int64_t find(int32_t I, int32_t J, int32_t K) const;
};

uint64_t morton3(uint32_t i, uint32_t j, uint32_t k);

// Builds `out` for `level` from caller coordinates.  `coarser` is the level-1
// tables (nullptr for the base level); its child array is updated on success.
// Returns an empty string on success, else the reason for rejection.
std::string build_level_tables(int level, bool is_base, int64_t n_oct, const int32_t* oct_ijk,
                               LevelTables* coarser, LevelTables* out);

}  // namespace amrfld
