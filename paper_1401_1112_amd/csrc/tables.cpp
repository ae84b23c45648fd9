// Oct tables of one level (host, built once per hierarchy).
#include "tables.h"

#include <algorithm>
#include <numeric>

namespace amrfld {

namespace {

uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffffu;
  x = (x | x << 32) & 0x1f00000000ffffULL;
  x = (x | x << 16) & 0x1f0000ff0000ffULL;
  x = (x | x << 8) & 0x100f00f00f00f00fULL;
  x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
  x = (x | x << 2) & 0x1249249249249249ULL;
  return x;
}

const int kOff[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};

}  // namespace

uint64_t morton3(uint32_t i, uint32_t j, uint32_t k) {
  return spread3(i) | (spread3(j) << 1) | (spread3(k) << 2);
}

int64_t LevelTables::find(int32_t I, int32_t J, int32_t K) const {
  const uint64_t k = morton3(uint32_t(I), uint32_t(J), uint32_t(K));
  auto it = std::lower_bound(key.begin(), key.end(), k);
  if (it == key.end() || *it != k) return -1;
  return int64_t(it - key.begin());
}

std::string build_level_tables(int level, bool is_base, int64_t n_oct, const int32_t* oct_ijk,
                               LevelTables* coarser, LevelTables* out) {
  const int64_t n_side = int64_t(1) << (level - 1);  // octs per axis on this level
  if (n_oct < 1) return "a level needs at least one oct";
  if (8 * n_oct > int64_t(0x7fffffff)) return "level too large for 32-bit slot indices";
  if (is_base && n_oct != n_side * n_side * n_side)
    return "the base level must list every oct of the box";
  for (int64_t o = 0; o < n_oct; ++o)
    for (int a = 0; a < 3; ++a) {
      const int32_t v = oct_ijk[3 * o + a];
      if (v < 0 || v >= n_side) return "oct coordinate out of range";
    }

  LevelTables t;
  t.level = level;
  t.n_oct = n_oct;
  std::vector<uint64_t> raw(n_oct);
  for (int64_t o = 0; o < n_oct; ++o)
    raw[o] = morton3(uint32_t(oct_ijk[3 * o]), uint32_t(oct_ijk[3 * o + 1]), uint32_t(oct_ijk[3 * o + 2]));
  std::vector<int64_t> order(n_oct);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return raw[a] < raw[b]; });
  t.key.resize(n_oct);
  t.ijk.resize(3 * n_oct);
  for (int64_t o = 0; o < n_oct; ++o) {
    t.key[o] = raw[order[o]];
    for (int a = 0; a < 3; ++a) t.ijk[3 * o + a] = oct_ijk[3 * order[o] + a];
    if (o > 0 && t.key[o] == t.key[o - 1]) return "duplicate oct";
  }

  t.nbr.assign(6 * n_oct, -1);
  t.cnb.assign(6 * n_oct, -1);
  t.parent.assign(n_oct, -1);
  t.child.assign(8 * n_oct, -1);
  t.n_leaf = 8 * n_oct;

  const int64_t c_side = n_side >> 1;  // octs per axis on the coarser level
  for (int64_t o = 0; o < n_oct; ++o) {
    const int32_t I = t.ijk[3 * o], J = t.ijk[3 * o + 1], K = t.ijk[3 * o + 2];
    for (int d = 0; d < kDirs; ++d) {
      const int64_t a = I + kOff[d][0], b = J + kOff[d][1], c = K + kOff[d][2];
      if (a < 0 || b < 0 || c < 0 || a >= n_side || b >= n_side || c >= n_side) continue;
      t.nbr[6 * o + d] = int32_t(t.find(int32_t(a), int32_t(b), int32_t(c)));
    }
    if (is_base) continue;
    // parent cell (I,J,K) at level-1 lives in coarse oct (I>>1, J>>1, K>>1)
    const int64_t po = coarser->find(I >> 1, J >> 1, K >> 1);
    if (po < 0) return "oct without a parent cell on the coarser level";
    const int pos = (I & 1) | ((J & 1) << 1) | ((K & 1) << 2);
    t.parent[o] = int32_t(8 * po + pos);
    for (int d = 0; d < kDirs; ++d) {
      const int64_t a = I + kOff[d][0], b = J + kOff[d][1], c = K + kOff[d][2];
      if (a < 0 || b < 0 || c < 0 || a >= n_side || b >= n_side || c >= n_side) continue;
      // the parent's face neighbour must exist at level-1 (neighbours within one level)
      const int64_t no = coarser->find(int32_t(a >> 1), int32_t(b >> 1), int32_t(c >> 1));
      if (no < 0) return "unbalanced hierarchy: a parent face neighbour is missing on the coarser level";
      if (t.nbr[6 * o + d] < 0) {
        const int npos = int(a & 1) | (int(b & 1) << 1) | (int(c & 1) << 2);
        t.cnb[6 * o + d] = int32_t(8 * no + npos);
      }
    }
  }
  (void)c_side;
  if (!is_base) {
    for (int64_t o = 0; o < n_oct; ++o) {
      coarser->child[t.parent[o]] = int32_t(o);
    }
    coarser->n_leaf -= n_oct;
  }
  *out = std::move(t);
  return std::string();
}

}  // namespace amrfld
