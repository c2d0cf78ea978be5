// Pruned uniform octree with Morton keys, near fields and interaction lists
// (Section 2 of arXiv 2408.07436; counts of Section 3.1).  Host code.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "internal.h"

namespace kifmm {

namespace {

uint64_t encode(int64_t ax, int64_t ay, int64_t az, int level) {
  uint64_t m = 0;
  for (int b = 0; b < level; ++b) {
    m |= (uint64_t)((ax >> b) & 1) << (3 * b);
    m |= (uint64_t)((ay >> b) & 1) << (3 * b + 1);
    m |= (uint64_t)((az >> b) & 1) << (3 * b + 2);
  }
  return m | ((uint64_t)1 << (3 * level));
}

void decode(uint64_t key, int level, int32_t a[3]) {
  a[0] = a[1] = a[2] = 0;
  for (int b = 0; b < level; ++b) {
    a[0] |= (int32_t)((key >> (3 * b)) & 1) << b;
    a[1] |= (int32_t)((key >> (3 * b + 1)) & 1) << b;
    a[2] |= (int32_t)((key >> (3 * b + 2)) & 1) << b;
  }
}

// index of key in a sorted key array, or -1
int32_t find(const std::vector<uint64_t>& keys, uint64_t key) {
  auto it = std::lower_bound(keys.begin(), keys.end(), key);
  if (it == keys.end() || *it != key) return -1;
  return (int32_t)(it - keys.begin());
}

int32_t find_anchor(const Level& lv, int level, int64_t ax, int64_t ay, int64_t az) {
  const int64_t n = (int64_t)1 << level;
  if (ax < 0 || ay < 0 || az < 0 || ax >= n || ay >= n || az >= n) return -1;
  return find(lv.keys, encode(ax, ay, az, level));
}

kifmm_status leaf_keys(const double* pts, int64_t n, int depth, const double o[3], double w,
                       std::vector<uint64_t>& keys) {
  keys.resize(n);
  const double scale = std::ldexp(1.0, depth);
  const int64_t top = ((int64_t)1 << depth) - 1;
  for (int64_t i = 0; i < n; ++i) {
    int64_t a[3];
    for (int c = 0; c < 3; ++c) {
      const double u = (pts[3 * i + c] - o[c]) / w;
      if (!(u >= 0.0 && u <= 1.0))
        return fail(KIFMM_EINVAL, "point " + std::to_string(i) + " lies outside the domain cube");
      int64_t ai = (int64_t)std::floor(u * scale);
      a[c] = ai > top ? top : ai;
    }
    keys[i] = encode(a[0], a[1], a[2], depth);
  }
  return KIFMM_OK;
}

void sort_points(const double* pts, const std::vector<uint64_t>& keys, std::vector<int64_t>& perm,
                 std::vector<double>& sorted, std::vector<uint64_t>& sorted_keys) {
  const int64_t n = (int64_t)keys.size();
  perm.resize(n);
  std::iota(perm.begin(), perm.end(), (int64_t)0);
  std::stable_sort(perm.begin(), perm.end(),
                   [&](int64_t a, int64_t b) { return keys[a] < keys[b]; });
  sorted.resize(3 * n);
  sorted_keys.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    std::memcpy(&sorted[3 * i], &pts[3 * perm[i]], 3 * sizeof(double));
    sorted_keys[i] = keys[perm[i]];
  }
}

void ranges(const std::vector<uint64_t>& sorted_keys, const std::vector<uint64_t>& leaves,
            std::vector<int32_t>& start, std::vector<int32_t>& end) {
  start.assign(leaves.size(), 0);
  end.assign(leaves.size(), 0);
  size_t j = 0;
  for (size_t i = 0; i < leaves.size(); ++i) {
    while (j < sorted_keys.size() && sorted_keys[j] < leaves[i]) ++j;
    start[i] = (int32_t)j;
    while (j < sorted_keys.size() && sorted_keys[j] == leaves[i]) ++j;
    end[i] = (int32_t)j;
  }
}

}  // namespace

int transfer_index(int tx, int ty, int tz) {
  if (std::max(std::abs(tx), std::max(std::abs(ty), std::abs(tz))) < 2) return -1;
  if (std::abs(tx) > 3 || std::abs(ty) > 3 || std::abs(tz) > 3) return -1;
  // rank in lexicographic order over [-3,3]^3 minus the inner [-1,1]^3 cube
  int idx = 0;
  for (int x = -3; x <= 3; ++x)
    for (int y = -3; y <= 3; ++y)
      for (int z = -3; z <= 3; ++z) {
        if (std::max(std::abs(x), std::max(std::abs(y), std::abs(z))) < 2) continue;
        if (x == tx && y == ty && z == tz) return idx;
        ++idx;
      }
  return -1;
}

void transfer_vector(int idx, int t[3]) {
  int i = 0;
  for (int x = -3; x <= 3; ++x)
    for (int y = -3; y <= 3; ++y)
      for (int z = -3; z <= 3; ++z) {
        if (std::max(std::abs(x), std::max(std::abs(y), std::abs(z))) < 2) continue;
        if (i == idx) {
          t[0] = x; t[1] = y; t[2] = z;
          return;
        }
        ++i;
      }
  t[0] = t[1] = t[2] = 0;
}

void direction_vector(int d, int D[3]) {
  int i = 0;
  for (int x = -1; x <= 1; ++x)
    for (int y = -1; y <= 1; ++y)
      for (int z = -1; z <= 1; ++z) {
        if (x == 0 && y == 0 && z == 0) continue;
        if (i == d) {
          D[0] = x; D[1] = y; D[2] = z;
          return;
        }
        ++i;
      }
}

kifmm_status build_tree(Tree& t, int depth, const double origin[3], double width, const double* src,
                        int64_t n_src, const double* tgt, int64_t n_tgt) {
  t = Tree();
  t.depth = depth;
  t.n_src = n_src;
  t.n_tgt = n_tgt;
  if (width > 0.0) {
    std::memcpy(t.origin, origin, sizeof(t.origin));
    t.width = width;
  } else {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (const double* set : {src, tgt}) {
      const int64_t n = set == src ? n_src : n_tgt;
      for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) {
          lo[c] = std::min(lo[c], set[3 * i + c]);
          hi[c] = std::max(hi[c], set[3 * i + c]);
        }
    }
    double ext = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
    if (!(ext > 0.0)) ext = 1.0;
    t.width = ext * (1.0 + 1e-12);
    for (int c = 0; c < 3; ++c) t.origin[c] = 0.5 * (lo[c] + hi[c]) - 0.5 * t.width;
  }

  std::vector<uint64_t> skeys, tkeys, sk_sorted, tk_sorted;
  kifmm_status st = leaf_keys(src, n_src, depth, t.origin, t.width, skeys);
  if (st != KIFMM_OK) return st;
  st = leaf_keys(tgt, n_tgt, depth, t.origin, t.width, tkeys);
  if (st != KIFMM_OK) return st;
  sort_points(src, skeys, t.src_perm, t.src_sorted, sk_sorted);
  sort_points(tgt, tkeys, t.tgt_perm, t.tgt_sorted, tk_sorted);

  // leaves: union of the non-empty source and target leaves
  t.levels.assign(depth + 1, Level());
  {
    std::vector<uint64_t> a(sk_sorted), b(tk_sorted);
    a.erase(std::unique(a.begin(), a.end()), a.end());
    b.erase(std::unique(b.begin(), b.end()), b.end());
    std::vector<uint64_t>& lv = t.levels[depth].keys;
    std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(lv));
  }
  for (int l = depth - 1; l >= 0; --l) {
    std::vector<uint64_t>& out = t.levels[l].keys;
    for (uint64_t k : t.levels[l + 1].keys) {
      const uint64_t pk = k >> 3;
      if (out.empty() || out.back() != pk) out.push_back(pk);
    }
  }
  for (int l = 0; l <= depth; ++l) {
    Level& lv = t.levels[l];
    lv.n = (int64_t)lv.keys.size();
    lv.anchor.resize(3 * lv.n);
    for (int64_t i = 0; i < lv.n; ++i) decode(lv.keys[i], l, &lv.anchor[3 * i]);
    lv.parent.assign(lv.n, -1);
    if (l < depth) lv.child.assign(8 * lv.n, -1);
  }
  for (int l = 1; l <= depth; ++l) {
    Level& lv = t.levels[l];
    Level& up = t.levels[l - 1];
    int64_t j = 0;
    for (int64_t i = 0; i < lv.n; ++i) {
      const uint64_t pk = lv.keys[i] >> 3;
      while (up.keys[j] != pk) ++j;
      lv.parent[i] = (int32_t)j;
      up.child[8 * j + (lv.keys[i] & 7)] = (int32_t)i;
    }
  }
  ranges(sk_sorted, t.levels[depth].keys, t.src_start, t.src_end);
  ranges(tk_sorted, t.levels[depth].keys, t.tgt_start, t.tgt_end);

  // interaction lists: children of the parent's neighbours that are not
  // adjacent to the box (Section 2, the M2L bullet)
  for (int l = 2; l <= depth; ++l) {
    Level& lv = t.levels[l];
    const Level& up = t.levels[l - 1];
    lv.il_offs.assign(lv.n + 1, 0);
    lv.il_src.clear();
    lv.il_t.clear();
    std::vector<std::pair<int32_t, int16_t>> row;
    for (int64_t i = 0; i < lv.n; ++i) {
      row.clear();
      const int32_t* a = &lv.anchor[3 * i];
      const int32_t* pa = &up.anchor[3 * lv.parent[i]];
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            const int32_t nb = find_anchor(up, l - 1, pa[0] + dx, pa[1] + dy, pa[2] + dz);
            if (nb < 0) continue;
            for (int o = 0; o < 8; ++o) {
              const int32_t s = up.child[8 * nb + o];
              if (s < 0) continue;
              const int32_t* sa = &lv.anchor[3 * s];
              const int tx = sa[0] - a[0], ty = sa[1] - a[1], tz = sa[2] - a[2];
              if (std::max(std::abs(tx), std::max(std::abs(ty), std::abs(tz))) <= 1) continue;
              row.emplace_back(s, (int16_t)transfer_index(tx, ty, tz));
            }
          }
      std::sort(row.begin(), row.end());
      for (auto& e : row) {
        lv.il_src.push_back(e.first);
        lv.il_t.push_back(e.second);
      }
      lv.il_offs[i + 1] = (int64_t)lv.il_src.size();
    }
    // sibling-cluster halos for the FFT form: clusters are the boxes of l-1
    lv.halo.assign((size_t)kNumDirections * up.n, -1);
    for (int64_t c = 0; c < up.n; ++c) {
      const int32_t* pa = &up.anchor[3 * c];
      for (int d = 0; d < kNumDirections; ++d) {
        int D[3];
        direction_vector(d, D);
        lv.halo[(size_t)d * up.n + c] = find_anchor(up, l - 1, pa[0] + D[0], pa[1] + D[1], pa[2] + D[2]);
      }
    }
  }

  // near fields of the leaves
  {
    const Level& lv = t.levels[depth];
    t.near_offs.assign(lv.n + 1, 0);
    t.near_src.clear();
    std::vector<int32_t> row;
    for (int64_t i = 0; i < lv.n; ++i) {
      row.clear();
      const int32_t* a = &lv.anchor[3 * i];
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            const int32_t s = find_anchor(lv, depth, a[0] + dx, a[1] + dy, a[2] + dz);
            if (s >= 0) row.push_back(s);
          }
      std::sort(row.begin(), row.end());
      t.near_src.insert(t.near_src.end(), row.begin(), row.end());
      t.near_offs[i + 1] = (int64_t)t.near_src.size();
    }
  }
  return KIFMM_OK;
}

}  // namespace kifmm
