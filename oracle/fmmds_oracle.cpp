/*
 * fmmds oracle: TEST INFRASTRUCTURE ONLY (see fmmds_oracle.h).
 *
 * Plain single-threaded CPU build of the FMM data structures, written from the
 * definitions of Hu, Gumerov and Duraiswami (arXiv 1301.1704):
 *   - boxes of an octree over the unit cube, Morton index n = 0..8^l - 1 at
 *     level l (Section 1.4);
 *   - points reordered by the Morton index of their finest-level box
 *     (Section 2.1, the Fixed-Grid-Method pseudo-sort, Algorithm 1);
 *   - bookmark (first point of each nonempty box) and nonempty-box index
 *     arrays (Section 2.2; Algorithm 3 in Section 2.3);
 *   - parent and children relations (Section 2.4; the parent is the Morton
 *     index shifted right by one level, Section 3.2);
 *   - E2 neighbor lists and E4 interaction lists of nonempty source boxes per
 *     nonempty receiver box (Section 1.4, Section 2.2, Algorithm 4), as
 *     ranks among the nonempty source boxes of that level.
 *
 * Nothing here is blocked, fused or reordered for speed: every table and list
 * is computed straight from its definition. Where the paper leaves a choice
 * open this file takes these readings:
 *   - order of points inside a box: ascending original index (the paper's
 *     pseudo-sort leaves it to run-time memory order, Section 2.1);
 *   - interleave: bit b of the x, y, z box coordinates goes to key bit 3b,
 *     3b+1, 3b+2 (the paper fixes no bit order; its one printed 2-D example
 *     refers to a missing figure);
 *   - E2 includes the box itself and the domain is not periodic;
 *   - E4 is the set difference of the parent's E2 children and the box's own
 *     E2, so it has at most 6^3 - 3^3 = 189 members;
 *   - list entries are in ascending source rank;
 *   - depth: with cluster size s > 0, the smallest level l in [2, max_level]
 *     whose fullest source box and fullest receiver box both hold at most s
 *     points; max_level if there is none; with s = 0, max_level.
 */
#include "fmmds_oracle.h"

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

namespace {

struct Level {
  std::vector<uint64_t> key;     // Morton index of each nonempty box, ascending
  std::vector<uint32_t> begin;   // first sorted point of each box, plus sentinel n
  std::vector<uint32_t> parent;  // rank of the parent box at level - 1
  std::vector<uint32_t> child;   // first child rank at level + 1, plus sentinel
};

struct PointSet {
  uint32_t n = 0;
  std::vector<uint32_t> perm;      // original index of each sorted point
  std::vector<float> sorted_xyz;   // xyz[perm[k]]
  std::vector<uint64_t> sorted_key;  // finest-level key of each sorted point
  std::vector<Level> lv;           // levels 0..depth
};

struct List {
  std::vector<uint32_t> off;
  std::vector<uint32_t> ent;
};

}  // namespace

struct oref_tree {
  uint32_t depth = 0, key_bits = 0, max_level = 0;
  bool shared = false, has_lists = false;
  PointSet src, recv;
  std::vector<List> e2, e4;  // indexed by level
  const PointSet& set(int s) const { return (s == 1 && !shared) ? recv : src; }
};

namespace {

// Section 1.4: the box of a point at level L has integer coordinates
// floor(x * 2^L) per axis. Scaling an FP32 value by 2^L is exact, so this is
// the exact floor of the real product.
inline uint32_t quantize(float x, uint32_t L) {
  return (uint32_t)std::floor(x * (float)(1u << L));
}

// Morton index: bit b of the x, y, z coordinates goes to bit 3b, 3b+1, 3b+2.
uint64_t interleave(uint32_t qx, uint32_t qy, uint32_t qz, uint32_t L) {
  uint64_t key = 0;
  for (uint32_t b = 0; b < L; ++b) {
    key |= (uint64_t)((qx >> b) & 1u) << (3 * b);
    key |= (uint64_t)((qy >> b) & 1u) << (3 * b + 1);
    key |= (uint64_t)((qz >> b) & 1u) << (3 * b + 2);
  }
  return key;
}

void deinterleave(uint64_t key, uint32_t L, int64_t c[3]) {
  c[0] = c[1] = c[2] = 0;
  for (uint32_t b = 0; b < L; ++b) {
    c[0] |= (int64_t)((key >> (3 * b)) & 1u) << b;
    c[1] |= (int64_t)((key >> (3 * b + 1)) & 1u) << b;
    c[2] |= (int64_t)((key >> (3 * b + 2)) & 1u) << b;
  }
}

bool in_unit_interval(float x) { return x >= 0.0f && x < 1.0f; }  // false for NaN

int point_keys(const float* xyz, uint32_t n, uint32_t L, uint64_t* out) {
  for (uint32_t i = 0; i < n; ++i) {
    const float x = xyz[3 * (size_t)i], y = xyz[3 * (size_t)i + 1], z = xyz[3 * (size_t)i + 2];
    if (!in_unit_interval(x) || !in_unit_interval(y) || !in_unit_interval(z)) return OREF_ERR_RANGE;
    out[i] = interleave(quantize(x, L), quantize(y, L), quantize(z, L), L);
  }
  return OREF_OK;
}

// Points ordered by (finest-level key, original index); then the per-level
// tables by their definitions.
int build_set(const float* xyz, uint32_t n, uint32_t L, PointSet& ps) {
  ps.n = n;
  std::vector<uint64_t> key(n);
  int st = point_keys(xyz, n, L, key.data());
  if (st != OREF_OK) return st;

  ps.perm.resize(n);
  for (uint32_t i = 0; i < n; ++i) ps.perm[i] = i;
  std::sort(ps.perm.begin(), ps.perm.end(), [&](uint32_t a, uint32_t b) {
    return key[a] != key[b] ? key[a] < key[b] : a < b;
  });
  ps.sorted_xyz.resize(3 * (size_t)n);
  ps.sorted_key.resize(n);
  for (uint32_t k = 0; k < n; ++k) {
    const uint32_t i = ps.perm[k];
    ps.sorted_xyz[3 * (size_t)k] = xyz[3 * (size_t)i];
    ps.sorted_xyz[3 * (size_t)k + 1] = xyz[3 * (size_t)i + 1];
    ps.sorted_xyz[3 * (size_t)k + 2] = xyz[3 * (size_t)i + 2];
    ps.sorted_key[k] = key[i];
  }

  // Nonempty boxes and bookmarks at every level 0..L (Algorithm 3): a box is
  // nonempty iff some point lies in it; its bookmark is its first point.
  ps.lv.assign(L + 1, Level());
  for (uint32_t l = 0; l <= L; ++l) {
    Level& lv = ps.lv[l];
    const uint32_t shift = 3 * (L - l);
    for (uint32_t k = 0; k < n; ++k) {
      const uint64_t kl = ps.sorted_key[k] >> shift;
      if (k == 0 || kl != (ps.sorted_key[k - 1] >> shift)) {
        lv.key.push_back(kl);
        lv.begin.push_back(k);
      }
    }
    lv.begin.push_back(n);
  }
  // Parent: the box whose index is this index shifted right by 3 bits.
  for (uint32_t l = 1; l <= L; ++l) {
    Level& lv = ps.lv[l];
    const std::vector<uint64_t>& up = ps.lv[l - 1].key;
    lv.parent.resize(lv.key.size());
    for (size_t j = 0; j < lv.key.size(); ++j) {
      const uint64_t pk = lv.key[j] >> 3;
      lv.parent[j] = (uint32_t)(std::lower_bound(up.begin(), up.end(), pk) - up.begin());
    }
  }
  // Children: the first box of level l+1 whose parent is j; sentinel n_{l+1}.
  for (uint32_t l = 0; l < L; ++l) {
    Level& lv = ps.lv[l];
    const Level& dn = ps.lv[l + 1];
    lv.child.assign(lv.key.size() + 1, 0);
    for (size_t k = 0; k < dn.key.size(); ++k)
      if (k == 0 || dn.parent[k] != dn.parent[k - 1]) lv.child[dn.parent[k]] = (uint32_t)k;
    lv.child[lv.key.size()] = (uint32_t)dn.key.size();
  }
  return OREF_OK;
}

uint32_t max_occupancy(const Level& lv) {
  uint32_t m = 0;
  for (size_t j = 0; j + 1 < lv.begin.size(); ++j) m = std::max(m, lv.begin[j + 1] - lv.begin[j]);
  return m;
}

// Membership of a box (by integer coordinates) among the nonempty source boxes
// of one level: a dense index table for small levels, binary search otherwise.
struct Lookup {
  const Level* lv = nullptr;
  uint32_t L = 0;
  std::vector<uint32_t> dense;  // rank, or 0xFFFFFFFF for an empty box
  Lookup(const Level& level, uint32_t l, bool allow_dense) : lv(&level), L(l) {
    if (allow_dense && 3 * l <= 27) {
      dense.assign((size_t)1 << (3 * l), 0xFFFFFFFFu);
      for (size_t j = 0; j < level.key.size(); ++j) dense[level.key[j]] = (uint32_t)j;
    }
  }
  int64_t rank(const int64_t c[3]) const {
    const int64_t m = (int64_t)1 << L;
    for (int d = 0; d < 3; ++d)
      if (c[d] < 0 || c[d] >= m) return -1;  // outside the domain: no box
    const uint64_t k = interleave((uint32_t)c[0], (uint32_t)c[1], (uint32_t)c[2], L);
    if (!dense.empty()) return dense[k] == 0xFFFFFFFFu ? -1 : (int64_t)dense[k];
    auto it = std::lower_bound(lv->key.begin(), lv->key.end(), k);
    if (it == lv->key.end() || *it != k) return -1;
    return it - lv->key.begin();
  }
};

// floor(v / 2), also for v < 0 (arithmetic shift).
inline int64_t floor_half(int64_t v) { return v >> 1; }
inline int64_t iabs(int64_t v) { return v < 0 ? -v : v; }

// E2(r): nonempty source boxes s at the level with max_d |c_s - c_r| <= 1.
// E4(r): nonempty source boxes s with max_d |c_s - c_r| >= 2 whose parent is
// within max_d |p_s - p_r| <= 1 of the receiver's parent (Section 1.4,
// E4(n, l) = E2(parent(n), l - 1) minus E2(n, l), taken over boxes).
// Entries sorted ascending.
void box_list(const Lookup& src, int kind, uint64_t recv_key, uint32_t l,
              std::vector<uint32_t>& out) {
  out.clear();
  int64_t cr[3];
  deinterleave(recv_key, l, cr);
  int64_t c[3];
  if (kind == 2) {
    for (int64_t dz = -1; dz <= 1; ++dz)
      for (int64_t dy = -1; dy <= 1; ++dy)
        for (int64_t dx = -1; dx <= 1; ++dx) {
          c[0] = cr[0] + dx; c[1] = cr[1] + dy; c[2] = cr[2] + dz;
          const int64_t r = src.rank(c);
          if (r >= 0) out.push_back((uint32_t)r);
        }
  } else {
    int64_t lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = 2 * (floor_half(cr[d]) - 1);
      hi[d] = 2 * (floor_half(cr[d]) + 1) + 1;
    }
    for (c[2] = lo[2]; c[2] <= hi[2]; ++c[2])
      for (c[1] = lo[1]; c[1] <= hi[1]; ++c[1])
        for (c[0] = lo[0]; c[0] <= hi[0]; ++c[0]) {
          int64_t cheb = 0, pcheb = 0;
          for (int d = 0; d < 3; ++d) {
            cheb = std::max(cheb, iabs(c[d] - cr[d]));
            pcheb = std::max(pcheb, iabs(floor_half(c[d]) - floor_half(cr[d])));
          }
          if (cheb < 2 || pcheb > 1) continue;
          const int64_t r = src.rank(c);
          if (r >= 0) out.push_back((uint32_t)r);
        }
  }
  std::sort(out.begin(), out.end());
}

int build_lists(oref_tree& t) {
  t.e2.assign(t.depth + 1, List());
  t.e4.assign(t.depth + 1, List());
  std::vector<uint32_t> tmp;
  for (uint32_t l = 2; l <= t.depth; ++l) {
    const Level& sl = t.set(0).lv[l];
    const Level& rl = t.set(1).lv[l];
    Lookup look(sl, l, true);
    for (int kind : {2, 4}) {
      List& L = (kind == 2) ? t.e2[l] : t.e4[l];
      L.off.assign(rl.key.size() + 1, 0);
      uint64_t total = 0;
      for (size_t j = 0; j < rl.key.size(); ++j) {
        box_list(look, kind, rl.key[j], l, tmp);
        L.off[j] = (uint32_t)total;
        total += tmp.size();
        if (total > 0xFFFFFFFFull) return OREF_ERR_OVERFLOW;
        L.ent.insert(L.ent.end(), tmp.begin(), tmp.end());
      }
      L.off[rl.key.size()] = (uint32_t)total;
    }
  }
  t.has_lists = true;
  return OREF_OK;
}

bool valid_set(int s) { return s == 0 || s == 1; }

}  // namespace

extern "C" {

int oref_point_keys(const float* xyz, uint32_t n, uint32_t level, uint64_t* keys_out) {
  if (!xyz || !keys_out || level > 21) return OREF_ERR_ARG;
  return point_keys(xyz, n, level, keys_out);
}

int oref_build(const float* src, uint32_t n_src, const float* recv, uint32_t n_recv,
               uint32_t key_bits, uint32_t cluster_s, uint32_t max_level, int with_lists,
               oref_tree** out) {
  if (!out) return OREF_ERR_ARG;
  *out = nullptr;
  const bool shared = (recv == nullptr);
  if (shared) n_recv = n_src;
  if (!src || n_src == 0 || n_recv == 0 || n_src >= 0xFFFFFFFFu || n_recv >= 0xFFFFFFFFu)
    return OREF_ERR_ARG;
  if (key_bits != 32 && key_bits != 64) return OREF_ERR_ARG;
  if (max_level < 2 || max_level > key_bits / 3) return OREF_ERR_ARG;
  oref_tree* t = new (std::nothrow) oref_tree();
  if (!t) return OREF_ERR_NOMEM;
  int st = OREF_OK;
  try {
    t->key_bits = key_bits;
    t->max_level = max_level;
    t->shared = shared;
    st = build_set(src, n_src, max_level, t->src);
    if (st == OREF_OK && !shared) st = build_set(recv, n_recv, max_level, t->recv);
    if (st == OREF_OK) {
      t->depth = max_level;
      if (cluster_s > 0) {
        for (uint32_t l = 2; l <= max_level; ++l) {
          if (max_occupancy(t->set(0).lv[l]) <= cluster_s &&
              max_occupancy(t->set(1).lv[l]) <= cluster_s) {
            t->depth = l;
            break;
          }
        }
      }
      // Drop levels below the chosen depth; the finest kept level has no
      // children.
      for (PointSet* ps : {&t->src, &t->recv}) {
        if (ps->lv.size() > t->depth + 1) ps->lv.resize(t->depth + 1);
        if (!ps->lv.empty()) ps->lv[t->depth].child.clear();
      }
      if (with_lists) st = build_lists(*t);
    }
  } catch (const std::bad_alloc&) {
    st = OREF_ERR_NOMEM;
  }
  if (st != OREF_OK) {
    delete t;
    return st;
  }
  *out = t;
  return OREF_OK;
}

void oref_free(oref_tree* t) { delete t; }

uint32_t oref_depth(const oref_tree* t) { return t ? t->depth : 0; }

uint32_t oref_n_points(const oref_tree* t, int set) {
  return (t && valid_set(set)) ? t->set(set).n : 0;
}

uint32_t oref_n_boxes(const oref_tree* t, int set, uint32_t level) {
  if (!t || !valid_set(set) || level > t->depth) return 0;
  return (uint32_t)t->set(set).lv[level].key.size();
}

uint32_t oref_max_occupancy(const oref_tree* t, int set, uint32_t level) {
  if (!t || !valid_set(set) || level > t->depth) return 0;
  return max_occupancy(t->set(set).lv[level]);
}

int oref_perm(const oref_tree* t, int set, uint32_t* out) {
  if (!t || !out || !valid_set(set)) return OREF_ERR_ARG;
  std::copy(t->set(set).perm.begin(), t->set(set).perm.end(), out);
  return OREF_OK;
}

int oref_sorted_xyz(const oref_tree* t, int set, float* out) {
  if (!t || !out || !valid_set(set)) return OREF_ERR_ARG;
  std::copy(t->set(set).sorted_xyz.begin(), t->set(set).sorted_xyz.end(), out);
  return OREF_OK;
}

int oref_keys(const oref_tree* t, int set, uint32_t level, uint64_t* out) {
  if (!t || !out || !valid_set(set)) return OREF_ERR_ARG;
  if (level > t->depth) return OREF_ERR_LEVEL;
  const Level& lv = t->set(set).lv[level];
  std::copy(lv.key.begin(), lv.key.end(), out);
  return OREF_OK;
}

int oref_begin(const oref_tree* t, int set, uint32_t level, uint32_t* out) {
  if (!t || !out || !valid_set(set)) return OREF_ERR_ARG;
  if (level > t->depth) return OREF_ERR_LEVEL;
  const Level& lv = t->set(set).lv[level];
  std::copy(lv.begin.begin(), lv.begin.end(), out);
  return OREF_OK;
}

int oref_parent(const oref_tree* t, int set, uint32_t level, uint32_t* out) {
  if (!t || !out || !valid_set(set)) return OREF_ERR_ARG;
  if (level < 1 || level > t->depth) return OREF_ERR_LEVEL;
  const Level& lv = t->set(set).lv[level];
  std::copy(lv.parent.begin(), lv.parent.end(), out);
  return OREF_OK;
}

int oref_child(const oref_tree* t, int set, uint32_t level, uint32_t* out) {
  if (!t || !out || !valid_set(set)) return OREF_ERR_ARG;
  if (level >= t->depth) return OREF_ERR_LEVEL;
  const Level& lv = t->set(set).lv[level];
  std::copy(lv.child.begin(), lv.child.end(), out);
  return OREF_OK;
}

int oref_list_sizes(const oref_tree* t, int kind, uint32_t level, uint32_t* n_recv_boxes,
                    uint64_t* n_entries) {
  if (!t || !n_recv_boxes || !n_entries || (kind != 2 && kind != 4) || !t->has_lists)
    return OREF_ERR_ARG;
  if (level < 2 || level > t->depth) return OREF_ERR_LEVEL;
  const List& L = (kind == 2) ? t->e2[level] : t->e4[level];
  *n_recv_boxes = (uint32_t)(L.off.size() - 1);
  *n_entries = L.ent.size();
  return OREF_OK;
}

int oref_list(const oref_tree* t, int kind, uint32_t level, uint32_t* offsets, uint32_t* entries) {
  if (!t || !offsets || !entries || (kind != 2 && kind != 4) || !t->has_lists) return OREF_ERR_ARG;
  if (level < 2 || level > t->depth) return OREF_ERR_LEVEL;
  const List& L = (kind == 2) ? t->e2[level] : t->e4[level];
  std::copy(L.off.begin(), L.off.end(), offsets);
  std::copy(L.ent.begin(), L.ent.end(), entries);
  return OREF_OK;
}

int oref_box_list(const oref_tree* t, int kind, uint32_t level, uint32_t recv_box,
                  uint32_t* entries) {
  if (!t || !entries || (kind != 2 && kind != 4)) return -OREF_ERR_ARG;
  if (level < 2 || level > t->depth) return -OREF_ERR_LEVEL;
  const Level& rl = t->set(1).lv[level];
  if (recv_box >= rl.key.size()) return -OREF_ERR_ARG;
  Lookup look(t->set(0).lv[level], level, false);
  std::vector<uint32_t> tmp;
  box_list(look, kind, rl.key[recv_box], level, tmp);
  std::copy(tmp.begin(), tmp.end(), entries);
  return (int)tmp.size();
}

// A level's source-box membership table, kept for repeated range queries.
struct oref_lookup {
  const oref_tree* t;
  uint32_t level;
  Lookup look;
  oref_lookup(const oref_tree* tree, uint32_t l)
      : t(tree), level(l), look(tree->set(0).lv[l], l, true) {}
};

oref_lookup* oref_lookup_open(const oref_tree* t, uint32_t level) {
  if (!t || level < 2 || level > t->depth) return nullptr;
  try {
    return new oref_lookup(t, level);
  } catch (const std::bad_alloc&) {
    return nullptr;
  }
}

void oref_lookup_close(oref_lookup* lk) { delete lk; }

int oref_list_range(const oref_lookup* lk, int kind, uint32_t r0, uint32_t r1,
                    uint32_t* offsets, uint32_t* entries) {
  if (!lk || !offsets || !entries || (kind != 2 && kind != 4)) return OREF_ERR_ARG;
  const Level& rl = lk->t->set(1).lv[lk->level];
  if (r0 > r1 || r1 > rl.key.size()) return OREF_ERR_ARG;
  std::vector<uint32_t> tmp;
  uint32_t total = 0;
  for (uint32_t j = r0; j < r1; ++j) {
    offsets[j - r0] = total;
    box_list(lk->look, kind, rl.key[j], lk->level, tmp);
    std::copy(tmp.begin(), tmp.end(), entries + total);
    total += (uint32_t)tmp.size();
  }
  offsets[r1 - r0] = total;
  return OREF_OK;
}


// ---------------------------------------------------------------------------
// Simulated partition and source box types (Section 3).
// ---------------------------------------------------------------------------

// Section 3.2: the boxes of the partition level l_par are given to the ranks
// in consecutive Morton ranges balanced by receiver points. Written out: the
// nonempty receiver box b at l_par whose first point (in Morton order) is the
// p-th of M goes to rank min(R - 1, floor(R * p / M)); every other Morton
// index at l_par takes the rank of the nearest nonempty receiver box before
// it, or rank 0 if there is none.
int oref_partition(const oref_tree* t, uint32_t l_par, uint32_t n_ranks, uint32_t* owner_out) {
  if (!t || !owner_out || n_ranks == 0) return OREF_ERR_ARG;
  if (l_par < 3 || l_par > t->depth || 3 * l_par > 30) return OREF_ERR_LEVEL;
  const Level& rl = t->set(1).lv[l_par];
  const uint64_t M = t->set(1).sorted_key.size();
  const uint64_t n_idx = 1ull << (3 * l_par);
  size_t b = 0;  // next nonempty receiver box
  uint32_t cur = 0;
  for (uint64_t m = 0; m < n_idx; ++m) {
    if (b < rl.key.size() && rl.key[b] == m) {
      const uint64_t p = rl.begin[b];
      cur = (uint32_t)std::min<uint64_t>(n_ranks - 1, (uint64_t)n_ranks * p / M);
      ++b;
    }
    owner_out[m] = cur;
  }
  return OREF_OK;
}

// Source box types for rank J (Section 3.1, Algorithm 6), levels 2..depth
// concatenated (level l's n_src_l entries after those of the levels below).
// DOMESTIC 0, EXPORT 1, IMPORT 2, ROOT 3, OTHER 4. Reading of the algorithm:
// the critical level is l_crit = l_par - 1 (l_par >= 3); below it every box
// is DOMESTIC. At l_crit a box whose nonempty source children (at l_par) are
// all on other ranks is IMPORT, one with children on J and elsewhere is ROOT;
// one with all children on J is EXPORT if some receiver box r at l_crit that
// has k in its M2L list E4(r) has a nonempty receiver child on another rank,
// else DOMESTIC. From l_par down, the owner of a box is the owner of its
// ancestor at l_par: a box on J is EXPORT if some receiver box on another rank
// has it in its E4 list, else DOMESTIC; a box on another rank is IMPORT if
// some receiver box on J has it in its E4 list, else OTHER.
int oref_box_types(const oref_tree* t, uint32_t l_par, const uint32_t* owner, uint32_t rank,
                   uint8_t* types_out) {
  enum { DOMESTIC = 0, EXPORT = 1, IMPORT = 2, ROOT = 3, OTHER = 4 };
  if (!t || !owner || !types_out) return OREF_ERR_ARG;
  if (l_par < 3 || l_par > t->depth || 3 * l_par > 30) return OREF_ERR_LEVEL;
  const uint32_t l_crit = l_par - 1;
  const PointSet& S = t->set(0);
  const PointSet& R = t->set(1);
  auto own = [&](uint64_t key, uint32_t l) { return owner[key >> (3 * (l - l_par))]; };
  std::vector<uint32_t> lst;
  size_t at = 0;
  for (uint32_t l = 2; l <= t->depth; ++l) {
    const Level& sl = S.lv[l];
    const Level& rl = R.lv[l];
    const size_t ns = sl.key.size();
    uint8_t* ty = types_out + at;
    at += ns;
    if (l < l_crit) {
      for (size_t k = 0; k < ns; ++k) ty[k] = DOMESTIC;
      continue;
    }
    Lookup look(sl, l, false);
    std::vector<char> needed_elsewhere(ns, 0), needed_here(ns, 0);
    if (l == l_crit) {
      // receiver boxes at l_crit with a nonempty receiver child on another rank
      const Level& rc = R.lv[l_par];
      for (size_t r = 0; r < rl.key.size(); ++r) {
        bool remote = false;
        for (size_t c = 0; c < rc.key.size(); ++c)
          if ((rc.key[c] >> 3) == rl.key[r] && own(rc.key[c], l_par) != rank) remote = true;
        if (!remote) continue;
        box_list(look, 4, rl.key[r], l, lst);
        for (uint32_t k : lst) needed_elsewhere[k] = 1;
      }
      const Level& sc = S.lv[l_par];
      for (size_t k = 0; k < ns; ++k) {
        bool on = false, off = false;
        for (size_t c = 0; c < sc.key.size(); ++c) {
          if ((sc.key[c] >> 3) != sl.key[k]) continue;
          if (own(sc.key[c], l_par) == rank) on = true;
          else off = true;
        }
        if (!on) ty[k] = IMPORT;
        else if (off) ty[k] = ROOT;
        else ty[k] = needed_elsewhere[k] ? EXPORT : DOMESTIC;
      }
      continue;
    }
    for (size_t r = 0; r < rl.key.size(); ++r) {
      const bool r_here = own(rl.key[r], l) == rank;
      box_list(look, 4, rl.key[r], l, lst);
      for (uint32_t k : lst) {
        const bool k_here = own(sl.key[k], l) == rank;
        if (k_here && !r_here) needed_elsewhere[k] = 1;
        if (!k_here && r_here) needed_here[k] = 1;
      }
    }
    for (size_t k = 0; k < ns; ++k) {
      if (own(sl.key[k], l) == rank) ty[k] = needed_elsewhere[k] ? EXPORT : DOMESTIC;
      else ty[k] = needed_here[k] ? IMPORT : OTHER;
    }
  }
  return OREF_OK;
}

// The type of one source box (level `level`, rank `box`), from the same
// definition as oref_box_types but without lists: the receiver boxes r with
// the box in E4(r) are found by enumerating the cells at Chebyshev distance
// >= 2 whose parents are within 1 (the E4 condition is symmetric in r and k)
// and looking them up among the nonempty receiver boxes. Returns the type, or
// minus a status code.
int oref_box_type_one(const oref_tree* t, uint32_t l_par, const uint32_t* owner, uint32_t rank,
                      uint32_t level, uint32_t box) {
  enum { DOMESTIC = 0, EXPORT = 1, IMPORT = 2, ROOT = 3, OTHER = 4 };
  if (!t || !owner) return -OREF_ERR_ARG;
  if (l_par < 3 || l_par > t->depth || 3 * l_par > 30) return -OREF_ERR_LEVEL;
  if (level < 2 || level > t->depth) return -OREF_ERR_LEVEL;
  const uint32_t l_crit = l_par - 1;
  const Level& sl = t->set(0).lv[level];
  if (box >= sl.key.size()) return -OREF_ERR_ARG;
  if (level < l_crit) return DOMESTIC;
  const uint64_t kk = sl.key[box];
  auto own = [&](uint64_t key, uint32_t l) { return owner[key >> (3 * (l - l_par))]; };
  auto has = [](const Level& lv, uint64_t key) {
    return std::binary_search(lv.key.begin(), lv.key.end(), key);
  };
  const Level& rl = t->set(1).lv[level];
  // nonempty receiver boxes r with kk in E4(r)
  std::vector<uint64_t> recv;
  int64_t ck[3];
  deinterleave(kk, level, ck);
  const int64_t m = (int64_t)1 << level;
  int64_t c[3];
  for (c[2] = 2 * (floor_half(ck[2]) - 1); c[2] <= 2 * (floor_half(ck[2]) + 1) + 1; ++c[2])
    for (c[1] = 2 * (floor_half(ck[1]) - 1); c[1] <= 2 * (floor_half(ck[1]) + 1) + 1; ++c[1])
      for (c[0] = 2 * (floor_half(ck[0]) - 1); c[0] <= 2 * (floor_half(ck[0]) + 1) + 1; ++c[0]) {
        bool inside = true;
        int64_t cheb = 0, pcheb = 0;
        for (int d = 0; d < 3; ++d) {
          inside = inside && c[d] >= 0 && c[d] < m;
          cheb = std::max(cheb, iabs(c[d] - ck[d]));
          pcheb = std::max(pcheb, iabs(floor_half(c[d]) - floor_half(ck[d])));
        }
        if (!inside || cheb < 2 || pcheb > 1) continue;
        const uint64_t rk = interleave((uint32_t)c[0], (uint32_t)c[1], (uint32_t)c[2], level);
        if (has(rl, rk)) recv.push_back(rk);
      }
  if (level == l_crit) {
    const Level& sc = t->set(0).lv[l_par];
    const Level& rc = t->set(1).lv[l_par];
    bool on = false, off = false;
    for (uint64_t o = 0; o < 8; ++o) {
      const uint64_t ch = (kk << 3) | o;
      if (!has(sc, ch)) continue;
      if (own(ch, l_par) == rank) on = true;
      else off = true;
    }
    if (!on) return IMPORT;
    if (off) return ROOT;
    for (uint64_t rk : recv)
      for (uint64_t o = 0; o < 8; ++o) {
        const uint64_t ch = (rk << 3) | o;
        if (has(rc, ch) && own(ch, l_par) != rank) return EXPORT;
      }
    return DOMESTIC;
  }
  const bool here = own(kk, level) == rank;
  for (uint64_t rk : recv) {
    const bool r_here = own(rk, level) == rank;
    if (here && !r_here) return EXPORT;
    if (!here && r_here) return IMPORT;
  }
  return here ? DOMESTIC : OTHER;
}

// ---------------------------------------------------------------------------
// Near-field sum over E2 (Algorithm 2 and a Laplace kernel).
// ---------------------------------------------------------------------------

// For every receiver point y (original order): phi = sum of q_i / |x_i - y|
// over the source points x_i of the E2 boxes of y's box at the finest level
// (Algorithm 2 gathers exactly these points), pairs at distance zero left
// out; abs_sum = the same with |q_i|. Charges in original source order, NULL
// for unit charges. FP64 from the FP32 coordinates; needs the lists.
int oref_near_field(const oref_tree* t, const float* charges, double* phi, double* abs_sum) {
  if (!t || !phi || !abs_sum || !t->has_lists) return OREF_ERR_ARG;
  const uint32_t D = t->depth;
  const PointSet& S = t->set(0);
  const PointSet& R = t->set(1);
  const Level& rl = R.lv[D];
  const Level& sl = S.lv[D];
  const List& e2 = t->e2[D];
  for (size_t b = 0; b + 1 < rl.begin.size(); ++b) {
    for (uint32_t k = rl.begin[b]; k < rl.begin[b + 1]; ++k) {
      const double y[3] = {R.sorted_xyz[3 * (size_t)k], R.sorted_xyz[3 * (size_t)k + 1],
                           R.sorted_xyz[3 * (size_t)k + 2]};
      double f = 0.0, a = 0.0;
      for (uint32_t e = e2.off[b]; e < e2.off[b + 1]; ++e) {
        const uint32_t sb = e2.ent[e];
        for (uint32_t i = sl.begin[sb]; i < sl.begin[sb + 1]; ++i) {
          const double dx = (double)S.sorted_xyz[3 * (size_t)i] - y[0];
          const double dy = (double)S.sorted_xyz[3 * (size_t)i + 1] - y[1];
          const double dz = (double)S.sorted_xyz[3 * (size_t)i + 2] - y[2];
          const double d = std::sqrt(dx * dx + dy * dy + dz * dz);
          if (d == 0.0) continue;
          const double q = charges ? (double)charges[S.perm[i]] : 1.0;
          f += q / d;
          a += std::fabs(q) / d;
        }
      }
      phi[R.perm[k]] = f;
      abs_sum[R.perm[k]] = a;
    }
  }
  return OREF_OK;
}

// The near-field sum of one receiver point (original index j) from the
// definition, without lists: the source boxes at Chebyshev distance <= 1 of
// the point's finest-level box are looked up among the nonempty source boxes.
int oref_near_field_one(const oref_tree* t, const float* charges, uint32_t j, double* phi,
                        double* abs_sum) {
  if (!t || !phi || !abs_sum) return OREF_ERR_ARG;
  const PointSet& S = t->set(0);
  const PointSet& R = t->set(1);
  if (j >= R.perm.size()) return OREF_ERR_ARG;
  const uint32_t D = t->depth;
  // position of j in the sorted receivers, and its coordinates
  const size_t k = std::find(R.perm.begin(), R.perm.end(), j) - R.perm.begin();
  const double y[3] = {R.sorted_xyz[3 * k], R.sorted_xyz[3 * k + 1], R.sorted_xyz[3 * k + 2]};
  int64_t cy[3];
  deinterleave(R.sorted_key[k] >> (3 * (t->max_level - D)), D, cy);
  const Level& sl = S.lv[D];
  Lookup look(sl, D, false);
  double f = 0.0, a = 0.0;
  int64_t c[3];
  for (c[2] = cy[2] - 1; c[2] <= cy[2] + 1; ++c[2])
    for (c[1] = cy[1] - 1; c[1] <= cy[1] + 1; ++c[1])
      for (c[0] = cy[0] - 1; c[0] <= cy[0] + 1; ++c[0]) {
        const int64_t sb = look.rank(c);
        if (sb < 0) continue;
        for (uint32_t i = sl.begin[sb]; i < sl.begin[sb + 1]; ++i) {
          const double dx = (double)S.sorted_xyz[3 * (size_t)i] - y[0];
          const double dy = (double)S.sorted_xyz[3 * (size_t)i + 1] - y[1];
          const double dz = (double)S.sorted_xyz[3 * (size_t)i + 2] - y[2];
          const double d = std::sqrt(dx * dx + dy * dy + dz * dz);
          if (d == 0.0) continue;
          const double q = charges ? (double)charges[S.perm[i]] : 1.0;
          f += q / d;
          a += std::fabs(q) / d;
        }
      }
  *phi = f;
  *abs_sum = a;
  return OREF_OK;
}

}  // extern "C"
