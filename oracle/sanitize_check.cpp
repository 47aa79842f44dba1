/*
 * Exercise of every oracle entry point for a sanitizer build (AddressSanitizer
 * and UndefinedBehaviorSanitizer): TEST INFRASTRUCTURE ONLY. The test suite
 * compiles this file together with fmmds_oracle.cpp with g++ and runs it; any
 * memory error or undefined behaviour aborts the run.
 */
#include "fmmds_oracle.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

namespace {

uint64_t g_state = 0x243F6A8885A308D3ull;
float unit() {  // uniform FP32 in [0, 1)
  g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
  return (float)(g_state >> 40) * (1.0f / 16777216.0f);
}

int fail(const char* what, int st) {
  std::fprintf(stderr, "sanitize_check: %s returned %d\n", what, st);
  return 1;
}

int exercise(const std::vector<float>& src, const std::vector<float>* recv, uint32_t kb,
             uint32_t s, uint32_t L) {
  const uint32_t ns = (uint32_t)(src.size() / 3);
  const uint32_t nr = recv ? (uint32_t)(recv->size() / 3) : 0;
  oref_tree* t = nullptr;
  int st = oref_build(src.data(), ns, recv ? recv->data() : nullptr, nr, kb, s, L, 1, &t);
  if (st != OREF_OK) return fail("oref_build", st);
  const uint32_t D = oref_depth(t);
  for (int set = 0; set < 2; ++set) {
    const uint32_t n = oref_n_points(t, set);
    std::vector<uint32_t> perm(n);
    std::vector<float> xyz(3 * (size_t)n);
    if ((st = oref_perm(t, set, perm.data())) != OREF_OK) return fail("oref_perm", st);
    if ((st = oref_sorted_xyz(t, set, xyz.data())) != OREF_OK) return fail("oref_sorted_xyz", st);
    for (uint32_t l = 0; l <= D; ++l) {
      const uint32_t nb = oref_n_boxes(t, set, l);
      std::vector<uint64_t> k(nb);
      std::vector<uint32_t> b(nb + 1), p(nb), c(nb + 1);
      (void)oref_max_occupancy(t, set, l);
      if ((st = oref_keys(t, set, l, k.data())) != OREF_OK) return fail("oref_keys", st);
      if ((st = oref_begin(t, set, l, b.data())) != OREF_OK) return fail("oref_begin", st);
      if (l >= 1 && (st = oref_parent(t, set, l, p.data())) != OREF_OK) return fail("oref_parent", st);
      if (l < D && (st = oref_child(t, set, l, c.data())) != OREF_OK) return fail("oref_child", st);
    }
  }
  for (uint32_t l = 2; l <= D; ++l) {
    oref_lookup* lk = oref_lookup_open(t, l);
    if (!lk) return fail("oref_lookup_open", -1);
    for (int kind : {2, 4}) {
      uint32_t nb = 0;
      uint64_t ne = 0;
      if ((st = oref_list_sizes(t, kind, l, &nb, &ne)) != OREF_OK) return fail("oref_list_sizes", st);
      std::vector<uint32_t> off(nb + 1), ent(ne + 1), roff(nb + 1), rent((size_t)nb * 189 + 1);
      if ((st = oref_list(t, kind, l, off.data(), ent.data())) != OREF_OK) return fail("oref_list", st);
      if ((st = oref_list_range(lk, kind, 0, nb, roff.data(), rent.data())) != OREF_OK)
        return fail("oref_list_range", st);
      for (uint32_t j = 0; j <= nb; ++j)
        if (roff[j] != off[j]) return fail("range offsets differ", (int)j);
      std::vector<uint32_t> one(189);
      for (uint32_t j = 0; j < nb; j += 1 + nb / 17)
        if (oref_box_list(t, kind, l, j, one.data()) < 0) return fail("oref_box_list", (int)j);
    }
    oref_lookup_close(lk);
  }
  for (uint32_t lp = 3; lp <= D && lp <= 5; ++lp) {
    std::vector<uint32_t> owner((size_t)1 << (3 * lp));
    if ((st = oref_partition(t, lp, 3, owner.data())) != OREF_OK) return fail("oref_partition", st);
    size_t total = 0;
    for (uint32_t l = 2; l <= D; ++l) total += oref_n_boxes(t, 0, l);
    std::vector<uint8_t> types(total + 1);
    for (uint32_t r = 0; r < 3; ++r) {
      if ((st = oref_box_types(t, lp, owner.data(), r, types.data())) != OREF_OK)
        return fail("oref_box_types", st);
      if (oref_box_type_one(t, lp, owner.data(), r, D, 0) < 0) return fail("oref_box_type_one", -1);
    }
  }
  const uint32_t m = oref_n_points(t, 1);
  std::vector<double> phi(m), abs_sum(m);
  std::vector<float> q(ns);
  for (auto& v : q) v = unit() - 0.5f;
  if ((st = oref_near_field(t, q.data(), phi.data(), abs_sum.data())) != OREF_OK)
    return fail("oref_near_field", st);
  double f1, a1;
  if ((st = oref_near_field_one(t, nullptr, m - 1, &f1, &a1)) != OREF_OK)
    return fail("oref_near_field_one", st);
  oref_free(t);
  return 0;
}

std::vector<float> points(uint32_t n, bool clustered) {
  std::vector<float> p(3 * (size_t)n);
  for (uint32_t i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) {
      float v = unit();
      if (clustered) v = 0.3f + 0.05f * v;
      p[3 * (size_t)i + d] = v;
    }
  return p;
}

}  // namespace

int main() {
  const std::vector<float> a = points(3000, false), b = points(2000, true);
  if (exercise(a, nullptr, 64, 0, 5)) return 1;
  if (exercise(a, &b, 32, 0, 6)) return 1;
  if (exercise(b, &a, 64, 40, 9)) return 1;
  const std::vector<float> one = {0.5f, 0.5f, 0.5f};
  if (exercise(one, &one, 64, 0, 21)) return 1;
  // error paths: NaN, out of range, bad arguments
  std::vector<float> bad = a;
  bad[7] = std::nanf("");
  oref_tree* t = nullptr;
  if (oref_build(bad.data(), 3000, nullptr, 0, 64, 0, 5, 1, &t) != OREF_ERR_RANGE) return 1;
  bad[7] = 1.0f;
  if (oref_build(bad.data(), 3000, nullptr, 0, 64, 0, 5, 1, &t) != OREF_ERR_RANGE) return 1;
  if (oref_build(a.data(), 3000, nullptr, 0, 32, 0, 11, 1, &t) != OREF_ERR_ARG) return 1;
  if (oref_build(nullptr, 3000, nullptr, 0, 64, 0, 5, 1, &t) != OREF_ERR_ARG) return 1;
  std::vector<uint64_t> keys(3000);
  if (oref_point_keys(a.data(), 3000, 21, keys.data()) != OREF_OK) return 1;
  std::puts("sanitize_check: ok");
  return 0;
}
