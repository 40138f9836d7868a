// Host-only driver for the library's planning code, built by
// tests/test_host_sanitize.py with AddressSanitizer and UndefinedBehavior-
// Sanitizer (no device code, no GPU): the planner, the tile choice, the
// planner dry run (famlies_analyze), the tile-table reader, the object
// registry and the indexing-vector bounds check.
//
//   driver analyze <cases>   one line per case: status, then (when OK) the
//                            plan summary and a checksum of the offsets
//   driver table <file>      load a tile table: "ok <entries>" or "err"
//   driver registry          token life cycle checks
//   driver bounds            offsets_in_span on crafted vectors
//
// Case file: whitespace-separated integers, per case
//   dtype compute, then for A, B, C: rank, extents..., strides..., labels...
#include <cstdint>
#include <cstdio>
#include <fstream>
#include <string>
#include <vector>

#include "famlies.h"
#include "internal.hpp"
#include "runtime.hpp"

using namespace famlies;

static bool read_tensor(std::istream& in, int32_t* rank, std::vector<int64_t>* e, std::vector<int64_t>* s,
                        std::vector<int32_t>* l) {
  if (!(in >> *rank)) return false;
  const int r = *rank < 0 ? 0 : *rank;
  e->assign((size_t)r, 0);
  s->assign((size_t)r, 0);
  l->assign((size_t)r, 0);
  for (auto& x : *e) in >> x;
  for (auto& x : *s) in >> x;
  for (auto& x : *l) in >> x;
  return (bool)in;
}

static int run_analyze(const char* path) {
  std::ifstream in(path);
  int dtype, compute;
  while (in >> dtype >> compute) {
    int32_t r[3];
    std::vector<int64_t> e[3], s[3];
    std::vector<int32_t> l[3];
    for (int t = 0; t < 3; ++t)
      if (!read_tensor(in, &r[t], &e[t], &s[t], &l[t])) return 2;
    famlies_tensor T[3];
    for (int t = 0; t < 3; ++t)
      T[t] = famlies_tensor{r[t], e[t].empty() ? nullptr : e[t].data(), s[t].empty() ? nullptr : s[t].data(),
                            l[t].empty() ? nullptr : l[t].data()};
    famlies_plan_info info;
    famlies_status st = famlies_analyze(dtype, compute, &T[0], &T[1], &T[2], &info, nullptr, 0);
    if (st != FAMLIES_OK) {
      std::printf("%d\n", st);
      continue;
    }
    const int64_t len = 2 * info.m + 2 * info.k + 2 * info.n + 3 * info.batch;
    std::vector<int64_t> offs((size_t)len + 1, 0);
    st = famlies_analyze(dtype, compute, &T[0], &T[1], &T[2], &info, offs.data(), len);
    uint64_t sum = 0;
    for (int64_t i = 0; i < len; ++i) sum += (uint64_t)offs[(size_t)i] * (uint64_t)(i % 97 + 1);
    std::printf("%d %lld %lld %lld %lld %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %llu\n", st,
                (long long)info.m, (long long)info.n, (long long)info.k, (long long)info.batch, info.swapped,
                info.x_kfast, info.y_kfast, info.n_i, info.n_j, info.n_p, info.n_batch, info.n_trace,
                info.n_diag, info.tile_m, info.tile_n, info.tile_k, info.split_k, info.index_bits, info.kernel,
                info.split_tiles, info.index_elements, (unsigned long long)sum);
  }
  return 0;
}

static int run_table(const char* path) {
  TileTable t;
  std::string err;
  if (t.load(path, &err))
    std::printf("ok %zu\n", t.entries.size());
  else
    std::printf("err\n");
  return 0;
}

static int run_registry() {
  int a = 0, b = 0;
  void* ta = registry_add(&a, ObjKind::kPlan);
  if (!ta || registry_get(ta, ObjKind::kPlan) != &a) return 10;
  if (registry_get(ta, ObjKind::kHandle) || registry_get(ta, ObjKind::kNetwork)) return 11;  // wrong kind
  if (registry_take(ta, ObjKind::kPlan) != &a) return 12;
  if (registry_get(ta, ObjKind::kPlan) || registry_take(ta, ObjKind::kPlan)) return 13;  // retired
  void* tb = registry_add(&b, ObjKind::kPlan);  // reuses the slot with the next generation
  if (!tb || tb == ta) return 14;
  if (registry_get(ta, ObjKind::kPlan)) return 15;  // the stale token stays rejected
  if (registry_get(tb, ObjKind::kPlan) != &b) return 16;
  if (registry_get(nullptr, ObjKind::kPlan) || registry_get(reinterpret_cast<void*>(0x12345678), ObjKind::kPlan))
    return 17;
  std::vector<void*> many;
  for (int i = 0; i < 1000; ++i) many.push_back(registry_add(&a, ObjKind::kHandle));
  for (void* t : many)
    if (registry_take(t, ObjKind::kHandle) != &a) return 18;
  if (registry_take(tb, ObjKind::kPlan) != &b) return 19;
  std::printf("registry ok\n");
  return 0;
}

static int run_bounds() {
  // a 3 x 4 column-major tensor (strides 1, 3) viewed as rows x cols
  const std::vector<int64_t> rows = {0, 1, 2}, cols = {0, 3, 6, 9}, batch = {0};
  const bool inside = offsets_in_span(rows, 3, cols, 4, batch, 1, 0, 11);
  const bool past = offsets_in_span(rows, 3, cols, 4, batch, 1, 0, 10);          // last element 11 > 10
  const bool before = offsets_in_span(rows, 3, cols, 4, {-1}, 1, 0, 11);         // first element -1 < 0
  const bool neg = offsets_in_span({0, -1, -2}, 3, cols, 4, batch, 1, -2, 9);     // negative row stride
  const bool empty = offsets_in_span(rows, 0, cols, 4, batch, 1, 5, 4);          // nothing addressed
  const bool short_vec = offsets_in_span(rows, 4, cols, 4, batch, 1, 0, 100);    // fewer entries than claimed
  std::printf("%d %d %d %d %d %d\n", inside, past, before, neg, empty, short_vec);
  return 0;
}

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  const std::string mode = argv[1];
  if (mode == "analyze" && argc == 3) return run_analyze(argv[2]);
  if (mode == "table" && argc == 3) return run_table(argv[2]);
  if (mode == "registry") return run_registry();
  if (mode == "bounds") return run_bounds();
  return 2;
}
