// Autotuner: time the candidate tile shapes (and split-K factors) on
// synthetic problems of each size class and record the fastest in the tile
// table.  The paper derives block sizes from an analytical model and encodes
// the choice per level in a control tree (Section "Building on important
// advances"); here the choice is measured on the device instead, once per
// size class, and stored as text.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>

#include "famlies.h"
#include "runtime.hpp"

namespace famlies {
namespace {

struct Buffers {
  void* a = nullptr;
  void* b = nullptr;
  void* c = nullptr;
  ~Buffers() {
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (c) (void)hipFree(c);
  }
};

// Median time (ms) of `reps` launches of a plan, after two warm-up launches.
famlies_status time_plan(famlies_plan_s* p, const Buffers& buf, hipStream_t s, int reps, float* ms) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(FAMLIES_ERR_DEVICE, "hipEventCreate");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(FAMLIES_ERR_DEVICE, "hipEventCreate");
  }
  std::vector<float> t;
  famlies_status st = FAMLIES_OK;
  for (int r = 0; r < reps + 2 && st == FAMLIES_OK; ++r) {
    (void)hipEventRecord(e0, s);
    st = execute_impl(p, 1.0, buf.a, buf.b, 0.0, buf.c, 0, s);
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) st = fail(FAMLIES_ERR_DEVICE, "hipEventSynchronize");
    float x = 0.f;
    (void)hipEventElapsedTime(&x, e0, e1);
    if (r >= 2) t.push_back(x);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != FAMLIES_OK) return st;
  std::sort(t.begin(), t.end());
  *ms = t[t.size() / 2];
  return FAMLIES_OK;
}

}  // namespace
}  // namespace famlies

using namespace famlies;

extern "C" {

static famlies_status tune_impl(famlies_handle htok, const char* table_path, int flags) {
  famlies_handle_s* h = handle_of(htok);
  if (!h || !table_path) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_tune: invalid argument");
  const bool quick = flags & 1;
  DeviceGuard dg(h->device);
  if (!dg.ok) return fail(FAMLIES_ERR_DEVICE, "cannot select the handle's device");
  // size classes: log2 of M, N, K; each operand at most 2^26 elements
  std::vector<int> lmn = quick ? std::vector<int>{6, 9, 12} : std::vector<int>{5, 6, 7, 8, 9, 10, 11, 12};
  std::vector<int> lks = quick ? std::vector<int>{6, 10} : std::vector<int>{5, 7, 9, 11, 13};
  const int64_t cap = (int64_t)1 << 26;
  Buffers buf;
  hipError_t e;
  if ((e = hipMalloc(&buf.a, cap * 8)) != hipSuccess || (e = hipMalloc(&buf.b, cap * 8)) != hipSuccess ||
      (e = hipMalloc(&buf.c, cap * 8)) != hipSuccess)
    return hip_fail(e, "famlies_tune: hipMalloc");
  if ((e = hipMemset(buf.a, 0, cap * 8)) != hipSuccess || (e = hipMemset(buf.b, 0, cap * 8)) != hipSuccess ||
      (e = hipMemset(buf.c, 0, cap * 8)) != hipSuccess)
    return hip_fail(e, "famlies_tune: hipMemset");
  hipStream_t s = nullptr;
  const int reps = quick ? 3 : 7;
  TileTable fresh;
  struct Mode2 {
    int dtype, compute;
  };
  const Mode2 modes[3] = {{FAMLIES_F64, FAMLIES_NATIVE}, {FAMLIES_F32, FAMLIES_NATIVE}, {FAMLIES_F32, FAMLIES_BF16X3}};
  for (const Mode2& md : modes) {
    for (int lm : lmn)
      for (int ln : lmn)
        for (int lk : lks) {
          const int64_t M = (int64_t)1 << lm, N = (int64_t)1 << ln, K = (int64_t)1 << lk;
          if (M * K > cap || K * N > cap || M * N > cap) continue;
          // C[m,n] = sum_k A[m,k] B[k,n]: A and B contiguous along k (the
          // K-gathered case), C contiguous along n (no operand exchange)
          const int64_t ea[2] = {M, K}, sa[2] = {K, 1};
          const int64_t eb[2] = {K, N}, sb[2] = {1, K};
          const int64_t ec[2] = {M, N}, sc[2] = {N, 1};
          const int32_t la[2] = {'m', 'k'}, lb[2] = {'k', 'n'}, lc[2] = {'m', 'n'};
          famlies_tensor A = {2, ea, sa, la}, B = {2, eb, sb, lb}, C = {2, ec, sc, lc};
          Analysis an;
          std::string err;
          if (analyze(md.dtype, md.compute, &A, &B, &C, &an, &err) != FAMLIES_OK) continue;
          std::vector<TileCfg> cands;
          for (int bt : {64, 128}) {
            TileCfg t;
            t.bm = t.bn = bt;
            t.bk = md.dtype == FAMLIES_F64 ? 16 : 32;
            t.split = 1;
            cands.push_back(t);
            const int64_t tiles = ((M + bt - 1) / bt) * ((N + bt - 1) / bt);
            for (int sp : {2, 4, 8, 16})
              if (tiles * sp <= 4 * h->num_cus && K / sp >= 2 * t.bk) {
                t.split = sp;
                cands.push_back(t);
              }
          }
          float best = 1e30f, best_nosplit = 1e30f;
          TileCfg bcfg = cands[0], bns = cands[0];
          for (const TileCfg& t : cands) {
            famlies_plan_s* p = nullptr;
            famlies_status st = make_plan(h, &p, md.dtype, md.compute, &A, &B, &C, &t);
            if (st != FAMLIES_OK) return st;
            const TileCfg eff = p->cfg;  // split after the planner's rounding
            float ms = 0.f;
            st = time_plan(p, buf, s, reps, &ms);
            destroy_plan(p);
            if (st != FAMLIES_OK) return st;
            if (ms < best) {
              best = ms;
              bcfg = eff;
            }
            if (eff.split == 1 && ms < best_nosplit) {
              best_nosplit = ms;
              bns = eff;
            }
          }
          TileTable::Entry en;
          en.kind = 0;
          en.dtype = md.dtype;
          en.compute = md.compute;
          en.lm = TileTable::log2c(an.M);
          en.ln = TileTable::log2c(an.N);
          en.lk = TileTable::log2c(an.K);
          en.cfg = bcfg;
          fresh.put(en);
          if (md.compute == FAMLIES_NATIVE) {  // batched kernel: no split-K
            en.kind = 1;
            en.cfg = bns;
            fresh.put(en);
          }
        }
  }
  std::string err;
  if (!fresh.save(table_path, &err)) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_tune: " + err);
  for (const auto& en : fresh.entries) h->table.put(en);
  return FAMLIES_OK;
}

famlies_status famlies_tune(famlies_handle htok, const char* table_path, int flags) {
  return no_throw("famlies_tune", [&] { return tune_impl(htok, table_path, flags); });
}

famlies_status famlies_load_tune_table(famlies_handle htok, const char* table_path) {
  famlies_handle_s* h = handle_of(htok);
  if (!h || !table_path) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_load_tune_table: invalid argument");
  return no_throw("famlies_load_tune_table", [&] {
    std::string err;
    if (!h->table.load(table_path, &err)) return fail(FAMLIES_ERR_INVALID_ARG, err);
    return FAMLIES_OK;
  });
}

}  // extern "C"
