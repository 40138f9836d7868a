// Autotuner: time the candidate tile shapes (and split-K factors) on
// synthetic problems of each size class and record the fastest in the tile
// table.  The paper derives block sizes from an analytical model and encodes
// the choice per level in a control tree (Section "Building on important
// advances"); here the choice is measured on the device instead, once per
// size class, and stored as text.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
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

// Median time (ms) of `reps` launches of a batched plan, after two warm-up
// launches.
famlies_status time_batch(famlies_plan_s* p, void* const* ptrs, int64_t n, hipStream_t s, int reps, float* ms) {
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
    st = batch_execute_impl(p, 1.0, 0.0, ptrs, ptrs + n, ptrs + 2 * n, s);
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

// Plain kernels: tile shape and split-K per size class, timed on one GEMM-
// shaped contraction C[m,n] = sum_k A[m,k] B[k,n] with A and B contiguous
// along k (the K-gathered case) and C contiguous along n.
famlies_status tune_plain(famlies_handle_s* h, const Buffers& buf, int64_t cap, bool quick, int reps,
                          TileTable* fresh) {
  const std::vector<int> lmn = quick ? std::vector<int>{6, 9, 12} : std::vector<int>{5, 6, 7, 8, 9, 10, 11, 12};
  const std::vector<int> lks = quick ? std::vector<int>{6, 10} : std::vector<int>{5, 7, 9, 11, 13};
  struct Mode2 {
    int dtype, compute;
  };
  const Mode2 modes[3] = {{FAMLIES_F64, FAMLIES_NATIVE}, {FAMLIES_F32, FAMLIES_NATIVE}, {FAMLIES_F32, FAMLIES_BF16X3}};
  hipStream_t s = nullptr;
  for (const Mode2& md : modes)
    for (int lm : lmn)
      for (int ln : lmn)
        for (int lk : lks) {
          const int64_t M = (int64_t)1 << lm, N = (int64_t)1 << ln, K = (int64_t)1 << lk;
          if (M * K > cap || K * N > cap || M * N > cap) continue;
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
            t.bk = md.dtype == FAMLIES_F64 ? 8 : 32;
            t.split = 1;
            cands.push_back(t);
            const int64_t tiles = ((M + bt - 1) / bt) * ((N + bt - 1) / bt);
            for (int sp : {2, 4, 8, 16})
              if (tiles * sp <= 4 * h->num_cus && K / sp >= 2 * t.bk) {
                t.split = sp;
                cands.push_back(t);
              }
          }
          float best = 1e30f;
          TileCfg bcfg = cands[0];
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
          }
          if (log_enabled())
            std::fprintf(stderr, "[famlies] tune plain dtype %d compute %d M %lld N %lld K %lld: %dx%dx%d split %d %.4f ms\n",
                         md.dtype, md.compute, (long long)M, (long long)N, (long long)K, bcfg.bm, bcfg.bn, bcfg.bk,
                         bcfg.split, best);
          TileTable::Entry en;
          en.kind = 0;
          en.dtype = md.dtype;
          en.compute = md.compute;
          en.lm = TileTable::log2c(an.M);
          en.ln = TileTable::log2c(an.N);
          en.lk = TileTable::log2c(an.K);
          en.cfg = bcfg;
          fresh->put(en);
        }
  return FAMLIES_OK;
}

// Batched kernel: tile class per size class, timed on the batched kernel
// itself.  Each size class runs as one batched launch of identical problems
// C_i[m,n] = sum_k A[m,k] B[k,n], A contiguous along k (X gathered along K)
// and B contiguous along n (Y gathered by rows), so that both loaders take
// part; the A and B data are shared by all problems, the C blocks are
// disjoint.  Enough problems are batched for about 2e10 flops and at least
// four items of the largest tile per resident workgroup (at most 4096
// problems, and as many as the scratch buffers hold), so every class fills
// the device and the time is throughput as in a large mixed batch.
famlies_status tune_batch(famlies_handle_s* h, const Buffers& buf, int64_t cap, bool quick, int reps,
                          TileTable* fresh) {
  const std::vector<int> lmn = quick ? std::vector<int>{5, 8, 11} : std::vector<int>{4, 5, 6, 7, 8, 9, 10, 11, 12};
  const std::vector<int> lks = quick ? std::vector<int>{6, 10} : std::vector<int>{4, 6, 8, 10, 12};
  constexpr int64_t kMaxProblems = 4096;
  constexpr double kTargetFlops = 2e10;
  void** ptrs = nullptr;  // device: A pointers | B pointers | C pointers
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&ptrs), 3 * kMaxProblems * sizeof(void*));
  if (e != hipSuccess) return hip_fail(e, "famlies_tune: hipMalloc");
  struct Free {
    void* p;
    ~Free() { (void)hipFree(p); }
  } free_ptrs{ptrs};
  std::vector<void*> host(3 * kMaxProblems);
  hipStream_t s = nullptr;
  for (int dtype : {FAMLIES_F64, FAMLIES_F32}) {
    const int64_t es = dtype == FAMLIES_F64 ? 8 : 4;
    for (int lm : lmn)
      for (int ln : lmn)
        for (int lk : lks) {
          const int64_t M = (int64_t)1 << lm, N = (int64_t)1 << ln, K = (int64_t)1 << lk;
          if (M * K > cap || K * N > cap || M * N > cap) continue;
          const int64_t items128 = ceil_div(M, 128) * ceil_div(N, 128);
          const int64_t min_items = 4 * 2 * (int64_t)h->num_cus;  // two resident workgroups per CU
          int64_t n = std::max<int64_t>((int64_t)std::ceil(kTargetFlops / (2.0 * M * N * K)),
                                        ceil_div(min_items, items128));
          n = std::max<int64_t>(1, std::min<int64_t>({n, kMaxProblems, cap * 8 / (M * N * es)}));
          const int64_t ea[2] = {M, K}, sa[2] = {K, 1};
          const int64_t eb[2] = {K, N}, sb[2] = {N, 1};
          const int64_t ec[2] = {M, N}, sc[2] = {N, 1};
          const int32_t la[2] = {'m', 'k'}, lb[2] = {'k', 'n'}, lc[2] = {'m', 'n'};
          const famlies_tensor A = {2, ea, sa, la}, B = {2, eb, sb, lb}, C = {2, ec, sc, lc};
          const std::vector<famlies_tensor> As((size_t)n, A), Bs((size_t)n, B), Cs((size_t)n, C);
          for (int64_t i = 0; i < n; ++i) {
            host[(size_t)i] = buf.a;
            host[(size_t)(n + i)] = buf.b;
            host[(size_t)(2 * n + i)] = static_cast<char*>(buf.c) + i * M * N * es;
          }
          if ((e = hipMemcpy(ptrs, host.data(), 3 * n * sizeof(void*), hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "famlies_tune: hipMemcpy");
          float best = 1e30f, tms[4] = {0.f, 0.f, 0.f, 0.f};
          int bcls = 0;
          for (int cls = 0; cls < 4; ++cls) {
            famlies_plan_s* p = nullptr;
            famlies_status st = batch_plan_make(h, &p, dtype, n, As.data(), Bs.data(), Cs.data(), cls);
            if (st != FAMLIES_OK) return st;
            float ms = 0.f;
            st = time_batch(p, ptrs, n, s, reps, &ms);
            destroy_plan(p);
            if (st != FAMLIES_OK) return st;
            tms[cls] = ms;
            if (ms < best) {
              best = ms;
              bcls = cls;
            }
          }
          if (log_enabled())
            std::fprintf(stderr,
                         "[famlies] tune batch %s M %lld N %lld K %lld x %lld: ms 64x64 %.4f 128x64 %.4f "
                         "64x128 %.4f 128x128 %.4f\n",
                         dtype == FAMLIES_F64 ? "f64" : "f32", (long long)M, (long long)N, (long long)K,
                         (long long)n, tms[0], tms[1], tms[2], tms[3]);
          TileTable::Entry en;
          en.kind = 1;
          en.dtype = dtype;
          en.compute = FAMLIES_NATIVE;
          en.lm = lm;
          en.ln = ln;
          en.lk = lk;
          en.cfg.bm = (bcls & 1) ? 128 : 64;
          en.cfg.bn = (bcls & 2) ? 128 : 64;
          en.cfg.bk = batch_slice_k();
          en.cfg.split = 1;
          fresh->put(en);
        }
  }
  return FAMLIES_OK;
}

}  // namespace
}  // namespace famlies

using namespace famlies;

extern "C" {

static famlies_status tune_impl(famlies_handle htok, const char* table_path, int flags) {
  famlies_handle_s* h = handle_of(htok);
  if (!h || !table_path) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_tune: invalid argument");
  const bool quick = flags & FAMLIES_TUNE_QUICK;
  const bool do_plain = !(flags & FAMLIES_TUNE_BATCH_ONLY), do_batch = !(flags & FAMLIES_TUNE_PLAIN_ONLY);
  if (!do_plain && !do_batch) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_tune: nothing to tune");
  DeviceGuard dg(h->device);
  if (!dg.ok) return fail(FAMLIES_ERR_DEVICE, "cannot select the handle's device");
  // each operand at most 2^26 elements
  const int64_t cap = (int64_t)1 << 26;
  Buffers buf;
  hipError_t e;
  if ((e = hipMalloc(&buf.a, cap * 8)) != hipSuccess || (e = hipMalloc(&buf.b, cap * 8)) != hipSuccess ||
      (e = hipMalloc(&buf.c, cap * 8)) != hipSuccess)
    return hip_fail(e, "famlies_tune: hipMalloc");
  if ((e = hipMemset(buf.a, 0, cap * 8)) != hipSuccess || (e = hipMemset(buf.b, 0, cap * 8)) != hipSuccess ||
      (e = hipMemset(buf.c, 0, cap * 8)) != hipSuccess)
    return hip_fail(e, "famlies_tune: hipMemset");
  const int reps = quick ? 3 : 7;
  TileTable fresh;
  famlies_status st = FAMLIES_OK;
  if (do_plain && (st = tune_plain(h, buf, cap, quick, reps, &fresh)) != FAMLIES_OK) return st;
  if (do_batch && (st = tune_batch(h, buf, cap, quick, reps, &fresh)) != FAMLIES_OK) return st;
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
