// Batched contractions: many independent, uneven problems in one persistent
// launch, and the autotuner that picks tile shapes per size class.
//
// The host plans every problem as a single contraction would be planned
// (labels, grouping, orientation, indexing vectors), then cuts all problems
// into (problem, tile) work items and deals them to a fixed grid of
// workgroups: problems are spread over the XCDs by estimated cost (so a
// problem's tiles share one L2; a problem larger than a quarter of an XCD's
// share is cut into runs of tiles first), and each XCD's items form one queue,
// the costliest items (largest padded K) first with a problem's tiles
// consecutive.  The
// workgroups of an XCD take items from its queue with an atomic counter, so
// a problem's tiles run side by side and no workgroup idles while its queue
// has work (longest-processing-time-first, decided as the launch runs).  The
// last workgroup of a queue to finish sets its counters back to zero, so a
// launch needs no clearing and can be captured in a HIP graph and replayed;
// launches of one batched plan must not overlap.  This is the
// on-GPU counterpart of running many tile-sized contractions (Approach,
// "Supporting tensor computations": tiling of tensors, tensor-of-tensors
// and dynamic blocking) and of block-size selection per problem (the
// control tree of Section "Building on important advances").
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "famlies.h"
#include "runtime.hpp"
#include "tile.hpp"

namespace famlies {

struct BatchProblemDev {
  int32_t M, N, K;
  int32_t flags;  // bit 0: swapped, bit 1: X gathered along K, bit 2: Y along K, bits 8..: tile class
  int64_t off;    // first entry of this problem's six indexing vectors in the pool
  int64_t xlo, ylo, clo;  // element shift from each base pointer to the operand's lowest element
  int32_t pos[6]; // vector starts relative to off: X rows, X k, Y k, Y cols, C rows, C cols
};

struct BatchItem {
  int32_t prob;
  int16_t tm, tn;
};

struct BatchArgs {
  const BatchProblemDev* probs;
  const BatchItem* items;
  const int32_t* q_start;  // items of queue q: [q_start[q], q_start[q+1]) (kXcds queues)
  int32_t* counters;       // [q]: next item of queue q; [kXcds + q]: workgroups done with it
  int32_t per_queue;       // workgroups serving each queue (workgroup w serves w % kXcds)
  const uint32_t* pool;     // indexing vectors: byte offsets from each operand's lowest element
  const void* const* A;
  const void* const* B;
  void* const* C;
  double alpha, beta;
};

// Tile classes of the batched kernel: BM x BN with BM, BN in {64, 128}
// (bit 0 of the class: BM = 128, bit 1: BN = 128).
constexpr int kBatchClasses = 4;
__host__ __device__ constexpr int batch_class_bm(int cls) { return (cls & 1) ? 128 : 64; }
__host__ __device__ constexpr int batch_class_bn(int cls) { return (cls & 2) ? 128 : 64; }

// Slices in flight of the batched item body (its K slice is
// batch_slice_k()).  The items are short in K (tens of slices) and their
// operands mostly miss L2, so the loads' lead time decides: FP32 takes
// 16-deep slices with two in flight (the lead of one 32-deep slice, in finer
// steps).  On the 20,000-problem workload, against 32-deep slices with one
// in flight: 174.6 -> 166.7 ms; 16-deep with one in flight (half the lead)
// 184.8 ms.  FP64 keeps one 16-deep slice in flight.
__host__ __device__ constexpr int batch_depth(int esize) { return esize == 4 ? 2 : 1; }

template <typename T, int BM, int BN, bool XK, bool YK>
__device__ __forceinline__ void run_item(const TileJob<uint32_t>& j, T* smem) {
  constexpr int BK = batch_slice_k();
  constexpr int kDepth = batch_depth(sizeof(T));
  PlainTile<T, BM, BN, BK, XK ? kKGather : kRowGather, YK ? kKGather : kRowGather, kDepth>::template run<uint32_t>(
      j, smem);
}

// One item of class (BM, BN); xy: bit 0 X gathered along K, bit 1 Y along K.
template <typename T, int BM, int BN>
__device__ __forceinline__ void run_class(int xy, const TileJob<uint32_t>& j, T* smem) {
  switch (xy) {
    case 0: run_item<T, BM, BN, false, false>(j, smem); break;
    case 1: run_item<T, BM, BN, true, false>(j, smem); break;
    case 2: run_item<T, BM, BN, false, true>(j, smem); break;
    default: run_item<T, BM, BN, true, true>(j, smem); break;
  }
}

// Wave-uniform copies (readfirstlane) of values every lane holds alike.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <typename P>
__device__ __forceinline__ P* uniform(P* p) {
  return reinterpret_cast<P*>(uniform(reinterpret_cast<int64_t>(p)));
}

template <typename T>
__global__ __launch_bounds__(kThreads, 2) void batch_contract(BatchArgs a) {
  constexpr int BK = batch_slice_k();
  constexpr int SM = PlainTile<T, 128, 128, BK, true, true>::SMEM;
  __shared__ T smem[SM];
  __shared__ int next;
  const int q = (int)blockIdx.x % kXcds;
  const int beg = a.q_start[q], count = a.q_start[q + 1] - beg;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(a.counters + q, 1);
    __syncthreads();
    const int it = uniform(next);
    if (it >= count) break;  // the counter only grows: every workgroup gets here
    // The item and its problem are the same for the whole workgroup: taking
    // every field through readfirstlane keeps the tile's addresses and sizes
    // in scalar registers (vector loads of them would hold ~70 VGPRs per
    // lane through the tile and push the kernel into spills).
    const BatchItem item = a.items[beg + it];
    const int prob = uniform(item.prob);
    const BatchProblemDev& P = a.probs[prob];
    const int flags = uniform(P.flags);
    const bool swapped = flags & 1;
    const int cls = flags >> 8;
    const uint32_t* o = uniform(a.pool + P.off);
    TileJob<uint32_t> j;
    j.x = uniform(static_cast<const T*>(swapped ? a.B[prob] : a.A[prob]) + P.xlo);
    j.y = uniform(static_cast<const T*>(swapped ? a.A[prob] : a.B[prob]) + P.ylo);
    j.c = uniform(static_cast<T*>(a.C[prob]) + P.clo);
    j.xmn = o + uniform(P.pos[0]);
    j.xk = o + uniform(P.pos[1]);
    j.yk = o + uniform(P.pos[2]);
    j.ymn = o + uniform(P.pos[3]);
    j.cm = o + uniform(P.pos[4]);
    j.cn = o + uniform(P.pos[5]);
    j.M = uniform(P.M);
    j.N = uniform(P.N);
    j.m0 = uniform((int)item.tm) * batch_class_bm(cls);
    j.n0 = uniform((int)item.tn) * batch_class_bn(cls);
    j.kbeg = 0;
    j.kend = uniform(P.K);
    j.alpha = a.alpha;
    j.beta = a.beta;
    j.work = nullptr;
    j.ldw = 0;
    j.x_nkb = j.y_nkb = 0;
    const int xy = (flags >> 1) & 3;
    switch (cls) {
      case 0: run_class<T, 64, 64>(xy, j, smem); break;
      case 1: run_class<T, 128, 64>(xy, j, smem); break;
      case 2: run_class<T, 64, 128>(xy, j, smem); break;
      default: run_class<T, 128, 128>(xy, j, smem); break;
    }
    __syncthreads();
  }
  // every workgroup of the queue has drawn past its end: the last one to
  // arrive clears the queue's counters for the next launch
  if (threadIdx.x == 0 && atomicAdd(a.counters + kXcds + q, 1) == a.per_queue - 1) {
    a.counters[q] = 0;
    a.counters[kXcds + q] = 0;
  }
}

struct BatchPlan {
  int dtype = FAMLIES_F32;
  int64_t n = 0;
  int grid = 0;
  void* d_buf = nullptr;  // probs | items | queues | scale list | pool, one allocation
  BatchArgs args{};
  int64_t n_items = 0;
  double flops = 0.0;
  std::vector<int> scale_only;  // problems with K == 0 (alpha*A.B vanishes)
  std::vector<int8_t> cls;      // tile class per problem, -1 when it has no tiles
  const int32_t* scale_dev = nullptr;
  ~BatchPlan() {
    if (d_buf) (void)hipFree(d_buf);
  }
};

void destroy_batch(BatchPlan* b) { delete b; }

void batch_info(const BatchPlan* b, famlies_plan_info* info) {
  std::memset(info, 0, sizeof *info);
  info->batch = b->n;
  info->flops = b->flops;
}

// Problems whose product term vanishes (K == 0, or every problem when
// alpha == 0): C = beta * C (beta == 0 writes zeros without reading C).  One
// workgroup per problem; `list` selects the problems, or all when null.
template <typename T>
__global__ __launch_bounds__(kThreads) void batch_scale(BatchArgs a, const int32_t* list, int n) {
  if ((int)blockIdx.x >= n) return;
  const int p = list ? list[blockIdx.x] : (int)blockIdx.x;
  const BatchProblemDev& P = a.probs[p];
  const uint32_t* o = a.pool + P.off;
  T* C = static_cast<T*>(a.C[p]) + P.clo;
  const int64_t mn = (int64_t)P.M * P.N;
  const T be = static_cast<T>(a.beta);
  for (int64_t i = threadIdx.x; i < mn; i += kThreads) {
    const int m = (int)(i / P.N), nn = (int)(i % P.N);
    auto* cp = global(at(C, (uint32_t)(o[P.pos[4] + m] + o[P.pos[5] + nn])));
    *cp = be != T(0) ? be * *cp : T(0);
  }
}

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

int batch_class_of(int bm, int bn) { return (bm >= 128 ? 1 : 0) | (bn >= 128 ? 2 : 0); }

// Tile class for a problem: the tile table's batched entry for its size class
// if present, else 128 along each of M and N that fills it, 64 otherwise.
static int pick_class(const famlies_handle_s* h, int dtype, const Analysis& an, bool* from_table) {
  TileCfg t;
  *from_table = h->table.lookup_batch(dtype, an.M, an.N, an.K, &t);
  if (*from_table) return batch_class_of(t.bm, t.bn);
  return batch_class_of(an.M >= 128 ? 128 : 64, an.N >= 128 ? 128 : 64);
}

famlies_status batch_plan_make(famlies_handle_s* h, famlies_plan_s** out, int dtype, int64_t n,
                               const famlies_tensor* A, const famlies_tensor* B, const famlies_tensor* C,
                               int force_cls) {
  *out = nullptr;
  if (force_cls >= kBatchClasses) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_batch_plan: bad tile class");
  if (n < 0 || (n > 0 && (!A || !B || !C))) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_batch_plan: bad arrays");
  if (n > (1 << 30)) return fail(FAMLIES_ERR_UNSUPPORTED, "famlies_batch_plan: too many problems");
  auto* bp = new (std::nothrow) BatchPlan();
  if (!bp) return fail(FAMLIES_ERR_ALLOC, "out of host memory");
  bp->dtype = dtype;
  bp->n = n;
  std::vector<BatchProblemDev> probs((size_t)n);
  bp->cls.assign((size_t)n, -1);
  std::vector<uint32_t> pool;
  std::vector<int64_t> tmp;
  struct Job {
    int32_t prob;
    int16_t tm, tn;
    double cost;
  };
  std::vector<std::vector<Job>> per_prob((size_t)n);
  std::vector<double> prob_cost((size_t)n, 0.0);
  int64_t table_hits = 0;
  const int BK = batch_slice_k();
  for (int64_t p = 0; p < n; ++p) {
    Analysis an;
    std::string err;
    int st = analyze(dtype, FAMLIES_NATIVE, &A[p], &B[p], &C[p], &an, &err);
    if (st != FAMLIES_OK) {
      delete bp;
      return fail(st, "problem " + std::to_string(p) + ": " + err);
    }
    if (an.L > 1) {
      delete bp;
      return fail(FAMLIES_ERR_UNSUPPORTED, "problem " + std::to_string(p) + ": batch modes in a batched plan");
    }
    const int64_t lim = (int64_t)1 << 30, es = an.esize;
    if ((an.x_span + 1) * es >= lim || (an.y_span + 1) * es >= lim || (an.c_span + 1) * es >= lim ||
        an.M >= lim || an.N >= lim || an.K >= lim) {
      delete bp;
      return fail(FAMLIES_ERR_UNSUPPORTED, "problem " + std::to_string(p) + ": too large for the batched kernel");
    }
    bool hit = false;
    const int cls = force_cls >= 0 ? force_cls : pick_class(h, dtype, an, &hit);
    table_hits += hit ? 1 : 0;
    const int bm = batch_class_bm(cls), bn = batch_class_bn(cls);
    BatchProblemDev& d = probs[(size_t)p];
    d.M = (int32_t)an.M;
    d.N = (int32_t)an.N;
    d.K = (int32_t)an.K;
    d.flags = (an.swapped ? 1 : 0) | (an.x_kfast ? 2 : 0) | (an.y_kfast ? 4 : 0) | (cls << 8);
    d.off = (int64_t)pool.size();
    d.xlo = an.x_lo;
    d.ylo = an.y_lo;
    d.clo = an.c_lo_mn;
    if (an.M == 0 || an.N == 0) continue;  // nothing to write
    const int64_t mp = cdiv(an.M, bm) * bm, np = cdiv(an.N, bn) * bn;
    const int64_t kp = cdiv(std::max<int64_t>(an.K, 1), BK) * BK + BK;
    const std::vector<Mode>* groups[6] = {&an.I, &an.P, &an.P, &an.J, &an.I, &an.J};
    const int which[6] = {0, 0, 1, 1, 2, 2};
    const int64_t len[6] = {an.M, an.K, an.K, an.N, an.M, an.N};
    const int64_t padded[6] = {mp, kp, kp, np, mp, np};
    const int64_t shift[6] = {an.x_lo, 0, 0, an.y_lo, an.c_lo_mn, 0};
    std::vector<int64_t> vecs[6];
    for (int v = 0; v < 6; ++v) {
      d.pos[v] = (int32_t)(pool.size() - d.off);
      offsets(*groups[v], which[v], len[v], padded[v], vecs[v]);
      for (int64_t x : vecs[v]) pool.push_back((uint32_t)(uint64_t)((x - shift[v]) * es));  // byte offsets, mod 2^32
    }
    // host-side bounds check of the vectors against the descriptors' spans
    const std::vector<int64_t> zero(1, 0);
    const int64_t x_lo = an.swapped ? an.b_lo : an.a_lo, x_hi = an.swapped ? an.b_hi : an.a_hi;
    const int64_t y_lo = an.swapped ? an.a_lo : an.b_lo, y_hi = an.swapped ? an.a_hi : an.b_hi;
    if ((an.K > 0 && (!offsets_in_span(vecs[0], an.M, vecs[1], an.K, zero, 1, x_lo, x_hi) ||
                      !offsets_in_span(vecs[3], an.N, vecs[2], an.K, zero, 1, y_lo, y_hi))) ||
        !offsets_in_span(vecs[4], an.M, vecs[5], an.N, zero, 1, an.c_lo, an.c_hi)) {
      delete bp;
      return fail(FAMLIES_ERR_BOUNDS, "problem " + std::to_string(p) +
                                          ": an indexing vector addresses outside its tensor's span");
    }
    if (an.K == 0) {
      bp->scale_only.push_back((int)p);
      continue;
    }
    bp->flops += 2.0 * (double)an.M * (double)an.N * (double)an.K;
    bp->cls[(size_t)p] = (int8_t)cls;
    const int tm = (int)cdiv(an.M, bm), tn = (int)cdiv(an.N, bn);
    if (tm > 32767 || tn > 32767) {
      delete bp;
      return fail(FAMLIES_ERR_UNSUPPORTED, "problem " + std::to_string(p) + ": more than 32767 tiles along M or N");
    }
    // cost model: MFMA work of the padded tile plus a fixed per-item overhead
    const double c = (double)bm * bn * (double)(cdiv(an.K, BK) * BK) + 64.0 * bm * bn;
    for (int jn = 0; jn < tn; ++jn)
      for (int jm = 0; jm < tm; ++jm) per_prob[(size_t)p].push_back({(int32_t)p, (int16_t)jm, (int16_t)jn, c});
    prob_cost[(size_t)p] = c * tm * tn;
  }
  if (pool.size() >= ((size_t)1 << 31)) {
    delete bp;
    return fail(FAMLIES_ERR_UNSUPPORTED, "famlies_batch_plan: indexing vectors exceed 2^31 entries");
  }
  // Grid: as many workgroups as can be resident at once, a multiple of the
  // XCD count (workgroup w serves queue w % 8).  No workgroup waits for
  // another: one that starts late finds its queue drained and leaves.
  int per_cu = 0;
  {
    DeviceGuard dg0(h->device);
    hipError_t oe = dtype == FAMLIES_F64
                        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_contract<double>, kThreads, 0)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_contract<float>, kThreads, 0);
    if (oe != hipSuccess || per_cu < 1) per_cu = 1;
  }
  const int grid = std::max(kXcds, (per_cu * h->num_cus) / kXcds * kXcds);
  // 1) problems -> XCDs, largest first, to the least-loaded XCD.  A problem
  //    costing more than a quarter of an XCD's fair share is first cut into
  //    runs of consecutive tiles (tiles of one Y panel stay together), each
  //    placed on its own: a batch of a few large problems then still spreads
  //    over every XCD.
  double total_cost = 0.0;
  for (double c : prob_cost) total_cost += c;
  const double unit_cap = total_cost / (4.0 * kXcds);
  struct Unit {
    int64_t prob;
    size_t first, count;
    double cost;
  };
  std::vector<Unit> units;
  for (int64_t p = 0; p < n; ++p) {
    const auto& js = per_prob[(size_t)p];
    if (js.empty()) continue;
    const double c = prob_cost[(size_t)p];
    const size_t parts = c > unit_cap ? std::min(js.size(), (size_t)std::ceil(c / unit_cap)) : 1;
    for (size_t u = 0; u < parts; ++u) {
      const size_t a0 = js.size() * u / parts, a1 = js.size() * (u + 1) / parts;
      units.push_back({p, a0, a1 - a0, c * (double)(a1 - a0) / (double)js.size()});
    }
  }
  std::stable_sort(units.begin(), units.end(), [](const Unit& a, const Unit& b) { return a.cost > b.cost; });
  std::vector<double> xload(kXcds, 0.0);
  std::vector<std::vector<Job>> xjobs(kXcds);
  for (const Unit& u : units) {
    int x = (int)(std::min_element(xload.begin(), xload.end()) - xload.begin());
    xload[(size_t)x] += u.cost;
    const auto& js = per_prob[(size_t)u.prob];
    for (size_t i = u.first; i < u.first + u.count; ++i) xjobs[(size_t)x].push_back(js[i]);
  }
  // 2) each XCD's queue: the costliest items first (item cost: the padded
  //    tile's MFMA work, so largest K first), a problem's tiles consecutive,
  //    so the workgroups that draw them run them side by side and the
  //    problem's operand panels are read once into the XCD's L2
  std::vector<BatchItem> items;
  std::vector<int32_t> q_start(kXcds + 1, 0);
  for (int x = 0; x < kXcds; ++x) {
    q_start[(size_t)x] = (int32_t)items.size();
    auto& js = xjobs[(size_t)x];
    std::stable_sort(js.begin(), js.end(), [](const Job& a, const Job& b) {
      return a.cost != b.cost ? a.cost > b.cost : a.prob < b.prob;
    });
    for (const Job& jb : js) items.push_back({jb.prob, jb.tm, jb.tn});
  }
  q_start[kXcds] = (int32_t)items.size();
  bp->grid = grid;
  bp->n_items = (int64_t)items.size();
  // one device allocation: probs | items | queue starts and counters | scale list | pool
  auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t s_probs = align(probs.size() * sizeof(BatchProblemDev) + 1);
  const size_t s_items = align(items.size() * sizeof(BatchItem) + 1);
  const size_t s_wg = align((q_start.size() + 2 * kXcds) * sizeof(int32_t));  // counters start at zero
  const size_t s_scale = align(bp->scale_only.size() * sizeof(int32_t) + 1);
  const size_t s_pool = align(pool.size() * sizeof(uint32_t) + 1);
  const size_t total = s_probs + s_items + s_wg + s_scale + s_pool;
  DeviceGuard dg(h->device);
  hipError_t e = hipMalloc(&bp->d_buf, total);
  if (e != hipSuccess) {
    delete bp;
    return hip_fail(e, "hipMalloc(batched plan)");
  }
  char* base = static_cast<char*>(bp->d_buf);
  // Staged through pinned host memory: a pageable copy of this size would go
  // through the runtime's staging buffer in many small pieces.
  char* host = nullptr;
  e = hipHostMalloc(reinterpret_cast<void**>(&host), total, hipHostMallocDefault);
  if (e != hipSuccess) {
    delete bp;
    return hip_fail(e, "hipHostMalloc(batched plan staging)");
  }
  std::memset(host, 0, total);
  std::memcpy(host, probs.data(), probs.size() * sizeof(BatchProblemDev));
  std::memcpy(host + s_probs, items.data(), items.size() * sizeof(BatchItem));
  std::memcpy(host + s_probs + s_items, q_start.data(), q_start.size() * sizeof(int32_t));
  std::memcpy(host + s_probs + s_items + s_wg, bp->scale_only.data(), bp->scale_only.size() * sizeof(int32_t));
  std::memcpy(host + s_probs + s_items + s_wg + s_scale, pool.data(), pool.size() * sizeof(uint32_t));
  e = hipMemcpy(bp->d_buf, host, total, hipMemcpyHostToDevice);
  (void)hipHostFree(host);
  if (e != hipSuccess) {
    delete bp;
    return hip_fail(e, "hipMemcpy(batched plan)");
  }
  bp->args.probs = reinterpret_cast<const BatchProblemDev*>(base);
  bp->args.items = reinterpret_cast<const BatchItem*>(base + s_probs);
  bp->args.q_start = reinterpret_cast<const int32_t*>(base + s_probs + s_items);
  bp->args.counters = reinterpret_cast<int32_t*>(base + s_probs + s_items) + q_start.size();
  bp->args.per_queue = grid / kXcds;
  bp->args.pool = reinterpret_cast<const uint32_t*>(base + s_probs + s_items + s_wg + s_scale);
  bp->scale_dev = reinterpret_cast<const int32_t*>(base + s_probs + s_items + s_wg);
  auto* p = new (std::nothrow) famlies_plan_s();
  if (!p) {
    delete bp;
    return fail(FAMLIES_ERR_ALLOC, "out of host memory");
  }
  p->h = h;
  p->an.dtype = dtype;
  p->an.esize = dtype == FAMLIES_F64 ? 8 : 4;
  p->batch = bp;
  if (log_enabled())
    std::fprintf(stderr,
                 "[famlies] batch plan %s: %lld problems, %lld (problem, tile) items, grid %d, %zu K = 0, "
                 "tile class from the table for %lld\n",
                 dtype == FAMLIES_F64 ? "f64" : "f32", (long long)n, (long long)bp->n_items, bp->grid,
                 bp->scale_only.size(), (long long)table_hits);
  *out = p;
  return FAMLIES_OK;
}

famlies_status batch_execute_impl(famlies_plan_s* p, double alpha, double beta, const void* const* A_dev,
                                  const void* const* B_dev, void* const* C_dev, void* stream) {
  if (!p || !p->batch) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_batch_execute: not a batched plan");
  BatchPlan* bp = p->batch;
  if (bp->n == 0) return FAMLIES_OK;
  if (!A_dev || !B_dev || !C_dev) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_batch_execute: null pointer array");
  DeviceGuard dg(p->h->device);
  if (!dg.ok) return fail(FAMLIES_ERR_DEVICE, "cannot select the plan's device");
  BatchArgs a = bp->args;
  a.A = A_dev;
  a.B = B_dev;
  a.C = C_dev;
  a.alpha = alpha;
  a.beta = beta;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool f64 = bp->dtype == FAMLIES_F64;
  if (alpha != 0.0) {
    if (bp->n_items > 0) {
      if (f64)
        hipLaunchKernelGGL(batch_contract<double>, dim3(bp->grid), dim3(kThreads), 0, s, a);
      else
        hipLaunchKernelGGL(batch_contract<float>, dim3(bp->grid), dim3(kThreads), 0, s, a);
    }
    const int ns = (int)bp->scale_only.size();
    if (ns > 0) {
      if (f64)
        hipLaunchKernelGGL(batch_scale<double>, dim3(ns), dim3(kThreads), 0, s, a, bp->scale_dev, ns);
      else
        hipLaunchKernelGGL(batch_scale<float>, dim3(ns), dim3(kThreads), 0, s, a, bp->scale_dev, ns);
    }
  } else {
    const int n = (int)bp->n;
    if (f64)
      hipLaunchKernelGGL(batch_scale<double>, dim3(n), dim3(kThreads), 0, s, a, nullptr, n);
    else
      hipLaunchKernelGGL(batch_scale<float>, dim3(n), dim3(kThreads), 0, s, a, nullptr, n);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "batched kernel launch");
  return FAMLIES_OK;
}

}  // namespace famlies

using namespace famlies;

extern "C" {

static famlies_status batch_plan_impl(famlies_handle htok, famlies_plan* out, int dtype, int64_t n,
                                      const famlies_tensor* A, const famlies_tensor* B, const famlies_tensor* C) {
  if (!out) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_batch_plan: null output pointer");
  *out = nullptr;
  famlies_handle_s* h = handle_of(htok);
  if (!h) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_batch_plan: invalid handle");
  famlies_plan_s* p = nullptr;
  famlies_status st = batch_plan_make(h, &p, dtype, n, A, B, C, -1);
  if (st != FAMLIES_OK) return st;
  void* tok = registry_add(p, ObjKind::kPlan);
  if (!tok) {
    destroy_plan(p);
    return fail(FAMLIES_ERR_ALLOC, "famlies_batch_plan: no free object slot");
  }
  *out = static_cast<famlies_plan>(tok);
  return FAMLIES_OK;
}

famlies_status famlies_batch_plan(famlies_handle htok, famlies_plan* out, int dtype, int64_t n,
                                  const famlies_tensor* A, const famlies_tensor* B, const famlies_tensor* C) {
  return no_throw("famlies_batch_plan", [&] { return batch_plan_impl(htok, out, dtype, n, A, B, C); });
}

famlies_status famlies_batch_plan_tiles(famlies_plan tok, int32_t* tile_m, int32_t* tile_n, int64_t n) {
  famlies_plan_s* p = plan_of(tok);
  if (!p || !p->batch) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_batch_plan_tiles: not a batched plan");
  if (!tile_m || !tile_n || n != p->batch->n)
    return fail(FAMLIES_ERR_INVALID_ARG, "famlies_batch_plan_tiles: bad arrays or count");
  for (int64_t i = 0; i < n; ++i) {
    const int c = p->batch->cls[(size_t)i];
    tile_m[i] = c < 0 ? 0 : batch_class_bm(c);
    tile_n[i] = c < 0 ? 0 : batch_class_bn(c);
  }
  return FAMLIES_OK;
}

famlies_status famlies_batch_execute(famlies_plan tok, double alpha, double beta, const void* const* A_dev,
                                     const void* const* B_dev, void* const* C_dev, void* stream) {
  famlies_plan_s* p = plan_of(tok);
  if (!p || !p->batch) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_batch_execute: not a batched plan");
  return batch_execute_impl(p, alpha, beta, A_dev, B_dev, C_dev, stream);
}

}  // extern "C"
