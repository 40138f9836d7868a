// C ABI: handles, plans, planning (tile choice, indexing-vector upload) and
// execution.  Errors are returned as famlies_status with a thread-local
// message (graceful error handling and bounds checking: Girder 1, "Code
// safety").
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "famlies.h"
#include "internal.hpp"
#include "launch.hpp"
#include "runtime.hpp"

namespace famlies {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

static std::mutex g_live_mu;
static std::set<const void*> g_live;  // live handles and plans (use-after-destroy check)

void register_live(const void* p) {
  std::lock_guard<std::mutex> lk(g_live_mu);
  g_live.insert(p);
}
void unregister_live(const void* p) {
  std::lock_guard<std::mutex> lk(g_live_mu);
  g_live.erase(p);
}
bool is_live(const void* p) {
  std::lock_guard<std::mutex> lk(g_live_mu);
  return g_live.count(p) != 0;
}

famlies_status fail(famlies_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

famlies_status hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? FAMLIES_ERR_ALLOC : FAMLIES_ERR_DEVICE;
}

// Make `device` current for the scope, restoring the caller's device after.
DeviceGuard::DeviceGuard(int device) {
  ok = hipGetDevice(&prev) == hipSuccess;
  if (ok && prev != device) ok = hipSetDevice(device) == hipSuccess;
  else if (ok) prev = -1;
}
DeviceGuard::~DeviceGuard() {
  if (prev >= 0) (void)hipSetDevice(prev);
}

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Step a4: tile shape and split-K.  A tile-table entry for the problem's
// size class wins.  Otherwise a small cost model picks the tile edge (128 or
// 64) and the number of K slices: the workgroups are dealt to the CUs two at
// a time (two share a CU at half rate each; a lone one runs at about 0.65 of
// the CU), so the busiest CU's time is
//     pairs * 2w + (odd ? w / 0.65 : 0),  w = work of one workgroup,
// a 64-edge tile does its flops at about 0.75 of the 128-edge rate, and each
// extra K slice costs a pass over the split tiles' partial sums (at HBM
// rate, measured in the same units).  Splitting is either whole (every tile
// in K slices) or of the tail only: when the tiles fill some rounds of two
// workgroups per CU and part of one more, the whole rounds run unsplit and
// only the tiles of the last round are cut into K slices, so that round
// spreads over every CU instead of leaving most of them idle.  The model
// only ranks candidates; it is not a timing.
TileCfg choose_tiles(const famlies_handle_s* h, const Analysis& an) {
  TileCfg t;
  const int bk = an.dtype == FAMLIES_F64 ? 16 : 32;
  t.bk = bk;
  if (an.M == 0 || an.N == 0 || an.K == 0) return t;
  if (h && h->table.lookup_plain(an, &t)) return t;
  const int cus = h ? h->num_cus : 256;
  // CU throughput in flop/s and HBM bandwidth in bytes/s (MI355X-class)
  const double cu_rate = (an.dtype == FAMLIES_F64 ? 78.6e12 : 157.3e12) / 256.0;
  const double hbm = 8.0e12 * cus / 256.0;
  const double es = an.esize;
  double best = 1e300;
  TileCfg pick = t;
  for (int bt : {128, 64}) {
    const int64_t tiles = ceil_div(an.M, bt) * ceil_div(an.N, bt) * an.L;
    const double eff = bt == 128 ? 1.0 : 0.75;
    for (int split : {1, 2, 3, 4, 6, 8, 12, 16}) {
      if (split > 1 && (an.L > 1 || an.K / split < 2 * bk)) continue;
      const int64_t units = tiles * split;
      const int64_t q = ceil_div(units, cus);  // workgroups on the busiest CU
      const double w = 2.0 * bt * bt * ((double)an.K / split) / (cu_rate * eff);
      double time = (double)(q / 2) * 2.0 * w + (q % 2 ? w / 0.65 : 0.0);
      if (split > 1) time += (double)split * an.M * an.N * es * 2.0 / hbm + 4e-6;
      if (time < best * 0.9) {  // prefer fewer slices / larger tiles unless clearly faster
        best = time;
        pick.bm = pick.bn = bt;
        pick.split = split;
        pick.tail = 0;
      }
    }
    // tail split: whole rounds unsplit, the last partial round in K slices
    const int64_t slots = 2 * (int64_t)cus, rem = tiles % slots;
    if (an.L == 1 && tiles > slots && rem > 0) {
      const double w = 2.0 * bt * bt * (double)an.K / (cu_rate * eff);
      const double head = (double)(tiles / slots) * 2.0 * w;
      for (int split : {2, 3, 4, 6, 8}) {
        if (an.K / split < 2 * bk) continue;
        const int64_t q = ceil_div(rem * split, cus);
        const double ws = w / split;
        const double time = head + (double)(q / 2) * 2.0 * ws + (q % 2 ? ws / 0.65 : 0.0) +
                            (double)split * rem * bt * bt * es * 2.0 / hbm + 4e-6;
        if (time < best * 0.95) {  // only the tail pays for partial sums
          best = time;
          pick.bm = pick.bn = bt;
          pick.split = split;
          pick.tail = (int)rem;
        }
      }
    }
  }
  return pick;
}

// Settle split-K: K slices of whole BK-blocks, and the number of tiles
// computed whole first (*head; every tile when there is no split).
static void finalize_split(TileCfg* t, int64_t K, int64_t ntiles, int* kchunk, int* head) {
  *head = (int)std::min<int64_t>(ntiles, INT32_MAX);
  if (t->split <= 1 || K <= t->bk) {
    t->split = 1;
    t->tail = 0;
    *kchunk = (int)std::max<int64_t>(K, 1);
    return;
  }
  int64_t chunk = ceil_div(ceil_div(K, t->split), t->bk) * t->bk;
  t->split = (int)ceil_div(K, chunk);
  *kchunk = (int)chunk;
  if (t->split <= 1) {
    t->split = 1;
    t->tail = 0;
    *kchunk = (int)K;
    return;
  }
  if (t->tail <= 0 || t->tail >= ntiles) t->tail = 0;  // every tile split
  *head = t->tail ? (int)(ntiles - t->tail) : 0;
}

static void fill_info(const Analysis& an, const TileCfg& t, int index_bits, int kernel,
                      famlies_plan_info* info) {
  std::memset(info, 0, sizeof *info);
  info->m = an.M;
  info->n = an.N;
  info->k = an.K;
  info->batch = an.L;
  info->n_batch = (int32_t)an.Lm.size();
  info->n_trace = an.n_trace;
  info->n_diag = an.n_diag;
  info->swapped = an.swapped;
  info->x_kfast = an.x_kfast;
  info->y_kfast = an.y_kfast;
  info->n_i = (int32_t)an.I.size();
  info->n_j = (int32_t)an.J.size();
  info->n_p = (int32_t)an.P.size();
  info->tile_m = t.bm;
  info->tile_n = t.bn;
  info->tile_k = t.bk;
  info->split_k = t.split;
  info->split_tiles = t.split > 1 ? (t.tail ? t.tail : (int32_t)(ceil_div(an.M, t.bm) * ceil_div(an.N, t.bn))) : 0;
  info->index_bits = index_bits;
  info->kernel = kernel;
  info->flops = 2.0 * (double)an.L * (double)an.M * (double)an.N * (double)an.K;
}

// 32: uint32 byte offsets from each operand's lowest element (every operand
// spans less than 4 GiB over its non-batch modes); 64: int64 element offsets.
static int index_bits_for(const Analysis& an) {
  const int64_t lim = ((int64_t)1 << 32) - 64;
  const int64_t es = an.esize;
  return ((an.x_span + 1) * es < lim && (an.y_span + 1) * es < lim && (an.c_span + 1) * es < lim) ? 32 : 64;
}

// Upload the indexing vectors (padded to the tile grid) into one device
// buffer: six OffT vectors (X rows, X k, Y k, Y cols, C rows, C cols), then
// the three int64 batch-offset vectors.  In the uint32 form every row vector
// is rebased by its operand's lowest offset and all six are scaled to bytes;
// sums row + col then land in [0, span) (unsigned wrap-around is exact).
// Block strides of the block-scatter layout (Approach, "Supporting tensor
// computations"): an operand gathered along K can be read with 16-byte loads
// when BK divides K (every slice whole), in every BK-block of K its indexing
// vector steps by exactly one element, and every run start (row offset +
// block start + batch offset, in elements from the base pointer) is a
// multiple of the 16-byte vector.
static bool affine_k_blocks(const std::vector<int64_t>& rows, int64_t nrows, const std::vector<int64_t>& ks,
                            int64_t K, int bk, const std::vector<int64_t>& batch, int64_t L, int64_t vk) {
  if (K < 1 || K % bk) return false;
  for (int64_t b = 0; b < K; b += bk) {
    const int64_t s0 = ks[(size_t)b];
    if (s0 % vk) return false;
    for (int64_t k = b + 1; k < std::min<int64_t>(K, b + bk); ++k)
      if (ks[(size_t)k] != s0 + (k - b)) return false;
  }
  for (int64_t m = 0; m < nrows; ++m)
    if (rows[(size_t)m] % vk) return false;
  for (int64_t l = 0; l < L; ++l)
    if (batch[(size_t)l] % vk) return false;
  return true;
}

// Affine-block flags of X and Y for a plan with K-slice depth bk; v holds
// the nine indexing vectors in upload() order.
static void vec_flags(const Analysis& an, int bk, int /*index_bits*/, const std::vector<int64_t>* v, bool* xv,
                      bool* yv) {
  *xv = *yv = false;
  const int64_t vk = 16 / an.esize;
  *xv = an.x_kfast && affine_k_blocks(v[0], an.M, v[1], an.K, bk, v[6], an.L, vk);
  *yv = an.y_kfast && affine_k_blocks(v[3], an.N, v[2], an.K, bk, v[7], an.L, vk);
}

static void all_offsets(const Analysis& an, std::vector<int64_t>* v) {
  const std::vector<Mode>* groups[9] = {&an.I, &an.P, &an.P, &an.J, &an.I, &an.J, &an.Lm, &an.Lm, &an.Lm};
  const int which[9] = {0, 0, 1, 1, 2, 2, 0, 1, 2};
  const int64_t len[9] = {an.M, an.K, an.K, an.N, an.M, an.N, an.L, an.L, an.L};
  for (int i = 0; i < 9; ++i) offsets(*groups[i], which[i], len[i], len[i], v[i]);
}

template <typename OffT>
static famlies_status upload(famlies_plan_s* p, int64_t mp, int64_t np, int64_t kp) {
  const Analysis& an = p->an;
  std::vector<int64_t> v[9];
  offsets(an.I, 0, an.M, mp, v[0]);
  offsets(an.P, 0, an.K, kp, v[1]);
  offsets(an.P, 1, an.K, kp, v[2]);
  offsets(an.J, 1, an.N, np, v[3]);
  offsets(an.I, 2, an.M, mp, v[4]);
  offsets(an.J, 2, an.N, np, v[5]);
  offsets(an.Lm, 0, an.L, an.L, v[6]);
  offsets(an.Lm, 1, an.L, an.L, v[7]);
  offsets(an.Lm, 2, an.L, an.L, v[8]);
  const bool bytes = sizeof(OffT) == 4;
  const int64_t es = an.esize;
  vec_flags(an, p->cfg.bk, bytes ? 32 : 64, v, &p->x_vec, &p->y_vec);
  const int64_t shift[6] = {an.x_lo, 0, 0, an.y_lo, an.c_lo_mn, 0};
  size_t n6 = 0;
  for (int i = 0; i < 6; ++i) n6 += v[i].size();
  const size_t b6 = (n6 * sizeof(OffT) + 7) & ~(size_t)7;
  const size_t total = b6 + 3 * (size_t)an.L * sizeof(int64_t);
  std::vector<char> host(total, 0);
  OffT* o = reinterpret_cast<OffT*>(host.data());
  size_t pos = 0;
  for (int i = 0; i < 6; ++i) {
    p->off_pos[i] = pos;
    for (int64_t x : v[i]) {
      if (bytes)
        o[pos++] = (OffT)(uint64_t)((x - shift[i]) * es);  // wraps modulo 2^32 on purpose
      else
        o[pos++] = (OffT)x;
    }
  }
  int64_t* lb = reinterpret_cast<int64_t*>(host.data() + b6);
  for (int i = 0; i < 3; ++i) {
    p->off_pos[6 + i] = (size_t)i * (size_t)an.L;
    for (int64_t l = 0; l < an.L; ++l) lb[i * an.L + l] = v[6 + i][(size_t)l];
  }
  p->batch_off_bytes = b6;
  hipError_t e = hipMalloc(&p->d_off, total);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(indexing vectors)");
  e = hipMemcpy(p->d_off, host.data(), total, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(indexing vectors)");
  return FAMLIES_OK;
}

template <typename OffT>
static PlainArgs<OffT> make_args(const famlies_plan_s* p, const void* x, const void* y, void* c,
                                 double alpha, double beta) {
  PlainArgs<OffT> a;
  const OffT* o = static_cast<const OffT*>(p->d_off);
  const int64_t* lb = reinterpret_cast<const int64_t*>(static_cast<const char*>(p->d_off) + p->batch_off_bytes);
  const bool bytes = sizeof(OffT) == 4;
  const int64_t es = p->an.esize;
  // in the byte form the kernel addresses each operand from its lowest element
  a.x = x ? static_cast<const char*>(x) + (bytes ? p->an.x_lo * es : 0) : nullptr;
  a.y = y ? static_cast<const char*>(y) + (bytes ? p->an.y_lo * es : 0) : nullptr;
  a.c = static_cast<char*>(c) + (bytes ? p->an.c_lo_mn * es : 0);
  a.xmn = o + p->off_pos[0];
  a.xk = o + p->off_pos[1];
  a.yk = o + p->off_pos[2];
  a.ymn = o + p->off_pos[3];
  a.cm = o + p->off_pos[4];
  a.cn = o + p->off_pos[5];
  a.xl = lb + p->off_pos[6];
  a.yl = lb + p->off_pos[7];
  a.cl = lb + p->off_pos[8];
  a.M = (int32_t)p->an.M;
  a.N = (int32_t)p->an.N;
  a.K = (int32_t)p->an.K;
  a.L = (int32_t)p->an.L;
  a.x_nkb = 0;
  a.y_nkb = 0;
  a.tiles_m = (int32_t)ceil_div(p->an.M, p->cfg.bm);
  a.tiles_n = (int32_t)ceil_div(p->an.N, p->cfg.bn);
  a.splits = p->cfg.split;
  a.kchunk = p->kchunk;
  a.head = p->head;
  a.alpha = alpha;
  a.beta = beta;
  a.work = p->d_work;
  return a;
}

famlies_status make_plan(famlies_handle h, famlies_plan* out, int dtype, int compute,
                         const famlies_tensor* A, const famlies_tensor* B, const famlies_tensor* C,
                         const TileCfg* force) {
  if (!out) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_plan_contract: null output pointer");
  *out = nullptr;
  if (!h || !is_live(h)) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_plan_contract: invalid handle");
  Analysis an;
  std::string err;
  int st = analyze(dtype, compute, A, B, C, &an, &err);
  if (st != FAMLIES_OK) return fail(st, err);
  const int64_t lim = ((int64_t)1 << 31) - 1024;
  if (an.M > lim || an.N > lim || an.K > lim || an.L > lim)
    return fail(FAMLIES_ERR_UNSUPPORTED, "a GEMM dimension exceeds 2^31 - 1024");
  DeviceGuard dg(h->device);
  if (!dg.ok) return fail(FAMLIES_ERR_DEVICE, "cannot select the handle's device");
  auto* p = new (std::nothrow) famlies_plan_s();
  if (!p) return fail(FAMLIES_ERR_ALLOC, "out of host memory");
  p->h = h;
  p->an = an;
  p->cfg = force ? *force : choose_tiles(h, an);
  p->index_bits = p->cfg.index_bits == 64 ? 64 : index_bits_for(an);
  const int ns = split_parts(compute);
  if (ns) {
    // the bf16 kernels split every tile or none: a tail split becomes none
    if (p->cfg.tail) {
      p->cfg.split = 1;
      p->cfg.tail = 0;
    }
    p->cfg.bk = 32;
    // bf16x3 on large problems: a 256 x 128 tile (128 x 64 per wave) halves
    // the LDS bytes per MFMA of the 128 x 128 tile (bf16x6 has three
    // accumulators per block and stays at 128 x 128).  It has registers for
    // one slice in flight and one workgroup per CU, so it is taken only when
    // both operands are element-gathered along K: a row-gathered operand
    // keeps the 128 x 128 tile with two slices in flight (ring o=48 v=192:
    // 186 -> 201 TFLOP/s FP32-equivalent), and an affine-block operand the
    // 128 x 128 tile at two workgroups per CU (ladder v=128 o=32: 284 -> 307).
    if (!force && ns == 2 && an.M >= 1024 && an.N >= 512 && p->cfg.split == 1 && an.x_kfast && an.y_kfast) {
      std::vector<int64_t> v[9];
      bool xv = false, yv = false;
      all_offsets(an, v);
      vec_flags(an, 32, index_bits_for(an), v, &xv, &yv);
      if (!xv && !yv) {
        p->cfg.bm = 256;
        p->cfg.bn = 128;
      }
    }
    if (!split_tile_supported(ns, p->cfg.bm, p->cfg.bn)) p->cfg.bm = p->cfg.bn = 128;
  } else if (!plain_tile_supported(dtype, p->cfg.bm, p->cfg.bn, p->cfg.bk)) {
    p->cfg.bm = p->cfg.bn = 128;
    p->cfg.bk = dtype == FAMLIES_F64 ? 16 : 32;
  }
  if (an.L > 1) p->cfg.split = 1;  // batch modes already multiply the tile count
  const int64_t ntiles = ceil_div(an.M, p->cfg.bm) * ceil_div(an.N, p->cfg.bn);
  finalize_split(&p->cfg, an.K, ntiles, &p->kchunk, &p->head);
  if (ntiles * p->cfg.split * an.L >= ((int64_t)1 << 31)) {
    delete p;
    return fail(FAMLIES_ERR_UNSUPPORTED, "the tile grid exceeds 2^31 workgroups");
  }
  const bool empty = an.M == 0 || an.N == 0;
  if (!empty) {
    const int64_t mp = ceil_div(std::max<int64_t>(an.M, 1), p->cfg.bm) * p->cfg.bm;
    const int64_t np = ceil_div(std::max<int64_t>(an.N, 1), p->cfg.bn) * p->cfg.bn;
    const int64_t kp = ceil_div(std::max<int64_t>(an.K, 1), p->cfg.bk) * p->cfg.bk + p->cfg.bk;
    st = p->index_bits == 32 ? upload<uint32_t>(p, mp, np, kp) : upload<int64_t>(p, mp, np, kp);
    if (st != FAMLIES_OK) {
      delete p;
      return st;
    }
    if (p->cfg.split > 1 && an.K > 0) {
      // plain kernels: one BM x BN block per split tile and K slice; bf16
      // kernels: one padded M x N plane of FP64 sums per K slice
      p->work_bytes = ns ? (size_t)p->cfg.split * (size_t)mp * (size_t)np * 8
                         : (size_t)p->cfg.split * (size_t)(ntiles - p->head) * (size_t)p->cfg.bm *
                               (size_t)p->cfg.bn * (size_t)an.esize;
      hipError_t e = hipMalloc(&p->d_work, p->work_bytes);
      if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipMalloc(split-K workspace)");
      }
    }
  }
  register_live(p);
  *out = p;
  return FAMLIES_OK;
}


}  // namespace famlies

famlies_plan_s::~famlies_plan_s() {
  if (d_off) (void)hipFree(d_off);
  if (d_work) (void)hipFree(d_work);
  if (batch) famlies::destroy_batch(batch);
}

using namespace famlies;

extern "C" {

const char* famlies_last_error(void) { return g_err.c_str(); }

const char* famlies_version(void) { return "famlies-mi355x 0.1 (gfx950)"; }

famlies_status famlies_create(famlies_handle* out, int device) {
  if (!out) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_create: null output pointer");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= n) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_create: no such device");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(FAMLIES_ERR_UNSUPPORTED, std::string("famlies_create: device is ") + prop.gcnArchName +
                                             ", this library is built for gfx950 only");
  auto* h = new (std::nothrow) famlies_handle_s();
  if (!h) return fail(FAMLIES_ERR_ALLOC, "famlies_create: out of host memory");
  h->device = device;
  h->num_cus = prop.multiProcessorCount;
  const char* tt = std::getenv("FAMLIES_TUNE_TABLE");
  if (tt && *tt) {
    std::string err;
    if (!h->table.load(tt, &err)) {
      delete h;
      return fail(FAMLIES_ERR_INVALID_ARG, "FAMLIES_TUNE_TABLE: " + err);
    }
  }
  register_live(h);
  *out = h;
  return FAMLIES_OK;
}

famlies_status famlies_destroy(famlies_handle h) {
  if (!h || !is_live(h)) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_destroy: invalid handle");
  unregister_live(h);
  delete h;
  return FAMLIES_OK;
}

famlies_status famlies_analyze(int dtype, int compute, const famlies_tensor* A, const famlies_tensor* B,
                               const famlies_tensor* C, famlies_plan_info* info, int64_t* offs,
                               int64_t offs_len) {
  if (!info) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_analyze: null info");
  Analysis an;
  std::string err;
  int st = analyze(dtype, compute, A, B, C, &an, &err);
  if (st != FAMLIES_OK) return fail(st, err);
  TileCfg t = choose_tiles(nullptr, an);
  if (split_parts(an.compute) && t.tail) {  // as in make_plan: no split for the bf16 kernels
    t.split = 1;
    t.tail = 0;
  }
  int kchunk = 0, head = 0;
  finalize_split(&t, an.K, ceil_div(an.M, t.bm) * ceil_div(an.N, t.bn), &kchunk, &head);
  const int ib = index_bits_for(an);
  std::vector<int64_t> v[9];
  bool xv = false, yv = false;
  if (an.M > 0 && an.N > 0) {
    all_offsets(an, v);
    vec_flags(an, t.bk, ib, v, &xv, &yv);
  }
  fill_info(an, t, ib, 1 + split_parts(an.compute) + (xv ? 16 : 0) + (yv ? 32 : 0), info);
  if (offs) {
    const int64_t need = 2 * an.M + 2 * an.K + 2 * an.N + 3 * an.L;
    if (offs_len < need) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_analyze: offsets buffer too short");
    if (an.M == 0 || an.N == 0) all_offsets(an, v);
    int64_t pos = 0;
    for (int i = 0; i < 9; ++i) {
      std::copy(v[i].begin(), v[i].end(), offs + pos);
      pos += (int64_t)v[i].size();
    }
  }
  return FAMLIES_OK;
}

famlies_status famlies_plan_contract(famlies_handle h, famlies_plan* out, int dtype, int compute,
                                     const famlies_tensor* A, const famlies_tensor* B,
                                     const famlies_tensor* C) {
  return make_plan(h, out, dtype, compute, A, B, C, nullptr);
}

famlies_status famlies_plan_destroy(famlies_plan p) {
  if (!p || !is_live(p)) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_plan_destroy: invalid plan");
  unregister_live(p);
  DeviceGuard dg(p->h->device);
  delete p;
  return FAMLIES_OK;
}

famlies_status famlies_plan_get_info(famlies_plan p, famlies_plan_info* info) {
  if (!p || !is_live(p) || !info) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_plan_get_info: invalid argument");
  fill_info(p->an, p->cfg, p->index_bits,
            1 + split_parts(p->an.compute) + (p->x_vec ? 16 : 0) + (p->y_vec ? 32 : 0), info);
  return FAMLIES_OK;
}

static bool overlaps(const void* p, int64_t plo, int64_t phi, const void* q, int64_t qlo, int64_t qhi,
                     int es) {
  if (plo > phi || qlo > qhi) return false;
  const intptr_t a0 = (intptr_t)p + plo * es, a1 = (intptr_t)p + (phi + 1) * es;
  const intptr_t b0 = (intptr_t)q + qlo * es, b1 = (intptr_t)q + (qhi + 1) * es;
  return a0 < b1 && b0 < a1;
}

static famlies_status execute_impl(famlies_plan p, double alpha, const void* A, const void* B, double beta,
                                   void* C, int packed, void* stream) {
  if (!p || !is_live(p) || p->batch) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_execute: invalid plan");
  const Analysis& an = p->an;
  if (an.M == 0 || an.N == 0) return FAMLIES_OK;
  const bool need_ab = alpha != 0.0 && an.K > 0;
  if (!C || (need_ab && (!A || !B))) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_execute: null data pointer");
  const uintptr_t al = (uintptr_t)an.esize - 1;
  if (((uintptr_t)C & al) || (need_ab && (((uintptr_t)A & al) || ((uintptr_t)B & al))))
    return fail(FAMLIES_ERR_ALIGN, "famlies_execute: data pointer not aligned to its element size");
  const bool pa = packed & 1, pb = packed & 2;
  size_t sza = 0, szb = 0;
  if (need_ab && pa) {
    famlies_status st = famlies_pack_size(p, 0, &sza);
    if (st != FAMLIES_OK) return st;
    if ((uintptr_t)A & 15) return fail(FAMLIES_ERR_ALIGN, "famlies_execute_packed: packed A not 16-byte aligned");
  }
  if (need_ab && pb) {
    famlies_status st = famlies_pack_size(p, 1, &szb);
    if (st != FAMLIES_OK) return st;
    if ((uintptr_t)B & 15) return fail(FAMLIES_ERR_ALIGN, "famlies_execute_packed: packed B not 16-byte aligned");
  }
  const int64_t es = an.esize;
  auto packed_overlap = [&](const void* q, size_t bytes) {
    return overlaps(C, an.c_lo, an.c_hi, q, 0, (int64_t)(bytes / (size_t)es) - 1, an.esize);
  };
  if (need_ab && ((pa ? packed_overlap(A, sza) : overlaps(C, an.c_lo, an.c_hi, A, an.a_lo, an.a_hi, an.esize)) ||
                  (pb ? packed_overlap(B, szb) : overlaps(C, an.c_lo, an.c_hi, B, an.b_lo, an.b_hi, an.esize))))
    return fail(FAMLIES_ERR_ALIAS, "famlies_execute: C overlaps A or B");
  DeviceGuard dg(p->h->device);
  if (!dg.ok) return fail(FAMLIES_ERR_DEVICE, "cannot select the plan's device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const void* x = an.swapped ? B : A;
  const void* y = an.swapped ? A : B;
  const bool xp = an.swapped ? pb : pa, yp = an.swapped ? pa : pb;
  PlainLaunch L;
  L.bm = p->cfg.bm;
  L.bn = p->cfg.bn;
  L.bk = p->cfg.bk;
  // affine-block 16-byte loads need a 16-byte aligned base pointer
  L.xm = xp ? 2 : (an.x_kfast ? (p->x_vec && !((uintptr_t)x & 15) ? 3 : 1) : 0);
  L.ym = yp ? 2 : (an.y_kfast ? (p->y_vec && !((uintptr_t)y & 15) ? 3 : 1) : 0);
  L.kind = (an.K == 0 || alpha == 0.0) ? PlainLaunch::kScale : PlainLaunch::kMain;
  hipError_t e;
  const int ns = split_parts(an.compute);
  if (ns && L.kind == PlainLaunch::kMain) {
    if (p->index_bits == 32) {
      PlainArgs<uint32_t> a = make_args<uint32_t>(p, x, y, C, alpha, beta);
      if (xp) {  // the packed buffer is addressed from its start, not through offsets
        a.x = x;
        a.x_nkb = (int32_t)((an.K + L.bk - 1) / L.bk);
      }
      if (yp) {
        a.y = y;
        a.y_nkb = (int32_t)((an.K + L.bk - 1) / L.bk);
      }
      e = launch_split(a, L, ns, s);
    } else {
      e = launch_split(make_args<int64_t>(p, x, y, C, alpha, beta), L, ns, s);
    }
  } else if (p->index_bits == 32) {
    PlainArgs<uint32_t> a = make_args<uint32_t>(p, x, y, C, alpha, beta);
    if (xp) {
      a.x = x;
      a.x_nkb = (int32_t)((an.K + L.bk - 1) / L.bk);
    }
    if (yp) {
      a.y = y;
      a.y_nkb = (int32_t)((an.K + L.bk - 1) / L.bk);
    }
    e = launch_plain(an.dtype, a, L, s);
  } else {
    e = launch_plain(an.dtype, make_args<int64_t>(p, x, y, C, alpha, beta), L, s);
  }
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return FAMLIES_OK;
}

famlies_status famlies_execute(famlies_plan p, double alpha, const void* A, const void* B, double beta,
                               void* C, void* stream) {
  return execute_impl(p, alpha, A, B, beta, C, 0, stream);
}

famlies_status famlies_execute_packed(famlies_plan p, double alpha, const void* A, const void* B, double beta,
                                      void* C, int packed, void* stream) {
  if (packed < 0 || packed > 3) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_execute_packed: packed must be 0..3");
  return execute_impl(p, alpha, A, B, beta, C, packed, stream);
}

}  // extern "C"
