// Host-side planning that touches no device: error state, tile choice,
// split-K settlement, the plan summary and the planner dry run
// (famlies_analyze).  Kept apart from the HIP sources so that it can be
// built and run on its own under the host sanitizers.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "famlies.h"
#include "internal.hpp"
#include "runtime.hpp"

namespace famlies {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

famlies_status fail(famlies_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

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
TileCfg choose_tiles(const famlies_handle_s* h, const Analysis& an, bool* from_table) {
  TileCfg t;
  const int bk = an.dtype == FAMLIES_F64 ? 8 : 32;
  t.bk = bk;
  if (from_table) *from_table = false;
  if (an.M == 0 || an.N == 0 || an.K == 0) return t;
  if (h && h->table.lookup_plain(an, &t)) {
    if (from_table) *from_table = true;
    return t;
  }
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
void finalize_split(TileCfg* t, int64_t K, int64_t ntiles, int* kchunk, int* head) {
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

void fill_info(const Analysis& an, const TileCfg& t, int index_bits, int kernel,
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
int index_bits_for(const Analysis& an) {
  const int64_t lim = ((int64_t)1 << 32) - 64;
  const int64_t es = an.esize;
  return ((an.x_span + 1) * es < lim && (an.y_span + 1) * es < lim && (an.c_span + 1) * es < lim) ? 32 : 64;
}

void index_form(const Analysis& an, int force, int* bits, bool* elem32) {
  // int32 element offsets: rebased row offsets lie in [0, span] and K
  // offsets in [-span, span], every sum in [0, span]: all below 2^31
  const int64_t lim = ((int64_t)1 << 31) - 64;
  const bool e32 = !int8_slices(an.compute) && an.x_span + 1 < lim && an.y_span + 1 < lim && an.c_span + 1 < lim;
  *elem32 = false;
  if (force == 64) {
    *bits = 64;
  } else if (force == kForceElem32 && e32) {
    *bits = 32;
    *elem32 = true;
  } else if (index_bits_for(an) == 32) {
    *bits = 32;
  } else if (e32) {
    *bits = 32;
    *elem32 = true;
  } else {
    *bits = 64;
  }
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
bool affine_k_blocks(const std::vector<int64_t>& rows, int64_t nrows, const std::vector<int64_t>& ks,
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
void vec_flags(const Analysis& an, int bk, int /*index_bits*/, const std::vector<int64_t>* v, bool* xv,
                      bool* yv) {
  *xv = *yv = false;
  const int64_t vk = 16 / an.esize;
  *xv = an.x_kfast && affine_k_blocks(v[0], an.M, v[1], an.K, bk, v[6], an.L, vk);
  *yv = an.y_kfast && affine_k_blocks(v[3], an.N, v[2], an.K, bk, v[7], an.L, vk);
}

void all_offsets(const Analysis& an, std::vector<int64_t>* v) {
  const std::vector<Mode>* groups[9] = {&an.I, &an.P, &an.P, &an.J, &an.I, &an.J, &an.Lm, &an.Lm, &an.Lm};
  const int which[9] = {0, 0, 1, 1, 2, 2, 0, 1, 2};
  const int64_t len[9] = {an.M, an.K, an.K, an.N, an.M, an.N, an.L, an.L, an.L};
  for (int i = 0; i < 9; ++i) offsets(*groups[i], which[i], len[i], len[i], v[i]);
}

int kernel_code(const Analysis& an, bool xv, bool yv) {
  if (int8_slices(an.compute)) return 8 + int8_slices(an.compute);
  return 1 + split_parts(an.compute) + (xv ? 16 : 0) + (yv ? 32 : 0);
}

TileCfg int8_tile() {
  TileCfg t;
  t.bm = 128;
  t.bn = 64;
  t.bk = 64;
  t.split = 1;
  t.tail = 0;
  return t;
}

bool log_enabled() {
  static const bool on = [] {
    const char* v = std::getenv("FAMLIES_LOG");
    return v && *v && std::strcmp(v, "0") != 0;
  }();
  return on;
}

// One line on stderr: what the planner decided (orientation, loaders, tile,
// split, index form -- index_bits 32: uint32 bytes, -32: int32 elements, 64:
// int64 elements -- and workspace).
void log_decision(const char* what, const Analysis& an, const TileCfg& cfg, int index_bits, bool x_vec,
                  bool y_vec, size_t work_bytes, bool table_hit) {
  static const char* loader[4] = {"rows", "k-gather", "packed", "k-affine"};
  const int xm = an.x_kfast ? (x_vec ? 3 : 1) : 0, ym = an.y_kfast ? (y_vec ? 3 : 1) : 0;
  static const char* int8_names[8] = {"", "", "", "int8x3", "int8x4", "int8x5", "int8x6", "int8x7"};
  const char* comp = an.compute == FAMLIES_BF16X3   ? "bf16x3"
                     : an.compute == FAMLIES_BF16X6 ? "bf16x6"
                     : int8_slices(an.compute)      ? int8_names[int8_slices(an.compute)]
                                                    : "native";
  std::fprintf(stderr,
               "[famlies] %s %s/%s M=%lld N=%lld K=%lld L=%lld swapped=%d groups=%zu/%zu/%zu/%zu "
               "trace=%d diag=%d X=%s Y=%s tile=%dx%dx%d split=%d split_tiles=%d index=%s "
               "workspace=%zu B%s\n",
               what, an.dtype == FAMLIES_F64 ? "f64" : "f32", comp, (long long)an.M, (long long)an.N,
               (long long)an.K, (long long)an.L, an.swapped ? 1 : 0, an.I.size(), an.J.size(), an.P.size(),
               an.Lm.size(), an.n_trace, an.n_diag, loader[xm], loader[ym], cfg.bm, cfg.bn, cfg.bk, cfg.split,
               cfg.split > 1 ? (cfg.tail ? cfg.tail : -1) : 0,
               index_bits == 32 ? "u32-bytes" : index_bits == -32 ? "i32-elements" : "i64-elements", work_bytes,
               table_hit ? " (tile table)" : "");
}

}  // namespace famlies

using namespace famlies;

extern "C" {

const char* famlies_last_error(void) { return g_err.c_str(); }

static famlies_status analyze_impl(int dtype, int compute, const famlies_tensor* A, const famlies_tensor* B,
                                   const famlies_tensor* C, famlies_plan_info* info, int64_t* offs,
                                   int64_t offs_len) {
  if (!info) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_analyze: null info");
  Analysis an;
  std::string err;
  int st = analyze(dtype, compute, A, B, C, &an, &err);
  if (st != FAMLIES_OK) return fail(st, err);
  if (an.M > kMaxGemmDim || an.N > kMaxGemmDim || an.K > kMaxGemmDim || an.L > kMaxGemmDim)
    return fail(FAMLIES_ERR_UNSUPPORTED, "a GEMM dimension exceeds 2^31 - 1024");
  TileCfg t = int8_slices(an.compute) ? int8_tile() : choose_tiles(nullptr, an);
  if (split_parts(an.compute) && t.tail) {  // as in make_plan: no split for the bf16 kernels
    t.split = 1;
    t.tail = 0;
  }
  if (split_parts(an.compute)) t.bk = split_slice_k(split_parts(an.compute));
  int kchunk = 0, head = 0;
  finalize_split(&t, an.K, ceil_div(an.M, t.bm) * ceil_div(an.N, t.bn), &kchunk, &head);
  int ib = 64;
  bool e32 = false;
  index_form(an, 0, &ib, &e32);
  std::vector<int64_t> v[9];
  bool xv = false, yv = false;
  if (an.M > 0 && an.N > 0) {
    all_offsets(an, v);
    vec_flags(an, t.bk, ib, v, &xv, &yv);
  }
  fill_info(an, t, ib, kernel_code(an, xv, yv), info);
  info->index_elements = ib == 64 || e32;
  if (log_enabled()) log_decision("analyze", an, t, e32 ? -32 : ib, xv, yv, 0, false);
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

famlies_status famlies_analyze(int dtype, int compute, const famlies_tensor* A, const famlies_tensor* B,
                               const famlies_tensor* C, famlies_plan_info* info, int64_t* offs,
                               int64_t offs_len) {
  return no_throw("famlies_analyze", [&] { return analyze_impl(dtype, compute, A, B, C, info, offs, offs_len); });
}

}  // extern "C"
