// Host-side data structures shared by the planner, the launchers and the C ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "famlies.h"

namespace famlies {

// One (possibly fused) mode of a group, with its stride in each operand of
// the kernel view: X (left, rows M), Y (right, columns N) and C.  A stride is
// 0 in an operand that does not hold the mode.
struct Mode {
  int32_t label;
  int64_t ext;
  int64_t sx, sy, sc;
  // Blocked enumeration: when the first two modes of a group carry blk > 0,
  // the group's index runs over blk0 x blk1 blocks of those two modes: inside
  // a block the first mode runs fastest, then the second; the blocks follow
  // the first mode, then the second; the remaining modes come last.
  int64_t blk = 0;
};

// Result of steps a1-a3 (label classification, grouping/fusion, orientation,
// gather directions).  The kernel computes
//   C(m,n) = sum_k X(m,k) * Y(k,n)
// with X(m,k) at x + xmn[m] + xk[k], Y(k,n) at y + yk[k] + ymn[n] and C(m,n)
// at c + cm[m] + cn[n]; each offset vector is the column-major odometer over
// its group's modes (first mode fastest; blocked over its first two modes
// when they carry block sizes), the same order for every operand holding the
// group (conformal partitioning).
//
// Labels that are not in exactly two tensors are folded into the same view:
// a label in all three tensors is a batch ("L") mode -- one independent GEMM
// per batch index, addressed through three more offset vectors; a label in
// only one input is summed inside the product, i.e. a contracted mode whose
// stride in the other input is 0; a label repeated within one input selects
// the diagonal, i.e. one mode whose stride is the sum of the repeats'.
struct Analysis {
  int dtype = 0, compute = 0;
  int64_t M = 0, N = 0, K = 0, L = 1;
  bool swapped = false;
  bool x_kfast = true, y_kfast = true;
  std::vector<Mode> I, J, P, Lm;
  // address spans (element offsets relative to the base pointer) of the user
  // tensors A, B, C: [lo, hi]; empty tensors have lo > hi.
  int64_t a_lo = 0, a_hi = -1, b_lo = 0, b_hi = -1, c_lo = 0, c_hi = -1;
  int64_t max_abs_x = 0, max_abs_y = 0, max_abs_c = 0;  // bounds on |offset sums|
  // Lowest element offset (<= 0) and reach (max - min offset) of each kernel
  // operand over its non-batch modes: X over I and P, Y over J and P, C over
  // I and J.  Offsets rebased by the lowest one are non-negative.
  int64_t x_lo = 0, y_lo = 0, c_lo_mn = 0;
  int64_t x_span = 0, y_span = 0, c_span = 0;
  int n_trace = 0, n_diag = 0;  // labels summed inside one input / repeated in an input
  int esize = 8;
};

int analyze(int dtype, int compute, const famlies_tensor* A, const famlies_tensor* B,
            const famlies_tensor* C, Analysis* out, std::string* err);

// Offset vector of length n_pad over `modes` using stride selector `which`
// (0: X, 1: Y, 2: C); entries beyond `n` are 0 (a valid address whenever the
// problem is non-empty).
void offsets(const std::vector<Mode>& modes, int which, int64_t n, int64_t n_pad,
             std::vector<int64_t>& out);

// Tile configuration of the plain kernels.
// TileCfg::index_bits value that asks for int32 element offsets.
constexpr int kForceElem32 = 33;

struct TileCfg {
  int bm = 128, bn = 128, bk = 16;
  int split = 1;
  // 0: automatic; 64: 64-bit indexing vectors even where 32 bits reach;
  // kForceElem32: 32-bit element offsets wherever they reach
  int index_bits = 0;
  // split > 1: how many tiles, the last ones in tile order, run as `split`
  // K slices each; the others run whole K first (0: every tile is split)
  int tail = 0;
};

// Host-side bounds check of indexing vectors: every address an operand's
// kernel view forms from the first na, nb, nl entries of a, b and l
// (a[i] + b[j] + l[k], element offsets) lies in [lo, hi].  The vectors are
// separable, so the extreme addresses are sums of each vector's extremes.
bool offsets_in_span(const std::vector<int64_t>& a, int64_t na, const std::vector<int64_t>& b, int64_t nb,
                     const std::vector<int64_t>& l, int64_t nl, int64_t lo, int64_t hi);

void set_error(const std::string& msg);

}  // namespace famlies
