// Kernel argument blocks (host-safe: no device code).
#pragma once

#include <stdint.h>

namespace famlies {

// Offsets are either uint32_t byte offsets from the operand's lowest element
// (when every operand spans less than 4 GiB) or int64_t element offsets from
// the base pointer.
template <typename OffT>
struct PlainArgs {
  const void* x;    // X, Y, C base pointers (the lowest element in the uint32_t form)
  const void* y;
  void* c;
  const OffT* xmn;  // X rows (M, padded)
  const OffT* xk;   // X contracted (K, padded)
  const OffT* yk;   // Y contracted (K, padded)
  const OffT* ymn;  // Y columns (N, padded)
  const OffT* cm;   // C rows (M, padded)
  const OffT* cn;   // C columns (N, padded)
  const int64_t* xl;  // batch offsets of X, Y, C in elements (L entries each)
  const int64_t* yl;
  const int64_t* cl;
  int32_t M, N, K, L;
  int32_t x_nkb, y_nkb;  // k-blocks per tile row of a pre-packed X / Y (0: not packed)
  int32_t tiles_m, tiles_n, splits, kchunk;
  // splits > 1: tiles [0, head) run whole first; tiles [head, tiles_m*tiles_n)
  // run as `splits` K slices each, writing partial sums to `work`
  int32_t head;
  double alpha, beta;
  void* work;       // split-K partials [splits][tile - head][BM*BN] (plain kernels; the bf16
                    // kernels use [splits][tiles_m*BM][tiles_n*BN] with head = 0)
};

}  // namespace famlies
