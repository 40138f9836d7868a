// Kernel argument blocks (host-safe: no device code).
#pragma once

#include <stdint.h>

namespace famlies {

template <typename OffT>
struct PlainArgs {
  const void* x;
  const void* y;
  void* c;
  const OffT* xmn;  // X rows (M, padded)
  const OffT* xk;   // X contracted (K, padded)
  const OffT* yk;   // Y contracted (K, padded)
  const OffT* ymn;  // Y columns (N, padded)
  const OffT* cm;   // C rows (M, padded)
  const OffT* cn;   // C columns (N, padded)
  const OffT* xl;   // batch offsets of X, Y, C (L entries each)
  const OffT* yl;
  const OffT* cl;
  int32_t M, N, K, L;
  int32_t tiles_m, tiles_n, splits, kchunk;
  double alpha, beta;
  void* work;       // split-K partials [splits][tiles_m*BM][tiles_n*BN]
};

}  // namespace famlies
