// Host-side launch interface between the C ABI and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include "args.hpp"
#include "famlies.h"

namespace famlies {

struct PlainLaunch {
  enum Kind { kMain = 0, kScale = 1 } kind = kMain;
  int bm = 128, bn = 128, bk = 16;
  int xm = 1, ym = 1;  // operand loader modes: 0 row-gathered, 1 K-gathered, 2 pre-packed
};

hipError_t launch_plain(int dtype, const PlainArgs<uint32_t>& a, const PlainLaunch& L, hipStream_t s);
hipError_t launch_plain(int dtype, const PlainArgs<int32_t>& a, const PlainLaunch& L, hipStream_t s);
hipError_t launch_plain(int dtype, const PlainArgs<int64_t>& a, const PlainLaunch& L, hipStream_t s);
bool plain_tile_supported(int dtype, int bm, int bn, int bk);

}  // namespace famlies
