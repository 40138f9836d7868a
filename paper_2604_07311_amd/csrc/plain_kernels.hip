// Plain FP64 / FP32 strided-contraction kernels, the split-K reduction and
// the K == 0 scaling kernel.
//
// One workgroup computes one BM x BN tile of C (in the kernel view
// C(m,n) = sum_k X(m,k) Y(k,n)) over one K range:
//   gather X and Y K-slices through the block-scatter indexing vectors into
//   double-buffered LDS  ->  2x2 waves, each a (BM/2)x(BN/2) MFMA tile
//   ->  alpha/beta scatter-update of C through C's indexing vectors
// (block-scatter mapping, Approach, "Supporting tensor computations"; the
// loops-around-a-micro-kernel structure of Fig. "five loops").
#include "launch.hpp"
#include "tile.hpp"

// Two workgroups per CU (waves per SIMD) for the plain kernels: the FP64 tile
// then keeps its accumulators in VGPRs within 256 registers, and a second
// workgroup hides the other's barrier and global-load latency.
#ifndef FAMLIES_PLAIN_WAVES_PER_EU
#define FAMLIES_PLAIN_WAVES_PER_EU 2
#endif

namespace famlies {

template <typename T, typename OffT, int BM, int BN, int BK, int XM, int YM>
__global__ __launch_bounds__(kThreads, FAMLIES_PLAIN_WAVES_PER_EU) void plain_contract(PlainArgs<OffT> a) {
  // Two slices in flight where the registers allow it: tiles with a
  // row-gathered operand and 32-bit offsets (one load per element along K,
  // so its slice takes longest to arrive), and tiles whose operands are both
  // read in affine 16-byte blocks (few registers per slice; FP64 only with
  // 32-bit offsets).  Measured on the ladder (both affine): FP64 82 -> 87 %,
  // FP32 83 -> 88 %, FP32 with 64-bit offsets 77 -> 85 % of peak.  FP64
  // slices are 8 deep (the FP64 MFMA takes 4 k's, so two steps per slice):
  // half the staging registers of 16-deep slices, which lets the FP64 tile
  // with a row-gathered operand keep two slices in flight too (ring o=48
  // v=192 83.1 -> 85.5 %; ladder 87.0 -> 87.7 %).  With both operands
  // element-gathered along K the deeper pipeline was no faster.
  static constexpr int kDepth =
      ((sizeof(OffT) == 4 && (XM == kRowGather || YM == kRowGather)) ||
       ((sizeof(OffT) == 4 || sizeof(T) == 4) && XM == kVecK && YM == kVecK))
          ? 2
          : 1;
  using Tile = PlainTile<T, BM, BN, BK, XM, YM, kDepth>;
  __shared__ T smem[Tile::SMEM];
  // Work units in launch order: without split-K, every tile of every batch
  // plane; with split-K, first the tiles [0, head) over all of K, then each
  // remaining tile once per K slice.  Each range is spread over the XCDs in
  // contiguous blocks, so neighbouring tiles share an L2.
  const int ntiles = a.tiles_m * a.tiles_n;
  int l = 0, split = -1, t;
  if (a.splits == 1) {
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    l = lid / ntiles;  // batch index
    t = lid % ntiles;
  } else if ((int)blockIdx.x < a.head) {
    t = xcd_remap(blockIdx.x, a.head);
  } else {
    const int ntail = ntiles - a.head;
    const int v = xcd_remap(blockIdx.x - a.head, gridDim.x - a.head);
    split = v / ntail;
    t = a.head + v % ntail;
  }
  const int pm = t % a.tiles_m, pn = t / a.tiles_m;  // M fastest: neighbours share Y's panel
  TileJob<OffT> j;
  // a pre-packed operand holds its batch planes back to back
  j.x = static_cast<const T*>(a.x) +
        (XM == kPacked ? (int64_t)l * a.tiles_m * a.x_nkb * (int64_t)(BM * BK) : a.xl[l]);
  j.y = static_cast<const T*>(a.y) +
        (YM == kPacked ? (int64_t)l * a.tiles_n * a.y_nkb * (int64_t)(BN * BK) : a.yl[l]);
  j.x_nkb = a.x_nkb;
  j.y_nkb = a.y_nkb;
  j.c = static_cast<T*>(a.c) + a.cl[l];
  j.xmn = a.xmn;
  j.xk = a.xk;
  j.yk = a.yk;
  j.ymn = a.ymn;
  j.cm = a.cm;
  j.cn = a.cn;
  j.M = a.M;
  j.N = a.N;
  j.m0 = pm * BM;
  j.n0 = pn * BN;
  j.kbeg = split < 0 ? 0 : split * a.kchunk;
  j.kend = split < 0 ? a.K : min(a.K, j.kbeg + a.kchunk);
  j.alpha = a.alpha;
  j.beta = a.beta;
  // partial sums of a split tile: its own dense BM x BN block
  j.ldw = BN;
  j.work = split < 0 ? nullptr
                     : static_cast<void*>(static_cast<T*>(a.work) +
                                          ((size_t)split * (size_t)(ntiles - a.head) + (size_t)(t - a.head)) *
                                              (size_t)(BM * BN));
  Tile::run(j, smem);
}

// For the split tiles: C = alpha * sum_s W[s] + beta * C, the K slices
// summed in index order so the result does not depend on scheduling.  One
// thread per element of a split tile (bm x bn blocks, row-major).
template <typename T, typename OffT>
__global__ __launch_bounds__(kThreads) void splitk_reduce(PlainArgs<OffT> a, int bm, int bn) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int ntail = a.tiles_m * a.tiles_n - a.head;
  const int64_t per = (int64_t)bm * bn;
  if (i >= ntail * per) return;
  const int tt = (int)(i / per), r = (int)(i % per);
  const int t = a.head + tt;
  const int m = (t % a.tiles_m) * bm + r / bn, n = (t / a.tiles_m) * bn + r % bn;
  if (m >= a.M || n >= a.N) return;
  const T* W = static_cast<const T*>(a.work);
  T s = T(0);
  for (int k = 0; k < a.splits; ++k) s += W[((size_t)k * ntail + tt) * per + r];
  T* cp = at(static_cast<T*>(a.c), (OffT)(a.cm[m] + a.cn[n]));
  const T al = static_cast<T>(a.alpha), be = static_cast<T>(a.beta);
  T v = al * s;
  if (be != T(0)) v += be * *cp;
  *cp = v;
}

// K == 0 or alpha == 0: C = beta * C (beta == 0 writes zeros without reading C).
template <typename T, typename OffT>
__global__ __launch_bounds__(kThreads) void scale_c(PlainArgs<OffT> a) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t mn = (int64_t)a.M * a.N;
  if (i >= mn * a.L) return;
  const int l = (int)(i / mn);
  const int64_t r = i % mn;
  const int m = (int)(r / a.N), n = (int)(r % a.N);
  T* cp = at(static_cast<T*>(a.c) + a.cl[l], (OffT)(a.cm[m] + a.cn[n]));
  const T be = static_cast<T>(a.beta);
  *cp = be != T(0) ? be * *cp : T(0);
}

// ------------------------------------------------------------------ dispatch
template <typename T, typename OffT, int BM, int BN, int BK, int XM, int YM>
static void launch_one(const PlainArgs<OffT>& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((plain_contract<T, OffT, BM, BN, BK, XM, YM>), dim3(grid), dim3(kThreads), 0, s, a);
}

// Gathered and affine-block operands (modes 0, 1, 3) with every offset form;
// pre-packed operands (mode 2) with byte offsets only.
template <typename T, typename OffT, int BM, int BN, int BK>
static hipError_t launch_tile(const PlainArgs<OffT>& a, int xm, int ym, int grid, hipStream_t s) {
  const int code = xm * 4 + ym;
  switch (code) {
    case 0: launch_one<T, OffT, BM, BN, BK, 0, 0>(a, grid, s); return hipGetLastError();
    case 1: launch_one<T, OffT, BM, BN, BK, 0, 1>(a, grid, s); return hipGetLastError();
    case 3: launch_one<T, OffT, BM, BN, BK, 0, 3>(a, grid, s); return hipGetLastError();
    case 4: launch_one<T, OffT, BM, BN, BK, 1, 0>(a, grid, s); return hipGetLastError();
    case 5: launch_one<T, OffT, BM, BN, BK, 1, 1>(a, grid, s); return hipGetLastError();
    case 7: launch_one<T, OffT, BM, BN, BK, 1, 3>(a, grid, s); return hipGetLastError();
    case 12: launch_one<T, OffT, BM, BN, BK, 3, 0>(a, grid, s); return hipGetLastError();
    case 13: launch_one<T, OffT, BM, BN, BK, 3, 1>(a, grid, s); return hipGetLastError();
    case 15: launch_one<T, OffT, BM, BN, BK, 3, 3>(a, grid, s); return hipGetLastError();
    default: break;
  }
  if constexpr (kByteOffsets<OffT>) {
    switch (code) {
      case 2: launch_one<T, OffT, BM, BN, BK, 0, 2>(a, grid, s); return hipGetLastError();
      case 6: launch_one<T, OffT, BM, BN, BK, 1, 2>(a, grid, s); return hipGetLastError();
      case 8: launch_one<T, OffT, BM, BN, BK, 2, 0>(a, grid, s); return hipGetLastError();
      case 9: launch_one<T, OffT, BM, BN, BK, 2, 1>(a, grid, s); return hipGetLastError();
      case 10: launch_one<T, OffT, BM, BN, BK, 2, 2>(a, grid, s); return hipGetLastError();
      case 11: launch_one<T, OffT, BM, BN, BK, 2, 3>(a, grid, s); return hipGetLastError();
      case 14: launch_one<T, OffT, BM, BN, BK, 3, 2>(a, grid, s); return hipGetLastError();
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

template <typename T, typename OffT>
static hipError_t launch_plain_t(const PlainArgs<OffT>& a, const PlainLaunch& L, hipStream_t s) {
  const int64_t mn = (int64_t)a.M * a.N;
  if (L.kind == PlainLaunch::kScale) {
    hipLaunchKernelGGL((scale_c<T, OffT>), dim3((int)((mn * a.L + kThreads - 1) / kThreads)), dim3(kThreads),
                       0, s, a);
    return hipGetLastError();
  }
  const int64_t ntiles = (int64_t)a.tiles_m * a.tiles_n;
  const int grid = (int)(a.splits == 1 ? ntiles * a.L : a.head + (ntiles - a.head) * a.splits);
  constexpr int BK = sizeof(T) == 8 ? 8 : 32;
  hipError_t e = hipErrorInvalidValue;
  if (L.bm == 128 && L.bn == 128 && L.bk == BK)
    e = launch_tile<T, OffT, 128, 128, BK>(a, L.xm, L.ym, grid, s);
  else if (L.bm == 64 && L.bn == 64 && L.bk == BK)
    e = launch_tile<T, OffT, 64, 64, BK>(a, L.xm, L.ym, grid, s);
  if (e != hipSuccess || a.splits == 1) return e;
  const int64_t red = (ntiles - a.head) * L.bm * L.bn;
  hipLaunchKernelGGL((splitk_reduce<T, OffT>), dim3((int)((red + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                     a, L.bm, L.bn);
  return hipGetLastError();
}

hipError_t launch_plain(int dtype, const PlainArgs<uint32_t>& a, const PlainLaunch& L, hipStream_t s) {
  return dtype == FAMLIES_F64 ? launch_plain_t<double, uint32_t>(a, L, s)
                              : launch_plain_t<float, uint32_t>(a, L, s);
}

hipError_t launch_plain(int dtype, const PlainArgs<int32_t>& a, const PlainLaunch& L, hipStream_t s) {
  return dtype == FAMLIES_F64 ? launch_plain_t<double, int32_t>(a, L, s)
                              : launch_plain_t<float, int32_t>(a, L, s);
}

hipError_t launch_plain(int dtype, const PlainArgs<int64_t>& a, const PlainLaunch& L, hipStream_t s) {
  return dtype == FAMLIES_F64 ? launch_plain_t<double, int64_t>(a, L, s)
                              : launch_plain_t<float, int64_t>(a, L, s);
}

bool plain_tile_supported(int dtype, int bm, int bn, int bk) {
  const int BK = dtype == FAMLIES_F64 ? 8 : 32;
  return bk == BK && ((bm == 128 && bn == 128) || (bm == 64 && bn == 64));
}

}  // namespace famlies
