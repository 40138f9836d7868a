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
#include "device.hpp"
#include "launch.hpp"

namespace famlies {

template <typename T, typename OffT, int BM, int BN, int BK, bool XK, bool YK>
__global__ __launch_bounds__(kThreads) void plain_contract(PlainArgs<OffT> a) {
  using MF = Mfma<T>;
  using GX = TileGather<T, OffT, BM, BK, XK>;
  using GY = TileGather<T, OffT, BN, BK, YK>;
  constexpr int WTM = BM / 2, WTN = BN / 2;
  constexpr int MB = WTM / MF::BS, NB = WTN / MF::BS;
  constexpr int KPG = BK / MF::KG;  // k's per lane group per slice
  constexpr int XS = BM * GX::LDK, YS = BN * GY::LDK;
  static_assert(MB >= 1 && NB >= 1 && BK % MF::KG == 0, "bad tile");
  __shared__ T smem[2 * (XS + YS)];

  const int tid = threadIdx.x;
  const int lane = tid % 64, wave = tid / 64;
  const int wm = wave / 2, wn = wave % 2;

  const int lid = xcd_remap(blockIdx.x, gridDim.x);
  const int ntiles = a.tiles_m * a.tiles_n;
  const int split = lid / ntiles;
  const int t = lid % ntiles;
  const int pm = t % a.tiles_m, pn = t / a.tiles_m;  // M fastest: neighbours share Y's panel
  const int m0 = pm * BM, n0 = pn * BN;
  const int kbeg = split * a.kchunk;
  const int kend = min(a.K, kbeg + a.kchunk);
  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;

  const T* __restrict__ X = static_cast<const T*>(a.x);
  const T* __restrict__ Y = static_cast<const T*>(a.y);

  GX gx;
  GY gy;
  gx.init(a.xmn, m0, tid);
  gy.init(a.ymn, n0, tid);

  typename MF::Acc acc[MB][NB];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = typename MF::Acc{};

  const int g = lane / MF::BS, r = lane % MF::BS;
  if (nk > 0) {
    gx.load(X, a.xk, kbeg, kend);
    gy.load(Y, a.yk, kbeg, kend);
    gx.store(smem);
    gy.store(smem + XS);
    __syncthreads();
    for (int it = 0; it < nk; ++it) {
      const int cur = it & 1;
      const bool more = it + 1 < nk;
      if (more) {
        const int kn = kbeg + (it + 1) * BK;
        gx.load(X, a.xk, kn, kend);
        gy.load(Y, a.yk, kn, kend);
      }
      const T* xs = smem + cur * (XS + YS);
      const T* ys = xs + XS;
#pragma unroll
      for (int s = 0; s < KPG; ++s) {
        T av[MB], bv[NB];
#pragma unroll
        for (int i = 0; i < MB; ++i)
          av[i] = xs[(wm * WTM + i * MF::BS + r) * GX::LDK + g * KPG + s];
#pragma unroll
        for (int j = 0; j < NB; ++j)
          bv[j] = ys[(wn * WTN + j * MF::BS + r) * GY::LDK + g * KPG + s];
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
          for (int j = 0; j < NB; ++j) acc[i][j] = MF::mma(av[i], bv[j], acc[i][j]);
      }
      if (more) {
        T* nx = smem + (cur ^ 1) * (XS + YS);
        gx.store(nx);
        gy.store(nx + XS);
      }
      __syncthreads();
    }
  }

  if (a.splits == 1) {
    T* __restrict__ C = static_cast<T*>(a.c);
    const T al = static_cast<T>(a.alpha), be = static_cast<T>(a.beta);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int n = n0 + wn * WTN + j * MF::BS + r;
      const OffT cn = a.cn[n];
#pragma unroll
      for (int i = 0; i < MB; ++i) {
#pragma unroll
        for (int e = 0; e < MF::NACC; ++e) {
          const int m = m0 + wm * WTM + i * MF::BS + MF::row(lane, e);
          if (m < a.M && n < a.N) {
            const OffT idx = a.cm[m] + cn;
            T v = al * acc[i][j][e];
            if (be != T(0)) v += be * C[idx];
            C[idx] = v;
          }
        }
      }
    }
  } else {
    // Partial sums of this K range, full padded tile, dense [m][n].
    const int ldw = a.tiles_n * BN;
    T* __restrict__ W = static_cast<T*>(a.work) + (size_t)split * (size_t)(a.tiles_m * BM) * ldw;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int n = n0 + wn * WTN + j * MF::BS + r;
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int e = 0; e < MF::NACC; ++e) {
          const int m = m0 + wm * WTM + i * MF::BS + MF::row(lane, e);
          W[(size_t)m * ldw + n] = acc[i][j][e];
        }
    }
  }
}

// C = alpha * sum_s W[s] + beta * C, the K slices summed in index order so
// the result does not depend on scheduling.
template <typename T, typename OffT>
__global__ __launch_bounds__(kThreads) void splitk_reduce(PlainArgs<OffT> a, int ldw, int rows) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= (int64_t)a.M * a.N) return;
  const int m = (int)(i / a.N), n = (int)(i % a.N);
  const T* W = static_cast<const T*>(a.work);
  const size_t plane = (size_t)rows * ldw;
  T s = T(0);
  for (int k = 0; k < a.splits; ++k) s += W[(size_t)k * plane + (size_t)m * ldw + n];
  T* C = static_cast<T*>(a.c);
  const OffT idx = a.cm[m] + a.cn[n];
  const T al = static_cast<T>(a.alpha), be = static_cast<T>(a.beta);
  T v = al * s;
  if (be != T(0)) v += be * C[idx];
  C[idx] = v;
}

// K == 0: C = beta * C (beta == 0 writes zeros without reading C).
template <typename T, typename OffT>
__global__ __launch_bounds__(kThreads) void scale_c(PlainArgs<OffT> a) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= (int64_t)a.M * a.N) return;
  const int m = (int)(i / a.N), n = (int)(i % a.N);
  T* C = static_cast<T*>(a.c);
  const OffT idx = a.cm[m] + a.cn[n];
  const T be = static_cast<T>(a.beta);
  C[idx] = be != T(0) ? be * C[idx] : T(0);
}

// ------------------------------------------------------------------ dispatch
template <typename T, typename OffT, int BM, int BN, int BK>
static hipError_t launch_tile(const PlainArgs<OffT>& a, bool xk, bool yk, int grid, hipStream_t s) {
  if (xk && yk)
    hipLaunchKernelGGL((plain_contract<T, OffT, BM, BN, BK, true, true>), dim3(grid), dim3(kThreads), 0, s, a);
  else if (xk)
    hipLaunchKernelGGL((plain_contract<T, OffT, BM, BN, BK, true, false>), dim3(grid), dim3(kThreads), 0, s, a);
  else if (yk)
    hipLaunchKernelGGL((plain_contract<T, OffT, BM, BN, BK, false, true>), dim3(grid), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL((plain_contract<T, OffT, BM, BN, BK, false, false>), dim3(grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

template <typename T, typename OffT>
static hipError_t launch_plain_t(const PlainArgs<OffT>& a, const PlainLaunch& L, hipStream_t s) {
  const int64_t mn = (int64_t)a.M * a.N;
  const int eg = (int)((mn + kThreads - 1) / kThreads);
  if (L.kind == PlainLaunch::kScale) {
    hipLaunchKernelGGL((scale_c<T, OffT>), dim3(eg), dim3(kThreads), 0, s, a);
    return hipGetLastError();
  }
  const int grid = a.tiles_m * a.tiles_n * a.splits;
  constexpr int BK = sizeof(T) == 8 ? 16 : 32;
  hipError_t e = hipErrorInvalidValue;
  if (L.bm == 128 && L.bn == 128 && L.bk == BK)
    e = launch_tile<T, OffT, 128, 128, BK>(a, L.xk, L.yk, grid, s);
  else if (L.bm == 64 && L.bn == 64 && L.bk == BK)
    e = launch_tile<T, OffT, 64, 64, BK>(a, L.xk, L.yk, grid, s);
  if (e != hipSuccess || a.splits == 1) return e;
  hipLaunchKernelGGL((splitk_reduce<T, OffT>), dim3(eg), dim3(kThreads), 0, s, a, a.tiles_n * L.bn,
                     a.tiles_m * L.bm);
  return hipGetLastError();
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
  const int BK = dtype == FAMLIES_F64 ? 16 : 32;
  return bk == BK && ((bm == 128 && bn == 128) || (bm == 64 && bn == 64));
}

}  // namespace famlies
