// One C tile of the kernel view C(m,n) = sum_k X(m,k) Y(k,n): the body shared
// by the single-problem kernels and the persistent batched kernel.
//
//   gather X, Y K-slices through the indexing vectors into double-buffered LDS
//   -> 2x2 waves, each a (BM/2)x(BN/2) MFMA tile
//   -> alpha/beta scatter-update of C, or FP partial sums for split-K
#pragma once

#include "device.hpp"

namespace famlies {

template <typename OffT>
struct TileJob {
  const void* x;
  const void* y;
  void* c;
  const OffT* xmn;
  const OffT* xk;
  const OffT* yk;
  const OffT* ymn;
  const OffT* cm;
  const OffT* cn;
  int M, N;
  int m0, n0, kbeg, kend;
  double alpha, beta;
  void* work;  // non-null: write partial sums here, dense [m][n] with leading dim ldw
  int ldw;
  int x_nkb, y_nkb;  // k-blocks per tile row of a pre-packed X / Y
};

// XM, YM: operand loader modes (kRowGather, kKGather, kPacked).
template <typename T, int BM, int BN, int BK, int XM, int YM>
struct PlainTile {
  using MF = Mfma<T>;
  template <typename OffT>
  using GX = Loader<T, OffT, BM, BK, XM>;
  template <typename OffT>
  using GY = Loader<T, OffT, BN, BK, YM>;
  static constexpr int LX = GX<int32_t>::LDK;
  static constexpr int LY = GY<int32_t>::LDK;
  static constexpr int XS = BM * LX, YS = BN * LY;
  static constexpr int SMEM = 2 * (XS + YS);  // elements of T
  static constexpr int WTM = BM / 2, WTN = BN / 2;
  static constexpr int MB = WTM / MF::BS, NB = WTN / MF::BS;
  static constexpr int KPG = BK / MF::KG;
  static_assert(MB >= 1 && NB >= 1 && BK % MF::KG == 0, "bad tile");

  template <typename OffT>
  __device__ __forceinline__ static void run(const TileJob<OffT>& j, T* smem) {
    const int tid = threadIdx.x;
    const int lane = tid % 64, wave = tid / 64;
    const int wm = wave / 2, wn = wave % 2;
    const int nk = j.kend > j.kbeg ? (j.kend - j.kbeg + BK - 1) / BK : 0;
    const T* __restrict__ X = static_cast<const T*>(j.x);
    const T* __restrict__ Y = static_cast<const T*>(j.y);

    GX<OffT> gx;
    GY<OffT> gy;
    gx.init(j.xmn, j.m0, tid);
    gy.init(j.ymn, j.n0, tid);
    if constexpr (XM == kPacked) gx.nkb = j.x_nkb;
    if constexpr (YM == kPacked) gy.nkb = j.y_nkb;

    typename MF::Acc acc[MB][NB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
      for (int jj = 0; jj < NB; ++jj) acc[i][jj] = typename MF::Acc{};

    const int g = lane / MF::BS, r = lane % MF::BS;
    if (nk > 0) {
      // pipeline: offsets two slices ahead, data one slice ahead, LDS double buffer
      gx.fetch_k(j.xk, j.kbeg);
      gy.fetch_k(j.yk, j.kbeg);
      gx.load(X);
      gy.load(Y);
      if (nk > 1) {
        gx.fetch_k(j.xk, j.kbeg + BK);
        gy.fetch_k(j.yk, j.kbeg + BK);
      }
      gx.store(smem, j.kbeg, j.kend);
      gy.store(smem + XS, j.kbeg, j.kend);
      __syncthreads();
      for (int it = 0; it < nk; ++it) {
        const int cur = it & 1;
        const bool more = it + 1 < nk;
        if (more) {
          gx.load(X);
          gy.load(Y);
          if (it + 2 < nk) {
            gx.fetch_k(j.xk, j.kbeg + (it + 2) * BK);
            gy.fetch_k(j.yk, j.kbeg + (it + 2) * BK);
          }
        }
        const T* xs = smem + cur * (XS + YS);
        const T* ys = xs + XS;
#pragma unroll
        for (int s = 0; s < KPG; ++s) {
          T av[MB], bv[NB];
#pragma unroll
          for (int i = 0; i < MB; ++i) av[i] = xs[(wm * WTM + i * MF::BS + r) * LX + g * KPG + s];
#pragma unroll
          for (int jj = 0; jj < NB; ++jj) bv[jj] = ys[(wn * WTN + jj * MF::BS + r) * LY + g * KPG + s];
#pragma unroll
          for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) acc[i][jj] = MF::mma(av[i], bv[jj], acc[i][jj]);
        }
        if (more) {
          T* nx = smem + (cur ^ 1) * (XS + YS);
          const int kn = j.kbeg + (it + 1) * BK;
          gx.store(nx, kn, j.kend);
          gy.store(nx + XS, kn, j.kend);
        }
        __syncthreads();
      }
    }

    if (j.work == nullptr) {
      T* __restrict__ C = static_cast<T*>(j.c);
      const T al = static_cast<T>(j.alpha), be = static_cast<T>(j.beta);
#pragma unroll
      for (int jj = 0; jj < NB; ++jj) {
        const int n = j.n0 + wn * WTN + jj * MF::BS + r;
        const OffT cn = j.cn[n];
#pragma unroll
        for (int i = 0; i < MB; ++i) {
#pragma unroll
          for (int e = 0; e < MF::NACC; ++e) {
            const int m = j.m0 + wm * WTM + i * MF::BS + MF::row(lane, e);
            if (m < j.M && n < j.N) {
              T* cp = at(C, (OffT)(j.cm[m] + cn));
              T v = al * acc[i][jj][e];
              if (be != T(0)) v += be * *cp;
              *cp = v;
            }
          }
        }
      }
    } else {
      T* __restrict__ W = static_cast<T*>(j.work);
#pragma unroll
      for (int jj = 0; jj < NB; ++jj) {
        const int n = j.n0 + wn * WTN + jj * MF::BS + r;
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
          for (int e = 0; e < MF::NACC; ++e) {
            const int m = j.m0 + wm * WTM + i * MF::BS + MF::row(lane, e);
            W[(size_t)m * j.ldw + n] = acc[i][jj][e];
          }
      }
    }
  }
};

}  // namespace famlies
