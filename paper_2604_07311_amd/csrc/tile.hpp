// One C tile of the kernel view C(m,n) = sum_k X(m,k) Y(k,n): the body shared
// by the single-problem kernels and the persistent batched kernel.
//
//   gather X, Y K-slices through the indexing vectors into double-buffered LDS
//   -> 2x2 waves, each a (BM/2)x(BN/2) MFMA tile
//   -> alpha/beta scatter-update of C, or FP partial sums for split-K
#pragma once

#include <type_traits>

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
  void* work;  // non-null: write partial sums here, the tile's block [m - m0][n - n0] with leading dim ldw
  int ldw;
  int x_nkb, y_nkb;  // k-blocks per tile row of a pre-packed X / Y
};

// XM, YM: operand loader modes (kRowGather, kKGather, kPacked, kVecK).  DEPTH: K
// slices whose data loads are in flight while a slice is multiplied (1: the
// next slice; 2: the next two, for latency-bound gathers when registers
// allow).
template <typename T, int BM, int BN, int BK, int XM, int YM, int DEPTH = 1>
struct PlainTile {
  using MF = Mfma<T>;
  template <typename OffT>
  using GX = Loader<T, OffT, BM, BK, XM, 1, DEPTH>;
  template <typename OffT>
  using GY = Loader<T, OffT, BN, BK, YM, 1, DEPTH>;
  static constexpr int LX = GX<int32_t>::LDK;
  static constexpr int LY = GY<int32_t>::LDK;
  static constexpr int XS = BM * LX, YS = BN * LY;
  static constexpr int SMEM = 2 * (XS + YS);  // elements of T
  static constexpr int WTM = BM / 2, WTN = BN / 2;
  static constexpr int MB = WTM / MF::BS, NB = WTN / MF::BS;
  static constexpr int KPG = BK / MF::KG;
  static_assert(MB >= 1 && NB >= 1 && BK % MF::KG == 0, "bad tile");
  static_assert(DEPTH == 1 || DEPTH == 2, "pipeline depth 1 or 2");

  // One slice from LDS buffer `xs` into the accumulators.
  __device__ __forceinline__ static void multiply(const T* xs, int wm, int wn, int g, int r,
                                                  typename MF::Acc (&acc)[MB][NB]) {
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
  }

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
    if constexpr (DEPTH == 1) {
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
          multiply(smem + cur * (XS + YS), wm, wn, g, r, acc);
          if (more) {
            T* nx = smem + (cur ^ 1) * (XS + YS);
            const int kn = j.kbeg + (it + 1) * BK;
            gx.store(nx, kn, j.kend);
            gy.store(nx + XS, kn, j.kend);
          }
          __syncthreads();
        }
      }
    } else if (nk > 0) {
      // DEPTH 2: slice s lives in register slot s % 2 and LDS buffer s % 2;
      // data two slices ahead, offsets three ahead.  Loads and offset
      // fetches are issued on every step, past the last slice too (their
      // slice index clamped to the last one, their data never stored): with
      // the same loads on every path the compiler's wait before a store
      // counts only the slice being stored, not the loads just issued.
      const int klast = j.kbeg + (nk - 1) * BK;
      auto kc = [&](int k0) { return k0 < klast ? k0 : klast; };
      gx.template fetch_k<0>(j.xk, j.kbeg);
      gy.template fetch_k<0>(j.yk, j.kbeg);
      gx.template load<0>(X);
      gy.template load<0>(Y);
      gx.template fetch_k<1>(j.xk, kc(j.kbeg + BK));
      gy.template fetch_k<1>(j.yk, kc(j.kbeg + BK));
      gx.template load<1>(X);
      gy.template load<1>(Y);
      gx.template fetch_k<0>(j.xk, kc(j.kbeg + 2 * BK));
      gy.template fetch_k<0>(j.yk, kc(j.kbeg + 2 * BK));
      gx.template store<0>(smem, j.kbeg, j.kend);
      gy.template store<0>(smem + XS, j.kbeg, j.kend);
      __syncthreads();
      // Step for slice `it` held in LDS buffer S (it % 2 == S): slot S is free
      // and holds the offsets of slice it + 2; slot S^1 holds slice it + 1.
      auto step = [&](auto sc, int it) {
        constexpr int S = decltype(sc)::value;
        gx.template load<S>(X);
        gy.template load<S>(Y);
        gx.template fetch_k<S ^ 1>(j.xk, kc(j.kbeg + (it + 3) * BK));
        gy.template fetch_k<S ^ 1>(j.yk, kc(j.kbeg + (it + 3) * BK));
        multiply(smem + S * (XS + YS), wm, wn, g, r, acc);
        if (it + 1 < nk) {
          T* nx = smem + (S ^ 1) * (XS + YS);
          const int kn = j.kbeg + (it + 1) * BK;
          gx.template store<S ^ 1>(nx, kn, j.kend);
          gy.template store<S ^ 1>(nx + XS, kn, j.kend);
        }
        __syncthreads();
      };
      for (int it = 0; it < nk; it += 2) {
        step(std::integral_constant<int, 0>{}, it);
        if (it + 1 < nk) step(std::integral_constant<int, 1>{}, it + 1);
      }
    }

    if (j.work == nullptr) {
      // Every read (the C indexing vectors, then C itself for beta != 0) is
      // issued before the first write: a write may alias any later read as
      // far as the compiler knows, so reads interleaved with writes would be
      // in flight one at a time.  Rows and columns past the edge take row 0
      // / column 0, a valid element whose value is never written back.
      T* __restrict__ C = static_cast<T*>(j.c);
      const T al = static_cast<T>(j.alpha), be = static_cast<T>(j.beta);
      OffT cmv[MB][MF::NACC], cnv[NB];
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int e = 0; e < MF::NACC; ++e) {
          const int m = j.m0 + wm * WTM + i * MF::BS + MF::row(lane, e);
          cmv[i][e] = j.cm[m < j.M ? m : 0];
        }
#pragma unroll
      for (int jj = 0; jj < NB; ++jj) {
        const int n = j.n0 + wn * WTN + jj * MF::BS + r;
        cnv[jj] = j.cn[n < j.N ? n : 0];
      }
#pragma unroll
      for (int jj = 0; jj < NB; ++jj) {
        const int n = j.n0 + wn * WTN + jj * MF::BS + r;
        T cv[MB][MF::NACC];
        if (be != T(0)) {
#pragma unroll
          for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int e = 0; e < MF::NACC; ++e) cv[i][e] = *global(at(C, (OffT)(cmv[i][e] + cnv[jj])));
        }
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
          for (int e = 0; e < MF::NACC; ++e) {
            const int m = j.m0 + wm * WTM + i * MF::BS + MF::row(lane, e);
            if (m < j.M && n < j.N) {
              T v = al * acc[i][jj][e];
              if (be != T(0)) v += be * cv[i][e];
              *global(at(C, (OffT)(cmv[i][e] + cnv[jj]))) = v;
            }
          }
      }
    } else {
      // partial sums into the tile's own block (tile-local rows and columns)
      T* __restrict__ W = static_cast<T*>(j.work);
#pragma unroll
      for (int jj = 0; jj < NB; ++jj) {
        const int n = wn * WTN + jj * MF::BS + r;
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
          for (int e = 0; e < MF::NACC; ++e) {
            const int m = wm * WTM + i * MF::BS + MF::row(lane, e);
            *global(W + (size_t)m * j.ldw + n) = acc[i][jj][e];
          }
      }
    }
  }
};

}  // namespace famlies
