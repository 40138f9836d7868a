// Split-bf16 precision paths: FP32 data, products on BF16 MFMA.
//
// Each FP32 operand value x is split while it is staged into LDS (the
// transform sits inside the packing step, as the paper does for T*A^T in its
// footnote on the sandwiched GEMM C := C - A T A^T) into NS bf16 parts:
//   bf16x3 (NS = 2): h = RNE_bf16(x), l = RNE_bf16(x - h);
//                    x*y ~= hh + (hl + lh)              (3 products)
//   bf16x6 (NS = 3): h, m = RNE_bf16(x - h), l = RNE_bf16(x - h - m);
//                    x*y ~= hh + (hm + mh) + (hl + mm + lh)   (6 products)
// (every difference is exact in FP32).  Products of the same order go to one
// FP32 MFMA accumulator (in bf16x6 the orders 1 and 2 share one); the
// epilogue adds the accumulators in FP64 together with alpha, beta and C,
// and stores FP32 (new and mixed precisions: Introduction, "Challenges";
// "Supporting new and mixed precisions").
#include "device.hpp"
#include "runtime.hpp"

namespace famlies {

// v_mfma_f32_32x32x16_bf16: lane l supplies 8 consecutive contraction
// entries of row (left) / column (right) l % 32 for contraction group l / 32;
// the accumulator layout is that of the 32x32 FP32 shape.
__device__ __forceinline__ f32x16 mma_bf16(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Split two floats into NS packed bf16 pairs (part t of both values in
// parts[t]); each residual x - (parts so far) is exact in FP32.
template <int NS>
__device__ __forceinline__ void split2(float x0, float x1, uint32_t* parts) {
  f32x2 r = {x0, x1};
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    const bf16x2 h = __builtin_convertvector(r, bf16x2);
    parts[t] = __builtin_bit_cast(uint32_t, h);
    if (t + 1 < NS) r = r - __builtin_convertvector(h, f32x2);
  }
}

// bf16 LDS tiles: [row][k] with 16-byte aligned rows of BK + 8 entries,
// BK the contraction slice per stage: 32 for bf16x3, 16 for bf16x6 (whose
// three part planes per operand then leave room in the CU's 160 KB of LDS
// for two workgroups).
template <int NS>
constexpr int kSplitBK = split_slice_k(NS);
template <int NS>
constexpr int kSplitLD = kSplitBK<NS> + 8;  // row pitch in bf16

// Write the split of a gathered slice into the NS part tiles (part t at
// tiles + t * tile_elems).  K-gathered threads own pairs of consecutive k's
// (one packed dword per row and part); row-gathered threads own a run of k's
// in one row (8-byte stores).  EDGE: the slice reaches past kend.
template <int NS, typename G, bool KFAST, bool EDGE, int S>
__device__ __forceinline__ void store_split(const G& gg, __bf16* tiles, int tile_elems, int k0, int kend) {
  if constexpr (KFAST) {
    static_assert(G::KVT == 2, "K-gathered bf16 split stores pairs of k");
#pragma unroll
    for (int i = 0; i < G::E / 2; ++i) {
      uint32_t p[NS];
      split2<NS>(gg.template val<EDGE, S>(2 * i, k0, kend), gg.template val<EDGE, S>(2 * i + 1, k0, kend), p);
      const int idx = gg.lds_index(2 * i, kSplitLD<NS>);
#pragma unroll
      for (int t = 0; t < NS; ++t) *reinterpret_cast<uint32_t*>(tiles + t * tile_elems + idx) = p[t];
    }
  } else if constexpr (G::E == 8) {
    // Two 4-k chunks per row (16-deep slices): both are split before either
    // is written, and lanes 16..31 of each half-wave write them in the other
    // order.  Measured on the bf16x6 ring: 2-3 % faster than splitting and
    // writing chunk by chunk, with the same LDS bank-conflict count (those
    // conflicts are not these stores').
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    uint32_t p[2][2][NS];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      split2<NS>(gg.template val<EDGE, S>(4 * q, k0, kend), gg.template val<EDGE, S>(4 * q + 1, k0, kend), p[q][0]);
      split2<NS>(gg.template val<EDGE, S>(4 * q + 2, k0, kend), gg.template val<EDGE, S>(4 * q + 3, k0, kend),
                 p[q][1]);
    }
    const bool rot = (threadIdx.x >> 4) & 1;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int idx = gg.lds_index(4 * (rot ? 1 - i : i), kSplitLD<NS>);
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const u32x2 w = {rot ? p[1 - i][0][t] : p[i][0][t], rot ? p[1 - i][1][t] : p[i][1][t]};
        *reinterpret_cast<u32x2*>(tiles + t * tile_elems + idx) = w;
      }
    }
  } else {
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
#pragma unroll
    for (int q = 0; q < G::E / 4; ++q) {
      uint32_t p0[NS], p1[NS];
      split2<NS>(gg.template val<EDGE, S>(4 * q, k0, kend), gg.template val<EDGE, S>(4 * q + 1, k0, kend), p0);
      split2<NS>(gg.template val<EDGE, S>(4 * q + 2, k0, kend), gg.template val<EDGE, S>(4 * q + 3, k0, kend), p1);
      const int idx = gg.lds_index(4 * q, kSplitLD<NS>);
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const u32x2 w = {p0[t], p1[t]};
        *reinterpret_cast<u32x2*>(tiles + t * tile_elems + idx) = w;
      }
    }
  }
}

// Operand loader of the split kernels: a gathered FP32 slice split at the
// LDS store (modes kRowGather, kKGather), or pre-packed bf16 parts copied as
// they are (kPacked: block (tile, kb) holds the NS part planes of BR x BK
// bf16, [row][k], zero-filled past the edges; see famlies_pack).  NSLOT
// slices in flight; each phase takes its slot as a template argument.
template <typename OffT, int BR, int NS, int MODE, int NSLOT = 1>
struct SplitLoader {
  static_assert(MODE == kRowGather || MODE == kKGather, "every other mode has its own loader");
  static constexpr bool KF = MODE == kKGather;
  using G = TileGather<float, OffT, BR, kSplitBK<NS>, KF, KF ? 2 : 1, NSLOT>;
  G g;
  int nkb = 0;
  __device__ __forceinline__ void init(const OffT* mnoff, int tile_r0, int tid) { g.init(mnoff, tile_r0, tid); }
  template <int S = 0>
  __device__ __forceinline__ void fetch_k(const OffT* koff, int k0) { g.template fetch_k<S>(koff, k0); }
  template <int S = 0>
  __device__ __forceinline__ void load(const void* base) { g.template load<S>(static_cast<const float*>(base)); }
  template <int S = 0>
  __device__ __forceinline__ void store(__bf16* tiles, int tile_elems, int k0, int kend) const {
    if (k0 + kSplitBK<NS> <= kend)
      store_split<NS, G, KF, false, S>(g, tiles, tile_elems, k0, kend);
    else
      store_split<NS, G, KF, true, S>(g, tiles, tile_elems, k0, kend);
  }
};

// Four consecutive k's of one row, split and written as 8-byte runs of
// bf16 per part (t-th part at tiles + t * tile_elems + idx).
template <int NS>
__device__ __forceinline__ void store_split4(float x0, float x1, float x2, float x3, __bf16* tiles, int tile_elems,
                                             int idx) {
  typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
  uint32_t p0[NS], p1[NS];
  split2<NS>(x0, x1, p0);
  split2<NS>(x2, x3, p1);
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    const u32x2 w = {p0[t], p1[t]};
    *reinterpret_cast<u32x2*>(tiles + t * tile_elems + idx) = w;
  }
}

// K-gathered from affine unit-stride K blocks: 16-byte loads of four k's
// (every slice whole: the planner takes this loader only when BK divides K).
template <typename OffT, int BR, int NS, int NSLOT>
struct SplitLoader<OffT, BR, NS, kVecK, NSLOT> {
  using G = VecKGather<float, OffT, BR, kSplitBK<NS>, NSLOT>;
  G g;
  int nkb = 0;
  __device__ __forceinline__ void init(const OffT* mnoff, int tile_r0, int tid) { g.init(mnoff, tile_r0, tid); }
  template <int S = 0>
  __device__ __forceinline__ void fetch_k(const OffT* koff, int k0) { g.template fetch_k<S>(koff, k0); }
  template <int S = 0>
  __device__ __forceinline__ void load(const void* base) { g.template load<S>(static_cast<const float*>(base)); }
  template <int S = 0>
  __device__ __forceinline__ void store(__bf16* tiles, int tile_elems, int, int) const {
#pragma unroll
    for (int i = 0; i < G::NR; ++i) {
      const auto v = g.v[S][i];
      store_split4<NS>(v[0], v[1], v[2], v[3], tiles, tile_elems, (g.r0 + i * G::RSTEP) * kSplitLD<NS> + g.kk0);
    }
  }
};

template <typename OffT, int BR, int NS, int NSLOT>
struct SplitLoader<OffT, BR, NS, kPacked, NSLOT> {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  static constexpr int BK = kSplitBK<NS>;
  static constexpr int NV = BR * BK / 8;                      // 16-byte vectors per part of a block
  static constexpr int VPT = (NV + kThreads - 1) / kThreads;  // per thread (the last one partly idle)
  u32x4 v[NSLOT][NS][VPT];
  int tile = 0, kb[NSLOT] = {}, nkb = 1, tid = 0;
  __device__ __forceinline__ void init(const OffT*, int tile_r0, int t) {
    tile = tile_r0 / BR;
    tid = t;
  }
  template <int S = 0>
  __device__ __forceinline__ void fetch_k(const OffT*, int k0) { kb[S] = k0 / BK; }
  template <int S = 0>
  __device__ __forceinline__ void load(const void* base) {
    const __bf16* blk = static_cast<const __bf16*>(base) + ((size_t)tile * nkb + kb[S]) * (size_t)(NS * BR * BK);
#pragma unroll
    for (int t = 0; t < NS; ++t)
#pragma unroll
      for (int q = 0; q < VPT; ++q)
        if (NV % kThreads == 0 || tid + q * kThreads < NV)
          v[S][t][q] = reinterpret_cast<const u32x4*>(blk + t * BR * BK)[tid + q * kThreads];
  }
  template <int S = 0>
  __device__ __forceinline__ void store(__bf16* tiles, int tile_elems, int, int) const {
#pragma unroll
    for (int t = 0; t < NS; ++t)
#pragma unroll
      for (int q = 0; q < VPT; ++q) {
        if (NV % kThreads != 0 && tid + q * kThreads >= NV) continue;
        const int e = (tid + q * kThreads) * 8;
        *reinterpret_cast<u32x4*>(tiles + t * tile_elems + (e / BK) * kSplitLD<NS> + e % BK) = v[S][t][q];
      }
  }
};

// One workgroup: a BM x BN tile of C, 2 x 2 waves of (BM/2) x (BN/2), each
// made of 32 x 32 MFMA blocks.
// Two slices in flight except for the 256-row tile, whose two accumulator
// sets fill the accumulation registers and whose loads would then spill.
template <typename OffT, int BM, int NS, int XM, int YM>
constexpr int kSplitDepth = BM == 256 ? 1 : 2;

// Two workgroups per CU for the 128 x 128 bf16x3 tile (256 registers per
// lane, two tiles' LDS in the CU's 160 KB) when its operands are read along K
// in affine blocks or pre-packed: they then fit with two slices in flight;
// measured: ring with pre-packed operands 254 -> 330, ladder v=192 o=48 260
// -> 275 TFLOP/s FP32-equivalent.  With 32-bit offsets one row-gathered
// operand is also allowed: that spills 5 to 24 registers, yet the second
// workgroup hides more than the spills cost (ring, A read along K in affine
// blocks and B row-gathered: 201 -> 261 TFLOP/s).  Both operands row-gathered
// or both element-gathered along K, 64-bit offsets with a row-gathered
// operand (74 to 111 registers spilled) and the other tiles stay at one.
// The 128 x 128 bf16x6 tile runs two workgroups per CU under the same
// operand conditions with 32-bit offsets: its 16-deep slices take 74 KB of
// LDS for both stages, and its two accumulator sets leave the registers for
// two slices in flight (ring 10.80 -> 9.02 ms, ladder v=128 o=32 3.31 ->
// 2.94 ms, ladder v=192 o=48 40.0 -> 35.6 ms against 32-deep slices at one
// workgroup per CU; bf16x3 with 16-deep slices was 4 to 9 % slower).
template <typename OffT, int BM, int NS, int XM, int YM>
constexpr int kSplitWgPerCu =
    (BM == 128 && !(XM == kKGather && YM == kKGather) && !(XM == kRowGather && YM == kRowGather) &&
     (NS == 2 ? ((XM != kRowGather && YM != kRowGather) || sizeof(OffT) == 4) : sizeof(OffT) == 4)) ? 2 : 1;

template <typename OffT, int BM, int BN, int XM, int YM, int NS>
__global__ __launch_bounds__(kThreads, (kSplitWgPerCu<OffT, BM, NS, XM, YM>)) void split_contract(PlainArgs<OffT> a) {
  constexpr int BK = kSplitBK<NS>, LD = kSplitLD<NS>;
  // Slices in flight: one workgroup per CU holds the accumulators, so the
  // next slice's loads must hide behind a single slice of bf16 MFMAs; two
  // slices in flight where the registers allow it.
  constexpr int DEPTH = kSplitDepth<OffT, BM, NS, XM, YM>;
  using GX = SplitLoader<OffT, BM, NS, XM, DEPTH>;
  using GY = SplitLoader<OffT, BN, NS, YM, DEPTH>;
  constexpr int WTM = BM / 2, WTN = BN / 2;
  constexpr int MB = WTM / 32, NB = WTN / 32;
  constexpr int XS = BM * LD, YS = BN * LD;  // bf16 elements per part tile
  constexpr int STAGE = NS * (XS + YS);            // all parts of both tiles
  __shared__ __attribute__((aligned(16))) __bf16 smem[2 * STAGE];

  const int tid = threadIdx.x;
  const int lane = tid % 64, wave = tid / 64;
  const int wm = wave / 2, wn = wave % 2;
  const int lid0 = xcd_remap(blockIdx.x, gridDim.x);
  const int ntiles = a.tiles_m * a.tiles_n;
  const int per_batch = ntiles * a.splits;
  const int l = lid0 / per_batch;  // batch index
  const int lid = lid0 % per_batch;
  const int split = lid / ntiles;
  const int t = lid % ntiles;
  const int pm = t % a.tiles_m, pn = t / a.tiles_m;
  const int m0 = pm * BM, n0 = pn * BN;
  const int kbeg = split * a.kchunk;
  const int kend = min(a.K, kbeg + a.kchunk);
  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  // a pre-packed operand holds its batch planes back to back
  const void* X = XM == kPacked ? static_cast<const void*>(static_cast<const __bf16*>(a.x) +
                                                           (int64_t)l * a.tiles_m * a.x_nkb * (int64_t)(NS * BM * BK))
                                : static_cast<const void*>(static_cast<const float*>(a.x) + a.xl[l]);
  const void* Y = YM == kPacked ? static_cast<const void*>(static_cast<const __bf16*>(a.y) +
                                                           (int64_t)l * a.tiles_n * a.y_nkb * (int64_t)(NS * BN * BK))
                                : static_cast<const void*>(static_cast<const float*>(a.y) + a.yl[l]);

  GX gx;
  GY gy;
  gx.init(a.xmn, m0, tid);
  gy.init(a.ymn, n0, tid);
  gx.nkb = a.x_nkb;
  gy.nkb = a.y_nkb;

  // acc[o]: products whose parts' orders sum to o; in bf16x6 the orders 1
  // and 2 (five products, each below 2^-8 |x||y|) share acc[1], so that two
  // workgroups fit per CU
  constexpr int NA = NS == 3 ? 2 : NS;
  auto slot_of = [](int o) { return o < NA ? o : NA - 1; };
  f32x16 acc[NA][MB][NB];
#pragma unroll
  for (int o = 0; o < NA; ++o)
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) acc[o][i][j] = f32x16{};

  const int g = lane / 32, r = lane % 32;
  auto stage_store = [&](auto sc, int buf, int k0) {
    constexpr int S = decltype(sc)::value;
    __bf16* base = smem + buf * STAGE;
    gx.template store<S>(base, XS, k0, kend);
    gy.template store<S>(base + NS * XS, YS, k0, kend);
  };
  auto multiply = [&](int cur) {
    const __bf16* xs = smem + cur * STAGE;
    const __bf16* ys = xs + NS * XS;
    // lane group g covers k in [g BK/2, (g + 1) BK/2) of the slice, in steps of 8
#pragma unroll
    for (int s = 0; s < BK / 16; ++s) {
      bf16x8 av[NS][MB], bv[NS][NB];
#pragma unroll
      for (int p = 0; p < NS; ++p) {
#pragma unroll
        for (int i = 0; i < MB; ++i)
          av[p][i] = *reinterpret_cast<const bf16x8*>(xs + p * XS + (wm * WTM + i * 32 + r) * LD + g * (BK / 2) + s * 8);
#pragma unroll
        for (int j = 0; j < NB; ++j)
          bv[p][j] = *reinterpret_cast<const bf16x8*>(ys + p * YS + (wn * WTN + j * 32 + r) * LD + g * (BK / 2) + s * 8);
      }
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
          for (int pa = 0; pa < NS; ++pa)
#pragma unroll
            for (int pb = 0; pa + pb < NS; ++pb)
              acc[slot_of(pa + pb)][i][j] = mma_bf16(av[pa][i], bv[pb][j], acc[slot_of(pa + pb)][i][j]);
    }
  };
  constexpr auto slot0 = std::integral_constant<int, 0>{};
  if (nk > 0) {
    if constexpr (DEPTH == 1) {
      gx.fetch_k(a.xk, kbeg);
      gy.fetch_k(a.yk, kbeg);
      gx.load(X);
      gy.load(Y);
      if (nk > 1) {
        gx.fetch_k(a.xk, kbeg + BK);
        gy.fetch_k(a.yk, kbeg + BK);
      }
      stage_store(slot0, 0, kbeg);
      __syncthreads();
      for (int it = 0; it < nk; ++it) {
        const int cur = it & 1;
        const bool more = it + 1 < nk;
        if (more) {
          gx.load(X);
          gy.load(Y);
          if (it + 2 < nk) {
            gx.fetch_k(a.xk, kbeg + (it + 2) * BK);
            gy.fetch_k(a.yk, kbeg + (it + 2) * BK);
          }
        }
        multiply(cur);
        if (more) stage_store(slot0, cur ^ 1, kbeg + (it + 1) * BK);
        __syncthreads();
      }
    } else {
      // Slice s in register slot s % 2 and LDS stage s % 2; data two slices
      // ahead, offsets three ahead.  The loads are issued on every step, past
      // the last slice too (slice index clamped, data never stored), so the
      // wait before a store covers only the slice being stored.
      const int klast = kbeg + (nk - 1) * BK;
      auto kc = [&](int k0) { return k0 < klast ? k0 : klast; };
      gx.template fetch_k<0>(a.xk, kbeg);
      gy.template fetch_k<0>(a.yk, kbeg);
      gx.template load<0>(X);
      gy.template load<0>(Y);
      gx.template fetch_k<1>(a.xk, kc(kbeg + BK));
      gy.template fetch_k<1>(a.yk, kc(kbeg + BK));
      gx.template load<1>(X);
      gy.template load<1>(Y);
      gx.template fetch_k<0>(a.xk, kc(kbeg + 2 * BK));
      gy.template fetch_k<0>(a.yk, kc(kbeg + 2 * BK));
      stage_store(slot0, 0, kbeg);
      __syncthreads();
      auto step = [&](auto sc, int it) {
        constexpr int S = decltype(sc)::value;
        gx.template load<S>(X);
        gy.template load<S>(Y);
        gx.template fetch_k<S ^ 1>(a.xk, kc(kbeg + (it + 3) * BK));
        gy.template fetch_k<S ^ 1>(a.yk, kc(kbeg + (it + 3) * BK));
        multiply(S);
        if (it + 1 < nk) stage_store(std::integral_constant<int, S ^ 1>{}, S ^ 1, kbeg + (it + 1) * BK);
        __syncthreads();
      };
      for (int it = 0; it < nk; it += 2) {
        step(std::integral_constant<int, 0>{}, it);
        if (it + 1 < nk) step(std::integral_constant<int, 1>{}, it + 1);
      }
    }
  }

  auto total = [&](int i, int j, int e) {
    double v = 0.0;
#pragma unroll
    for (int o = NA - 1; o >= 0; --o) v += (double)acc[o][i][j][e];  // smallest order first
    return v;
  };
  if (a.splits == 1) {
    float* __restrict__ C = static_cast<float*>(a.c) + a.cl[l];
    // Every read (indexing vectors, then C for beta != 0) before the first
    // write, so that the reads are in flight together rather than one per
    // element; past the edge row 0 / column 0 is read and never written.
    OffT cmv[MB][16], cnv[NB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int m = m0 + wm * WTM + i * 32 + Mfma<float>::row(lane, e);
        cmv[i][e] = a.cm[m < a.M ? m : 0];
      }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int n = n0 + wn * WTN + j * 32 + r;
      cnv[j] = a.cn[n < a.N ? n : 0];
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int n = n0 + wn * WTN + j * 32 + r;
      float cv[MB][16];
      if (a.beta != 0.0) {
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
          for (int e = 0; e < 16; ++e) cv[i][e] = *at(C, (OffT)(cmv[i][e] + cnv[j]));
      }
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int m = m0 + wm * WTM + i * 32 + Mfma<float>::row(lane, e);
          if (m < a.M && n < a.N) {
            double v = a.alpha * total(i, j, e);
            if (a.beta != 0.0) v += a.beta * (double)cv[i][e];
            *at(C, (OffT)(cmv[i][e] + cnv[j])) = (float)v;
          }
        }
    }
  } else {
    const int ldw = a.tiles_n * BN;
    double* __restrict__ W = static_cast<double*>(a.work) + (size_t)split * (size_t)(a.tiles_m * BM) * ldw;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int n = n0 + wn * WTN + j * 32 + r;
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int m = m0 + wm * WTM + i * 32 + Mfma<float>::row(lane, e);
          W[(size_t)m * ldw + n] = total(i, j, e);
        }
    }
  }
}

template <typename OffT>
__global__ __launch_bounds__(kThreads) void split_reduce(PlainArgs<OffT> a, int ldw, int rows) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= (int64_t)a.M * a.N) return;
  const int m = (int)(i / a.N), n = (int)(i % a.N);
  const double* W = static_cast<const double*>(a.work);
  const size_t plane = (size_t)rows * ldw;
  double s = 0.0;
  for (int k = 0; k < a.splits; ++k) s += W[(size_t)k * plane + (size_t)m * ldw + n];
  float* cp = at(static_cast<float*>(a.c), (OffT)(a.cm[m] + a.cn[n]));
  double v = a.alpha * s;
  if (a.beta != 0.0) v += a.beta * (double)*cp;
  *cp = (float)v;
}

template <typename OffT, int BM, int BN, int NS, int XM, int YM>
static void launch_split_one(const PlainArgs<OffT>& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((split_contract<OffT, BM, BN, XM, YM, NS>), dim3(grid), dim3(kThreads), 0, s, a);
}

// Gathered and affine-block operands with every offset form; pre-packed
// operands with byte offsets only.
template <typename OffT, int BM, int BN, int NS>
static hipError_t launch_split_tile(const PlainArgs<OffT>& a, int xm, int ym, int grid, hipStream_t s) {
  const int code = xm * 4 + ym;
  switch (code) {
    case 0: launch_split_one<OffT, BM, BN, NS, 0, 0>(a, grid, s); return hipGetLastError();
    case 1: launch_split_one<OffT, BM, BN, NS, 0, 1>(a, grid, s); return hipGetLastError();
    case 3: launch_split_one<OffT, BM, BN, NS, 0, 3>(a, grid, s); return hipGetLastError();
    case 4: launch_split_one<OffT, BM, BN, NS, 1, 0>(a, grid, s); return hipGetLastError();
    case 5: launch_split_one<OffT, BM, BN, NS, 1, 1>(a, grid, s); return hipGetLastError();
    case 7: launch_split_one<OffT, BM, BN, NS, 1, 3>(a, grid, s); return hipGetLastError();
    case 12: launch_split_one<OffT, BM, BN, NS, 3, 0>(a, grid, s); return hipGetLastError();
    case 13: launch_split_one<OffT, BM, BN, NS, 3, 1>(a, grid, s); return hipGetLastError();
    case 15: launch_split_one<OffT, BM, BN, NS, 3, 3>(a, grid, s); return hipGetLastError();
    default: break;
  }
  if constexpr (kByteOffsets<OffT>) {
    switch (code) {
      case 2: launch_split_one<OffT, BM, BN, NS, 0, 2>(a, grid, s); return hipGetLastError();
      case 6: launch_split_one<OffT, BM, BN, NS, 1, 2>(a, grid, s); return hipGetLastError();
      case 8: launch_split_one<OffT, BM, BN, NS, 2, 0>(a, grid, s); return hipGetLastError();
      case 9: launch_split_one<OffT, BM, BN, NS, 2, 1>(a, grid, s); return hipGetLastError();
      case 10: launch_split_one<OffT, BM, BN, NS, 2, 2>(a, grid, s); return hipGetLastError();
      case 11: launch_split_one<OffT, BM, BN, NS, 2, 3>(a, grid, s); return hipGetLastError();
      case 14: launch_split_one<OffT, BM, BN, NS, 3, 2>(a, grid, s); return hipGetLastError();
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

template <typename OffT>
static hipError_t launch_split_t(const PlainArgs<OffT>& a, const PlainLaunch& L, int ns, hipStream_t s) {
  const int grid = a.tiles_m * a.tiles_n * a.splits * a.L;
  hipError_t e = hipErrorInvalidValue;
  if (ns == 2) {
    if (L.bm == 256 && L.bn == 128)
      e = launch_split_tile<OffT, 256, 128, 2>(a, L.xm, L.ym, grid, s);
    else if (L.bm == 128 && L.bn == 128)
      e = launch_split_tile<OffT, 128, 128, 2>(a, L.xm, L.ym, grid, s);
    else if (L.bm == 64 && L.bn == 64)
      e = launch_split_tile<OffT, 64, 64, 2>(a, L.xm, L.ym, grid, s);
  } else if (ns == 3) {
    if (L.bm == 128 && L.bn == 128)
      e = launch_split_tile<OffT, 128, 128, 3>(a, L.xm, L.ym, grid, s);
    else if (L.bm == 64 && L.bn == 64)
      e = launch_split_tile<OffT, 64, 64, 3>(a, L.xm, L.ym, grid, s);
  }
  if (e != hipSuccess || a.splits == 1) return e;
  const int64_t mn = (int64_t)a.M * a.N;
  hipLaunchKernelGGL((split_reduce<OffT>), dim3((int)((mn + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                     s, a, a.tiles_n * L.bn, a.tiles_m * L.bm);
  return hipGetLastError();
}

hipError_t launch_split(const PlainArgs<uint32_t>& a, const PlainLaunch& L, int ns, hipStream_t s) {
  return launch_split_t(a, L, ns, s);
}
hipError_t launch_split(const PlainArgs<int32_t>& a, const PlainLaunch& L, int ns, hipStream_t s) {
  return launch_split_t(a, L, ns, s);
}
hipError_t launch_split(const PlainArgs<int64_t>& a, const PlainLaunch& L, int ns, hipStream_t s) {
  return launch_split_t(a, L, ns, s);
}
bool split_tile_supported(int ns, int bm, int bn) {
  if (ns == 3) return (bm == 128 && bn == 128) || (bm == 64 && bn == 64);
  return (bm == 256 && bn == 128) || (bm == 128 && bn == 128) || (bm == 64 && bn == 64);
}

}  // namespace famlies
