// FP64 contraction emulated on 8-bit integer products (INT8 MFMA).
//
// A new precision placed inside the GEMM the way the paper places
// transformations in the packing step ("Supporting new and mixed
// precisions"; Introduction, "Challenges"): the operands are sliced while
// they are packed, and the GEMM runs on the slices.  The slicing is the
// error-free splitting of Ozaki, Ogita, Oishi and Rump in the integer form of
// Ootomo, Ozaki and Yokota:
//   1. every row of X's GEMM view (and column of Y's) is scaled by a power
//      of two, 2^-e with e the smallest integer such that
//      max|v| <= (127/128) 2^e;
//   2. each scaled value is cut into S signed digits by exact rounding to
//      nearest (d_t = rint(2^7 r), r <- 2^7 r - d_t; |d_1| <= 127 since the
//      scale keeps |v| <= 127/128, |d_t| <= 64 after it);
//   3. for every digit pair (t, u) with t + u <= S + 1 the digit products are
//      summed exactly in int32 on v_mfma_i32_32x32x32_i8, pairs of one
//      diagonal t + u into one accumulator (exact while the sum stays below
//      2^31, so long K runs in chunks flushed to FP64);
//   4. C = alpha 2^(ex+ey) sum_d 2^-7d S_d + beta C, in FP64.
//
// int8_slice: one workgroup per 64 rows of one operand view, all of K:
//   pass 1 the row maxima -> exponents, pass 2 the digits -> digit planes
//   stored tile-major, [l][t][tile][k block][row in tile][64 k] (int8), the
//   layout int8_gemm copies straight into LDS.
// int8_gemm: one workgroup per 128 x 64 tile of C, 2 x 2 waves of 64 x 32;
//   the S planes of X and Y for 32 contracted indices sit in one of two LDS
//   buffers (the next step's are loaded meanwhile) and every wave keeps one
//   int32 accumulator set per digit diagonal (S sets of 32 registers, in the
//   accumulation registers).  S is 3 to 7 (seven sets: 224 accumulation
//   registers, 126 KB of LDS).
#include "launch.hpp"
#include "runtime.hpp"
#include "tile.hpp"

namespace famlies {

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));

constexpr int kI8K = 64;        // contracted indices (bytes of one digit plane) per K slice
constexpr int kI8SliceRows = 64;  // rows per slicing workgroup
constexpr int kI8Pitch = 80;    // LDS row pitch in bytes: 64 + 16 (16-byte aligned, spreads banks)
constexpr int kI8BM = 128, kI8BN = 64;
constexpr int kExpNonFinite = 0x7fffffff;  // exponent of a row holding Inf or NaN

// K slices whose digit products stay exact in int32: one diagonal sums at
// most S pairs of products |d_t d_u| <= 127^2 per contracted index.
constexpr int int8_chunk_slices(int S) { return (int)(2147483647LL / (64LL * S * 127 * 127)); }

template <typename OffT>
struct SliceArgs {
  const void* src;      // operand base (its lowest element in the uint32 form)
  const OffT* rows;     // row offsets (R valid)
  const OffT* ks;       // contracted offsets (K valid)
  const int64_t* bl;    // batch offsets in elements (L)
  int8_t* planes;       // [L][S][tiles][nkb][tile_rows][64]
  int32_t* exps;        // [L][tiles * tile_rows]
  double* pmax;         // partial row maxima [L][ksplit][tiles * tile_rows] (+Inf: a non-finite value)
  int32_t R, K, L;
  int32_t tile_rows, tiles, nkb;
  int32_t ksplit, kbper;  // K ranges per row block, 64-blocks per range
};

// ---------------------------------------------------------------- slicing
// Two kernels over (row block of 64, K range) workgroups, so that a long K
// spreads over many workgroups: int8_rowmax writes each range's row maxima,
// int8_digits reduces them for its rows (the first range's workgroup also
// writes the exponents) and cuts its range into digit planes.  The partial
// maxima are reduced in range order: no atomics, deterministic.
//
// Operand read modes: lanes along rows (row-gathered), lanes along k with
// one load per element (K-gathered), or lanes along k with 16-byte loads of
// runs of consecutive k (K blocks that are affine unit-stride runs with
// 16-byte aligned starts, the block strides of the block-scatter layout).
constexpr int kSliceRows = 0, kSliceK = 1, kSliceKVec = 2;

// Step 1: the smallest e with m <= (127/128) 2^e (0 for m == 0), so that
// every scaled value's first digit rint(2^7 v) stays within [-127, 127].
__device__ __forceinline__ int slice_exponent(double m) {
  if (m == 0.0) return 0;
  int e;
  const double f = frexp(m, &e);
  return f <= 127.0 / 128.0 ? e : e + 1;
}

// One workgroup's view of a slicing job: 64 rows from row0, K blocks
// [kb0, kb1).  Thread layout: 16 elements each, 4 rows x 4 consecutive k
// (lanes along k, 16 lanes per row) or 1 row x 4 runs of 4 consecutive k
// (lanes along rows).
template <typename OffT, int MODE>
struct SliceTile {
  static constexpr bool KF = MODE != kSliceRows;
  const SliceArgs<OffT>& a;
  OffT* srow;  // LDS: the 64 row offsets
  OffT* sk;    // LDS: one block's 64 contracted offsets
  const double* base;
  int tid, l, row0, kb0, kb1, kq, rg, rr, kg;
  __device__ SliceTile(const SliceArgs<OffT>& args, OffT* sr, OffT* skk) : a(args), srow(sr), sk(skk) {
    tid = threadIdx.x;
    const int rblocks = a.tiles * (a.tile_rows / kI8SliceRows);
    const int per_l = rblocks * a.ksplit;
    l = blockIdx.x / per_l;
    const int w = blockIdx.x % per_l;
    row0 = (w / a.ksplit) * kI8SliceRows;
    kb0 = (w % a.ksplit) * a.kbper;
    kb1 = min(a.nkb, kb0 + a.kbper);
    base = static_cast<const double*>(a.src) + a.bl[l];
    kq = KF ? tid % 16 : 0;
    rg = KF ? tid / 16 : 0;
    rr = KF ? 0 : tid % 64;
    kg = KF ? 0 : tid / 64;
    if (tid < kI8SliceRows) srow[tid] = row0 + tid < a.R ? a.rows[row0 + tid] : (OffT)0;
  }
  __device__ int row_of(int j) const { return KF ? rg + 16 * j : rr; }
  __device__ int kin(int j) const { return KF ? 4 * kq : 4 * (kg + 4 * j); }  // first of 4 k's in the block
  // stage block kb's offsets in LDS (barriers on both sides)
  __device__ void stage_k(int kb) {
    __syncthreads();
    if (tid < kI8K) sk[tid] = kb * kI8K + tid < a.K ? a.ks[kb * kI8K + tid] : (OffT)0;
    __syncthreads();
  }
  __device__ void load(int kb, double (&v)[4][4]) const {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = row_of(j), k0 = kin(j);
      const bool rok = row0 + r < a.R;
      const OffT ro = srow[r];
      if constexpr (MODE == kSliceKVec) {
        // a whole affine block (the mode needs K a multiple of 64)
        typedef double f64x2 __attribute__((ext_vector_type(2)));
        const double* p = at(base, (OffT)(ro + sk[k0]));
        const f64x2 lo = rok ? *global(reinterpret_cast<const f64x2*>(p)) : f64x2{0.0, 0.0};
        const f64x2 hi = rok ? *global(reinterpret_cast<const f64x2*>(p) + 1) : f64x2{0.0, 0.0};
        v[j][0] = lo[0];
        v[j][1] = lo[1];
        v[j][2] = hi[0];
        v[j][3] = hi[1];
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int k = kb * kI8K + k0 + c;
          v[j][c] = (rok && k < a.K) ? *global(at(base, (OffT)(ro + sk[k0 + c]))) : 0.0;
        }
      }
    }
  }
};

// Partial row maxima of one K range (+Inf marks a row holding Inf or NaN).
template <typename OffT, int MODE>
__global__ __launch_bounds__(kThreads) void int8_rowmax(SliceArgs<OffT> a) {
  __shared__ OffT srow[kI8SliceRows], sk[kI8K];
  __shared__ double smax[4][kI8SliceRows];
  SliceTile<OffT, MODE> st(a, srow, sk);
  constexpr bool KF = SliceTile<OffT, MODE>::KF;
  double m[4] = {0.0, 0.0, 0.0, 0.0};
  for (int kb = st.kb0; kb < st.kb1; ++kb) {
    st.stage_k(kb);
    double v[4][4];
    st.load(kb, v);
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double x = v[j][c];
        m[KF ? j : 0] = __builtin_isfinite(x) ? fmax(m[KF ? j : 0], fabs(x)) : __builtin_inf();
      }
  }
  const int64_t rows_pad = (int64_t)a.tiles * a.tile_rows;
  double* out = a.pmax + ((int64_t)st.l * a.ksplit + st.kb0 / a.kbper) * rows_pad + st.row0;
  if constexpr (KF) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
      for (int sh = 1; sh < 16; sh <<= 1) m[j] = fmax(m[j], __shfl_xor(m[j], sh, 16));
      if (st.kq == 0) out[st.row_of(j)] = m[j];
    }
  } else {
    smax[st.kg][st.rr] = m[0];
    __syncthreads();
    if (st.tid < kI8SliceRows)
      out[st.tid] = fmax(fmax(smax[0][st.tid], smax[1][st.tid]), fmax(smax[2][st.tid], smax[3][st.tid]));
  }
}

// Exponents from the partial maxima, then the digits of one K range (step 2:
// exact rounding to nearest), staged in LDS and written out as 16-byte rows
// of the planes.
template <typename OffT, int S, int MODE>
__global__ __launch_bounds__(kThreads) void int8_digits(SliceArgs<OffT> a) {
  __shared__ __attribute__((aligned(16))) unsigned char dig[S * kI8SliceRows * kI8Pitch];
  __shared__ OffT srow[kI8SliceRows], sk[kI8K];
  __shared__ int sexp[kI8SliceRows];
  SliceTile<OffT, MODE> st(a, srow, sk);
  const int tid = st.tid;
  const int64_t rows_pad = (int64_t)a.tiles * a.tile_rows;
  if (tid < kI8SliceRows) {
    const double* pm = a.pmax + (int64_t)st.l * a.ksplit * rows_pad + st.row0 + tid;
    double m = 0.0;
    for (int q = 0; q < a.ksplit; ++q) m = fmax(m, pm[q * rows_pad]);
    const int e = m == __builtin_inf() ? kExpNonFinite : slice_exponent(m);
    sexp[tid] = e;
    if (st.kb0 == 0) a.exps[(int64_t)st.l * rows_pad + st.row0 + tid] = e;
  }
  const int tile = st.row0 / a.tile_rows, rin = st.row0 % a.tile_rows;
  for (int kb = st.kb0; kb < st.kb1; ++kb) {
    st.stage_k(kb);  // its first barrier also orders sexp and the previous block's dig reads
    double v[4][4];
    st.load(kb, v);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = st.row_of(j);
      const int e = sexp[r];
      uint32_t packed[S];
#pragma unroll
      for (int t = 0; t < S; ++t) packed[t] = 0u;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double rem = e == kExpNonFinite ? 0.0 : ldexp(v[j][c], -e);
#pragma unroll
        for (int t = 0; t < S; ++t) {
          const double y = rem * 128.0;  // exact
          const double q = rint(y);      // nearest, ties to even
          rem = y - q;                   // exact
          packed[t] |= ((uint32_t)(int)q & 0xffu) << (8 * c);
        }
      }
#pragma unroll
      for (int t = 0; t < S; ++t)
        *reinterpret_cast<uint32_t*>(&dig[(t * kI8SliceRows + r) * kI8Pitch + st.kin(j)]) = packed[t];
    }
    __syncthreads();
    // 64 rows x 64 bytes per plane: 256 chunks of 16 bytes, one per thread
    const int cr = tid / 4, cc = tid % 4;
#pragma unroll
    for (int t = 0; t < S; ++t) {
      const i32x4 w = *reinterpret_cast<const i32x4*>(&dig[(t * kI8SliceRows + cr) * kI8Pitch + 16 * cc]);
      const int64_t blk = (((int64_t)st.l * S + t) * a.tiles + tile) * a.nkb + kb;
      *global(reinterpret_cast<i32x4*>(a.planes + (blk * a.tile_rows + rin + cr) * kI8K + 16 * cc)) = w;
    }
  }
}

// K ranges per row block: enough workgroups to fill the chip (about 2048)
// with ranges of whole 64-blocks.
__host__ __device__ inline void slice_split(int64_t rblocks_l, int nkb, int* ksplit, int* kbper) {
  int64_t want = (2048 + rblocks_l - 1) / rblocks_l;
  if (want < 1) want = 1;
  if (want > nkb) want = nkb;
  *kbper = (int)((nkb + want - 1) / want);
  *ksplit = (nkb + *kbper - 1) / *kbper;
}

// ---------------------------------------------------------------- GEMM
template <typename OffT>
struct Int8GemmArgs {
  PlainArgs<OffT> p;         // C, its indexing vectors, sizes, alpha, beta
  const int8_t* xp;          // X digit planes [L][S][tiles_m][nkb][128][64]
  const int8_t* yp;          // Y digit planes [L][S][tiles_n][nkb][64][64]
  const int32_t* xe;         // X row exponents [L][tiles_m * 128]
  const int32_t* ye;         // Y column exponents [L][tiles_n * 64]
  int32_t nkb;               // K slices of the planes
  int32_t kb0, kb1;          // the K slices this launch sums (at most one exact int32 chunk)
};

// 32 x 32 accumulator layout of the 32x32 MFMA shapes: element r of lane l
// is row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.
__device__ __forceinline__ int acc_row(int l, int r) { return 8 * (r / 4) + 4 * (l / 32) + (r % 4); }

// LDS of the GEMM: two buffers, each the S planes of X (128 rows) and Y (64
// rows) for 32 contracted indices, rows 48 bytes apart (32 + 16: the MFMA
// operand reads of 16 consecutive rows cover all 64 banks once).
constexpr int kI8Step = 32;
constexpr int kI8StepPitch = 48;
// Steps whose global loads are in flight while one is multiplied: two up to
// six digit slices (the second register set fits beside the S accumulator
// sets), one at seven.  The loads are plane chunks that mostly miss L2; with
// one step of lead (about 0.5 us of MFMA work) the GEMM waited on them.
constexpr int int8_gemm_lead(int S) { return S <= 6 ? 2 : 1; }

template <typename OffT, int S>
__global__ __launch_bounds__(kThreads, 1) void int8_gemm(Int8GemmArgs<OffT> g) {
  constexpr int XB = S * kI8BM * kI8StepPitch, YB = S * kI8BN * kI8StepPitch;  // bytes per buffer
  __shared__ __attribute__((aligned(16))) unsigned char smem[2 * (XB + YB)];
  const PlainArgs<OffT>& a = g.p;
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int wm = wave % 2, wn = wave / 2;  // wave tile: rows 64 wm .., columns 32 wn ..
  const int ntiles = a.tiles_m * a.tiles_n;
  const int lid = xcd_remap(blockIdx.x, gridDim.x);
  const int l = lid / ntiles, t = lid % ntiles;
  const int pm = t % a.tiles_m, pn = t / a.tiles_m;  // M fastest: neighbours share Y's panel
  const int8_t* xb = g.xp + ((int64_t)l * S * a.tiles_m + pm) * (int64_t)g.nkb * (kI8BM * kI8K);
  const int8_t* yb = g.yp + ((int64_t)l * S * a.tiles_n + pn) * (int64_t)g.nkb * (kI8BN * kI8K);
  const int64_t xplane = (int64_t)a.tiles_m * g.nkb * (kI8BM * kI8K);  // stride between X planes
  const int64_t yplane = (int64_t)a.tiles_n * g.nkb * (kI8BN * kI8K);
  // A step is 32 contracted indices, half of a 64-k block of the planes:
  // per plane X 128 rows x 32 bytes (one 16-byte chunk per thread), Y 64 rows
  // x 32 bytes (threads < 128).  Chunk c: row c / 2, bytes 16 (c % 2).
  // One step of one plane: X 128 rows x 32 bytes, one 16-byte chunk per
  // thread; Y 64 rows x 32 bytes, with two register sets one 8-byte chunk
  // per thread (half the registers), with one a 16-byte chunk per thread of
  // the first 128.  Each group of 8 lanes stores 8 consecutive rows at one
  // chunk offset (16-byte chunks), or 8 rows at two neighbouring offsets
  // (8-byte chunks): at the 48-byte pitch their LDS banks are disjoint.
  constexpr int NL = int8_gemm_lead(S);
  constexpr bool kYHalf = NL == 2;
  typedef int i32x2 __attribute__((ext_vector_type(2)));
  typedef typename std::conditional<kYHalf, i32x2, i32x4>::type ychunk_t;
  const int crow = ((tid >> 4) << 3) | (tid & 7), cofs = 16 * ((tid >> 3) & 1);
  const int yrow = kYHalf ? ((tid >> 5) << 3) | ((tid >> 1) & 7) : crow;
  const int yofs = kYHalf ? 8 * (2 * ((tid >> 4) & 1) + (tid & 1)) : cofs;
  const bool ythr = kYHalf || tid < 2 * kI8BN;
  constexpr int kStepsPerBlock = kI8K / kI8Step;
  const int st0 = kStepsPerBlock * g.kb0, st1 = kStepsPerBlock * g.kb1;
  i32x4 rx[NL][S];
  ychunk_t ry[NL][S];
  // loads of step st into register set Q (steps past the last re-read it;
  // their data is never stored)
  auto fetch = [&](auto qc, int st) {
    constexpr int Q = decltype(qc)::value;
    st = st < st1 ? st : st1 - 1;
    const int64_t blk = (int64_t)(st / kStepsPerBlock), half = kI8Step * (st % kStepsPerBlock);
#pragma unroll
    for (int t2 = 0; t2 < S; ++t2) {
      rx[Q][t2] = *global(reinterpret_cast<const i32x4*>(xb + t2 * xplane + blk * (kI8BM * kI8K) + crow * kI8K +
                                                         half + cofs));
      if (ythr)
        ry[Q][t2] = *global(reinterpret_cast<const ychunk_t*>(yb + t2 * yplane + blk * (kI8BN * kI8K) +
                                                              yrow * kI8K + half + yofs));
    }
  };
  auto stash = [&](auto qc, int buf) {
    constexpr int Q = decltype(qc)::value;
    unsigned char* bx = smem + buf * (XB + YB);
    unsigned char* by = bx + XB;
#pragma unroll
    for (int t2 = 0; t2 < S; ++t2) {
      *reinterpret_cast<i32x4*>(&bx[(t2 * kI8BM + crow) * kI8StepPitch + cofs]) = rx[Q][t2];
      if (ythr) *reinterpret_cast<ychunk_t*>(&by[(t2 * kI8BN + yrow) * kI8StepPitch + yofs]) = ry[Q][t2];
    }
  };
  i32x16 acc[S][2];
#pragma unroll
  for (int d = 0; d < S; ++d)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[d][b][r] = 0;
  const int fr = lane % 32, fk = 16 * (lane / 32);  // operand fragment: row / column, k offset
  // C update from the exact int32 sums of this launch's K chunk:
  // C = alpha 2^(ex+ey) sum_d 2^-7d S_d + beta C, the sum over diagonals from
  // the lightest to the heaviest (a later chunk runs with beta = 1).
  auto update_c = [&]() {
    const int64_t mrow0 = (int64_t)pm * kI8BM + wm * 64, ncol = (int64_t)pn * kI8BN + wn * 32 + fr;
    if (ncol >= a.N) return;
    const int ey = g.ye[(int64_t)l * a.tiles_n * kI8BN + ncol];
    double* C = static_cast<double*>(a.c) + a.cl[l];
    const OffT cn = a.cn[ncol];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t m = mrow0 + 32 * b + acc_row(lane, r);
        if (m >= a.M) continue;
        const int ex = g.xe[(int64_t)l * a.tiles_m * kI8BM + m];
        double v = 0.0;
#pragma unroll
        for (int d = S - 1; d >= 0; --d) v += ldexp((double)acc[d][b][r], -7 * (d + 2));
        v = (ex == kExpNonFinite || ey == kExpNonFinite) ? __builtin_nan("") : ldexp(v, ex + ey);
        double* cp = at(C, (OffT)(a.cm[m] + cn));
        double out = a.alpha * v;
        if (a.beta != 0.0) out += a.beta * *cp;
        *cp = out;
      }
  };
  // Steps [st0, st1) through two LDS buffers and NL register sets: step st
  // is in set st % NL and buffer (st - st0) % 2.  A step first loads step
  // st + NL into its own set (stored into LDS by the step before), then
  // multiplies, then stores step st + 1 into the other buffer (its loads were
  // issued NL - 1 steps earlier): one barrier per step.
  auto multiply = [&](int buf) {
    const unsigned char* bx = smem + buf * (XB + YB);
    const unsigned char* by = bx + XB;
    i32x4 yf[S];
#pragma unroll
    for (int u = 0; u < S; ++u)
      yf[u] = *reinterpret_cast<const i32x4*>(&by[(u * kI8BN + wn * 32 + fr) * kI8StepPitch + fk]);
#pragma unroll
    for (int t2 = 0; t2 < S; ++t2) {
      const i32x4 x0 = *reinterpret_cast<const i32x4*>(&bx[(t2 * kI8BM + wm * 64 + fr) * kI8StepPitch + fk]);
      const i32x4 x1 = *reinterpret_cast<const i32x4*>(&bx[(t2 * kI8BM + wm * 64 + 32 + fr) * kI8StepPitch + fk]);
      // pairs (t2, u) with t2 + u <= S - 1 (0-based digits): diagonal d = t2 + u
#pragma unroll
      for (int u = 0; u + t2 < S; ++u) {
        acc[t2 + u][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(x0, yf[u], acc[t2 + u][0], 0, 0, 0);
        acc[t2 + u][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(x1, yf[u], acc[t2 + u][1], 0, 0, 0);
      }
    }
  };
  constexpr auto set0 = std::integral_constant<int, 0>{};
  fetch(set0, st0);
  if constexpr (NL == 2) fetch(std::integral_constant<int, 1>{}, st0 + 1);
  stash(set0, 0);
  __syncthreads();
  auto step = [&](auto qc, int st) {
    constexpr int Q = decltype(qc)::value;
    const int cur = (st - st0) & 1;
    const bool more = st + 1 < st1;
    if constexpr (NL == 1) {
      if (more) fetch(set0, st + 1);
    } else {
      fetch(qc, st + NL);
    }
    multiply(cur);
    if (more) stash(std::integral_constant<int, (Q + 1) % NL>{}, cur ^ 1);
    __syncthreads();
  };
  for (int st = st0; st < st1; st += NL) {
    step(set0, st);
    if constexpr (NL == 2)
      if (st + 1 < st1) step(std::integral_constant<int, 1>{}, st + 1);
  }
  update_c();
}

// ---------------------------------------------------------------- launch
template <typename OffT, int S, int MODE>
static void launch_slice_mode(const SliceArgs<OffT>& sa, int grid, hipStream_t s) {
  hipLaunchKernelGGL((int8_rowmax<OffT, MODE>), dim3(grid), dim3(kThreads), 0, s, sa);
  hipLaunchKernelGGL((int8_digits<OffT, S, MODE>), dim3(grid), dim3(kThreads), 0, s, sa);
}

template <typename OffT, int S>
static void launch_slice(const SliceArgs<OffT>& sa, int mode, hipStream_t s) {
  const int grid = sa.L * sa.tiles * (sa.tile_rows / kI8SliceRows) * sa.ksplit;
  if (mode == kSliceKVec)
    launch_slice_mode<OffT, S, kSliceKVec>(sa, grid, s);
  else if (mode == kSliceK)
    launch_slice_mode<OffT, S, kSliceK>(sa, grid, s);
  else
    launch_slice_mode<OffT, S, kSliceRows>(sa, grid, s);
}

// Workspace layout of an INT8 plan: X planes | Y planes | X exponents |
// Y exponents | X partial maxima | Y partial maxima.
struct Int8Layout {
  int64_t nkb, tm, tn, xsplit, xper, ysplit, yper;
  int64_t xplanes, yplanes, xexp, yexp, xmax, ymax;  // bytes
  Int8Layout(int S, int64_t M, int64_t N, int64_t K, int64_t L) {
    nkb = (K + kI8K - 1) / kI8K;
    tm = (M + kI8BM - 1) / kI8BM;
    tn = (N + kI8BN - 1) / kI8BN;
    int a, b;
    slice_split(L * tm * (kI8BM / kI8SliceRows), (int)nkb, &a, &b);
    xsplit = a;
    xper = b;
    slice_split(L * tn * (kI8BN / kI8SliceRows), (int)nkb, &a, &b);
    ysplit = a;
    yper = b;
    xplanes = L * S * tm * nkb * (kI8BM * kI8K);
    yplanes = L * S * tn * nkb * (kI8BN * kI8K);
    xexp = L * tm * kI8BM * 4;
    yexp = L * tn * kI8BN * 4;
    xmax = L * xsplit * tm * kI8BM * 8;
    ymax = L * ysplit * tn * kI8BN * 8;
  }
  int64_t total() const { return xplanes + yplanes + xexp + yexp + xmax + ymax; }
};

template <typename OffT, int S>
static hipError_t launch_int8_s(const PlainArgs<OffT>& a, int xmode, int ymode, hipStream_t s) {
  const Int8Layout lay(S, a.M, a.N, a.K, a.L);
  const int nkb = (int)lay.nkb;
  int8_t* xp = static_cast<int8_t*>(a.work);
  int8_t* yp = xp + lay.xplanes;
  int32_t* xe = reinterpret_cast<int32_t*>(yp + lay.yplanes);
  int32_t* ye = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(xe) + lay.xexp);
  double* xm = reinterpret_cast<double*>(reinterpret_cast<char*>(ye) + lay.yexp);
  double* ym = reinterpret_cast<double*>(reinterpret_cast<char*>(xm) + lay.xmax);
  SliceArgs<OffT> sx{a.x, a.xmn, a.xk, a.xl, xp, xe, xm, a.M, a.K, a.L, kI8BM, a.tiles_m, nkb,
                     (int)lay.xsplit, (int)lay.xper};
  SliceArgs<OffT> sy{a.y, a.ymn, a.yk, a.yl, yp, ye, ym, a.N, a.K, a.L, kI8BN, a.tiles_n, nkb,
                     (int)lay.ysplit, (int)lay.yper};
  launch_slice<OffT, S>(sx, xmode, s);
  launch_slice<OffT, S>(sy, ymode, s);
  // one launch per K chunk whose int32 sums stay exact, ordered on the stream
  const int chunk = int8_chunk_slices(S);
  const int grid = a.L * a.tiles_m * a.tiles_n;
  for (int kb0 = 0; kb0 < nkb; kb0 += chunk) {
    Int8GemmArgs<OffT> g{a, xp, yp, xe, ye, nkb, kb0, min(nkb, kb0 + chunk)};
    if (kb0 > 0) g.p.beta = 1.0;  // later chunks add to C
    hipLaunchKernelGGL((int8_gemm<OffT, S>), dim3(grid), dim3(kThreads), 0, s, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

template <typename OffT>
static hipError_t launch_int8_t(const PlainArgs<OffT>& a, int slices, int xmode, int ymode, hipStream_t s) {
  switch (slices) {
    case 3: return launch_int8_s<OffT, 3>(a, xmode, ymode, s);
    case 4: return launch_int8_s<OffT, 4>(a, xmode, ymode, s);
    case 5: return launch_int8_s<OffT, 5>(a, xmode, ymode, s);
    case 6: return launch_int8_s<OffT, 6>(a, xmode, ymode, s);
    case 7: return launch_int8_s<OffT, 7>(a, xmode, ymode, s);
    default: return hipErrorInvalidValue;
  }
}

// xmode / ymode: 0 row-gathered, 1 K-gathered, 2 K-gathered in affine blocks
hipError_t launch_int8(const PlainArgs<uint32_t>& a, int slices, int xmode, int ymode, hipStream_t s) {
  return launch_int8_t(a, slices, xmode, ymode, s);
}
hipError_t launch_int8(const PlainArgs<int64_t>& a, int slices, int xmode, int ymode, hipStream_t s) {
  return launch_int8_t(a, slices, xmode, ymode, s);
}

size_t int8_work_bytes(int slices, int64_t M, int64_t N, int64_t K, int64_t L) {
  return (size_t)Int8Layout(slices, M, N, K, L).total();
}

}  // namespace famlies
