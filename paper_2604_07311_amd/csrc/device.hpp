// Device building blocks of the contraction kernels (gfx950 / CDNA4).
//
// Structure follows the paper's GEMM layering (the BLIS refactoring as loops
// around a micro-kernel with packed operands, Fig. "five loops around the
// micro-kernel"), re-cut for a GPU: the workgroup grid replaces the outer
// cache-blocking loops, the block-scatter gather into LDS replaces packing
// into contiguous panels (Approach, "Supporting tensor computations"), and
// wave-level MFMA tiles replace the register micro-kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "args.hpp"

namespace famlies {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;  // 4 waves of 64 lanes
constexpr int kXcds = 8;       // MI355X: 8 XCDs, 32 CUs each

// Workgroups are dealt round-robin to the XCDs (id % 8).  Renumber them so
// that consecutive logical tile ids land on the same XCD and share its L2.
__device__ __forceinline__ int xcd_remap(int bid, int total) {
  int q = total / kXcds, r = total % kXcds;
  int xcd = bid % kXcds, idx = bid / kXcds;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// Element at `off` from `base`: uint32_t offsets count bytes (an SGPR base
// plus a 32-bit VGPR offset per load); int32_t and int64_t offsets count
// elements (int32_t for operands past 4 GiB but under 2^31 elements: 32-bit
// registers per offset like the byte form).
template <typename T>
__device__ __forceinline__ T* at(T* base, uint32_t off) {
  typedef typename std::conditional<std::is_const<T>::value, const char, char>::type byte;
  return reinterpret_cast<T*>(reinterpret_cast<byte*>(base) + off);
}
template <typename T>
__device__ __forceinline__ T* at(T* base, int32_t off) {
  return base + (int64_t)off;
}
template <typename T>
__device__ __forceinline__ T* at(T* base, int64_t off) {
  return base + off;
}

// Offsets that count bytes (the uint32_t form) rather than elements.
template <typename OffT>
constexpr bool kByteOffsets = std::is_same<OffT, uint32_t>::value;

// Operands always live in global memory.  Loads and stores through these
// helpers say so, so they compile to global (not flat) instructions even when
// the pointer was read from memory, as in the batched kernel: a flat load
// takes a 64-bit VGPR address and is counted by the LDS wait counter too.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* global(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* global(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}
template <typename T, typename OffT>
__device__ __forceinline__ T gload(const T* base, OffT off) {
  return *global(at(base, off));
}

// MFMA shapes.  In every shape the lane index l selects the row (of the left
// operand) and the column (of the right operand) as l % BS, and the group
// l / BS selects the contraction index, the same way for both operands, so
// any consistent assignment of tile k's to (group, step) is valid.
template <typename T>
struct Mfma;

template <>
struct Mfma<double> {  // v_mfma_f64_16x16x4_f64
  static constexpr int BS = 16, KG = 4, NACC = 4;
  using Acc = f64x4;
  __device__ __forceinline__ static Acc mma(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of accumulator element r held by lane l (column is l % 16)
  __device__ __forceinline__ static int row(int l, int r) { return (l / 16) + 4 * r; }
};

template <>
struct Mfma<float> {  // v_mfma_f32_32x32x2_f32
  static constexpr int BS = 32, KG = 2, NACC = 16;
  using Acc = f32x16;
  __device__ __forceinline__ static Acc mma(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int l, int r) {
    return 8 * (r / 4) + 4 * (l / 32) + (r % 4);
  }
};

// Gather of one operand tile (BR rows of the free dimension x BK contracted
// indices) from strided global memory through the block-scatter indexing
// vectors into LDS laid out [row][k] with leading dimension LDK (16-byte
// aligned rows, padded by 16 bytes so that the MFMA operand reads and the
// stores below are free of bank conflicts).
//
// KFAST (the operand's smallest stride is a contracted mode): lanes run along
// k; each thread owns KV consecutive k's (KV = 1 for the plain kernels, 2 for
// the bf16 split, whose stores pack pairs) in E / KV rows.
// Row-fast (otherwise): lanes run along the rows, each thread owns one row and
// a run of E consecutive k's, stored to LDS as 16-byte vectors.
// Rows past the problem edge carry offset 0 (a valid address) and only feed
// accumulator rows that are never stored; k's past the edge are stored as 0.
//
// The phases are split so a K loop can pipeline them: fetch_k() loads the
// contracted-index offsets of a future slice, load() issues the data loads of
// the next slice (nothing waits on them until store()), store() writes the
// slice into LDS, zeroing k >= kend.  Element j of a thread is
// (row j / KV, k j % KV) in the KFAST case and (row 0, k j) otherwise.
// NSLOT > 1 keeps that many slices in flight: each phase takes the slot it
// works on as a template argument.
template <typename T, typename OffT, int BR, int BK, bool KFAST, int KV = 1, int NSLOT = 1>
struct TileGather {
  static constexpr int E = BR * BK / kThreads;
  static constexpr int KVT = KV;                  // KFAST: consecutive k's per thread
  static constexpr int LDK = BK + 16 / (int)sizeof(T);
  static constexpr int VK = 16 / (int)sizeof(T);  // k's per 16-byte vector
  static constexpr int KT = BK / KV;              // KFAST: threads along k
  static constexpr int RSTEP = kThreads / KT;     // KFAST: row step between a thread's rows
  static constexpr int KPH = kThreads / BR;       // row-fast: threads sharing one row
  static_assert(E >= 1 && E % KV == 0, "tile too small for the workgroup");
  static_assert(KFAST ? (kThreads % KT == 0 && BR % RSTEP == 0)
                      : (kThreads % BR == 0 && BK % KPH == 0 && E % VK == 0),
                "tile shape does not divide the workgroup");

  OffT mn[KFAST ? E / KV : 1];  // row offsets, fixed for the tile
  OffT ko[NSLOT][KFAST ? KV : E];  // contracted-index offsets of a slice to load
  T v[NSLOT][E];
  int r0, kk0;  // first row; first k of the thread's run

  __device__ __forceinline__ void init(const OffT* __restrict__ mnoff, int tile_r0, int tid) {
    if constexpr (KFAST) {
      kk0 = (tid % KT) * KV;
      r0 = tid / KT;
#pragma unroll
      for (int i = 0; i < E / KV; ++i) mn[i] = mnoff[tile_r0 + r0 + i * RSTEP];
    } else {
      r0 = tid % BR;
      // The k run is the same for a whole wave, but its offsets are fetched
      // with vector loads on purpose: scalar loads share the LDS wait
      // counter, and every wait for an MFMA operand read would then also wait
      // for the offsets of a slice two steps ahead.
      kk0 = (tid / BR) * E;
      mn[0] = mnoff[tile_r0 + r0];
    }
  }

  // Offsets of slice [k0, k0 + BK); koff must hold k0 + BK entries.  Row-fast
  // runs are read as 16-byte vectors: every indexing vector starts on a
  // 64-byte boundary and k0 + kk0 is a multiple of E.
  static constexpr int OV = 16 / (int)sizeof(OffT);
  template <int S = 0>
  __device__ __forceinline__ void fetch_k(const OffT* __restrict__ koff, int k0) {
    if constexpr (!KFAST && E % OV == 0) {
      typedef OffT ovec_t __attribute__((ext_vector_type(16 / sizeof(OffT))));
      const ovec_t* src = reinterpret_cast<const ovec_t*>(koff + k0 + kk0);
#pragma unroll
      for (int q = 0; q < E / OV; ++q) {
        const ovec_t w = src[q];
#pragma unroll
        for (int u = 0; u < OV; ++u) ko[S][q * OV + u] = w[u];
      }
    } else {
#pragma unroll
      for (int u = 0; u < (KFAST ? KV : E); ++u) ko[S][u] = koff[k0 + kk0 + u];
    }
  }

  template <int S = 0>
  __device__ __forceinline__ void load(const T* __restrict__ base) {
#pragma unroll
    for (int j = 0; j < E; ++j)
      v[S][j] = KFAST ? gload(base, (OffT)(mn[j / KV] + ko[S][j % KV])) : gload(base, (OffT)(mn[0] + ko[S][j]));
  }

  __device__ __forceinline__ int krel(int j) const { return kk0 + (KFAST ? j % KV : j); }

  // Value of element j of the slice starting at k0 (0 past kend).
  template <int S = 0>
  __device__ __forceinline__ T value(int j, int k0, int kend) const {
    return k0 + krel(j) < kend ? v[S][j] : T(0);
  }

  // value() where EDGE, the raw element otherwise (slices wholly inside K).
  template <bool EDGE, int S = 0>
  __device__ __forceinline__ T val(int j, int k0, int kend) const {
    return EDGE ? value<S>(j, k0, kend) : v[S][j];
  }

  __device__ __forceinline__ int lds_index(int j, int ldk) const {
    return KFAST ? (r0 + (j / KV) * RSTEP) * ldk + kk0 + j % KV : r0 * ldk + kk0 + j;
  }

  // Store the slice to LDS, zeroing k's past kend.  Only the last slice of a
  // K range can hold such k's, so the test is skipped (a uniform branch) on
  // every other slice.
  template <bool EDGE, int S>
  __device__ __forceinline__ void store_impl(T* __restrict__ lds, int k0, int kend) const {
    if constexpr (KFAST) {
#pragma unroll
      for (int j = 0; j < E; ++j) lds[lds_index(j, LDK)] = val<EDGE, S>(j, k0, kend);
    } else {
      typedef T vec_t __attribute__((ext_vector_type(16 / sizeof(T))));
#pragma unroll
      for (int q = 0; q < E / VK; ++q) {
        vec_t w;
#pragma unroll
        for (int u = 0; u < VK; ++u) w[u] = val<EDGE, S>(q * VK + u, k0, kend);
        *reinterpret_cast<vec_t*>(lds + r0 * LDK + kk0 + q * VK) = w;
      }
    }
  }
  template <int S = 0>
  __device__ __forceinline__ void store(T* __restrict__ lds, int k0, int kend) const {
    if (k0 + BK <= kend)
      store_impl<false, S>(lds, k0, kend);
    else
      store_impl<true, S>(lds, k0, kend);
  }
};

// Loader for a pre-packed operand (the packing step hoisted out of repeated
// calls: Girder 2, "Enabling optimizations across layers").  The packed
// buffer holds the operand tile by tile in the kernel's order: block
// (tile, kb) is BR x BK elements stored [row][k] densely, zero-filled past the
// problem edges, blocks ordered tile-major (tile * nkb + kb).  A slice is then
// a contiguous run of 16-byte vectors: no indexing vectors, no edge tests.
template <typename T, int BR, int BK, int NSLOT = 1>
struct PackedGather {
  static constexpr int VK = 16 / (int)sizeof(T);
  static constexpr int LDK = BK + VK;
  static constexpr int NV = BR * BK / VK;  // vectors per block
  static constexpr int VPT = NV / kThreads;
  static_assert(NV % kThreads == 0 && BK % VK == 0, "packed block does not divide the workgroup");
  typedef T vec_t __attribute__((ext_vector_type(16 / sizeof(T))));
  vec_t v[NSLOT][VPT];
  int tile = 0, kb[NSLOT] = {}, nkb = 1, tid = 0;

  template <typename OffT>
  __device__ __forceinline__ void init(const OffT* /*unused*/, int tile_r0, int t) {
    tile = tile_r0 / BR;
    tid = t;
  }
  template <int S = 0, typename OffT>
  __device__ __forceinline__ void fetch_k(const OffT* /*unused*/, int k0) {
    kb[S] = k0 / BK;
  }
  template <int S = 0>
  __device__ __forceinline__ void load(const T* __restrict__ base) {
    const vec_t* blk = reinterpret_cast<const vec_t*>(base + ((size_t)tile * nkb + kb[S]) * (size_t)(BR * BK));
#pragma unroll
    for (int q = 0; q < VPT; ++q) v[S][q] = *global(blk + tid + q * kThreads);
  }
  template <int S = 0>
  __device__ __forceinline__ void store(T* __restrict__ lds, int /*k0*/, int /*kend*/) const {
#pragma unroll
    for (int q = 0; q < VPT; ++q) {
      const int e = (tid + q * kThreads) * VK;
      *reinterpret_cast<vec_t*>(lds + (e / BK) * LDK + e % BK) = v[S][q];
    }
  }
};

// Loader for a K-gathered operand stored in affine blocks (the block-scatter
// layout's block strides, Approach, "Supporting tensor computations"): in
// every BK-slice of K the indexing vector is a progression of step one
// element, and every run start is 16-byte aligned, so a row's slice is a
// contiguous run in memory.  Each thread reads VK consecutive k's of a row
// with one 16-byte load instead of VK gathered loads and takes one offset per
// slice.  Every slice is whole (the planner takes this loader only when BK
// divides K, and split-K chunks are whole slices): a load with a fallback
// for a partial slice made the compiler copy the other operand's freshly
// loaded registers at the join, waiting for those loads on every step.
template <typename T, typename OffT, int BR, int BK, int NSLOT = 1>
struct VecKGather {
  static constexpr int VK = 16 / (int)sizeof(T);
  // one element in offset units: bytes for the byte form, else 1
  static constexpr int kStep = kByteOffsets<OffT> ? (int)sizeof(T) : 1;
  static constexpr int LDK = BK + VK;
  static constexpr int KT = BK / VK;           // threads along k
  static constexpr int RSTEP = kThreads / KT;  // rows between a thread's runs
  static constexpr int NR = BR / RSTEP;        // runs per thread
  static_assert(BK % VK == 0 && kThreads % KT == 0 && BR % RSTEP == 0, "tile shape does not divide the workgroup");
  typedef T vec_t __attribute__((ext_vector_type(16 / sizeof(T))));
  OffT mn[NR];
  OffT ko[NSLOT];
  vec_t v[NSLOT][NR];
  int r0 = 0, kk0 = 0;

  __device__ __forceinline__ void init(const OffT* __restrict__ mnoff, int tile_r0, int tid) {
    kk0 = (tid % KT) * VK;
    r0 = tid / KT;
#pragma unroll
    for (int i = 0; i < NR; ++i) mn[i] = mnoff[tile_r0 + r0 + i * RSTEP];
  }
  template <int S = 0>
  __device__ __forceinline__ void fetch_k(const OffT* __restrict__ koff, int k0) {
    ko[S] = koff[k0 + kk0];
  }
  template <int S = 0>
  __device__ __forceinline__ void load(const T* __restrict__ base) {
#pragma unroll
    for (int i = 0; i < NR; ++i) v[S][i] = *global(reinterpret_cast<const vec_t*>(at(base, (OffT)(mn[i] + ko[S]))));
  }
  template <int S = 0>
  __device__ __forceinline__ void store(T* __restrict__ lds, int /*k0*/, int /*kend*/) const {
#pragma unroll
    for (int i = 0; i < NR; ++i) *reinterpret_cast<vec_t*>(lds + (r0 + i * RSTEP) * LDK + kk0) = v[S][i];
  }
};

// Operand loaders by mode: 0 row-gathered, 1 K-gathered, 2 pre-packed,
// 3 K-gathered from affine unit-stride blocks.
enum { kRowGather = 0, kKGather = 1, kPacked = 2, kVecK = 3 };
template <int MODE>
constexpr bool known_mode() {
  static_assert(MODE >= kRowGather && MODE <= kVecK, "unknown loader mode");
  return true;
}
template <typename T, typename OffT, int BR, int BK, int MODE, int KV = 1, int NSLOT = 1,
          bool = known_mode<MODE>()>
using Loader = typename std::conditional<
    MODE == kPacked, PackedGather<T, BR, BK, NSLOT>,
    typename std::conditional<MODE == kVecK, VecKGather<T, OffT, BR, BK, NSLOT>,
                              TileGather<T, OffT, BR, BK, MODE == kKGather, KV, NSLOT>>::type>::type;

}  // namespace famlies
