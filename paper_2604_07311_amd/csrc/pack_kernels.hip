// Pre-packing of one operand into the kernel's tile order (the packing step
// hoisted out of repeated calls: Girder 2, "Enabling optimizations across
// layers" -- packing moved up into a higher layer so it is paid once for an
// operand that many contractions read).  Block (tile, kb) of the packed
// buffer is BR x BK elements stored [row][k], zero-filled past the problem
// edges, blocks ordered tile-major (tile * nkb + kb), batch planes back to
// back.  For the split-bf16 modes each block holds the NS bf16 part planes of
// the split that the kernels would otherwise do while staging.
#include "device.hpp"
#include "launch.hpp"
#include "runtime.hpp"

namespace famlies {

template <typename OffT>
struct PackArgs {
  const void* src;       // operand base (the lowest element in the 32-bit form)
  const OffT* mn;        // row offsets (padded to the tile grid)
  const OffT* ko;        // contracted offsets (padded)
  const int64_t* bl;     // batch offsets (elements)
  void* dst;
  int32_t R, K, L, tiles, nkb;
};

template <typename T, typename OffT, int BR, int BK>
__global__ __launch_bounds__(kThreads) void pack_plain(PackArgs<OffT> p) {
  const int64_t total = (int64_t)p.L * p.tiles * p.nkb * BR * BK;
  T* dst = static_cast<T*>(p.dst);
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total; e += (int64_t)gridDim.x * kThreads) {
    const int kin = (int)(e % BK);
    int64_t t = e / BK;
    const int r = (int)(t % BR);
    t /= BR;
    const int kb = (int)(t % p.nkb);
    t /= p.nkb;
    const int tile = (int)(t % p.tiles);
    const int l = (int)(t / p.tiles);
    const int m = tile * BR + r, k = kb * BK + kin;
    T v = T(0);
    if (m < p.R && k < p.K) v = *at(static_cast<const T*>(p.src) + p.bl[l], (OffT)(p.mn[m] + p.ko[k]));
    dst[e] = v;
  }
}

template <typename OffT, int BR, int NS>
__global__ __launch_bounds__(kThreads) void pack_split(PackArgs<OffT> p) {
  constexpr int BK = split_slice_k(NS);
  const int64_t total = (int64_t)p.L * p.tiles * p.nkb * BR * BK;
  __bf16* dst = static_cast<__bf16*>(p.dst);
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total; e += (int64_t)gridDim.x * kThreads) {
    const int kin = (int)(e % BK);
    int64_t t = e / BK;
    const int r = (int)(t % BR);
    const int64_t blk = t / BR;  // (l * tiles + tile) * nkb + kb
    const int kb = (int)(blk % p.nkb);
    const int tile = (int)((blk / p.nkb) % p.tiles);
    const int l = (int)(blk / p.nkb / p.tiles);
    const int m = tile * BR + r, k = kb * BK + kin;
    float x = 0.f;
    if (m < p.R && k < p.K) x = *at(static_cast<const float*>(p.src) + p.bl[l], (OffT)(p.mn[m] + p.ko[k]));
    __bf16* out = dst + blk * (int64_t)(NS * BR * BK) + r * BK + kin;
#pragma unroll
    for (int q = 0; q < NS; ++q) {  // the same RNE split as the kernels' staging
      const __bf16 h = static_cast<__bf16>(x);
      out[q * BR * BK] = h;
      x = x - static_cast<float>(h);
    }
  }
}

template <typename OffT>
static hipError_t launch_pack_t(const PackArgs<OffT>& a, int dtype, int ns, int br, int bk, hipStream_t s) {
  const int64_t total = (int64_t)a.L * a.tiles * a.nkb * br * bk;
  const int grid = (int)std::min<int64_t>((total + kThreads - 1) / kThreads, 8192);
  if (ns == 0) {
    if (dtype == FAMLIES_F64 && br == 128 && bk == 8)
      hipLaunchKernelGGL((pack_plain<double, OffT, 128, 8>), dim3(grid), dim3(kThreads), 0, s, a);
    else if (dtype == FAMLIES_F64 && br == 64 && bk == 8)
      hipLaunchKernelGGL((pack_plain<double, OffT, 64, 8>), dim3(grid), dim3(kThreads), 0, s, a);
    else if (dtype == FAMLIES_F32 && br == 128 && bk == 32)
      hipLaunchKernelGGL((pack_plain<float, OffT, 128, 32>), dim3(grid), dim3(kThreads), 0, s, a);
    else if (dtype == FAMLIES_F32 && br == 64 && bk == 32)
      hipLaunchKernelGGL((pack_plain<float, OffT, 64, 32>), dim3(grid), dim3(kThreads), 0, s, a);
    else
      return hipErrorInvalidValue;
  } else if (bk != split_slice_k(ns)) {
    return hipErrorInvalidValue;
  } else if (ns == 2 && br == 256) {
    hipLaunchKernelGGL((pack_split<OffT, 256, 2>), dim3(grid), dim3(kThreads), 0, s, a);
  } else if (ns == 2 && br == 128) {
    hipLaunchKernelGGL((pack_split<OffT, 128, 2>), dim3(grid), dim3(kThreads), 0, s, a);
  } else if (ns == 2 && br == 64) {
    hipLaunchKernelGGL((pack_split<OffT, 64, 2>), dim3(grid), dim3(kThreads), 0, s, a);
  } else if (ns == 3 && br == 128) {
    hipLaunchKernelGGL((pack_split<OffT, 128, 3>), dim3(grid), dim3(kThreads), 0, s, a);
  } else if (ns == 3 && br == 64) {
    hipLaunchKernelGGL((pack_split<OffT, 64, 3>), dim3(grid), dim3(kThreads), 0, s, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pack(const PackArgs<uint32_t>& a, int dtype, int ns, int br, int bk, hipStream_t s) {
  return launch_pack_t(a, dtype, ns, br, bk, s);
}

}  // namespace famlies

using namespace famlies;

namespace {

// Kernel-view side of a user operand, whether the plan can pack it, and the
// packed geometry.
struct PackGeom {
  bool x;         // the operand is the kernel's X (rows M) rather than Y (rows N)
  int br, bk;     // block shape
  int64_t rows, tiles, nkb;
  size_t bytes;
};

famlies_status pack_geom(famlies_plan_s* p, int operand, PackGeom* g) {
  if (!p || p->batch) return fail(FAMLIES_ERR_INVALID_ARG, "pack: invalid plan");
  if (operand != 0 && operand != 1) return fail(FAMLIES_ERR_INVALID_ARG, "pack: operand must be 0 (A) or 1 (B)");
  const Analysis& an = p->an;
  const int ns = split_parts(an.compute);
  if (int8_slices(an.compute)) return fail(FAMLIES_ERR_UNSUPPORTED, "pack: INT8 plans slice their operands themselves");
  g->x = (operand == 0) != an.swapped;
  g->br = g->x ? p->cfg.bm : p->cfg.bn;
  g->bk = p->cfg.bk;
  const bool tile_ok = ns ? split_tile_supported(ns, p->cfg.bm, p->cfg.bn)
                          : plain_tile_supported(an.dtype, p->cfg.bm, p->cfg.bn, p->cfg.bk);
  if (!tile_ok || p->index_bits != 32 || p->elem32)
    return fail(FAMLIES_ERR_UNSUPPORTED, "pack: an operand of this plan spans 4 GiB or more (no packed kernel)");
  if (an.M == 0 || an.N == 0 || an.K == 0) return fail(FAMLIES_ERR_UNSUPPORTED, "pack: empty problem");
  g->rows = g->x ? an.M : an.N;
  g->tiles = (g->rows + g->br - 1) / g->br;
  g->nkb = (an.K + g->bk - 1) / g->bk;
  const size_t es = ns ? 2 * (size_t)ns : (size_t)an.esize;
  g->bytes = (size_t)an.L * (size_t)g->tiles * (size_t)g->nkb * (size_t)g->br * (size_t)g->bk * es;
  return FAMLIES_OK;
}

}  // namespace

namespace famlies {

famlies_status pack_size_impl(famlies_plan_s* p, int operand, size_t* bytes) {
  if (!bytes) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_pack_size: null output");
  PackGeom g;
  famlies_status st = pack_geom(p, operand, &g);
  if (st != FAMLIES_OK) return st;
  *bytes = g.bytes;
  return FAMLIES_OK;
}

famlies_status pack_impl(famlies_plan_s* p, int operand, const void* src, void* dst, void* stream) {
  PackGeom g;
  famlies_status st = pack_geom(p, operand, &g);
  if (st != FAMLIES_OK) return st;
  if (!src || !dst) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_pack: null pointer");
  const Analysis& an = p->an;
  const uintptr_t al = (uintptr_t)an.esize - 1;
  if (((uintptr_t)src & al) || ((uintptr_t)dst & 15))
    return fail(FAMLIES_ERR_ALIGN, "famlies_pack: src must be element-aligned, dst 16-byte aligned");
  DeviceGuard dg(p->h->device);
  if (!dg.ok) return fail(FAMLIES_ERR_DEVICE, "cannot select the plan's device");
  const uint32_t* o = static_cast<const uint32_t*>(p->d_off);
  const int64_t* lb = reinterpret_cast<const int64_t*>(static_cast<const char*>(p->d_off) + p->batch_off_bytes);
  PackArgs<uint32_t> a;
  const int64_t es = an.esize;
  a.src = static_cast<const char*>(src) + (g.x ? an.x_lo : an.y_lo) * es;
  a.mn = o + p->off_pos[g.x ? 0 : 3];
  a.ko = o + p->off_pos[g.x ? 1 : 2];
  a.bl = lb + p->off_pos[g.x ? 6 : 7];
  a.dst = dst;
  a.R = (int32_t)g.rows;
  a.K = (int32_t)an.K;
  a.L = (int32_t)an.L;
  a.tiles = (int32_t)g.tiles;
  a.nkb = (int32_t)g.nkb;
  hipError_t e = launch_pack(a, an.dtype, split_parts(an.compute), g.br, g.bk, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "pack kernel launch");
  return FAMLIES_OK;
}

}  // namespace famlies

extern "C" {

famlies_status famlies_pack_size(famlies_plan tok, int operand, size_t* bytes) {
  return pack_size_impl(plan_of(tok), operand, bytes);
}

famlies_status famlies_pack(famlies_plan tok, int operand, const void* src, void* dst, void* stream) {
  return pack_impl(plan_of(tok), operand, src, dst, stream);
}

}  // extern "C"
