// C ABI: handles, plans, planning (tile choice, indexing-vector upload) and
// execution.  Errors are returned as famlies_status with a thread-local
// message (graceful error handling and bounds checking: Girder 1, "Code
// safety").
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "famlies.h"
#include "internal.hpp"
#include "launch.hpp"
#include "runtime.hpp"

// Device scratch of famlies_contract_noalloc: the indexing vectors and
// split-K partial sums of the call in flight, one copy per device, held until
// the process ends.  Host code never passes `scratch` itself to a kernel or
// a copy (in host code the name is only a stand-in): the device address is
// resolved per device with hipGetSymbolAddress and kept (g_scratch_addr).
static constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace famlies {

static std::mutex g_scratch_mu;
static void* g_scratch_addr[64] = {};

// The scratch array's address on `device` (resolved once, with that device
// current).
static famlies_status scratch_address(int device, void** out) {
  if (device < 0 || device >= 64) return fail(FAMLIES_ERR_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    DeviceGuard dg(device);
    if (!dg.ok) return fail(FAMLIES_ERR_DEVICE, "cannot select the device");
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(FAMLIES_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned null");
    g_scratch_addr[device] = ptr;
  }
  *out = g_scratch_addr[device];
  return FAMLIES_OK;
}

famlies_status hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? FAMLIES_ERR_ALLOC : FAMLIES_ERR_DEVICE;
}

// Make `device` current for the scope, restoring the caller's device after.
DeviceGuard::DeviceGuard(int device) {
  ok = hipGetDevice(&prev) == hipSuccess;
  if (ok && prev != device) ok = hipSetDevice(device) == hipSuccess;
  else if (ok) prev = -1;
}
DeviceGuard::~DeviceGuard() {
  if (prev >= 0) (void)hipSetDevice(prev);
}

template <typename OffT>
static famlies_status index_image(famlies_plan_s* p, int64_t mp, int64_t np, int64_t kp, std::vector<char>* image) {
  const Analysis& an = p->an;
  std::vector<int64_t> v[9];
  offsets(an.I, 0, an.M, mp, v[0]);
  offsets(an.P, 0, an.K, kp, v[1]);
  offsets(an.P, 1, an.K, kp, v[2]);
  offsets(an.J, 1, an.N, np, v[3]);
  offsets(an.I, 2, an.M, mp, v[4]);
  offsets(an.J, 2, an.N, np, v[5]);
  offsets(an.Lm, 0, an.L, an.L, v[6]);
  offsets(an.Lm, 1, an.L, an.L, v[7]);
  offsets(an.Lm, 2, an.L, an.L, v[8]);
  // 32-bit forms rebase the row vectors to each operand's lowest element;
  // the byte form also scales every offset to bytes
  const bool rebase = sizeof(OffT) == 4, bytes = std::is_same<OffT, uint32_t>::value;
  const int64_t es = an.esize;
  vec_flags(an, p->cfg.bk, sizeof(OffT) == 4 ? 32 : 64, v, &p->x_vec, &p->y_vec);
  const int64_t shift[6] = {an.x_lo, 0, 0, an.y_lo, an.c_lo_mn, 0};
  size_t n6 = 0;
  for (int i = 0; i < 6; ++i) n6 += v[i].size();
  const size_t b6 = (n6 * sizeof(OffT) + 7) & ~(size_t)7;
  const size_t total = b6 + 3 * (size_t)an.L * sizeof(int64_t);
  std::vector<char>& host = *image;
  host.assign(total, 0);
  OffT* o = reinterpret_cast<OffT*>(host.data());
  size_t pos = 0;
  for (int i = 0; i < 6; ++i) {
    p->off_pos[i] = pos;
    for (int64_t x : v[i]) {
      if (bytes)
        o[pos++] = (OffT)(uint64_t)((x - shift[i]) * es);  // wraps modulo 2^32 on purpose
      else if (rebase)
        o[pos++] = (OffT)(x - shift[i]);  // |value| < 2^31 (index_form)
      else
        o[pos++] = (OffT)x;
    }
  }
  int64_t* lb = reinterpret_cast<int64_t*>(host.data() + b6);
  for (int i = 0; i < 3; ++i) {
    p->off_pos[6 + i] = (size_t)i * (size_t)an.L;
    for (int64_t l = 0; l < an.L; ++l) lb[i * an.L + l] = v[6 + i][(size_t)l];
  }
  p->batch_off_bytes = b6;
  // host-side bounds check of the vectors against the descriptors' spans
  const int64_t x_lo = an.swapped ? an.b_lo : an.a_lo, x_hi = an.swapped ? an.b_hi : an.a_hi;
  const int64_t y_lo = an.swapped ? an.a_lo : an.b_lo, y_hi = an.swapped ? an.a_hi : an.b_hi;
  if ((an.K > 0 && (!offsets_in_span(v[0], an.M, v[1], an.K, v[6], an.L, x_lo, x_hi) ||
                    !offsets_in_span(v[3], an.N, v[2], an.K, v[7], an.L, y_lo, y_hi))) ||
      !offsets_in_span(v[4], an.M, v[5], an.N, v[8], an.L, an.c_lo, an.c_hi))
    return fail(FAMLIES_ERR_BOUNDS, "planner: an indexing vector addresses outside its tensor's span");
  return FAMLIES_OK;
}

template <typename OffT>
static PlainArgs<OffT> make_args(const famlies_plan_s* p, const void* x, const void* y, void* c,
                                 double alpha, double beta) {
  PlainArgs<OffT> a;
  const OffT* o = static_cast<const OffT*>(p->d_off);
  const int64_t* lb = reinterpret_cast<const int64_t*>(static_cast<const char*>(p->d_off) + p->batch_off_bytes);
  const bool rebased = sizeof(OffT) == 4;
  const int64_t es = p->an.esize;
  // in the 32-bit forms the kernel addresses each operand from its lowest element
  a.x = x ? static_cast<const char*>(x) + (rebased ? p->an.x_lo * es : 0) : nullptr;
  a.y = y ? static_cast<const char*>(y) + (rebased ? p->an.y_lo * es : 0) : nullptr;
  a.c = static_cast<char*>(c) + (rebased ? p->an.c_lo_mn * es : 0);
  a.xmn = o + p->off_pos[0];
  a.xk = o + p->off_pos[1];
  a.yk = o + p->off_pos[2];
  a.ymn = o + p->off_pos[3];
  a.cm = o + p->off_pos[4];
  a.cn = o + p->off_pos[5];
  a.xl = lb + p->off_pos[6];
  a.yl = lb + p->off_pos[7];
  a.cl = lb + p->off_pos[8];
  a.M = (int32_t)p->an.M;
  a.N = (int32_t)p->an.N;
  a.K = (int32_t)p->an.K;
  a.L = (int32_t)p->an.L;
  a.x_nkb = 0;
  a.y_nkb = 0;
  a.tiles_m = (int32_t)ceil_div(p->an.M, p->cfg.bm);
  a.tiles_n = (int32_t)ceil_div(p->an.N, p->cfg.bn);
  a.splits = p->cfg.split;
  a.kchunk = p->kchunk;
  a.head = p->head;
  a.alpha = alpha;
  a.beta = beta;
  a.work = p->d_work;
  return a;
}

// Planning decisions and the host image of the indexing vectors, touching no
// device memory: p->cfg, the split settlement, the loader flags, the vector
// positions and p->work_bytes (the split-K workspace the plan needs).
// *image is left empty when C has no elements.
static famlies_status prepare_plan(famlies_handle_s* h, famlies_plan_s* p, int dtype, int compute,
                                   const famlies_tensor* A, const famlies_tensor* B, const famlies_tensor* C,
                                   const TileCfg* force, std::vector<char>* image) {
  Analysis an;
  std::string err;
  int st = analyze(dtype, compute, A, B, C, &an, &err);
  if (st != FAMLIES_OK) return fail(st, err);
  const int64_t lim = kMaxGemmDim;
  if (an.M > lim || an.N > lim || an.K > lim || an.L > lim)
    return fail(FAMLIES_ERR_UNSUPPORTED, "a GEMM dimension exceeds 2^31 - 1024");
  p->h = h;
  p->an = an;
  const int i8 = int8_slices(compute);
  p->cfg = i8 ? int8_tile() : force ? *force : choose_tiles(h, an, &p->table_hit);
  if (i8 && force) p->cfg.index_bits = force->index_bits;
  index_form(an, p->cfg.index_bits, &p->index_bits, &p->elem32);
  const int ns = split_parts(compute);
  if (i8) {
    // fixed tile (int8_tile): no split-K, no tile table
  } else if (ns) {
    // the bf16 kernels split every tile or none: a tail split becomes none
    if (p->cfg.tail) {
      p->cfg.split = 1;
      p->cfg.tail = 0;
    }
    p->cfg.bk = split_slice_k(ns);
    // bf16x3 on large problems: a 256 x 128 tile (128 x 64 per wave) halves
    // the LDS bytes per MFMA of the 128 x 128 tile (bf16x6 stays at 128 x 128
    // with 16-deep slices, two workgroups per CU).  It has registers for
    // one slice in flight and one workgroup per CU, so it is taken only when
    // both operands are element-gathered along K: a row-gathered operand
    // keeps the 128 x 128 tile with two slices in flight (ring o=48 v=192:
    // 186 -> 201 TFLOP/s FP32-equivalent), and an affine-block operand the
    // 128 x 128 tile at two workgroups per CU (ladder v=128 o=32: 284 -> 307).
    if (!force && ns == 2 && an.M >= 1024 && an.N >= 512 && p->cfg.split == 1 && an.x_kfast && an.y_kfast) {
      std::vector<int64_t> v[9];
      bool xv = false, yv = false;
      all_offsets(an, v);
      vec_flags(an, 32, index_bits_for(an), v, &xv, &yv);
      if (!xv && !yv) {
        p->cfg.bm = 256;
        p->cfg.bn = 128;
      }
    }
    if (!split_tile_supported(ns, p->cfg.bm, p->cfg.bn)) p->cfg.bm = p->cfg.bn = 128;
  } else if (!plain_tile_supported(dtype, p->cfg.bm, p->cfg.bn, p->cfg.bk)) {
    p->cfg.bm = p->cfg.bn = 128;
    p->cfg.bk = dtype == FAMLIES_F64 ? 8 : 32;
  }
  if (an.L > 1) p->cfg.split = 1;  // batch modes already multiply the tile count
  const int64_t ntiles = ceil_div(an.M, p->cfg.bm) * ceil_div(an.N, p->cfg.bn);
  finalize_split(&p->cfg, an.K, ntiles, &p->kchunk, &p->head);
  if (ntiles * p->cfg.split * an.L >= ((int64_t)1 << 31))
    return fail(FAMLIES_ERR_UNSUPPORTED, "the tile grid exceeds 2^31 workgroups");
  image->clear();
  p->work_bytes = 0;
  if (an.M == 0 || an.N == 0) return FAMLIES_OK;
  const int64_t mp = ceil_div(std::max<int64_t>(an.M, 1), p->cfg.bm) * p->cfg.bm;
  const int64_t np = ceil_div(std::max<int64_t>(an.N, 1), p->cfg.bn) * p->cfg.bn;
  const int64_t kp = ceil_div(std::max<int64_t>(an.K, 1), p->cfg.bk) * p->cfg.bk + p->cfg.bk;
  st = p->index_bits == 64 ? index_image<int64_t>(p, mp, np, kp, image)
       : p->elem32          ? index_image<int32_t>(p, mp, np, kp, image)
                            : index_image<uint32_t>(p, mp, np, kp, image);
  if (st != FAMLIES_OK) return st;
  if (i8 && an.K > 0) {
    p->work_bytes = int8_work_bytes(i8, an.M, an.N, an.K, an.L);  // digit planes and exponents
  } else if (p->cfg.split > 1 && an.K > 0) {
    // plain kernels: one BM x BN block per split tile and K slice; bf16
    // kernels: one padded M x N plane of FP64 sums per K slice
    p->work_bytes = ns ? (size_t)p->cfg.split * (size_t)mp * (size_t)np * 8
                       : (size_t)p->cfg.split * (size_t)(ntiles - p->head) * (size_t)p->cfg.bm *
                             (size_t)p->cfg.bn * (size_t)an.esize;
  }
  return FAMLIES_OK;
}

famlies_status make_plan(famlies_handle h, famlies_plan* out, int dtype, int compute,
                         const famlies_tensor* A, const famlies_tensor* B, const famlies_tensor* C,
                         const TileCfg* force) {
  if (!out) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_plan_contract: null output pointer");
  *out = nullptr;
  if (!h) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_plan_contract: invalid handle");
  DeviceGuard dg(h->device);
  if (!dg.ok) return fail(FAMLIES_ERR_DEVICE, "cannot select the handle's device");
  auto* p = new (std::nothrow) famlies_plan_s();
  if (!p) return fail(FAMLIES_ERR_ALLOC, "out of host memory");
  struct Owner {  // frees the plan on every early return and if planning throws
    famlies_plan_s** q;
    ~Owner() {
      if (*q) delete *q;
    }
  } owner{&p};
  std::vector<char> image;
  famlies_status st = prepare_plan(h, p, dtype, compute, A, B, C, force, &image);
  if (st != FAMLIES_OK) return st;
  if (!image.empty()) {
    hipError_t e = hipMalloc(&p->d_off, image.size());
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(indexing vectors)");
    e = hipMemcpy(p->d_off, image.data(), image.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(indexing vectors)");
  }
  if (p->work_bytes) {
    hipError_t e = hipMalloc(&p->d_work, p->work_bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(split-K workspace)");
  }
  if (log_enabled()) log_plan(p);
  *out = p;
  p = nullptr;  // owned by the caller now
  return FAMLIES_OK;
}

void log_plan(const famlies_plan_s* p) {
  log_decision("plan", p->an, p->cfg, p->elem32 ? -32 : p->index_bits, p->x_vec, p->y_vec, p->work_bytes,
               p->table_hit);
}

void destroy_plan(famlies_plan_s* p) {
  if (!p) return;
  DeviceGuard dg(p->h->device);
  delete p;
}

}  // namespace famlies

famlies_plan_s::~famlies_plan_s() {
  if (owns_device && d_off) (void)hipFree(d_off);
  if (owns_device && d_work) (void)hipFree(d_work);
  if (batch) famlies::destroy_batch(batch);
}

using namespace famlies;

extern "C" {

const char* famlies_version(void) { return "famlies-mi355x 0.1 (gfx950)"; }

famlies_status famlies_create(famlies_handle* out, int device) {
  if (!out) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_create: null output pointer");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= n) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_create: no such device");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(FAMLIES_ERR_UNSUPPORTED, std::string("famlies_create: device is ") + prop.gcnArchName +
                                             ", this library is built for gfx950 only");
  auto* h = new (std::nothrow) famlies_handle_s();
  if (!h) return fail(FAMLIES_ERR_ALLOC, "famlies_create: out of host memory");
  h->device = device;
  h->num_cus = prop.multiProcessorCount;
  {
    famlies_status st = scratch_address(device, &h->scratch);
    if (st != FAMLIES_OK) {
      delete h;
      return st;
    }
  }
  const char* tt = std::getenv("FAMLIES_TUNE_TABLE");
  if (tt && *tt) {
    std::string err;
    if (!h->table.load(tt, &err)) {
      delete h;
      return fail(FAMLIES_ERR_INVALID_ARG, "FAMLIES_TUNE_TABLE: " + err);
    }
  }
  void* tok = registry_add(h, ObjKind::kHandle);
  if (!tok) {
    delete h;
    return fail(FAMLIES_ERR_ALLOC, "famlies_create: no free object slot");
  }
  *out = static_cast<famlies_handle>(tok);
  return FAMLIES_OK;
}

famlies_status famlies_destroy(famlies_handle tok) {
  auto* h = static_cast<famlies_handle_s*>(registry_take(tok, ObjKind::kHandle));
  if (!h) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_destroy: invalid handle");
  delete h;
  return FAMLIES_OK;
}

famlies_status famlies_plan_contract(famlies_handle htok, famlies_plan* out, int dtype, int compute,
                                     const famlies_tensor* A, const famlies_tensor* B,
                                     const famlies_tensor* C) {
  if (!out) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_plan_contract: null output pointer");
  *out = nullptr;
  famlies_plan_s* p = nullptr;
  famlies_status st = no_throw("famlies_plan_contract",
                               [&] { return make_plan(handle_of(htok), &p, dtype, compute, A, B, C, nullptr); });
  if (st != FAMLIES_OK) return st;
  void* tok = registry_add(p, ObjKind::kPlan);
  if (!tok) {
    destroy_plan(p);
    return fail(FAMLIES_ERR_ALLOC, "famlies_plan_contract: no free object slot");
  }
  *out = static_cast<famlies_plan>(tok);
  return FAMLIES_OK;
}

famlies_status famlies_plan_destroy(famlies_plan tok) {
  auto* p = static_cast<famlies_plan_s*>(registry_take(tok, ObjKind::kPlan));
  if (!p) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_plan_destroy: invalid plan");
  destroy_plan(p);
  return FAMLIES_OK;
}

famlies_status famlies_plan_get_info(famlies_plan tok, famlies_plan_info* info) {
  famlies_plan_s* p = plan_of(tok);
  if (!p || !info) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_plan_get_info: invalid argument");
  if (p->batch) {
    batch_info(p->batch, info);
    return FAMLIES_OK;
  }
  fill_info(p->an, p->cfg, p->index_bits, kernel_code(p->an, p->x_vec, p->y_vec), info);
  info->index_elements = p->index_bits == 64 || p->elem32;
  return FAMLIES_OK;
}

static bool overlaps(const void* p, int64_t plo, int64_t phi, const void* q, int64_t qlo, int64_t qhi,
                     int es) {
  if (plo > phi || qlo > qhi) return false;
  const intptr_t a0 = (intptr_t)p + plo * es, a1 = (intptr_t)p + (phi + 1) * es;
  const intptr_t b0 = (intptr_t)q + qlo * es, b1 = (intptr_t)q + (qhi + 1) * es;
  return a0 < b1 && b0 < a1;
}

}  // extern "C"

namespace famlies {

famlies_status execute_impl(famlies_plan_s* p, double alpha, const void* A, const void* B, double beta,
                            void* C, int packed, void* stream) {
  if (!p || p->batch) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_execute: invalid plan");
  const Analysis& an = p->an;
  if (an.M == 0 || an.N == 0) return FAMLIES_OK;
  const bool need_ab = alpha != 0.0 && an.K > 0;
  if (!C || (need_ab && (!A || !B))) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_execute: null data pointer");
  const uintptr_t al = (uintptr_t)an.esize - 1;
  if (((uintptr_t)C & al) || (need_ab && (((uintptr_t)A & al) || ((uintptr_t)B & al))))
    return fail(FAMLIES_ERR_ALIGN, "famlies_execute: data pointer not aligned to its element size");
  const bool pa = packed & 1, pb = packed & 2;
  size_t sza = 0, szb = 0;
  if (need_ab && pa) {
    famlies_status st = pack_size_impl(p, 0, &sza);
    if (st != FAMLIES_OK) return st;
    if ((uintptr_t)A & 15) return fail(FAMLIES_ERR_ALIGN, "famlies_execute_packed: packed A not 16-byte aligned");
  }
  if (need_ab && pb) {
    famlies_status st = pack_size_impl(p, 1, &szb);
    if (st != FAMLIES_OK) return st;
    if ((uintptr_t)B & 15) return fail(FAMLIES_ERR_ALIGN, "famlies_execute_packed: packed B not 16-byte aligned");
  }
  const int64_t es = an.esize;
  auto packed_overlap = [&](const void* q, size_t bytes) {
    return overlaps(C, an.c_lo, an.c_hi, q, 0, (int64_t)(bytes / (size_t)es) - 1, an.esize);
  };
  if (need_ab && ((pa ? packed_overlap(A, sza) : overlaps(C, an.c_lo, an.c_hi, A, an.a_lo, an.a_hi, an.esize)) ||
                  (pb ? packed_overlap(B, szb) : overlaps(C, an.c_lo, an.c_hi, B, an.b_lo, an.b_hi, an.esize))))
    return fail(FAMLIES_ERR_ALIAS, "famlies_execute: C overlaps A or B");
  DeviceGuard dg(p->h->device);
  if (!dg.ok) return fail(FAMLIES_ERR_DEVICE, "cannot select the plan's device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const void* x = an.swapped ? B : A;
  const void* y = an.swapped ? A : B;
  const bool xp = an.swapped ? pb : pa, yp = an.swapped ? pa : pb;
  PlainLaunch L;
  L.bm = p->cfg.bm;
  L.bn = p->cfg.bn;
  L.bk = p->cfg.bk;
  // affine-block 16-byte loads need a 16-byte aligned base pointer
  L.xm = xp ? 2 : (an.x_kfast ? (p->x_vec && !((uintptr_t)x & 15) ? 3 : 1) : 0);
  L.ym = yp ? 2 : (an.y_kfast ? (p->y_vec && !((uintptr_t)y & 15) ? 3 : 1) : 0);
  L.kind = (an.K == 0 || alpha == 0.0) ? PlainLaunch::kScale : PlainLaunch::kMain;
  hipError_t e;
  const int ns = split_parts(an.compute);
  const int i8 = int8_slices(an.compute);
  if (i8 && (pa || pb)) return fail(FAMLIES_ERR_UNSUPPORTED, "famlies_execute_packed: no packed operands for INT8 plans");
  if (i8 && L.kind == PlainLaunch::kMain) {
    // slicer read modes: affine K blocks (the plan's block-stride flags, for
    // slices of 64 and a 16-byte aligned base) with 16-byte loads
    const int xmode = an.x_kfast ? (p->x_vec && !((uintptr_t)x & 15) ? 2 : 1) : 0;
    const int ymode = an.y_kfast ? (p->y_vec && !((uintptr_t)y & 15) ? 2 : 1) : 0;
    e = p->index_bits == 32 ? launch_int8(make_args<uint32_t>(p, x, y, C, alpha, beta), i8, xmode, ymode, s)
                            : launch_int8(make_args<int64_t>(p, x, y, C, alpha, beta), i8, xmode, ymode, s);
  } else if (ns && L.kind == PlainLaunch::kMain) {
    if (p->elem32) {
      e = launch_split(make_args<int32_t>(p, x, y, C, alpha, beta), L, ns, s);
    } else if (p->index_bits == 32) {
      PlainArgs<uint32_t> a = make_args<uint32_t>(p, x, y, C, alpha, beta);
      if (xp) {  // the packed buffer is addressed from its start, not through offsets
        a.x = x;
        a.x_nkb = (int32_t)((an.K + L.bk - 1) / L.bk);
      }
      if (yp) {
        a.y = y;
        a.y_nkb = (int32_t)((an.K + L.bk - 1) / L.bk);
      }
      e = launch_split(a, L, ns, s);
    } else {
      e = launch_split(make_args<int64_t>(p, x, y, C, alpha, beta), L, ns, s);
    }
  } else if (p->elem32) {
    e = launch_plain(an.dtype, make_args<int32_t>(p, x, y, C, alpha, beta), L, s);
  } else if (p->index_bits == 32) {
    PlainArgs<uint32_t> a = make_args<uint32_t>(p, x, y, C, alpha, beta);
    if (xp) {
      a.x = x;
      a.x_nkb = (int32_t)((an.K + L.bk - 1) / L.bk);
    }
    if (yp) {
      a.y = y;
      a.y_nkb = (int32_t)((an.K + L.bk - 1) / L.bk);
    }
    e = launch_plain(an.dtype, a, L, s);
  } else {
    e = launch_plain(an.dtype, make_args<int64_t>(p, x, y, C, alpha, beta), L, s);
  }
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return FAMLIES_OK;
}

}  // namespace famlies

extern "C" {

famlies_status famlies_execute(famlies_plan tok, double alpha, const void* A, const void* B, double beta,
                               void* C, void* stream) {
  return execute_impl(plan_of(tok), alpha, A, B, beta, C, 0, stream);
}

famlies_status famlies_execute_packed(famlies_plan tok, double alpha, const void* A, const void* B, double beta,
                                      void* C, int packed, void* stream) {
  if (packed < 0 || packed > 3) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_execute_packed: packed must be 0..3");
  return execute_impl(plan_of(tok), alpha, A, B, beta, C, packed, stream);
}

}  // extern "C"

// famlies_plan_contract + famlies_execute in one call whose device data (the
// indexing vectors and any split-K partial sums) live in the static scratch
// array instead of plan-owned allocations.
static famlies_status contract_noalloc_impl(famlies_handle htok, int dtype, int compute, double alpha,
                                            const famlies_tensor* A, const void* a, const famlies_tensor* B,
                                            const void* b, double beta, const famlies_tensor* C, void* c,
                                            void* stream) {
  famlies_handle_s* h = handle_of(htok);
  if (!h || !h->scratch) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_contract_noalloc: invalid handle");
  DeviceGuard dg(h->device);
  if (!dg.ok) return fail(FAMLIES_ERR_DEVICE, "cannot select the handle's device");
  famlies_plan_s p;
  p.owns_device = false;
  std::vector<char> image;
  famlies_status st = prepare_plan(h, &p, dtype, compute, A, B, C, nullptr, &image);
  if (st != FAMLIES_OK) return st;
  const size_t off_bytes = (image.size() + 255) & ~(size_t)255;
  if (off_bytes + p.work_bytes > kNoAllocScratchBytes)
    return fail(FAMLIES_ERR_UNSUPPORTED,
                "famlies_contract_noalloc: the call needs " + std::to_string(off_bytes + p.work_bytes) +
                    " bytes of scratch (indexing vectors and split-K partial sums); the maximum is " +
                    std::to_string(kNoAllocScratchBytes));
  p.d_off = h->scratch;
  p.d_work = p.work_bytes ? static_cast<char*>(h->scratch) + off_bytes : nullptr;
  if (log_enabled()) log_plan(&p);
  if (!image.empty()) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    // stream-ordered after earlier work on the stream (which may still read
    // the scratch); the wait lets the host image go when the call returns
    hipError_t e = hipMemcpyAsync(p.d_off, image.data(), image.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(indexing vectors to scratch)");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  }
  return execute_impl(&p, alpha, a, b, beta, c, 0, stream);
}

extern "C" {

famlies_status famlies_contract_noalloc(famlies_handle h, int dtype, int compute, double alpha,
                                        const famlies_tensor* A, const void* a, const famlies_tensor* B,
                                        const void* b, double beta, const famlies_tensor* C, void* c,
                                        void* stream) {
  return no_throw("famlies_contract_noalloc", [&] {
    return contract_noalloc_impl(h, dtype, compute, alpha, A, a, B, b, beta, C, c, stream);
  });
}

}  // extern "C"
