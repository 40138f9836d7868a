// Handle, plan and tile-table objects behind the opaque C ABI pointers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"
#include "launch.hpp"

namespace famlies {

// Tile table: the tuned choice of tile shape per problem size class (the
// role the paper gives the control tree -- encoding block-size choices per
// level, Section "Building on important advances", "Nesting of algorithms
// and blockings" -- reduced to one level).  A size class is the triple of
// ceil(log2) of M, N and K, per dtype and compute mode.
struct TileTable {
  struct Entry {
    int kind;  // 0 plain, 1 batched
    int dtype, compute;
    int lm, ln, lk;
    TileCfg cfg;
  };
  std::vector<Entry> entries;
  static int log2c(int64_t x);
  bool lookup_plain(const Analysis& an, TileCfg* out) const;
  bool lookup_batch(int dtype, int64_t m, int64_t n, int64_t k, TileCfg* out) const;
  bool load(const std::string& path, std::string* err);
  bool save(const std::string& path, std::string* err) const;
  void put(const Entry& e);
};

struct BatchPlan;
void destroy_batch(BatchPlan* b);
// famlies_plan_get_info of a batched plan: batch = problems, flops = total.
void batch_info(const BatchPlan* b, famlies_plan_info* info);

}  // namespace famlies

struct famlies_handle_s {
  int device = 0;
  int num_cus = 256;
  famlies::TileTable table;
  // device address of the library's static scratch array on this handle's
  // device (famlies_contract_noalloc), resolved once when the handle is made
  void* scratch = nullptr;
};

struct famlies_plan_s {
  famlies_handle_s* h = nullptr;
  famlies::Analysis an;
  famlies::TileCfg cfg;
  int index_bits = 32;
  bool elem32 = false;     // index_bits 32: int32 element offsets (else uint32 byte offsets)
  int kchunk = 0;
  int head = 0;            // split-K plans: tiles computed whole before the split ones
  void* d_off = nullptr;   // six OffT indexing vectors, then three int64 batch vectors
  size_t batch_off_bytes = 0;
  size_t off_pos[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  // X / Y are K-gathered from affine unit-stride K blocks with 16-byte
  // aligned run starts (given a 16-byte aligned base pointer)
  bool x_vec = false, y_vec = false;
  bool table_hit = false;  // the tile came from the handle's tile table
  void* d_work = nullptr;  // split-K partial sums
  size_t work_bytes = 0;
  famlies::BatchPlan* batch = nullptr;  // set for batched plans
  bool owns_device = true;  // false: d_off / d_work point into the static scratch array
  ~famlies_plan_s();
};

namespace famlies {

struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int device);
  ~DeviceGuard();
};

famlies_status fail(famlies_status st, const std::string& msg);
famlies_status hip_fail(hipError_t e, const char* what);

// Runs f() so that nothing throws across the C ABI: a host allocation
// failure becomes FAMLIES_ERR_ALLOC, any other C++ exception
// FAMLIES_ERR_INVALID_ARG.
template <typename F>
famlies_status no_throw(const char* where, F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(FAMLIES_ERR_ALLOC, std::string(where) + ": out of host memory");
  } catch (const std::exception& e) {
    return fail(FAMLIES_ERR_INVALID_ARG, std::string(where) + ": " + e.what());
  }
}

// GEMM dimensions the single-contraction kernels index with 32-bit ints.
constexpr int64_t kMaxGemmDim = ((int64_t)1 << 31) - 1024;

// The opaque pointers of the C ABI are generation-counted tokens (see
// registry.cpp): registry_add returns the token for a new object (null when
// out of slots), registry_get resolves a token of kind k (null when it is
// unknown, retired or of another kind), registry_take resolves it and
// retires it.
enum class ObjKind : uint32_t { kHandle = 1, kPlan = 2, kNetwork = 3 };
void* registry_add(void* obj, ObjKind k);
void* registry_get(const void* tok, ObjKind k);
void* registry_take(const void* tok, ObjKind k);
inline famlies_handle_s* handle_of(const void* tok) {
  return static_cast<famlies_handle_s*>(registry_get(tok, ObjKind::kHandle));
}
inline famlies_plan_s* plan_of(const void* tok) {
  return static_cast<famlies_plan_s*>(registry_get(tok, ObjKind::kPlan));
}

// Plan decisions are written to stderr when the environment variable
// FAMLIES_LOG is set to a non-empty value other than "0".
bool log_enabled();
void log_plan(const famlies_plan_s* p);
void log_decision(const char* what, const Analysis& an, const TileCfg& cfg, int index_bits, bool x_vec,
                  bool y_vec, size_t work_bytes, bool table_hit);

// Internal forms of the ABI calls, on resolved objects.
famlies_status execute_impl(famlies_plan_s* p, double alpha, const void* A, const void* B, double beta,
                            void* C, int packed, void* stream);
famlies_status pack_size_impl(famlies_plan_s* p, int operand, size_t* bytes);
famlies_status pack_impl(famlies_plan_s* p, int operand, const void* src, void* dst, void* stream);
void destroy_plan(famlies_plan_s* p);
// from_table (may be null) is set when the handle's tile table decided.
TileCfg choose_tiles(const famlies_handle_s* h, const Analysis& an, bool* from_table = nullptr);

// Host planning helpers (plan_host.cpp).
int64_t ceil_div(int64_t a, int64_t b);
// Settle split-K: K slices of whole BK-blocks, and the number of tiles
// computed whole first (*head; every tile when there is no split).
void finalize_split(TileCfg* t, int64_t K, int64_t ntiles, int* kchunk, int* head);
void fill_info(const Analysis& an, const TileCfg& t, int index_bits, int kernel, famlies_plan_info* info);
// famlies_plan_info.kernel of a plan (xv, yv: affine-block loaders of X, Y).
int kernel_code(const Analysis& an, bool xv, bool yv);
// The fixed tile of the INT8 kernels: 128 x 64 outputs, K slices of 64.
TileCfg int8_tile();
// 32: uint32 byte offsets from each operand's lowest element (every operand
// spans less than 4 GiB over its non-batch modes); 64: int64 element offsets.
int index_bits_for(const Analysis& an);
// The indexing-vector form of a plan: *bits 32 with *elem32 false (uint32
// byte offsets), 32 with *elem32 true (int32 element offsets from each
// operand's lowest element: spans of 4 GiB and more but under 2^31
// elements; not for INT8 plans, whose slicer reads bytes or int64), or 64
// (int64 element offsets).  force: TileCfg::index_bits (0 automatic, 64, or
// kForceElem32: int32 element offsets wherever they reach).
void index_form(const Analysis& an, int force, int* bits, bool* elem32);
// Affine-block flags of X and Y for a plan with K-slice depth bk; v holds
// the nine indexing vectors in upload order.
void vec_flags(const Analysis& an, int bk, int index_bits, const std::vector<int64_t>* v, bool* xv, bool* yv);
// The nine indexing vectors, unpadded: X rows, X k, Y k, Y cols, C rows,
// C cols, batch offsets of X, Y, C.
void all_offsets(const Analysis& an, std::vector<int64_t>* v);
// Plan a batch of n contractions for the persistent batched kernel;
// force_cls >= 0 gives every problem that tile class (0: 64 x 64, 1: 128 x 64,
// 2: 64 x 128, 3: 128 x 128), -1 takes it from the tile table or the default
// rule.  The plan is not registered.
famlies_status batch_plan_make(famlies_handle_s* h, famlies_plan_s** out, int dtype, int64_t n,
                               const famlies_tensor* A, const famlies_tensor* B, const famlies_tensor* C,
                               int force_cls);
famlies_status batch_execute_impl(famlies_plan_s* p, double alpha, double beta, const void* const* A_dev,
                                  const void* const* B_dev, void* const* C_dev, void* stream);
// Tile class of the batched kernel with tile BM x BN (each 64 or 128).
int batch_class_of(int bm, int bn);
// Plan one contraction; `force` (may be null) overrides the tile choice.
famlies_status make_plan(famlies_handle_s* h, famlies_plan_s** out, int dtype, int compute,
                         const famlies_tensor* A, const famlies_tensor* B, const famlies_tensor* C,
                         const TileCfg* force);

// Split-bf16 kernels: ns = 2 (bf16x3) or 3 (bf16x6) parts per operand.
hipError_t launch_split(const PlainArgs<uint32_t>& a, const PlainLaunch& L, int ns, hipStream_t s);
hipError_t launch_split(const PlainArgs<int32_t>& a, const PlainLaunch& L, int ns, hipStream_t s);
hipError_t launch_split(const PlainArgs<int64_t>& a, const PlainLaunch& L, int ns, hipStream_t s);
bool split_tile_supported(int ns, int bm, int bn);
inline int split_parts(int compute) { return compute == FAMLIES_BF16X6 ? 3 : compute == FAMLIES_BF16X3 ? 2 : 0; }
// Contraction slice (BK) of the split-bf16 kernels with ns parts per operand:
// 32 for bf16x3, 16 for bf16x6 (three part planes per operand in LDS).
constexpr int split_slice_k(int ns) { return ns == 3 ? 16 : 32; }
// Contraction slice of the batched kernel's items (both element types).
constexpr int batch_slice_k() { return 16; }
// FP64 on INT8 MFMA: the number of digit slices, 0 for other compute modes.
inline int int8_slices(int compute) {
  return compute >= FAMLIES_INT8X3 && compute <= FAMLIES_INT8X7 ? compute - FAMLIES_INT8X3 + 3 : 0;
}
// xmode / ymode: 0 row-gathered, 1 K-gathered, 2 K-gathered in affine blocks
hipError_t launch_int8(const PlainArgs<uint32_t>& a, int slices, int xmode, int ymode, hipStream_t s);
hipError_t launch_int8(const PlainArgs<int64_t>& a, int slices, int xmode, int ymode, hipStream_t s);
// Workspace of an INT8 plan: the digit planes of X and Y and their row /
// column exponents.
size_t int8_work_bytes(int slices, int64_t M, int64_t N, int64_t K, int64_t L);

}  // namespace famlies
