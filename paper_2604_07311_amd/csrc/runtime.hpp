// Handle, plan and tile-table objects behind the opaque C ABI pointers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
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

}  // namespace famlies

struct famlies_handle_s {
  int device = 0;
  int num_cus = 256;
  famlies::TileTable table;
};

struct famlies_plan_s {
  famlies_handle_s* h = nullptr;
  famlies::Analysis an;
  famlies::TileCfg cfg;
  int index_bits = 32;
  int kchunk = 0;
  int head = 0;            // split-K plans: tiles computed whole before the split ones
  void* d_off = nullptr;   // six OffT indexing vectors, then three int64 batch vectors
  size_t batch_off_bytes = 0;
  size_t off_pos[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  // X / Y are K-gathered from affine unit-stride K blocks with 16-byte
  // aligned run starts (given a 16-byte aligned base pointer)
  bool x_vec = false, y_vec = false;
  void* d_work = nullptr;  // split-K partial sums
  size_t work_bytes = 0;
  famlies::BatchPlan* batch = nullptr;  // set for batched plans
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
void register_live(const void* p);
void unregister_live(const void* p);
bool is_live(const void* p);
TileCfg choose_tiles(const famlies_handle_s* h, const Analysis& an);
// Plan one contraction; `force` (may be null) overrides the tile choice.
famlies_status make_plan(famlies_handle_s* h, famlies_plan_s** out, int dtype, int compute,
                         const famlies_tensor* A, const famlies_tensor* B, const famlies_tensor* C,
                         const TileCfg* force);

// Split-bf16 kernels: ns = 2 (bf16x3) or 3 (bf16x6) parts per operand.
hipError_t launch_split(const PlainArgs<uint32_t>& a, const PlainLaunch& L, int ns, hipStream_t s);
hipError_t launch_split(const PlainArgs<int64_t>& a, const PlainLaunch& L, int ns, hipStream_t s);
bool split_tile_supported(int ns, int bm, int bn);
inline int split_parts(int compute) { return compute == FAMLIES_BF16X6 ? 3 : compute == FAMLIES_BF16X3 ? 2 : 0; }

}  // namespace famlies
