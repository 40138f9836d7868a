// Batched contractions and the autotuner (entry points).
#include <hip/hip_runtime.h>

#include <string>

#include "famlies.h"
#include "runtime.hpp"

namespace famlies {
struct BatchPlan {};
void destroy_batch(BatchPlan* b) { delete b; }
}  // namespace famlies

using namespace famlies;

extern "C" {

famlies_status famlies_batch_plan(famlies_handle h, famlies_plan* out, int dtype, int64_t n,
                                  const famlies_tensor* A, const famlies_tensor* B, const famlies_tensor* C) {
  if (out) *out = nullptr;
  return fail(FAMLIES_ERR_UNSUPPORTED, "famlies_batch_plan: not available in this build");
}

famlies_status famlies_batch_execute(famlies_plan p, double alpha, double beta, const void* const* A_dev,
                                     const void* const* B_dev, void* const* C_dev, void* stream) {
  return fail(FAMLIES_ERR_UNSUPPORTED, "famlies_batch_execute: not available in this build");
}

famlies_status famlies_tune(famlies_handle h, const char* table_path, int flags) {
  return fail(FAMLIES_ERR_UNSUPPORTED, "famlies_tune: not available in this build");
}

famlies_status famlies_load_tune_table(famlies_handle h, const char* table_path) {
  if (!h || !is_live(h) || !table_path) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_load_tune_table: invalid argument");
  std::string err;
  if (!h->table.load(table_path, &err)) return fail(FAMLIES_ERR_INVALID_ARG, err);
  return FAMLIES_OK;
}

}  // extern "C"
