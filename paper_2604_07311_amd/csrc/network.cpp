// Contraction networks: an ordered sequence of contractions over named
// tensors, some supplied by the caller and some intermediates owned by the
// network, planned once and run as one call (sequences of contractions in a
// tensor network: Girder 5, tensor functionality; packing hoisted out of the
// repeated calls for operands that stay constant: Girder 2, "Enabling
// optimizations across layers").
//
// compile() plans every step, allocates the intermediates and the packed
// buffers; execute() packs each operand marked constant the first time it
// runs after that operand was (re)bound, then launches the steps in order on
// one stream.  After the first execute a run allocates nothing and does not
// synchronise, so it can be captured into a HIP graph.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <vector>

#include "famlies.h"
#include "runtime.hpp"

namespace famlies {

struct NetTensor {
  int32_t rank = 0;
  int64_t ext[FAMLIES_MAX_RANK] = {};
  int64_t str[FAMLIES_MAX_RANK] = {};
  int32_t lab[FAMLIES_MAX_RANK] = {};
  bool intermediate = false;
  void* ptr = nullptr;      // bound (user) or owned (intermediate) base pointer
  void* owned = nullptr;    // allocation of an intermediate
  int64_t lo = 0;           // lowest element offset (for intermediates' allocation)
  uint64_t version = 0;     // bumped on every bind

  famlies_tensor desc() const { return famlies_tensor{rank, ext, str, lab}; }
};

struct NetStep {
  double alpha, beta;
  int32_t a, b, c;
  bool pack_a, pack_b;
  famlies_plan_s* plan = nullptr;
  void* packed[2] = {nullptr, nullptr};   // packed copies of A / B
  uint64_t packed_version[2] = {0, 0};    // version of the source when packed (0: never)
};

}  // namespace famlies

struct famlies_network_s {
  famlies_handle_s* h = nullptr;
  int dtype = FAMLIES_F64, compute = FAMLIES_NATIVE;
  std::vector<famlies::NetTensor> tensors;
  std::vector<famlies::NetStep> steps;
  bool compiled = false;
  ~famlies_network_s() {
    for (auto& s : steps) {
      if (s.plan) famlies::destroy_plan(s.plan);
      for (void* q : s.packed)
        if (q) (void)hipFree(q);
    }
    for (auto& t : tensors)
      if (t.owned) (void)hipFree(t.owned);
  }
};

using namespace famlies;

static famlies_network_s* network_of(const void* tok) {
  return static_cast<famlies_network_s*>(registry_get(tok, ObjKind::kNetwork));
}

extern "C" {

famlies_status famlies_network_create(famlies_handle htok, famlies_network* out, int dtype, int compute) {
  if (!out) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_network_create: null output");
  *out = nullptr;
  famlies_handle_s* h = handle_of(htok);
  if (!h) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_network_create: invalid handle");
  if (dtype != FAMLIES_F64 && dtype != FAMLIES_F32) return fail(FAMLIES_ERR_INVALID_ARG, "bad dtype");
  if (compute < FAMLIES_NATIVE || compute > FAMLIES_BF16X6 || (compute != FAMLIES_NATIVE && dtype != FAMLIES_F32))
    return fail(FAMLIES_ERR_INVALID_ARG, "bad compute mode for this dtype");
  auto* n = new (std::nothrow) famlies_network_s();
  if (!n) return fail(FAMLIES_ERR_ALLOC, "out of host memory");
  n->h = h;
  n->dtype = dtype;
  n->compute = compute;
  void* tok = registry_add(n, ObjKind::kNetwork);
  if (!tok) {
    delete n;
    return fail(FAMLIES_ERR_ALLOC, "famlies_network_create: no free object slot");
  }
  *out = static_cast<famlies_network>(tok);
  return FAMLIES_OK;
}

famlies_status famlies_network_destroy(famlies_network tok) {
  auto* n = static_cast<famlies_network_s*>(registry_take(tok, ObjKind::kNetwork));
  if (!n) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_network_destroy: invalid network");
  DeviceGuard dg(n->h->device);
  delete n;
  return FAMLIES_OK;
}

static famlies_status add_tensor_impl(famlies_network tok, const famlies_tensor* desc, int intermediate,
                                      int32_t* id) {
  famlies_network_s* n = network_of(tok);
  if (!n || !desc || !id) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_network_add_tensor: bad argument");
  if (n->compiled) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_network_add_tensor: network already compiled");
  if (desc->rank < 0 || desc->rank > FAMLIES_MAX_RANK || (desc->rank > 0 && (!desc->extents || !desc->strides || !desc->labels)))
    return fail(FAMLIES_ERR_INVALID_ARG, "famlies_network_add_tensor: bad descriptor");
  NetTensor t;
  t.rank = desc->rank;
  for (int d = 0; d < t.rank; ++d) {
    if (desc->extents[d] < 0) return fail(FAMLIES_ERR_INVALID_ARG, "negative extent");
    t.ext[d] = desc->extents[d];
    t.str[d] = desc->strides[d];
    t.lab[d] = desc->labels[d];
  }
  t.intermediate = intermediate != 0;
  n->tensors.push_back(t);
  *id = (int32_t)n->tensors.size() - 1;
  return FAMLIES_OK;
}

famlies_status famlies_network_add_tensor(famlies_network tok, const famlies_tensor* desc, int intermediate,
                                          int32_t* id) {
  return no_throw("famlies_network_add_tensor", [&] { return add_tensor_impl(tok, desc, intermediate, id); });
}

famlies_status famlies_network_add_contraction(famlies_network tok, double alpha, int32_t a, int32_t b, double beta,
                                               int32_t c, int flags) {
  famlies_network_s* n = network_of(tok);
  if (!n) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_network_add_contraction: invalid network");
  if (n->compiled) return fail(FAMLIES_ERR_INVALID_ARG, "network already compiled");
  const int32_t nt = (int32_t)n->tensors.size();
  if (a < 0 || a >= nt || b < 0 || b >= nt || c < 0 || c >= nt)
    return fail(FAMLIES_ERR_INVALID_ARG, "famlies_network_add_contraction: tensor id out of range");
  if (c == a || c == b) return fail(FAMLIES_ERR_ALIAS, "famlies_network_add_contraction: C is also an input");
  if (n->steps.size() >= (size_t)1 << 20) return fail(FAMLIES_ERR_UNSUPPORTED, "too many network steps");
  NetStep s;
  s.alpha = alpha;
  s.beta = beta;
  s.a = a;
  s.b = b;
  s.c = c;
  s.pack_a = flags & FAMLIES_NET_PACK_A;
  s.pack_b = flags & FAMLIES_NET_PACK_B;
  return no_throw("famlies_network_add_contraction", [&] {
    n->steps.push_back(s);
    return FAMLIES_OK;
  });
}

static famlies_status compile_impl(famlies_network tok) {
  famlies_network_s* n = network_of(tok);
  if (!n) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_network_compile: invalid network");
  if (n->compiled) return FAMLIES_OK;
  DeviceGuard dg(n->h->device);
  if (!dg.ok) return fail(FAMLIES_ERR_DEVICE, "cannot select the network's device");
  const int64_t es = n->dtype == FAMLIES_F64 ? 8 : 4;
  // intermediates: allocate the address span of each layout
  for (auto& t : n->tensors) {
    if (!t.intermediate) continue;
    int64_t lo = 0, hi = 0;
    bool empty = false;
    for (int d = 0; d < t.rank; ++d) {
      if (t.ext[d] == 0) empty = true;
      const int64_t r = (t.ext[d] - 1) * t.str[d];
      if (r < 0) lo += r; else hi += r;
    }
    const size_t bytes = empty ? (size_t)es : (size_t)(hi - lo + 1) * (size_t)es;
    hipError_t e = hipMalloc(&t.owned, bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(network intermediate)");
    e = hipMemset(t.owned, 0, bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMemset(network intermediate)");
    t.lo = lo;
    t.ptr = static_cast<char*>(t.owned) - lo * es;
  }
  for (auto& s : n->steps) {
    famlies_tensor A = n->tensors[(size_t)s.a].desc(), B = n->tensors[(size_t)s.b].desc(),
                   C = n->tensors[(size_t)s.c].desc();
    famlies_status st = make_plan(n->h, &s.plan, n->dtype, n->compute, &A, &B, &C, nullptr);
    if (st != FAMLIES_OK) return st;
    for (int op = 0; op < 2; ++op) {
      if (!(op == 0 ? s.pack_a : s.pack_b)) continue;
      size_t bytes = 0;
      st = pack_size_impl(s.plan, op, &bytes);
      if (st == FAMLIES_ERR_UNSUPPORTED) {  // this plan has no packed kernel: gather instead
        (op == 0 ? s.pack_a : s.pack_b) = false;
        continue;
      }
      if (st != FAMLIES_OK) return st;
      hipError_t e = hipMalloc(&s.packed[op], bytes);
      if (e != hipSuccess) return hip_fail(e, "hipMalloc(network packed operand)");
    }
  }
  n->compiled = true;
  return FAMLIES_OK;
}

famlies_status famlies_network_compile(famlies_network tok) {
  return no_throw("famlies_network_compile", [&] { return compile_impl(tok); });
}

famlies_status famlies_network_bind(famlies_network tok, int32_t id, void* ptr) {
  famlies_network_s* n = network_of(tok);
  if (!n) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_network_bind: invalid network");
  if (id < 0 || id >= (int32_t)n->tensors.size()) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_network_bind: bad id");
  NetTensor& t = n->tensors[(size_t)id];
  if (t.intermediate) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_network_bind: tensor is an intermediate");
  t.ptr = ptr;
  t.version += 1;
  return FAMLIES_OK;
}

famlies_status famlies_network_tensor_ptr(famlies_network tok, int32_t id, void** ptr) {
  famlies_network_s* n = network_of(tok);
  if (!n || !ptr) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_network_tensor_ptr: bad argument");
  if (id < 0 || id >= (int32_t)n->tensors.size()) return fail(FAMLIES_ERR_INVALID_ARG, "bad tensor id");
  *ptr = n->tensors[(size_t)id].ptr;
  return FAMLIES_OK;
}

famlies_status famlies_network_execute(famlies_network tok, void* stream) {
  famlies_network_s* n = network_of(tok);
  if (!n) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_network_execute: invalid network");
  if (!n->compiled) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_network_execute: compile the network first");
  for (const auto& t : n->tensors)
    if (!t.intermediate && !t.ptr) return fail(FAMLIES_ERR_INVALID_ARG, "famlies_network_execute: unbound tensor");
  for (auto& s : n->steps) {
    const NetTensor& ta = n->tensors[(size_t)s.a];
    const NetTensor& tb = n->tensors[(size_t)s.b];
    const NetTensor& tc = n->tensors[(size_t)s.c];
    const void* A = ta.ptr;
    const void* B = tb.ptr;
    int mask = 0;
    const NetTensor* src[2] = {&ta, &tb};
    for (int op = 0; op < 2; ++op) {
      if (!(op == 0 ? s.pack_a : s.pack_b)) continue;
      // Constant operands are packed once per binding; an intermediate
      // changes every run, so it is packed every run.
      const uint64_t v = src[op]->intermediate ? 0 : src[op]->version;
      if (src[op]->intermediate || s.packed_version[op] != v) {
        famlies_status st = pack_impl(s.plan, op, src[op]->ptr, s.packed[op], stream);
        if (st != FAMLIES_OK) return st;
        s.packed_version[op] = v;
      }
      (op == 0 ? A : B) = s.packed[op];
      mask |= 1 << op;
    }
    famlies_status st = execute_impl(s.plan, s.alpha, A, B, s.beta, tc.ptr, mask, stream);
    if (st != FAMLIES_OK) return st;
  }
  return FAMLIES_OK;
}

}  // extern "C"
