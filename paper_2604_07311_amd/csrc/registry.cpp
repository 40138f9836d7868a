// Generation-counted object registry behind the opaque C ABI pointers
// (graceful handling of misuse: Girder 1, "Code safety").
//
// A famlies_handle, famlies_plan or famlies_network given to the caller is a
// token, not the object's address:
//     bits 63..32  generation of the slot when the object was registered
//     bits 31..4   slot index + 1
//     bits  3..0   object kind
// Destroying an object retires its token by bumping the slot's generation, so
// a stale token is rejected even after the slot (or the object's old address)
// is reused by a new object; a token of one kind is rejected where another
// kind is expected.
#include <cstdint>
#include <mutex>
#include <vector>

#include "runtime.hpp"

namespace famlies {

namespace {

struct Slot {
  void* obj = nullptr;
  uint32_t gen = 1;
  uint32_t kind = 0;
};

std::mutex g_mu;
std::vector<Slot> g_slots;
std::vector<uint32_t> g_free;

constexpr uint64_t kKindMask = 0xF;
constexpr uint64_t kIndexMask = 0x0FFFFFFF;

Slot* find(const void* tok, ObjKind k, uint32_t* index) {
  const uint64_t t = (uint64_t)(uintptr_t)tok;
  if ((t & kKindMask) != (uint64_t)k) return nullptr;
  const uint64_t i = (t >> 4) & kIndexMask;
  if (i == 0 || i > g_slots.size()) return nullptr;
  Slot& s = g_slots[(size_t)(i - 1)];
  if (!s.obj || s.kind != (uint32_t)k || s.gen != (uint32_t)(t >> 32)) return nullptr;
  *index = (uint32_t)(i - 1);
  return &s;
}

}  // namespace

void* registry_add(void* obj, ObjKind k) {
  if (!obj) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  uint32_t i;
  if (!g_free.empty()) {
    i = g_free.back();
    g_free.pop_back();
  } else {
    if (g_slots.size() >= kIndexMask) return nullptr;
    g_slots.emplace_back();
    i = (uint32_t)(g_slots.size() - 1);
  }
  Slot& s = g_slots[i];
  s.obj = obj;
  s.kind = (uint32_t)k;
  const uint64_t tok = ((uint64_t)s.gen << 32) | ((uint64_t)(i + 1) << 4) | (uint64_t)k;
  return reinterpret_cast<void*>((uintptr_t)tok);
}

void* registry_get(const void* tok, ObjKind k) {
  std::lock_guard<std::mutex> lk(g_mu);
  uint32_t i = 0;
  Slot* s = find(tok, k, &i);
  return s ? s->obj : nullptr;
}

void* registry_take(const void* tok, ObjKind k) {
  std::lock_guard<std::mutex> lk(g_mu);
  uint32_t i = 0;
  Slot* s = find(tok, k, &i);
  if (!s) return nullptr;
  void* obj = s->obj;
  s->obj = nullptr;
  s->kind = 0;
  s->gen = s->gen + 1 == 0 ? 1 : s->gen + 1;  // 2^32 destroys of one slot before a token repeats
  g_free.push_back(i);
  return obj;
}

}  // namespace famlies
