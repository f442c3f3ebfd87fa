// Device memory of the library: hipMalloc / hipFree, or a caller's
// allocator (for instance a framework's caching allocator) registered with
// cpr_set_allocator.  Contexts and networks take the allocator in force when
// they are created and return every block to it.
#include <mutex>

#include "internal.h"

namespace {
std::mutex g_mtx;
DevAlloc g_alloc;   // both callbacks null: hipMalloc / hipFree
}  // namespace

DevAlloc current_allocator() {
  std::lock_guard<std::mutex> lock(g_mtx);
  return g_alloc;
}

hipError_t dev_malloc(const DevAlloc& a, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 1;
  if (!a.alloc) return hipMalloc(p, bytes);
  *p = a.alloc(bytes, a.user);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}

void dev_free(const DevAlloc& a, void* p) {
  if (!p) return;
  if (!a.alloc) {
    hipFree(p);
    return;
  }
  a.free(p, a.user);
}

extern "C" int cpr_set_allocator(void* (*alloc)(size_t bytes, void* user), void (*release)(void* ptr, void* user),
                                 void* user) {
  if ((alloc == nullptr) != (release == nullptr)) return CPR_EINVAL;
  std::lock_guard<std::mutex> lock(g_mtx);
  g_alloc.alloc = alloc;
  g_alloc.free = release;
  g_alloc.user = alloc ? user : nullptr;
  return CPR_OK;
}
