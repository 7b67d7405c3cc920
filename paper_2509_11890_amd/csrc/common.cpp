// Error text across the C boundary and the caching device allocator.
#include "common.hpp"

#include <map>
#include <mutex>

namespace ttipm {

static thread_local std::string g_last_error;

void set_last_error(const std::string& msg) { g_last_error = msg; }
const char* last_error() { return g_last_error.c_str(); }

namespace {
struct Pool {
  std::mutex mu;
  std::map<size_t, std::vector<void*>> free_lists;   // size class -> blocks
  size_t in_use = 0;
};
Pool& pool() {
  static Pool* p = new Pool();   // never destroyed: blocks live until process exit
  return *p;
}
size_t size_class(size_t bytes) {
  size_t c = 256;
  while (c < bytes) c <<= 1;
  return c;
}
}  // namespace

void* pool_alloc(size_t bytes) {
  const size_t cls = size_class(bytes);
  Pool& P = pool();
  {
    std::lock_guard<std::mutex> g(P.mu);
    auto it = P.free_lists.find(cls);
    if (it != P.free_lists.end() && !it->second.empty()) {
      void* p = it->second.back();
      it->second.pop_back();
      P.in_use += cls;
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, cls);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    pool_trim();
    e = hipMalloc(&p, cls);
  }
  if (e != hipSuccess)
    throw Error(TT_ERR_ALLOC, "hipMalloc of " + std::to_string(cls) + " bytes failed: " + hipGetErrorString(e));
  std::lock_guard<std::mutex> g(P.mu);
  P.in_use += cls;
  return p;
}

void pool_free(void* p, size_t bytes) {
  if (!p) return;
  const size_t cls = size_class(bytes);
  Pool& P = pool();
  std::lock_guard<std::mutex> g(P.mu);
  P.free_lists[cls].push_back(p);
  P.in_use -= cls;
}

size_t pool_bytes_in_use() { return pool().in_use; }

void pool_trim() {
  Pool& P = pool();
  std::lock_guard<std::mutex> g(P.mu);
  (void)hipDeviceSynchronize();
  for (auto& kv : P.free_lists)
    for (void* p : kv.second) (void)hipFree(p);
  P.free_lists.clear();
}

}  // namespace ttipm
