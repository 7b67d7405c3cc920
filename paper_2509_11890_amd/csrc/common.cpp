// Error text across the C boundary and the caching device allocator.
#include "common.hpp"

#include <algorithm>
#include <map>
#include <string>
#include <vector>
#include <mutex>

namespace ttipm {

static thread_local std::string g_last_error;

void set_last_error(const std::string& msg) { g_last_error = msg; }
const char* last_error() { return g_last_error.c_str(); }

namespace {
// Freed blocks are reused without waiting for the stream: correct as long as
// one stream does all the work that touches the blocks of one free list.  A
// thread running work on a stream of its own therefore caches its frees in a
// pool of its own (pool_local_begin / pool_local_end).
struct Pool {
  std::mutex mu;
  std::map<size_t, std::vector<void*>> free_lists;   // size class -> blocks
  long long in_use = 0;
};
Pool& global_pool() {
  static Pool* p = new Pool();   // never destroyed: blocks live until process exit
  return *p;
}
thread_local Pool* t_pool = nullptr;

struct Arena {
  char* base = nullptr;
  size_t cap = 0, top = 0, peak = 0;
  struct Blk { size_t off, end; bool freed; };
  std::vector<Blk> stack;
};
thread_local Arena* t_arena = nullptr;
Pool& pool() { return t_pool ? *t_pool : global_pool(); }
size_t size_class(size_t bytes) {
  size_t c = 256;
  while (c < bytes) c <<= 1;
  return c;
}
}  // namespace

void* pool_alloc(size_t bytes) {
  if (t_arena) {
    Arena& A = *t_arena;
    const size_t off = (A.top + 255) & ~size_t(255);
    if (off + bytes > A.cap)
      throw Error(TT_ERR_ARG, "workspace too small: needs more than " + std::to_string(A.cap) + " bytes");
    A.stack.push_back({off, off + bytes, false});
    A.top = off + bytes;
    A.peak = std::max(A.peak, A.top);
    return A.base + off;
  }
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
  if (t_arena) {
    Arena& A = *t_arena;
    char* q = static_cast<char*>(p);
    if (q >= A.base && q < A.base + A.cap) {
      const size_t off = (size_t)(q - A.base);
      for (auto it = A.stack.rbegin(); it != A.stack.rend(); ++it)
        if (it->off == off && !it->freed) {
          it->freed = true;
          break;
        }
      while (!A.stack.empty() && A.stack.back().freed) A.stack.pop_back();
      A.top = A.stack.empty() ? 0 : A.stack.back().end;
      return;
    }
  }
  const size_t cls = size_class(bytes);
  Pool& P = pool();
  std::lock_guard<std::mutex> g(P.mu);
  P.free_lists[cls].push_back(p);
  P.in_use -= cls;
}

size_t pool_bytes_in_use() {
  const long long n = pool().in_use;
  return n > 0 ? (size_t)n : 0;
}

ArenaScope::ArenaScope(void* base, size_t bytes) {
  if (t_arena) throw Error(TT_ERR_ARG, "nested workspace scopes");
  t_arena = new Arena();
  t_arena->base = static_cast<char*>(base);
  t_arena->cap = bytes;
}

ArenaScope::~ArenaScope() {
  delete t_arena;
  t_arena = nullptr;
}

size_t ArenaScope::peak() const { return t_arena ? t_arena->peak : 0; }

void pool_local_begin() {
  if (!t_pool) t_pool = new Pool();
}

void pool_local_end() {
  if (!t_pool) return;
  Pool& G = global_pool();
  {
    std::lock_guard<std::mutex> g(G.mu);
    for (auto& kv : t_pool->free_lists) {
      auto& dst = G.free_lists[kv.first];
      dst.insert(dst.end(), kv.second.begin(), kv.second.end());
    }
    G.in_use += t_pool->in_use;
  }
  delete t_pool;
  t_pool = nullptr;
}

namespace {
const char* const kProfNames[PK_COUNT] = {"gemm_f64_kernel", "gemm_bf16_kernel", "jacobi_svd_kernel",
                                          "panel_lu_kernel", "lanczos_min_kernel", "dense_1wg_kernels"};
struct ProfRec {
  hipEvent_t a, b;
  int kernel;
  double flops, bytes;
};
struct Prof {
  std::mutex mu;
  bool on = false;
  int period = 1;
  long launches[PK_COUNT] = {};
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> spare;
};
Prof& prof() {
  static Prof* p = new Prof();
  return *p;
}
hipEvent_t prof_event(Prof& P) {
  if (!P.spare.empty()) {
    hipEvent_t e = P.spare.back();
    P.spare.pop_back();
    return e;
  }
  hipEvent_t e;
  TT_HIP(hipEventCreate(&e));
  return e;
}
}  // namespace

ProfLaunch prof_launch(int kernel, double flops, double bytes) {
  Prof& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  if (!P.on) return {};
  const long n = P.launches[kernel]++;
  if (n % P.period) return {};
  ProfRec r{prof_event(P), prof_event(P), kernel, flops, bytes};
  P.recs.push_back(r);
  return {r.a, r.b};
}

void prof_start(int period) {
  Prof& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  for (ProfRec& r : P.recs) {
    P.spare.push_back(r.a);
    P.spare.push_back(r.b);
  }
  P.recs.clear();
  for (long& x : P.launches) x = 0;
  P.period = period > 0 ? period : 1;
  P.on = true;
}

int prof_stop(tt_kernel_stat* out, int cap) {
  Prof& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  P.on = false;
  tt_kernel_stat st[PK_COUNT] = {};
  for (int k = 0; k < PK_COUNT; ++k) {
    std::snprintf(st[k].name, sizeof(st[k].name), "%s", kProfNames[k]);
    st[k].launches = P.launches[k];
  }
  for (ProfRec& r : P.recs) {
    TT_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    TT_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    tt_kernel_stat& x = st[r.kernel];
    x.timed += 1;
    x.time_ms += ms;
    x.flops += r.flops;
    x.bytes += r.bytes;
    P.spare.push_back(r.a);
    P.spare.push_back(r.b);
  }
  P.recs.clear();
  const int n = cap < PK_COUNT ? cap : PK_COUNT;
  for (int k = 0; k < n; ++k) out[k] = st[k];
  return PK_COUNT;
}

void pool_trim() {
  Pool& P = pool();
  std::lock_guard<std::mutex> g(P.mu);
  (void)hipDeviceSynchronize();
  for (auto& kv : P.free_lists)
    for (void* p : kv.second) (void)hipFree(p);
  P.free_lists.clear();
}

}  // namespace ttipm
