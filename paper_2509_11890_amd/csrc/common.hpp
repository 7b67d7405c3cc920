// Shared host-side helpers of the TT-IPM library: error reporting across the C
// ABI, HIP status checks and a small device-buffer type.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "../../include/ttipm.h"

namespace ttipm {

// Error carried from inside the library to the C boundary as a status code.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

#define TT_HIP(call)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      throw ::ttipm::Error(TT_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_) + \
                                           " at " + __FILE__ + ":" + std::to_string(__LINE__)); \
  } while (0)

#define TT_REQUIRE(cond, msg)                                                                   \
  do {                                                                                          \
    if (!(cond)) throw ::ttipm::Error(TT_ERR_ARG, std::string(msg) + " (" #cond ") at " +     \
                                                      __FILE__ + ":" + std::to_string(__LINE__)); \
  } while (0)

// Caching device allocator: freed blocks are kept per power-of-two size class
// and handed out again, so the many short-lived intermediates of a sweep do not
// pay hipMalloc/hipFree (hipFree synchronises the device).  All library work is
// ordered on the caller's stream, so a block reused by a later launch on that
// stream cannot overlap its previous user.
void* pool_alloc(size_t bytes);
void pool_free(void* p, size_t bytes);
size_t pool_bytes_in_use();
void pool_trim();
// The calling thread caches its frees apart from the shared pool until
// pool_local_end, which hands them over; the thread's stream must be
// synchronised by then.
void pool_local_begin();
void pool_local_end();

// While an ArenaScope is alive, every pool allocation of the calling thread is
// served from the caller-provided device region [base, base + bytes) instead
// of the pool (as a stack: a freed block at the top is reclaimed, so scoped
// temporaries reuse the space).  An allocation that does not fit throws
// TT_ERR_ARG.  Blocks taken from the region must be freed before the scope
// ends, and the stream that used them synchronised.
class ArenaScope {
 public:
  ArenaScope(void* base, size_t bytes);
  ~ArenaScope();
  ArenaScope(const ArenaScope&) = delete;
  ArenaScope& operator=(const ArenaScope&) = delete;
  size_t peak() const;
};

// Owning device buffer of doubles.  Grows, never shrinks.
class DevBuf {
 public:
  DevBuf() = default;
  explicit DevBuf(size_t n) { reserve(n); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p_(o.p_), n_(o.n_) { o.p_ = nullptr; o.n_ = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p_ = o.p_; n_ = o.n_; o.p_ = nullptr; o.n_ = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void reserve(size_t n) {
    if (n <= n_) return;
    release();
    p_ = pool_alloc((n ? n : 1) * sizeof(double));
    n_ = n;
  }
  double* get() const { return static_cast<double*>(p_); }
  size_t size() const { return n_; }
  void release() {
    if (p_) pool_free(p_, (n_ ? n_ : 1) * sizeof(double));
    p_ = nullptr;
    n_ = 0;
  }

 private:
  void* p_ = nullptr;
  size_t n_ = 0;
};

inline hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

// Event timing of selected kernels (tt_profile_start / tt_profile_stop).  While
// profiling is on, every period-th launch of an instrumented kernel is
// bracketed by HIP events recorded on the launch stream; its algorithmic flops
// and bytes are recorded with it.
enum ProfKernel { PK_GEMM_F64 = 0, PK_GEMM_BF16, PK_JACOBI_SVD, PK_PANEL_LU, PK_LANCZOS, PK_DENSE_1WG, PK_COUNT };
// A timed launch carries a start and a stop event that the dispatch itself
// records (hipExtLaunchKernel), so the measured time is the kernel's execution
// without the launch gap that separately recorded events would include.
struct ProfLaunch {
  hipEvent_t start = nullptr, stop = nullptr;   // null: this launch is not timed
};
ProfLaunch prof_launch(int kernel, double flops, double bytes);
void prof_start(int period);
int prof_stop(tt_kernel_stat* out, int cap);

// hipLaunchKernelGGL with the launch counted (and every period-th one timed)
// as an instance of the instrumented kernel `kernel`.
template <typename F, typename... Args>
void launch_prof(int kernel, double flops, double bytes, F func, dim3 grid, dim3 block, unsigned shmem, hipStream_t s,
                 Args... args) {
  const ProfLaunch pl = prof_launch(kernel, flops, bytes);
  if (pl.start)
    hipExtLaunchKernelGGL(func, grid, block, shmem, s, pl.start, pl.stop, 0u, args...);
  else
    hipLaunchKernelGGL(func, grid, block, shmem, s, args...);
}

// Number of blocks for n items with b threads per block (at least 1).
inline unsigned nblocks(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b > 0 ? (n + b - 1) / b : 1); }

}  // namespace ttipm
