// Static scratch of the allocation-free local product (tt_local_matvec_noalloc):
// one file-scope device array, whose address on each device is looked up once,
// with that device current, and kept.
#include <mutex>

#include "common.hpp"
#include "noalloc.hpp"

namespace ttipm {

namespace {

constexpr size_t kScratchDoubles = size_t(8) << 20;   // 64 MiB

__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

}  // namespace

double* noalloc_scratch(size_t* n_doubles) {
  int dev = 0;
  TT_HIP(hipGetDevice(&dev));
  TT_REQUIRE(dev >= 0 && dev < kMaxDevices, "device index out of range");
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_scratch[dev]) {
    // the array's name is a host-side stand-in; kernels get this address
    void* p = nullptr;
    TT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    TT_REQUIRE(p != nullptr, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch[dev] = static_cast<double*>(p);
  }
  *n_doubles = kScratchDoubles;
  return g_scratch[dev];
}

}  // namespace ttipm
