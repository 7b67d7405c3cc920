// Static device scratch for the allocation-free entry point.
#pragma once

#include <cstddef>

namespace ttipm {

// Device address (current device) of the library's static scratch array and
// its size in doubles.  The address is looked up on the first call per device.
double* noalloc_scratch(size_t* n_doubles);

}  // namespace ttipm
