// The fixed per-device scratch array of the allocation-free solve.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace gwr {

// Bytes of the scratch array (per device).
constexpr size_t SCRATCH_BYTES = (size_t)256 << 20;

// Look up the array's address on `device` (once per device; later calls
// return the first result).  Called by gw_solve_noalloc, which has made
// that device current.
hipError_t scratch_init(int device);

// The address scratch_init found, or nullptr if it has not run or failed.
void* scratch_ptr(int device);

}  // namespace gwr
