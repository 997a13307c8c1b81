// noalloc.h -- device scratch of the allocation-free entry points (see noalloc.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace lbm {

// Doubles in the scratch array: per-workgroup partial sums of the diagnostic reduction
// (6 per workgroup, at most kMaxDiagBlocks workgroups) followed by the 8 final sums.
constexpr uint32_t kNoAllocFinal = 6u * (uint32_t)kMaxDiagBlocks;
constexpr uint32_t kNoAllocDoubles = kNoAllocFinal + 8u;
constexpr int kNoAllocMaxDevices = 64;

// Look up the scratch array's address on `device` (once per device; the device is made
// current for the lookup and the previous one restored).  Returns the HIP status of the lookup.
hipError_t noalloc_setup(int device);
// The address found by noalloc_setup for `device`; hipErrorNotInitialized if it never ran or
// failed there.
hipError_t noalloc_scratch(int device, double **ptr);
// out[k] = scale * sums[k] for k = 0, 1 (device to device, on stream s).
hipError_t noalloc_scale2(const double *sums, double scale, double *out, hipStream_t s);

}  // namespace lbm
