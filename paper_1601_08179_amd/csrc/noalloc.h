// Fixed device workspace of semcond_apply_noalloc (see noalloc.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace semcond {

// Size of the per-device array: 32 MiB, i.e. 2 N_s k <= 4 Mi FP64 values.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;

// Look up the array's device address on the current device (once per device;
// later calls return at once).  Called by semcond_create.
hipError_t noalloc_scratch_init();
// The looked-up address on device dev, or nullptr before noalloc_scratch_init
// ran with dev current.
void* noalloc_scratch(int dev);

}  // namespace semcond
