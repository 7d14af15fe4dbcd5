// noalloc.h -- the fixed device workspace behind stixels_compute_noalloc.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace stx {

// Bytes of the fixed workspace (one per GPU): at 1024x440 with 128
// disparities it holds a scratch slot for every one of the 204 columns;
// larger frames run with fewer resident workgroups.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;

// Looks up the device address of the fixed workspace on `device`, which must
// be the current device; once per device (later calls return at once).
hipError_t noalloc_setup(int device);

}  // namespace stx
