// Device staging array of cum_update_noalloc (defined in noalloc.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace cum {

// Bytes of the fixed staging array: X_new and X_old of one call together.
constexpr size_t NOALLOC_STAGE_BYTES = (size_t)16 << 20;

// Device address of the current device's staging array (looked up with
// hipGetSymbolAddress on the first call per device, then cached).
hipError_t noalloc_stage(void** ptr);

}  // namespace cum
