// Library-internal declarations shared between translation units (not part
// of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace xs21 {

// The statically allocated scratch array (static_scratch.hip): its size, the
// per-device address lookup (call once per device with that device current;
// idempotent) and the address found for `device` (nullptr before the lookup).
size_t static_scratch_bytes();
hipError_t static_scratch_init(int device);
void* static_scratch(int device);

}  // namespace xs21
