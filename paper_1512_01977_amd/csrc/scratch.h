// Device scratch of the allocation-free entry points (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace lbm {

// Bytes of the scratch array each GPU holds (until the process ends).
size_t scratch_bytes();
// Looks up, once per device, the address of the current device's copy of the scratch array
// (hipGetSymbolAddress with that device current).  Called at handle set-up.
hipError_t scratch_attach();
// The address recorded for device `dev`, or nullptr if scratch_attach has not run there.
void* scratch_ptr(int dev);

}  // namespace lbm
