// Host helper for kernel launches whose status is read back.
#pragma once

#include <hip/hip_runtime.h>

namespace bspl {

// hipLaunchKernelGGL reports a failed launch only through hipGetLastError,
// which also returns any earlier failure on the calling thread (a failed
// allocation, say).  Clear that before launches whose status is read so.
inline void clear_last_error() { (void)hipGetLastError(); }

}  // namespace bspl
