// Events used only to time device work.
#ifndef SYMLAT_TIMING_H
#define SYMLAT_TIMING_H

#include <hip/hip_runtime.h>

namespace symlat {

// Recording such an event skips the system-scope fence (cache write-back and
// invalidate) a default event performs, which would otherwise be charged to
// the work being timed.
inline hipError_t timing_event_create(hipEvent_t* e) {
  return hipEventCreateWithFlags(e, hipEventDisableSystemFence);
}

}  // namespace symlat

#endif  // SYMLAT_TIMING_H
