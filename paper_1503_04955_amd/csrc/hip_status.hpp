// HIP status handling shared by the library's translation units: every failed HIP call is
// recorded per host thread (dkss_last_hip_error) before the entry point returns DKSS_EHIP.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/dkss.h"

namespace dkss {

// Record e if it is an error; DKSS_OK or DKSS_EHIP.
int note_hip(hipError_t e);

// Clear an error left by earlier, unrelated runtime calls of this thread, so that the launch
// check of an entry point reports only its own launches.
inline void clear_stale_hip_error() { (void)hipGetLastError(); }

// Status of the launches since the last check.
inline int launch_status() { return note_hip(hipGetLastError()); }

}  // namespace dkss
