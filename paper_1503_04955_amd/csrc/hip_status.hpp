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

// Carries of a product of nw words whose words and per-64-word generate / propagate masks were
// written by a decode kernel (each word's sum reduced to its low 32 bits plus the previous
// word's high part, leaving at most a 1-bit carry per word).  cin01 and the masks hold
// ceil(nw / 64) entries, seg_gp and seg_cin ceil(nw / 16384).  Enqueued on s.
int carry_resolve(uint32_t* c, long long nw, unsigned long long* gmask, unsigned long long* pmask,
                  unsigned char* cin01, unsigned char* seg_gp, unsigned char* seg_cin, hipStream_t s);

}  // namespace dkss
