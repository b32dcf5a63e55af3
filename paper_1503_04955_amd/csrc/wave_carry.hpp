// Carry propagation across the 64 lanes of a wavefront, for multi-limb numbers laid out one limb
// per lane per row (row i = limbs 64 i .. 64 i + 63): a lane's limb generates a carry (G) or
// propagates one (P: all ones for an addition, zero for a subtraction), and the carries into all
// lanes of the row are the carries of one 64-bit addition of the masks.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dkss {

__device__ __forceinline__ int wave_lane() { return (int)(threadIdx.x & 63); }

// Carries into the 64 lanes of a row: lane l generates (G) or propagates (P, disjoint from G) a
// carry; c enters lane 0.  Bit l of the result is the carry into lane l; *cout gets the carry
// out of lane 63.  (The carries of the 64-bit addition (G | P) + G + c are exactly these.)
__device__ __forceinline__ unsigned long long row_carries(unsigned long long G, unsigned long long P,
                                                          uint32_t c, uint32_t* cout) {
    const unsigned long long A = G | P;
    const unsigned long long t = A + G;
    const unsigned long long S = t + c;
    *cout = (uint32_t)((t < A) | (S < t));
    return S ^ A ^ G;
}

__device__ __forceinline__ uint32_t lane_bit(unsigned long long C) { return (uint32_t)(C >> wave_lane()) & 1u; }

}  // namespace dkss
