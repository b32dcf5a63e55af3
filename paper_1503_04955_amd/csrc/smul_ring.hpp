// Arithmetic on elements of Z/(2^K + 1)Z (K = 2048 LW bits) by one wavefront, for the SMUL
// kernels: an element is W = 64 LW limbs in LDS (lane l owns limbs l, l + 64, ...) and a top word
// that is 1 only for the value 2^K.  Header-only; every function is device code.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "wave_carry.hpp"

namespace {

using dkss::lane_bit;
using dkss::row_carries;

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// Orders the wavefront's LDS accesses (they are performed in issue order; this keeps the
// compiler from moving them across the point).
__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t bit_of(unsigned long long C) { return lane_bit(C); }

// x += v (v < 2^32 added at limb 0) over W limbs; returns the carry out of the top limb.
__device__ uint32_t fw_add_small(uint32_t* x, uint32_t v, int W) {
    const int l = lane_id();
    uint32_t c = 0;
    for (int w0 = 0; w0 < W; w0 += 64) {
        const uint32_t a = x[w0 + l];
        const uint32_t b = (w0 == 0 && l == 0) ? v : 0u;
        uint32_t s = a + b;
        const unsigned long long G = __ballot(s < a);
        const unsigned long long P = __ballot(s == 0xFFFFFFFFu);
        s += bit_of(row_carries(G, P, c, &c));
        x[w0 + l] = s;
    }
    wsync();
    return c;
}

// x -= v (v < 2^32 subtracted at limb 0) over W limbs; returns the borrow out of the top limb.
__device__ uint32_t fw_sub_small(uint32_t* x, uint32_t v, int W) {
    const int l = lane_id();
    uint32_t c = 0;
    for (int w0 = 0; w0 < W; w0 += 64) {
        const uint32_t a = x[w0 + l];
        const uint32_t b = (w0 == 0 && l == 0) ? v : 0u;
        uint32_t d = a - b;
        const unsigned long long G = __ballot(a < b);
        const unsigned long long P = __ballot(d == 0u);
        d -= bit_of(row_carries(G, P, c, &c));
        x[w0 + l] = d;
    }
    wsync();
    return c;
}

// The value x + T 2^K (x below 2^K in W limbs, T in [-3, 3]) reduced mod 2^K + 1 into [0, 2^K]:
// it is x - T (2^K = -1).  x is rewritten; returns the new top (1 only for 2^K, x then 0).
// The common cases change limb 0 alone; the rest propagate a carry or borrow.
__device__ uint32_t fw_norm(uint32_t* x, int T, int W) {
    wsync();
    if (T == 0) return 0;
    const uint32_t x0 = x[0];
    if (T > 0) {
        if (x0 >= (uint32_t)T) {
            if (lane_id() == 0) x[0] = x0 - (uint32_t)T;
            wsync();
            return 0;
        }
        if (!fw_sub_small(x, (uint32_t)T, W)) return 0;
        // x - T < 0: the value is x - T + 2^K + 1, the wrapped difference plus 1; a carry out
        // means the value 2^K
        return fw_add_small(x, 1u, W);
    }
    const uint32_t v = (uint32_t)(-T);
    if (x0 <= 0xFFFFFFFFu - v) {
        if (lane_id() == 0) x[0] = x0 + v;
        wsync();
        return 0;
    }
    if (!fw_add_small(x, v, W)) return 0;
    // x + v = 2^K + x' with x' < v (all limbs but limb 0 are zero): the value is x' - 1
    const uint32_t xs = x[0];
    if (xs == 0) return 1;                       // -1 = 2^K: x stays 0
    if (lane_id() == 0) x[0] = xs - 1u;
    wsync();
    return 0;
}

// x (canonical, top xt) times 2^t mod 2^K + 1 for 0 < t < K, in place; returns the new top.
// Below 2^K, x 2^t = Lo + H 2^K with Lo = (x << t) mod 2^K and H = x >> (K - t), so the result
// is Lo - H (plus 2^K + 1 if negative).  For x = 2^K (= -1) it is 2^K + 1 - 2^t.
template <int LW>
__device__ uint32_t fw_shift(uint32_t* x, uint32_t xt, int t) {
    constexpr int W = 64 * LW;
    constexpr int K = 32 * W;
    const int l = lane_id();
    wsync();
    if (xt) {
#pragma unroll
        for (int i = 0; i < LW; ++i) {
            const int w = 64 * i + l;
            const int lo = 32 * w;
            uint32_t v = lo + 32 <= t ? 0u : lo >= t ? 0xFFFFFFFFu : (0xFFFFFFFFu << (t - lo));
            if (w == 0) v |= 1u;
            x[w] = v;
        }
        wsync();
        return 0;
    }
    const int tq = t >> 5, tb = t & 31;
    const int u = K - t, uq = u >> 5, ub = u & 31;
    uint32_t lo[LW], hi[LW];
#pragma unroll
    for (int i = 0; i < LW; ++i) {
        const int w = 64 * i + l;
        const uint32_t a1 = w - tq >= 0 ? x[w - tq] : 0u;
        const uint32_t a0 = w - tq - 1 >= 0 ? x[w - tq - 1] : 0u;
        lo[i] = tb ? (a1 << tb) | (a0 >> (32 - tb)) : a1;
        const uint32_t b0 = w + uq < W ? x[w + uq] : 0u;
        const uint32_t b1 = w + uq + 1 < W ? x[w + uq + 1] : 0u;
        hi[i] = ub ? (b0 >> ub) | (b1 << (32 - ub)) : b0;
    }
    wsync();
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < LW; ++i) {
        uint32_t d = lo[i] - hi[i];
        const unsigned long long G = __ballot(lo[i] < hi[i]);
        const unsigned long long P = __ballot(d == 0u);
        d -= bit_of(row_carries(G, P, c, &c));
        x[64 * i + l] = d;
    }
    // Lo - H = d - c 2^K = d + c (mod 2^K + 1)
    return fw_norm(x, -(int)c, W);
}

// x = -x mod 2^K + 1 (canonical x with top xt); returns the new top.  For 0 < x < 2^K,
// 2^K + 1 - x = ~x + 2 (K-bit complement).
template <int LW>
__device__ uint32_t fw_neg(uint32_t* x, uint32_t xt) {
    constexpr int W = 64 * LW;
    const int l = lane_id();
    wsync();
    if (xt) {
#pragma unroll
        for (int i = 0; i < LW; ++i) x[64 * i + l] = (64 * i + l) == 0 ? 1u : 0u;
        wsync();
        return 0;
    }
    bool nz = false;
#pragma unroll
    for (int i = 0; i < LW; ++i) nz = nz || x[64 * i + l] != 0u;
    if (__ballot(nz) == 0ull) return 0;
#pragma unroll
    for (int i = 0; i < LW; ++i) x[64 * i + l] = ~x[64 * i + l];
    return fw_norm(x, -2, W);
}

}  // namespace
