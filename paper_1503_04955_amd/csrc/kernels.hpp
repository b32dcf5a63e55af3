// Device-side building blocks for DKSS multiplication on gfx950: multi-limb arithmetic modulo
// q = p^z and products in R = (Z/qZ)[alpha]/(alpha^m + 1).
//
// Representations
//  - In HBM a residue mod q is L uint32 limbs, little-endian, canonical in [0, q).
//  - For products a residue is re-expressed in D digits of 28 bits (D = ceil(32L/28)).  A
//    28x28-bit digit product is below 2^56, so up to 255 of them add into one 64-bit column
//    without carry handling: each digit product is a single v_mad_u64_u32 into its column.
//  - Products are reduced by Montgomery's method in radix 2^28 with K digit steps,
//    R' = 2^(28K) > 64 q, so one final subtraction makes the result canonical.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dkss {

constexpr int kMaxL = 8;
constexpr int kMaxD = 10;
constexpr uint32_t kMask28 = (1u << 28) - 1;

// Modulus constants passed by value to every kernel.
struct QConst {
    uint32_t q[kMaxL];       // q in 32-bit limbs
    uint32_t qd[kMaxD + 2];  // q in 28-bit digits
    uint32_t qinv28;         // -q^-1 mod 2^28
    uint32_t kpw[kMaxD + 2]; // digits of (2M)^-1 R'^2 mod q: rescales a pointwise product
};

template <int L>
struct Dig {
    static constexpr int D = (32 * L + 27) / 28;          // 28-bit digits per residue
    static constexpr int K = (32 * L + 6 + 27) / 28;      // Montgomery steps: 2^(28K) > 64 q
    static constexpr int NC = K + D + 1;                  // 64-bit columns of a product sum
    static constexpr int NI = (253 - K) / D;              // products per column between carries
};

// ----- limb arithmetic ------------------------------------------------------------------------

template <int L>
__device__ __forceinline__ bool geq_q(const uint32_t* x, const QConst& Q) {
#pragma unroll
    for (int i = L - 1; i >= 0; --i) {
        if (x[i] != Q.q[i]) return x[i] > Q.q[i];
    }
    return true;
}

// x -= q (caller knows x >= q, possibly with a carry bit above the top limb)
template <int L>
__device__ __forceinline__ void sub_q(uint32_t* x, const QConst& Q) {
    uint64_t borrow = 0;
#pragma unroll
    for (int i = 0; i < L; ++i) {
        uint64_t t = (uint64_t)x[i] - Q.q[i] - borrow;
        x[i] = (uint32_t)t;
        borrow = (t >> 63) & 1;
    }
}

// r = x + y mod q
template <int L>
__device__ __forceinline__ void mod_add(uint32_t* r, const uint32_t* x, const uint32_t* y,
                                        const QConst& Q) {
    uint64_t c = 0;
#pragma unroll
    for (int i = 0; i < L; ++i) {
        c += (uint64_t)x[i] + y[i];
        r[i] = (uint32_t)c;
        c >>= 32;
    }
    if (c || geq_q<L>(r, Q)) sub_q<L>(r, Q);
}

// r = x - y mod q
template <int L>
__device__ __forceinline__ void mod_sub(uint32_t* r, const uint32_t* x, const uint32_t* y,
                                        const QConst& Q) {
    uint64_t borrow = 0;
#pragma unroll
    for (int i = 0; i < L; ++i) {
        uint64_t t = (uint64_t)x[i] - y[i] - borrow;
        r[i] = (uint32_t)t;
        borrow = (t >> 63) & 1;
    }
    if (borrow) {
        uint64_t c = 0;
#pragma unroll
        for (int i = 0; i < L; ++i) {
            c += (uint64_t)r[i] + Q.q[i];
            r[i] = (uint32_t)c;
            c >>= 32;
        }
    }
}

// r = q - x (x in [0, q]; r = q for x = 0, which is harmless inside a product)
template <int L>
__device__ __forceinline__ void neg_q(uint32_t* r, const uint32_t* x, const QConst& Q) {
    uint64_t borrow = 0;
#pragma unroll
    for (int i = 0; i < L; ++i) {
        uint64_t t = (uint64_t)Q.q[i] - x[i] - borrow;
        r[i] = (uint32_t)t;
        borrow = (t >> 63) & 1;
    }
}

// ----- limbs <-> 28-bit digits --------------------------------------------------------------

template <int L>
__device__ __forceinline__ void limbs_to_digits(const uint32_t* x, uint32_t* d) {
    constexpr int D = Dig<L>::D;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const int bit = 28 * k;
        const int w = bit / 32, s = bit % 32;
        uint64_t v = x[w];
        if (w + 1 < L) v |= (uint64_t)x[w + 1] << 32;
        d[k] = (uint32_t)(v >> s) & kMask28;
    }
}

// D+1 digits (value below 2^(32L+1)) -> L limbs and the bit at 2^(32L)
template <int L>
__device__ __forceinline__ uint32_t digits_to_limbs(const uint32_t* d, uint32_t* x) {
#pragma unroll
    for (int w = 0; w < L; ++w) {
        const int bit = 32 * w;
        const int k = bit / 28, s = bit % 28;
        uint64_t v = ((uint64_t)d[k + 1] << 28) | d[k];
        x[w] = (uint32_t)(v >> s);
    }
    const int k = (32 * L) / 28, s = (32 * L) % 28;
    return (d[k] >> s) & 1;
}

// ----- Montgomery reduction of a column sum ---------------------------------------------------

// col holds S = sum_k col[k] 2^(28k) with S < 64 q^2 (any split into 64-bit columns whose
// running totals stay below 2^64).  Writes S 2^(-28K) mod q, canonical, to x.
template <int L>
__device__ __forceinline__ void redc_cols(uint64_t* col, const QConst& Q, uint32_t* x) {
    using G = Dig<L>;
#pragma unroll
    for (int i = 0; i < G::K; ++i) {
        uint32_t s = (uint32_t)col[i] & kMask28;
        uint32_t u = (s * Q.qinv28) & kMask28;
#pragma unroll
        for (int y = 0; y < G::D; ++y) col[i + y] += (uint64_t)u * Q.qd[y];
        col[i + 1] += col[i] >> 28;
    }
    uint32_t dg[G::D + 1];
    uint64_t carry = 0;
#pragma unroll
    for (int k = 0; k <= G::D; ++k) {
        uint64_t v = col[G::K + k] + carry;
        dg[k] = (uint32_t)v & kMask28;
        carry = v >> 28;
    }
    uint32_t hi = digits_to_limbs<L>(dg, x);
    if (hi || geq_q<L>(x, Q)) sub_q<L>(x, Q);
}

template <int L>
__device__ __forceinline__ void normalize_cols(uint64_t* col) {
    using G = Dig<L>;
#pragma unroll
    for (int k = 0; k + 1 < G::NC; ++k) {
        col[k + 1] += col[k] >> 28;
        col[k] &= kMask28;
    }
}

// One output coefficient j of a product in R:
//   S_j = sum_{i<m} T[i] * E[(j - i - r) mod 2m],
// T = m residues (digits), E = 2m residues (digits) holding x_0..x_{m-1}, q-x_0..q-x_{m-1}, the
// negacyclic extension of x (alpha^m = -1).  Then S_j = coefficient j of T * alpha^r * x.
// Returns S_j 2^(-28K) mod q in limbs.
template <int L>
__device__ __forceinline__ void rprod_coeff(const uint32_t* T, const uint32_t* E, int log2m, int j,
                                            int r, const QConst& Q, uint32_t* out) {
    using G = Dig<L>;
    const int m = 1 << log2m;
    const int mask2 = 2 * m - 1;
    uint64_t col[G::NC];
#pragma unroll
    for (int k = 0; k < G::NC; ++k) col[k] = 0;
    int idx = (j - r) & mask2;
    for (int i = 0; i < m; ++i) {
        uint32_t tv[G::D], ev[G::D];
#pragma unroll
        for (int x = 0; x < G::D; ++x) {
            tv[x] = T[i * G::D + x];
            ev[x] = E[idx * G::D + x];
        }
#pragma unroll
        for (int x = 0; x < G::D; ++x)
#pragma unroll
            for (int y = 0; y < G::D; ++y) col[x + y] += (uint64_t)tv[x] * ev[y];
        idx = (idx - 1) & mask2;
        if ((i + 1) % G::NI == 0) normalize_cols<L>(col);
    }
    redc_cols<L>(col, Q, out);
}

// x * k mod q 2^(-28K) for a constant k given in digits (a scalar Montgomery product)
template <int L>
__device__ __forceinline__ void mont_scalar(const uint32_t* x, const uint32_t* kd, const QConst& Q,
                                            uint32_t* out) {
    using G = Dig<L>;
    uint32_t xd[G::D];
    limbs_to_digits<L>(x, xd);
    uint64_t col[G::NC];
#pragma unroll
    for (int k = 0; k < G::NC; ++k) col[k] = 0;
#pragma unroll
    for (int a = 0; a < G::D; ++a)
#pragma unroll
        for (int b = 0; b < G::D; ++b) col[a + b] += (uint64_t)xd[a] * kd[b];
    redc_cols<L>(col, Q, out);
}

}  // namespace dkss
