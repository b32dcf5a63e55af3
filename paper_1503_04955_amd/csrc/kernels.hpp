// Device-side building blocks for DKSS multiplication on gfx950: arithmetic modulo q = p^z on
// residues in 28-bit digits, and products in R = (Z/qZ)[alpha]/(alpha^m + 1).
//
// Representation
//  - A residue mod q is D = ceil((32L+1)/28) digits of 28 bits, least significant first, each
//    digit in [0, 2^28), the value canonical in [0, q), with L = ceil(bits(q)/32); or, in the
//    tight format of a modulus below 2^(28D - 1), one digit fewer (fmt_D).  The format code C
//    (L and the tight bit) is the template parameter of every kernel.  Since 2q < 2^(28D), sums
//    of two residues never leave D digits.
//  - A 28x28-bit digit product is below 2^56, so up to 255 of them add into one 64-bit column
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
    uint32_t qd[kMaxD + 2];  // q in 28-bit digits
    uint32_t qinv28;         // -q^-1 mod 2^28
    uint32_t kpw[kMaxD + 2]; // digits of (2M)^-1 R'^2 mod q: rescales a pointwise product
    uint32_t ql[kMaxL];      // q in 32-bit limbs
    int se;                  // e >= 1 when q = 1 + qd[e] 2^(28e) + qd[e+1] 2^(28(e+1)), else 0
};

// A residue format C: L = C & 15 limbs of 32 bits; with bit 4 set ("tight") the modulus is below
// 2^(28 D - 1) for one 28-bit digit fewer than 32L bits need, D = floor(32L / 28), so that the
// digit products of a product in R shrink by that digit (q of 83 bits: 3 limbs, 3 digits instead
// of 4).  A plan takes the tight format whenever its q fits it.
__host__ __device__ constexpr int fmt_L(int C) { return C & 15; }
__host__ __device__ constexpr bool fmt_tight(int C) { return (C & 16) != 0; }
__host__ __device__ constexpr int fmt_D(int C) { return (32 * fmt_L(C) + 28) / 28 - (fmt_tight(C) ? 1 : 0); }
// bits of the largest modulus the format holds
__host__ __device__ constexpr int fmt_qbits(int C) { return fmt_tight(C) ? 28 * fmt_D(C) - 1 : 32 * fmt_L(C); }
// Montgomery steps: 2^(28K) > 64 q
__host__ __device__ constexpr int fmt_K(int C) { return (fmt_qbits(C) + 6 + 27) / 28; }
__host__ __device__ constexpr int fmt_code(int L, bool tight) { return L | (tight ? 16 : 0); }

template <int C>
struct Dig {
    static constexpr int L = fmt_L(C);
    static constexpr int D = fmt_D(C);                    // 28-bit digits per residue (2q fits)
    static constexpr int K = fmt_K(C);                    // Montgomery steps: 2^(28K) > 64 q
    static constexpr int E = (fmt_qbits(C) - 1) / 28;     // digit of the top bit of the largest q
    static constexpr int NC = K + D + 1;                  // 64-bit columns of a product sum
    static constexpr int NI = (253 - K) / D;              // products per column between carries
    // LDS strides: a staged ring element's residues (and the limb-form residues of levels that
    // also multiply) are laid out at an odd number of words, so that lanes reading consecutive
    // residues hit distinct banks
    static constexpr int DS = D | 1;                      // words per staged residue (digits)
    static constexpr int LS = L | 1;                      // words per residue in limbs
};

// ----- digit arithmetic mod q -----------------------------------------------------------------

// x >= q ?  (the borrow out of the top digit of x - q)
template <int C>
__host__ __device__ __forceinline__ bool dgeq_q(const uint32_t* x, const QConst& Q) {
    constexpr int L = fmt_L(C);
    constexpr int D = Dig<C>::D;
    uint32_t b = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const uint32_t t = x[k] - Q.qd[k] - b;
        b = t >> 31;
    }
    return b == 0;
}

// x -= q (x >= q)
template <int C>
__host__ __device__ __forceinline__ void dsub_q(uint32_t* x, const QConst& Q) {
    constexpr int L = fmt_L(C);
    constexpr int D = Dig<C>::D;
    uint32_t b = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const uint32_t t = x[k] - Q.qd[k] - b;
        x[k] = t & kMask28;
        b = t >> 31;
    }
}

// r = x + y mod q
template <int C>
__host__ __device__ __forceinline__ void dmod_add(uint32_t* r, const uint32_t* x, const uint32_t* y,
                                         const QConst& Q) {
    constexpr int L = fmt_L(C);
    constexpr int D = Dig<C>::D;
    uint32_t s[D], d[D];
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const uint32_t t = x[k] + y[k] + c;
        s[k] = t & kMask28;
        c = t >> 28;
    }
    uint32_t b = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const uint32_t t = s[k] - Q.qd[k] - b;
        d[k] = t & kMask28;
        b = t >> 31;
    }
    // s < 2q < 2^(28D): nothing carries out of the top digit; s >= q iff no borrow
#pragma unroll
    for (int k = 0; k < D; ++k) r[k] = b ? s[k] : d[k];
}

// r = x - y mod q
template <int C>
__host__ __device__ __forceinline__ void dmod_sub(uint32_t* r, const uint32_t* x, const uint32_t* y,
                                         const QConst& Q) {
    constexpr int L = fmt_L(C);
    constexpr int D = Dig<C>::D;
    uint32_t d[D];
    uint32_t b = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const uint32_t t = x[k] - y[k] - b;
        d[k] = t & kMask28;
        b = t >> 31;
    }
    const uint32_t mask = 0u - b;        // add q back if x < y
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const uint32_t t = d[k] + (Q.qd[k] & mask) + c;
        r[k] = t & kMask28;
        c = t >> 28;
    }
}

// r = q - x (x in [0, q]; r = q for x = 0, which is harmless inside a product)
template <int C>
__host__ __device__ __forceinline__ void dneg_q(uint32_t* r, const uint32_t* x, const QConst& Q) {
    constexpr int L = fmt_L(C);
    constexpr int D = Dig<C>::D;
    uint32_t b = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const uint32_t t = Q.qd[k] - x[k] - b;
        r[k] = t & kMask28;
        b = t >> 31;
    }
}

// 32-bit limbs of a residue given in digits
template <int C>
__host__ __device__ __forceinline__ void digits_to_limbs(const uint32_t* d, uint32_t* x) {
    constexpr int L = fmt_L(C);
    constexpr int D = Dig<C>::D;
#pragma unroll
    for (int w = 0; w < L; ++w) {
        const int bit = 32 * w;
        const int k = bit / 28, s = bit % 28;
        uint64_t v = d[k];
        if (k + 1 < D) v |= (uint64_t)d[k + 1] << 28;
        if (k + 2 < D) v |= (uint64_t)d[k + 2] << 56;
        x[w] = (uint32_t)(v >> s);
    }
}

// 28-bit digits of a residue given in 32-bit limbs
template <int C>
__host__ __device__ __forceinline__ void limbs_to_digits(const uint32_t* x, uint32_t* d) {
    constexpr int L = fmt_L(C);
    constexpr int D = Dig<C>::D;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const int bit = 28 * k;
        const int w = bit >> 5, s = bit & 31;
        uint64_t v = w < L ? x[w] : 0u;
        if (w + 1 < L) v |= (uint64_t)x[w + 1] << 32;
        d[k] = (uint32_t)(v >> s) & kMask28;
    }
}

// ----- arithmetic mod q on 32-bit limbs (the FFT passes) ----------------------------------------
// A residue in L limbs, canonical in [0, q); additions use the hardware carry (add/sub with carry
// chains): 2q < 2^(32L + 1), the carry out of the top limb is the extra bit.

// r = x + y mod q, q given by its limbs ql
template <int C>
__host__ __device__ __forceinline__ void lmod_add(uint32_t* r, const uint32_t* x, const uint32_t* y,
                                                  const uint32_t* ql) {
    constexpr int L = fmt_L(C);
    uint32_t s[L], d[L];
    unsigned int c = 0, b = 0;
#pragma unroll
    for (int k = 0; k < L; ++k) s[k] = __builtin_addc(x[k], y[k], c, &c);
#pragma unroll
    for (int k = 0; k < L; ++k) d[k] = __builtin_subc(s[k], ql[k], b, &b);
    const bool ge = c || !b;                 // x + y >= q
#pragma unroll
    for (int k = 0; k < L; ++k) r[k] = ge ? d[k] : s[k];
}

// r = x - y mod q, q given by its limbs ql
template <int C>
__host__ __device__ __forceinline__ void lmod_sub(uint32_t* r, const uint32_t* x, const uint32_t* y,
                                                  const uint32_t* ql) {
    constexpr int L = fmt_L(C);
    uint32_t d[L];
    unsigned int b = 0, c = 0;
#pragma unroll
    for (int k = 0; k < L; ++k) d[k] = __builtin_subc(x[k], y[k], b, &b);
    const uint32_t mask = 0u - b;            // add q back if x < y
#pragma unroll
    for (int k = 0; k < L; ++k) r[k] = __builtin_addc(d[k], ql[k] & mask, c, &c);
}

// ----- Montgomery reduction of a column sum ---------------------------------------------------

// The K Montgomery steps for a modulus q = 1 + qd[E] 2^(28E) + qd[E+1] 2^(28(E+1)), such as a
// prime h 2^n + 1 with n >= 28 (the thesis's kind of prime, Sec. 3.2.2 and Sec. 4.6):
// -q^-1 = -1 mod 2^28, and of the D digit products of a step only two are not zero.
template <int C, int E>
__host__ __device__ __forceinline__ void redc_steps_sparse(uint64_t* col, const QConst& Q) {
    constexpr int L = fmt_L(C);
    using G = Dig<C>;
#pragma unroll
    for (int i = 0; i < G::K; ++i) {
        const uint32_t u = (0u - (uint32_t)col[i]) & kMask28;
        col[i + 1] += (col[i] + u) >> 28;
        col[i + E] += (uint64_t)u * Q.qd[E];
        if (E + 1 < G::D) col[i + E + 1] += (uint64_t)u * Q.qd[E + 1];
    }
}

// col holds S = sum_k col[k] 2^(28k) with S < 64 q^2 (any split into 64-bit columns whose
// running totals stay below 2^64).  The K Montgomery steps leave S 2^(-28K) mod q, below 2q, in
// columns K .. K+D-1; its D digits (carries resolved) go to d.
template <int C>
__host__ __device__ __forceinline__ void redc_digits(uint64_t* col, const QConst& Q, uint32_t* d) {
    constexpr int L = fmt_L(C);
    using G = Dig<C>;
    if (Q.se == G::E) {
        redc_steps_sparse<C, G::E>(col, Q);
    } else {
#pragma unroll
        for (int i = 0; i < G::K; ++i) {
            uint32_t s = (uint32_t)col[i] & kMask28;
            uint32_t u = (s * Q.qinv28) & kMask28;
#pragma unroll
            for (int y = 0; y < G::D; ++y) col[i + y] += (uint64_t)u * Q.qd[y];
            col[i + 1] += col[i] >> 28;
        }
    }
    uint64_t carry = 0;
#pragma unroll
    for (int k = 0; k < G::D; ++k) {
        uint64_t v = col[G::K + k] + carry;
        d[k] = (uint32_t)v & kMask28;
        carry = v >> 28;
    }
}

// S 2^(-28K) mod q, canonical, in digits
template <int C>
__host__ __device__ __forceinline__ void redc_cols(uint64_t* col, const QConst& Q, uint32_t* x) {
    constexpr int L = fmt_L(C);
    redc_digits<C>(col, Q, x);
    if (dgeq_q<C>(x, Q)) dsub_q<C>(x, Q);
}

// S 2^(-28K) mod q, canonical, in L limbs: the value (below 2q < 2^(32L+1)) as L limbs and its
// bit 32L (zero in a tight format, where 2q < 2^(28D) <= 2^(32L)), then one subtraction of q on
// limbs with the hardware borrow
template <int C>
__host__ __device__ __forceinline__ void redc_cols_limbs(uint64_t* col, const QConst& Q, uint32_t* x) {
    constexpr int L = fmt_L(C);
    uint32_t d[Dig<C>::D], s[L];
    redc_digits<C>(col, Q, d);
    digits_to_limbs<C>(d, x);
    uint32_t top = 0;
    if constexpr (!fmt_tight(C)) top = (d[(32 * L) / 28] >> ((32 * L) % 28)) & 1u;
    unsigned int b = 0;
#pragma unroll
    for (int k = 0; k < L; ++k) s[k] = __builtin_subc(x[k], Q.ql[k], b, &b);
    const bool ge = top || !b;
#pragma unroll
    for (int k = 0; k < L; ++k) x[k] = ge ? s[k] : x[k];
}

template <int C>
__host__ __device__ __forceinline__ void normalize_cols(uint64_t* col) {
    constexpr int L = fmt_L(C);
    using G = Dig<C>;
#pragma unroll
    for (int k = 0; k + 1 < G::NC; ++k) {
        col[k + 1] += col[k] >> 28;
        col[k] &= kMask28;
    }
}

// col[x + y] += t_x x_y over the D x D digit pairs of one term
template <int C>
__host__ __device__ __forceinline__ void rprod_term(uint64_t* col, const uint32_t* tp, const uint32_t* xp) {
    constexpr int L = fmt_L(C);
    using G = Dig<C>;
    uint32_t tv[G::D], xv[G::D];
#pragma unroll
    for (int x = 0; x < G::D; ++x) {
        tv[x] = tp[x];
        xv[x] = xp[x];
    }
#pragma unroll
    for (int x = 0; x < G::D; ++x)
#pragma unroll
        for (int y = 0; y < G::D; ++y) col[x + y] += (uint64_t)tv[x] * xv[y];
}

// One output coefficient j of t * alpha^r * x in R, reduced by Montgomery.  With alpha^m = -1
// (so alpha^(2m) = 1), the term t_i x_k lands on coefficient j with sign + when
// i + k + r = j (mod 2m) and with sign - when i + k + r = j + m (mod 2m); for each k exactly one
// i < m does one of the two, hence
//   c_j = sum_{k<m} x_k T_((j - r - k) mod 2m),  T_w = t_w (w < m),  T_w = q - t_(w-m) (w >= m).
// The operand is staged rotated (stage_pos): TP holds T_i at position (i + m + r) mod 2m, at a
// stride of DS words, so that term k of coefficient j is the entry at position j + m - k for
// every r; X holds x_0..x_(m-1) at D words.  The lanes of one element read the same x_k (one
// LDS address) and m consecutive staged entries (odd stride), and the lanes of all elements of
// a wavefront read the same positions, whatever their twiddles.
// Returns c_j 2^(-28K) mod q, canonical, in digits (LIMBS: in L limbs).  FM > 0: log2m = FM is
// known at compile time and the sum is unrolled (no address arithmetic per term).
template <int C, bool LIMBS = false, int FM = 0>
__host__ __device__ __forceinline__ void rprod_coeff(const uint32_t* TP, const uint32_t* X, int log2m, int j,
                                            const QConst& Q, uint32_t* out) {
    constexpr int L = fmt_L(C);
    using G = Dig<C>;
    const int m = FM > 0 ? 1 << FM : 1 << log2m;
    uint64_t col[G::NC];
#pragma unroll
    for (int k = 0; k < G::NC; ++k) col[k] = 0;
    int w = j + m;
    rprod_term<C>(col, TP + w * G::DS, X);      // k = 0 ahead of the loop: the columns start from it
    if constexpr (FM > 0) {
#pragma unroll
        for (int k = 1; k < (1 << FM); ++k) {
            --w;
            rprod_term<C>(col, TP + w * G::DS, X + k * G::D);
            if ((k + 1) % G::NI == 0) normalize_cols<C>(col);
        }
    } else {
        for (int k = 1; k < m; ++k) {
            --w;
            rprod_term<C>(col, TP + w * G::DS, X + k * G::D);
            if ((k + 1) % G::NI == 0) normalize_cols<C>(col);
        }
    }
    if (LIMBS) redc_cols_limbs<C>(col, Q, out);
    else redc_cols<C>(col, Q, out);
}

// Position in the staging area of entry i < 2m of the operand T of rprod_coeff for a product
// by t alpha^r (r >= 0)
__host__ __device__ __forceinline__ int stage_pos(int i, int r, int log2m) {
    return (i + (1 << log2m) + r) & ((2 << log2m) - 1);
}

// LDS layout of the products in R, chosen so that the 64/m elements one wavefront serves read
// distinct banks (64 banks of 4 bytes; also 32 banks within each half of the wavefront):
//  - staging (stage_words): one element's operand, 2m residues at DS words, then m spare
//    words.  Every lane reads position j + m - k of its element's area (rprod_coeff).  The area
//    of element g starts at g (2m DS + m) = g m (2 DS + 1) words: modulo 64 these bases are the
//    64/m multiples of m DS in some order (DS and 2 DS + 1 are odd), so the words read, DS
//    (base / DS + position) + y, run over 64/m disjoint runs of m consecutive multiples of DS,
//    one bank each.
//  - digits (elem_words): an element's m residues at D words, then the fewest words (a
//    multiple of the widest read of a residue, 1, 2 or 4 words) that put the broadcast reads of
//    the wavefront's elements on disjoint banks.
__host__ __device__ constexpr int stage_words(int m, int DS) { return 2 * m * DS + (m < 64 ? m : 0); }

__host__ __device__ constexpr int elem_words(int m, int D) {
    const int width = D % 4 == 0 ? 4 : D % 2 == 0 ? 2 : 1;
    const int n = m < 64 ? 64 / m : 1;                 // elements per wavefront
    for (int pad = 0; pad < 64; pad += width) {
        const int ew = m * D + pad;
        bool ok = true;
        for (int g1 = 0; g1 < n && ok; ++g1)
            for (int g2 = g1 + 1; g2 < n && ok; ++g2) {
                const int d64 = ((g2 - g1) * ew) & 63, d32 = d64 & 31;
                const bool same_half = (g1 < n / 2) == (g2 < n / 2);
                ok = d64 >= width && 64 - d64 >= width &&
                     (!same_half || (d32 >= width && 32 - d32 >= width));
            }
        if (ok) return ew;
    }
    return m * D;
}

// x * k 2^(-28K) mod q for a constant k given in digits (a scalar Montgomery product)
template <int C>
__host__ __device__ __forceinline__ void mont_scalar(const uint32_t* x, const uint32_t* kd, const QConst& Q,
                                            uint32_t* out) {
    constexpr int L = fmt_L(C);
    using G = Dig<C>;
    uint64_t col[G::NC];
#pragma unroll
    for (int k = 0; k < G::NC; ++k) col[k] = 0;
#pragma unroll
    for (int a = 0; a < G::D; ++a)
#pragma unroll
        for (int b = 0; b < G::D; ++b) col[a + b] += (uint64_t)x[a] * kd[b];
    redc_cols<C>(col, Q, out);
}

}  // namespace dkss
