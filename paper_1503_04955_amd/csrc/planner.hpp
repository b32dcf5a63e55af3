// Host-side planning for DKSS multiplication: parameter choice and the ring constants that the
// GPU kernels need.  Pure C++ (no HIP): a small fixed-width unsigned integer type and modular
// arithmetic by shift-and-add, used only at plan time.
#pragma once
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace dkss {

// LDS bytes one workgroup may use for an FFT column (two buffers)
constexpr long long kLdsBytes = 65536;

// Unsigned integer of up to kWords 64-bit words, little-endian.  Sized for moduli p^z below
// 2^512 and their double-width intermediates.
struct Big {
    static constexpr int kWords = 17;
    uint64_t w[kWords] = {};

    static Big of(uint64_t v) { Big b; b.w[0] = v; return b; }
    bool is_zero() const;
    int bitlen() const;
    bool bit(int i) const { return (w[i / 64] >> (i % 64)) & 1; }
    int cmp(const Big& o) const;
    bool operator==(const Big& o) const { return cmp(o) == 0; }
    bool operator!=(const Big& o) const { return cmp(o) != 0; }
    Big shl(int s) const;
    Big shr(int s) const;
    Big add(const Big& o) const;          // no overflow check beyond kWords
    Big sub(const Big& o) const;          // requires *this >= o
    Big mul(const Big& o) const;          // truncated to kWords words
    uint32_t limb32(int i) const { return (uint32_t)(w[i / 2] >> (32 * (i % 2))); }
};

// Arithmetic modulo an odd modulus q (any size up to 2^512): double-and-add multiplication.
struct ModQ {
    Big q;
    explicit ModQ(const Big& qq) : q(qq) {}
    Big reduce(const Big& x) const;                     // x mod q by binary long division
    Big add(const Big& x, const Big& y) const;          // x, y < q
    Big sub(const Big& x, const Big& y) const;
    Big mul(const Big& x, const Big& y) const;
    Big pow(const Big& x, const Big& e) const;
    Big half(const Big& x) const;                       // x / 2 mod q
};

// Plan for one parameter tuple.
struct Plan {
    // parameters (Sec. 3.2 Steps 1-2)
    int log2_M = 0, log2_m = 0, u = 0, p_bits = 0, z = 1;
    std::vector<int> radix_log2;      // FFT level split, sum = log2_M + 1
    uint64_t cutoff_bits = 0;
    // prime and constants (Sec. 3.2.2-3.2.3)
    Big p, q;                         // prime and modulus p^z
    uint64_t h = 0;                   // p = h * 2^n + 1
    int n = 0;
    uint64_t zeta = 0;                // generator of F_p^*
    Big omega;                        // principal 2M-th root of unity mod q
    std::vector<Big> rho;             // m coefficients of rho
    int q_bits = 0;
    int L = 0;                        // uint32 limbs per residue
    int fmt = 0;                      // the kernels' residue format: L, and whether q fits one
                                      // 28-bit digit fewer than 32L bits need (kernels.hpp)
    // key for caching device tables
    std::string key() const;
    long long M() const { return 1LL << log2_M; }
    int m() const { return 1 << log2_m; }
    long long mu_top() const { return M() / m(); }
};

// Thesis parameter rule (Sec. 4.1).  N = bits of the longer operand.  Returns false if no
// tuple exists (N too large for the limits below).
bool thesis_params(uint64_t N, int* log2_M, int* log2_m, int* u, int* p_bits);

// Candidate tuple c (0 <= c < kNumCandidates) for N.  t_min is the smallest log2(Mm) for which
// a prime modulus p >= 2 Mm 2^(2u) (u = ceil(2N/Mm)) has at most 256 bits.
//   c < 18:  z = 1, Mm = 2^(t_min + c / 6), m = 2^(c % 6 + 1), p of the fewest whole 32-bit limbs,
//            or of 28 D - 1 bits where that many bits hold it in one 28-bit digit fewer than the
//            limbs would take (D = ceil((bits + 1) / 28) < ceil((32 limbs + 1) / 28))
//   c >= 18: z = 2 (q = p^2, Sec. 3.2 Step 2 with the Hensel lift of Sec. 3.2.3), Mm = 2^t_min,
//            m = 2^(c - 17), p of the fewest bits with p^2 > Mm 2^(2u)
// False if M < m or no modulus.
constexpr int kNumCandidatesZ1 = 18;
constexpr int kNumCandidates = 24;
bool candidate_params(uint64_t N, int c, int* log2_M, int* log2_m, int* u, int* p_bits, int* z);

// Smallest odd h with p = h*2^n + 1 prime, n = bits - bitlen(h), n >= min_n (Sec. 4.6).
bool proth_prime(int bits, int min_n, Big* p, uint64_t* h, int* n);

// Fill p, q, zeta, omega, rho of a plan whose parameters are set.  Returns false if the tuple
// is infeasible (no prime, p^z below Mm 2^(2u), q too large).
bool compute_constants(Plan* P);

// Default FFT level split: levels of radix 2m (capped by what one workgroup stages in LDS),
// then the remainder (the thesis's recursion, Sec. 4.2).
std::vector<int> default_radices(int log2_M, int log2_m, int L);
int max_radix_log2(int log2_m, int L);

}  // namespace dkss
