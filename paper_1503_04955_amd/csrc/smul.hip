// libdkss: Schoenhage-Strassen multiplication (the thesis's SMUL, Sec. 2.9) on gfx950, in its
// outermost form for the full product (Sec. 2.9.3, optimizations: a cyclic convolution with
// omega = 2^(2K/n), no weights, nonnegative convolution sums, n | 2K).
//
// Pipeline of one product c = a*b, on one HIP stream:
//   k_smul_encode     Step 1: n coefficients of s bits, one ring element of K = 32 W bits each
//   k_smul_level      Steps 3-4: radix-2 decimation in frequency over columns of r elements
//                     staged in LDS (natural order in, bit-reversed out); every multiplication by
//                     a root of unity is a cyclic shift
//   k_smul_pointwise  Step 5: products in R = Z/(2^K + 1)Z (schoolbook on 28-bit digits, the
//                     2K-bit product folded with 2^K = -1), times 1/n = -2^(K - log2 n); or
//                     the same with the 2K-bit product as exact 8-bit products on the matrix
//                     cores (k_smul_pointwise_mx, smul_mx.hip; K <= 32768)
//   k_smul_level      Steps 6-7: radix-2 decimation in time with omega^-1 (bit-reversed in,
//                     natural out)
//   k_smul_decode     Step 10: the coefficients c_k added at bit s k, the carries resolved by
//                     the DKSS decode's carry kernels
//
// Ring elements: W = 64 Lw limbs (Lw = 1, 2, 4, ..., 32), value in [0, 2^K]: the W limbs hold
// the value below 2^K and a separate word per element (its "top") is 1 only for the value 2^K.
// Arithmetic on an element is done by one wavefront: lane l owns limbs l, l + 64, l + 128, ...
// (row i = limbs 64 i .. 64 i + 63), so LDS accesses of a row are conflict-free, and carries
// cross a row by one 64-bit addition of the lanes' generate and propagate masks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>

#include "../../include/dkss.h"
#include "hip_status.hpp"
#include "smul_ring.hpp"
#include "wave_carry.hpp"

using namespace dkss;

namespace dkss {
// Step 5 on the matrix cores (smul_mx.hip): elements of 64 lw limbs, lw <= 16
bool smul_mx_supported(int lw);
int smul_pointwise_mx(int lw, long long n, uint32_t* A, uint32_t* At, const uint32_t* B, const uint32_t* Bt,
                      int log2n, hipStream_t s);
}  // namespace dkss

namespace {

constexpr int kT = 256;                   // threads per workgroup: four wavefronts
constexpr int kTL = 512;                  // threads per workgroup of a transform level: eight wavefronts
constexpr int kMaxLw = 32;                // limbs per lane: W <= 2048, K <= 65536
constexpr size_t kColumnBytes = 65536;    // LDS for the elements of one level column

// s = x + y into X and d = x - y into Y (canonical inputs with tops xt, yt, in LDS); returns
// the tops of s and d in *st, *dt.
template <int LW>
__device__ void fw_addsub(uint32_t* X, uint32_t xt, uint32_t* Y, uint32_t yt, uint32_t* st, uint32_t* dt) {
    constexpr int W = 64 * LW;
    const int l = lane_id();
    wsync();
    uint32_t cs = 0, bd = 0;
#pragma unroll
    for (int i = 0; i < LW; ++i) {
        const int w = 64 * i + l;
        const uint32_t a = X[w], b = Y[w];
        uint32_t s = a + b, d = a - b;
        const unsigned long long Gs = __ballot(s < a);
        const unsigned long long Ps = __ballot(s == 0xFFFFFFFFu);
        const unsigned long long Gd = __ballot(a < b);
        const unsigned long long Pd = __ballot(d == 0u);
        s += bit_of(row_carries(Gs, Ps, cs, &cs));
        d -= bit_of(row_carries(Gd, Pd, bd, &bd));
        X[w] = s;
        Y[w] = d;
    }
    // x + y = s + (cs + xt + yt) 2^K,  x - y = d + (xt - yt - bd) 2^K
    *st = fw_norm(X, (int)(cs + xt + yt), W);
    *dt = fw_norm(Y, (int)xt - (int)yt - (int)bd, W);
}

struct SmulLevel {
    long long n;
    int log2n;
    int log2r;        // radix of the level
    int log2H;        // stride of a column's elements
};

// One level of the transform over n elements of W = 64 LW limbs: a workgroup takes the column
// of r elements base + j H (j < r) into LDS and runs the level's log2 r radix-2 stages on it, one
// wavefront per butterfly.  DIT = 0: decimation in frequency, stages of span r/2 .. 1 (global
// span h = hl H): x, y -> x + y, (x - y) omega^(i n / 2h) with i = base + (j mod hl) H mod h.
// DIT = 1: decimation in time with omega^-1, spans 1 .. r/2: x, y -> x + omega^(-i n / 2h) y,
// x - omega^(-i n / 2h) y.  omega^e = 2^(e 2K / n): the exponent i n / 2h is the shift i K / h.
template <int LW, int DIT>
__global__ __launch_bounds__(kTL) void k_smul_level(uint32_t* __restrict__ poly, uint32_t* __restrict__ tops,
                                                   SmulLevel A) {
    constexpr int W = 64 * LW;
    constexpr int K = 32 * W;
    extern __shared__ uint32_t sm[];
    const int r = 1 << A.log2r;
    uint32_t* E = sm;                             // r elements of W limbs
    uint32_t* T = sm + (size_t)r * W;             // their tops
    const long long H = 1LL << A.log2H;
    const long long col = blockIdx.x;
    const long long c = col & (H - 1);
    const long long base = ((col >> A.log2H) << (A.log2H + A.log2r)) + c;
    for (int idx = threadIdx.x; idx < r * W; idx += kTL) {
        const int j = idx / W, w = idx - j * W;
        E[idx] = poly[(size_t)(base + j * H) * W + w];
    }
    if ((int)threadIdx.x < r) T[threadIdx.x] = tops[base + threadIdx.x * H];
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    for (int st = 0; st < A.log2r; ++st) {
        const int lh = DIT ? st : A.log2r - 1 - st;   // log2 of the local span hl
        const int hl = 1 << lh;
        for (int b = wave; b < r / 2; b += kTL / 64) {
            const int j = ((b >> lh) << (lh + 1)) + (b & (hl - 1));
            // twiddle shift i K / h, i = c + (j mod hl) H < h = hl H (so the shift is below K)
            const long long i = c + (long long)(b & (hl - 1)) * H;
            const int t = (int)(i * (K >> (lh + A.log2H)));
            uint32_t* X = E + (size_t)j * W;
            uint32_t* Y = E + (size_t)(j + hl) * W;
            const uint32_t xt = T[j], yt = T[j + hl];
            uint32_t nx, ny;
            if (!DIT) {
                uint32_t dt;
                fw_addsub<LW>(X, xt, Y, yt, &nx, &dt);
                ny = t ? fw_shift<LW>(Y, dt, t) : dt;
            } else if (t == 0) {
                fw_addsub<LW>(X, xt, Y, yt, &nx, &ny);
            } else {
                // omega^-e y = 2^(2K - t) y = -(2^(K - t) y) =: -z; then x - z, x + z
                const uint32_t zt = fw_shift<LW>(Y, yt, K - t);
                fw_addsub<LW>(X, xt, Y, zt, &nx, &ny);       // X = x + z, Y = x - z
                // swap the two results: limbs through registers, one row at a time
                const int l = lane_id();
#pragma unroll
                for (int q = 0; q < LW; ++q) {
                    const uint32_t u = X[64 * q + l];
                    X[64 * q + l] = Y[64 * q + l];
                    Y[64 * q + l] = u;
                }
                const uint32_t tmp = nx;
                nx = ny;
                ny = tmp;
            }
            wsync();
            if (lane_id() == 0) {
                T[j] = nx;
                T[j + hl] = ny;
            }
            wsync();
        }
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < r * W; idx += kTL) {
        const int j = idx / W, w = idx - j * W;
        poly[(size_t)(base + j * H) * W + w] = E[idx];
    }
    if ((int)threadIdx.x < r) tops[base + threadIdx.x * H] = T[threadIdx.x];
}

// Step 1: element e limb j = bits [s e + 32 j, s e + 32 j + 32) of x, cut to the coefficient's s
// bits (zero beyond x's limbs); tops 0.  One thread per limb.
__global__ __launch_bounds__(kT) void k_smul_encode(uint32_t* __restrict__ poly, uint32_t* __restrict__ tops,
                                                    const uint32_t* __restrict__ x, long long xlen, int s,
                                                    long long n, int log2W) {
    const long long idx = (long long)blockIdx.x * kT + threadIdx.x;
    if (idx >= (n << log2W)) return;
    const long long e = idx >> log2W;
    const int j = (int)(idx & ((1 << log2W) - 1));
    if (j == 0) tops[e] = 0;
    const int nb = s - 32 * j;                 // the coefficient's bits left at limb j
    uint32_t v = 0;
    if (nb > 0) {
        const long long bit = (long long)s * e + 32LL * j;
        const long long wi = bit >> 5;
        const int sh = (int)(bit & 31);
        const uint32_t lo = wi < xlen ? x[wi] : 0u;
        const uint32_t hi = wi + 1 < xlen ? x[wi + 1] : 0u;
        v = sh ? (lo >> sh) | (hi << (32 - sh)) : lo;
        if (nb < 32) v &= (1u << nb) - 1u;
    }
    poly[idx] = v;
}

// Words of the LDS of the componentwise products for W limbs per element: the two factors,
// their 28-bit digits, the column sums (28-bit low part and a 64-bit high part), the words'
// 64-bit sums and the product's 2W words.
__host__ __device__ constexpr int pw_digits(int W) { return (32 * W + 27) / 28; }
// columns per block of the column sums: 2 Dg columns in 512 blocks (two per thread), odd so that
// the lanes' strided digit reads fall on distinct banks
__host__ __device__ constexpr int pw_cb(int W) { return ((2 * pw_digits(W) + 2 * kT - 1) / (2 * kT)) | 1; }
__host__ __device__ constexpr size_t pw_lds_words(int W) {
    return 2 * (size_t)W + 2 * (size_t)pw_digits(W) + 4 * (size_t)pw_cb(W) + 3 * 2 * (size_t)pw_digits(W);
}

// Step 5 with the scaling of Step 9: element k of A becomes A_k B_k 2^(-log2 n) mod 2^K + 1.
// One workgroup per element.  The factors below 2^K go to 28-bit digits; thread t sums the
// columns t, t + 256, ... of their product (64-bit accumulators, the part above 28 bits moved
// out every 128 terms); the 2K-bit product is assembled word by word from the columns and its
// carries resolved by one wavefront, which then folds it (P_lo - P_hi, 2^K = -1) and scales it
// by 2^(-log2 n) = -2^(K - log2 n).  A factor equal to 2^K (= -1) makes the product the other
// factor's negation.  B == A for a squaring.
template <int LW>
__global__ __launch_bounds__(kT) void k_smul_pointwise(uint32_t* Ap, uint32_t* At, const uint32_t* Bp,
                                                       const uint32_t* Bt, int log2n) {
    constexpr int W = 64 * LW;
    constexpr int K = 32 * W;
    constexpr int Dg = pw_digits(W);
    constexpr int NC = 2 * Dg;                    // columns 0 .. 2 Dg - 2, and one more for the carry
    constexpr int CB = pw_cb(W);
    constexpr int PADL = 2 * CB;
    extern __shared__ uint32_t sm[];
    uint32_t* XA = sm;
    uint32_t* XB = XA + W;
    uint32_t* AD = XB + W;                        // Dg digits, then CB zeros
    uint32_t* BP = AD + Dg + CB;                  // 2 CB zeros, Dg digits, CB zeros
    uint32_t* BD = BP + PADL;
    uint32_t* C0 = BP + PADL + Dg + CB;           // NC low parts
    uint64_t* C1 = reinterpret_cast<uint64_t*>(C0 + NC + (NC & 1));   // NC high parts
    // once the columns are summed: the 2W word sums over the factors and digits (4W <= 2W +
    // 2 Dg words), then the 2W product words over the columns
    uint64_t* V = reinterpret_cast<uint64_t*>(sm);
    uint32_t* PW = C0;
    const size_t k = blockIdx.x;
    uint32_t* a = Ap + k * W;
    const uint32_t* b = Bp + k * W;
    for (int i = threadIdx.x; i < W; i += kT) {
        XA[i] = a[i];
        XB[i] = b[i];
    }
    const uint32_t at = At[k], bt = Bt[k];
    __syncthreads();
    const bool wave0 = threadIdx.x < 64;
    uint32_t* R = XA;                             // the result, in place of the first factor
    uint32_t rt = 0;
    if (at | bt) {
        // (-1) (-1) = 1; (-1) y = -y
        if (wave0) {
            if (at && bt) {
                for (int i = lane_id(); i < W; i += 64) R[i] = i == 0 ? 1u : 0u;
                rt = 0;
            } else if (at) {
                for (int i = lane_id(); i < W; i += 64) R[i] = XB[i];
                rt = fw_neg<LW>(R, 0);
            } else {
                rt = fw_neg<LW>(R, 0);
            }
        }
    } else {
        for (int d = threadIdx.x; d < Dg; d += kT) {
            const int bit = 28 * d, w = bit >> 5, sh = bit & 31;
            const uint64_t va = (uint64_t)XA[w] | ((w + 1 < W ? (uint64_t)XA[w + 1] : 0ull) << 32);
            const uint64_t vb = (uint64_t)XB[w] | ((w + 1 < W ? (uint64_t)XB[w + 1] : 0ull) << 32);
            AD[d] = (uint32_t)(va >> sh) & 0x0FFFFFFFu;
            BD[d] = (uint32_t)(vb >> sh) & 0x0FFFFFFFu;
        }
        if ((int)threadIdx.x < CB) {
            AD[Dg + threadIdx.x] = 0;
            BD[Dg + threadIdx.x] = 0;
        }
        if ((int)threadIdx.x < PADL) BP[threadIdx.x] = 0;
        __syncthreads();
        // columns c0 .. c0 + CB - 1 of a block: sum over i of A_i B_(c - i).  The B digits of the
        // block's CB columns at step i, B_(c0 + k - i) (k < CB), sit in registers, position k in
        // slot (k - i) mod CB, so one new digit per step enters; out-of-range digits are the
        // zero padding.  512 blocks of CB columns are centred on the 2 Dg - 1 columns, so that
        // blocks t and 511 - t, thread t's two, are mirror images with equal work.
        static_assert(2 * kT * CB >= 2 * Dg, "the blocks cover every column");
        constexpr int OFF = (2 * kT * CB - (2 * Dg - 1)) / 2;
        for (int hb = 0; hb < 2; ++hb) {
            const int c0 = (hb ? 2 * kT - 1 - (int)threadIdx.x : (int)threadIdx.x) * CB - OFF;
            uint64_t acc[CB], hi[CB];
#pragma unroll
            for (int k = 0; k < CB; ++k) acc[k] = hi[k] = 0;
            const int ilo = c0 - (Dg - 1) > 0 ? c0 - (Dg - 1) : 0;
            const int ihi = c0 + CB - 1 < Dg - 1 ? c0 + CB - 1 : Dg - 1;
            if (ihi >= ilo) {
                const int ngroups = (ihi - ilo + CB) / CB;
                uint32_t buf[CB];
#pragma unroll
                for (int k = 0; k < CB; ++k) buf[k] = BD[c0 + k - ilo];
                for (int g = 0; g < ngroups; ++g) {
                    const int ib = ilo + g * CB;
                    uint32_t av[CB], bv[CB];              // the group's digits, loaded together
#pragma unroll
                    for (int r = 0; r < CB; ++r) {
                        av[r] = AD[ib + r];
                        bv[r] = BD[c0 - (ib + r) - 1];
                    }
#pragma unroll
                    for (int r = 0; r < CB; ++r) {
                        const uint64_t a_i = av[r];
#pragma unroll
                        for (int k = 0; k < CB; ++k) acc[k] += a_i * buf[(k - r + CB) % CB];
                        buf[CB - 1 - r] = bv[r];
                    }
                    if ((g & 15) == 15) {          // at most 16 CB products of 2^56 per term
#pragma unroll
                        for (int k = 0; k < CB; ++k) {
                            hi[k] += acc[k] >> 28;
                            acc[k] &= 0x0FFFFFFFull;
                        }
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < CB; ++k) {
                if (c0 + k >= 0 && c0 + k < NC) {
                    C0[c0 + k] = (uint32_t)(acc[k] & 0x0FFFFFFFull);
                    C1[c0 + k] = hi[k] + (acc[k] >> 28);
                }
            }
        }
        __syncthreads();
        // the product is sum_c e_c 2^(28 c), e_c = C0[c] + C1[c - 1] < 2^42; word w sums the
        // pieces of the e_c that overlap it (at most 5)
        for (int w = threadIdx.x; w < 2 * W; w += kT) {
            uint64_t s = 0;
            const int clo = (32 * w - 63) / 28 > 0 ? (32 * w - 63) / 28 : 0;
            const int chi = (32 * w + 31) / 28 < NC - 1 ? (32 * w + 31) / 28 : NC - 1;
            for (int c = clo; c <= chi; ++c) {
                const uint64_t e = (uint64_t)C0[c] + (c ? C1[c - 1] : 0ull);
                const int o = 32 * w - 28 * c;
                if (o >= 0) {
                    if (o < 64) s += (uint32_t)(e >> o);
                } else if (o > -32) {
                    s += (uint32_t)(e << (-o));
                }
            }
            V[w] = s;
        }
        __syncthreads();
        if (wave0) {
            // x_w = low(V_w) + high(V_(w-1)) < 2^32 + 8: a 1-bit carry per word
            const int l = lane_id();
            uint32_t c = 0;
            for (int w0 = 0; w0 < 2 * W; w0 += 64) {
                const int w = w0 + l;
                const uint64_t x = (V[w] & 0xFFFFFFFFull) + (w ? (V[w - 1] >> 32) : 0ull);
                uint32_t y = (uint32_t)x;
                const unsigned long long G = __ballot((x >> 32) != 0);
                const unsigned long long P = __ballot(y == 0xFFFFFFFFu);
                y += bit_of(row_carries(G, P, c, &c));
                PW[w] = y;
            }
            wsync();
            // P = P_hi 2^K + P_lo = P_lo - P_hi (mod 2^K + 1)
            uint32_t bo = 0;
            for (int w0 = 0; w0 < W; w0 += 64) {
                const int w = w0 + l;
                const uint32_t x = PW[w], y = PW[W + w];
                uint32_t d = x - y;
                const unsigned long long G = __ballot(x < y);
                const unsigned long long P = __ballot(d == 0u);
                d -= bit_of(row_carries(G, P, bo, &bo));
                R[w] = d;
            }
            rt = fw_norm(R, -(int)bo, W);
        }
    }
    if (wave0) {
        // times 2^(-log2 n) = 2^(2K - log2 n) = -2^(K - log2 n)
        rt = fw_shift<LW>(R, rt, K - log2n);
        rt = fw_neg<LW>(R, rt);
        for (int i = lane_id(); i < W; i += 64) a[i] = R[i];
        if (lane_id() == 0) At[k] = rt;
    }
}

// Step 10: output word w sums the pieces of the coefficients c_k (k < n, value below 2^K, at bit
// s k) that overlap it; then low 32 bits + the previous word's high part and the generate /
// propagate masks per 64 words, as the DKSS decode writes them for the carry kernels.
__global__ __launch_bounds__(kT) void k_smul_decode(uint32_t* __restrict__ out, long long nw,
                                                    const uint32_t* __restrict__ poly, long long n, int W, int s,
                                                    unsigned long long* __restrict__ gmask,
                                                    unsigned long long* __restrict__ pmask) {
    __shared__ uint32_t hiv[kT + 1];
    const long long K = 32LL * W;
    const long long w0 = (long long)blockIdx.x * kT;
    const long long w = w0 + threadIdx.x;
    auto word_sum = [&](long long ww) -> uint64_t {
        uint64_t V = 0;
        // coefficients with s k < 32 ww + 32 and s k + K > 32 ww
        const long long lo_excl = 32 * ww - K;
        long long k0 = lo_excl < 0 ? 0 : lo_excl / s + 1;
        long long k1 = (32 * ww + 31) / s;
        if (k1 > n - 1) k1 = n - 1;
        for (long long kk = k0; kk <= k1; ++kk) {
            const long long o = 32 * ww - (long long)s * kk;
            const uint32_t* e = poly + (size_t)kk * W;
            if (o >= 0) {
                const int q = (int)(o >> 5), b = (int)(o & 31);
                const uint32_t x0 = e[q];
                const uint32_t x1 = q + 1 < W ? e[q + 1] : 0u;
                V += b ? (x0 >> b) | (x1 << (32 - b)) : x0;
            } else {
                V += e[0] << (int)(-o);
            }
        }
        return V;
    };
    uint64_t V = 0, Vprev = 0;
    if (w < nw) V = word_sum(w);
    if (threadIdx.x == 0 && w0 > 0 && w0 < nw) Vprev = word_sum(w0 - 1);
    hiv[threadIdx.x + 1] = (uint32_t)(V >> 32);
    if (threadIdx.x == 0) hiv[0] = (uint32_t)(Vprev >> 32);
    __syncthreads();
    const uint64_t x = (uint64_t)(uint32_t)V + hiv[threadIdx.x];
    const uint32_t y = (uint32_t)x;
    const bool g = w < nw && (x >> 32) != 0;
    const bool pr = w < nw && y == 0xFFFFFFFFu;
    const unsigned long long G = __ballot(g);
    const unsigned long long P = __ballot(pr);
    if (w < nw) out[w] = y;
    if ((threadIdx.x & 63) == 0 && w < nw) {
        gmask[w >> 6] = G;
        pmask[w >> 6] = P;
    }
}

// ----- host side -------------------------------------------------------------------------------

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct SmulPlan {
    int log2n = 0, lw = 0, W = 0, K = 0, s = 0;
    int products = 1;         // Step 5: 1 digit schoolbook on the vector units, 2 matrix cores
    long long n = 0;
    int nlev = 0;
    int lr[24] = {};          // radices (log2) of the forward levels, top level first
};

int lw_index(int lw) {
    switch (lw) {
        case 1: return 0;
        case 2: return 1;
        case 4: return 2;
        case 8: return 3;
        case 16: return 4;
        case 32: return 5;
        default: return -1;
    }
}

// Feasibility of (log2 n, lw) for a product of alen x blen limbs: s = ceil(32 (alen + blen) / n),
// the coefficient counts na + nb - 1 <= n (no cyclic wrap), the largest convolution sum
// min(na, nb) (2^s - 1)^2 below 2^K, and n | 2K.
bool smul_fits(size_t alen, size_t blen, int log2n, int lw, int* s_out) {
    if (log2n < 1 || log2n > 30 || lw_index(lw) < 0) return false;
    const long long n = 1LL << log2n;
    const long long K = 2048LL * lw;
    if ((2 * K) % n) return false;
    const long long bits = 32LL * (long long)(alen + blen);
    const long long s = (bits + n - 1) / n;
    if (s < 1 || s > K) return false;
    const long long na = std::max(1LL, (32LL * (long long)alen + s - 1) / s);
    const long long nb = std::max(1LL, (32LL * (long long)blen + s - 1) / s);
    if (na + nb - 1 > n) return false;
    int lg = 0;
    while ((1LL << lg) < std::min(na, nb)) ++lg;
    if (2 * s + lg > K) return false;
    *s_out = (int)s;
    return true;
}

void smul_levels(SmulPlan* P) {
    int rmax = 0;
    while ((size_t)(2LL << rmax) * (size_t)P->W * 4 <= kColumnBytes) ++rmax;   // 2^rmax W 4 <= budget
    rmax = std::max(1, std::min(rmax, 8));
    const int nlev = (P->log2n + rmax - 1) / rmax;
    P->nlev = nlev;
    for (int i = 0; i < nlev; ++i) P->lr[i] = P->log2n / nlev + (i < P->log2n % nlev ? 1 : 0);
}

// Modelled cost, in units of a digit product: the componentwise products (digit form: n (K / 28)^2
// digit products; matrix-core form: that cost times the ratio of the two forms' measured launch
// times at the same ring, 0.50 both at lw = 4 (n = 2^14) and at lw = 16 (n = 2^16)), and the
// transforms, 3 (levels) n W limbs through HBM and the butterflies.
constexpr double kMxRatio = 0.50;
double smul_products_cost(long long n, int W, int products) {
    const double K = 32.0 * W;
    const double digits = (double)n * (K / 28.0) * (K / 28.0);
    return products == 2 ? kMxRatio * digits : digits;
}
double smul_cost(long long n, int W, int nlev, int products) {
    return smul_products_cost(n, W, products) + 3.0 * (double)nlev * (double)n * W * 120.0;
}

int smul_plan(size_t alen, size_t blen, const dkss_smul_params* p, SmulPlan* P) {
    if (alen == 0 || blen == 0) return DKSS_OK;
    const int want = p ? (int)p->products : 0;
    if (want < 0 || want > 2) return DKSS_EINVAL;
    int best_n = -1, best_lw = 0, best_s = 0, best_pr = 1;
    double best = 0;
    for (int lg = 1; lg <= 24; ++lg) {
        for (int lw = 1; lw <= kMaxLw; lw *= 2) {
            if (p && p->log2_n && (int)p->log2_n != lg) continue;
            if (p && p->lw && (int)p->lw != lw) continue;
            int s = 0;
            if (!smul_fits(alen, blen, lg, lw, &s)) continue;
            SmulPlan T;
            T.log2n = lg;
            T.W = 64 * lw;
            smul_levels(&T);
            for (int pr = 1; pr <= 2; ++pr) {
                if ((want && pr != want) || (pr == 2 && !smul_mx_supported(lw))) continue;
                const double c = smul_cost(1LL << lg, 64 * lw, T.nlev, pr);
                if (best_n < 0 || c < best) {
                    best = c;
                    best_n = lg;
                    best_lw = lw;
                    best_s = s;
                    best_pr = pr;
                }
            }
        }
    }
    if (best_n < 0) return DKSS_ERANGE;
    P->products = best_pr;
    P->log2n = best_n;
    P->n = 1LL << best_n;
    P->lw = best_lw;
    P->W = 64 * best_lw;
    P->K = 32 * P->W;
    P->s = best_s;
    smul_levels(P);
    if ((unsigned long long)P->n * (unsigned long long)P->W >= (1ull << 32)) return DKSS_ERANGE;
    return DKSS_OK;
}

struct SmulWs {
    uint32_t *A, *B, *At, *Bt;
    unsigned long long *gmask, *pmask;
    unsigned char *cin01, *seg_gp, *seg_cin;
    size_t bytes;
};

SmulWs smul_layout(const SmulPlan& P, size_t nw, bool need_b, char* base) {
    SmulWs w{};
    const size_t pb = (size_t)P.n * P.W * 4;
    const size_t nwaves = (nw + 63) / 64;
    const size_t nseg = (nwaves + kT - 1) / kT;
    size_t off = 0;
    w.A = (uint32_t*)(base + off);
    off += al256(pb);
    w.B = (uint32_t*)(base + off);
    off += need_b ? al256(pb) : 0;
    w.At = (uint32_t*)(base + off);
    off += al256((size_t)P.n * 4);
    w.Bt = (uint32_t*)(base + off);
    off += need_b ? al256((size_t)P.n * 4) : 0;
    w.gmask = (unsigned long long*)(base + off);
    off += al256(nwaves * 8);
    w.pmask = (unsigned long long*)(base + off);
    off += al256(nwaves * 8);
    w.cin01 = (unsigned char*)(base + off);
    off += al256(nwaves);
    w.seg_gp = (unsigned char*)(base + off);
    off += al256(nseg);
    w.seg_cin = (unsigned char*)(base + off);
    off += al256(nseg);
    w.bytes = off;
    return w;
}

template <int LW>
int launch_transform(const SmulPlan& P, uint32_t* poly, uint32_t* tops, bool inverse, hipStream_t s) {
    int acc = 0;
    for (int li = 0; li < P.nlev; ++li) {
        // forward: levels top-down; inverse: bottom-up
        const int lev = inverse ? P.nlev - 1 - li : li;
        acc = 0;
        for (int q = 0; q <= lev; ++q) acc += P.lr[q];
        SmulLevel A;
        A.n = P.n;
        A.log2n = P.log2n;
        A.log2r = P.lr[lev];
        A.log2H = P.log2n - acc;
        const size_t lds = ((size_t)P.W << A.log2r) * 4 + ((size_t)4 << A.log2r);
        const unsigned cols = (unsigned)(P.n >> A.log2r);
        if (inverse)
            hipLaunchKernelGGL((k_smul_level<LW, 1>), dim3(cols), dim3(kTL), lds, s, poly, tops, A);
        else
            hipLaunchKernelGGL((k_smul_level<LW, 0>), dim3(cols), dim3(kTL), lds, s, poly, tops, A);
    }
    return launch_status();
}

template <int LW>
int launch_pointwise(const SmulPlan& P, uint32_t* A, uint32_t* At, const uint32_t* B, const uint32_t* Bt,
                     hipStream_t s) {
    if (P.products == 2) return smul_pointwise_mx(LW, P.n, A, At, B, Bt, P.log2n, s);
    const size_t lds = pw_lds_words(64 * LW) * 4;
    hipLaunchKernelGGL(k_smul_pointwise<LW>, dim3((unsigned)P.n), dim3(kT), lds, s, A, At, B, Bt, P.log2n);
    return launch_status();
}

template <template <int> class F, typename... Args>
int dispatch_lw(int lw, Args&&... args) {
    switch (lw) {
        case 1: return F<1>::run(args...);
        case 2: return F<2>::run(args...);
        case 4: return F<4>::run(args...);
        case 8: return F<8>::run(args...);
        case 16: return F<16>::run(args...);
        case 32: return F<32>::run(args...);
        default: return DKSS_ERANGE;
    }
}

template <int LW>
struct Transform {
    static int run(const SmulPlan& P, uint32_t* poly, uint32_t* tops, bool inverse, hipStream_t s) {
        return launch_transform<LW>(P, poly, tops, inverse, s);
    }
};

template <int LW>
struct Pointwise {
    static int run(const SmulPlan& P, uint32_t* A, uint32_t* At, const uint32_t* B, const uint32_t* Bt,
                   hipStream_t s) {
        return launch_pointwise<LW>(P, A, At, B, Bt, s);
    }
};

int encode(const SmulPlan& P, uint32_t* poly, uint32_t* tops, const uint32_t* x, size_t xlen, hipStream_t s) {
    const long long total = P.n * P.W;
    int log2W = 0;
    while ((1 << log2W) < P.W) ++log2W;
    hipLaunchKernelGGL(k_smul_encode, dim3((unsigned)((total + kT - 1) / kT)), dim3(kT), 0, s, poly, tops, x,
                       (long long)xlen, P.s, P.n, log2W);
    return launch_status();
}

void to_params(const SmulPlan& P, dkss_smul_params* out) {
    memset(out, 0, sizeof *out);
    out->log2_n = (uint32_t)P.log2n;
    out->lw = (uint32_t)P.lw;
    out->s = (uint32_t)P.s;
    out->K = (uint32_t)P.K;
    out->n_levels = (uint32_t)P.nlev;
    out->products = (uint32_t)P.products;
}

bool overlap(const void* x, size_t xb, const void* y, size_t yb) {
    const char* a = (const char*)x;
    const char* b = (const char*)y;
    return a < b + yb && b < a + xb;
}

__global__ void k_smul_zero(uint32_t* c, long long nw) {
    const long long i = (long long)blockIdx.x * kT + threadIdx.x;
    if (i < nw) c[i] = 0;
}

}  // namespace

extern "C" {

int dkss_smul_select(size_t alen, size_t blen, dkss_smul_params* out) {
    if (!out) return DKSS_EINVAL;
    if (alen == 0 || blen == 0) {
        memset(out, 0, sizeof *out);
        return DKSS_OK;
    }
    SmulPlan P;
    int rc = smul_plan(alen, blen, nullptr, &P);
    if (rc) return rc;
    to_params(P, out);
    return DKSS_OK;
}

int dkss_smul_workspace_bytes(size_t alen, size_t blen, const dkss_smul_params* p, size_t* out) {
    if (!out) return DKSS_EINVAL;
    *out = 0;
    if (alen == 0 || blen == 0) return DKSS_OK;
    SmulPlan P;
    int rc = smul_plan(alen, blen, p, &P);
    if (rc) return rc;
    *out = smul_layout(P, alen + blen, true, nullptr).bytes;
    return DKSS_OK;
}

int dkss_smul(uint32_t* c, const uint32_t* a, size_t alen, const uint32_t* b, size_t blen,
              const dkss_smul_params* p, void* ws, size_t ws_bytes, dkss_stream_t st) {
    clear_stale_hip_error();
    hipStream_t s = (hipStream_t)st;
    if (!c || (alen && !a) || (blen && !b)) return DKSS_EINVAL;
    const size_t nw = alen + blen;
    if ((alen && overlap(c, nw * 4, a, alen * 4)) || (blen && overlap(c, nw * 4, b, blen * 4))) return DKSS_EINVAL;
    if (alen == 0 || blen == 0) {
        if (nw) hipLaunchKernelGGL(k_smul_zero, dim3((unsigned)((nw + kT - 1) / kT)), dim3(kT), 0, s, c, (long long)nw);
        return launch_status();
    }
    SmulPlan P;
    int rc = smul_plan(alen, blen, p, &P);
    if (rc) return rc;
    const bool squaring = a == b && alen == blen;
    if (!ws || ((uintptr_t)ws & 255)) return DKSS_EINVAL;
    SmulWs w = smul_layout(P, nw, !squaring, (char*)ws);
    if (ws_bytes < w.bytes) return DKSS_ENOSPC;
    if ((rc = encode(P, w.A, w.At, a, alen, s))) return rc;
    if ((rc = dispatch_lw<Transform>(P.lw, P, w.A, w.At, false, s))) return rc;
    const uint32_t* Bp = w.A;
    const uint32_t* Bt = w.At;
    if (!squaring) {
        if ((rc = encode(P, w.B, w.Bt, b, blen, s))) return rc;
        if ((rc = dispatch_lw<Transform>(P.lw, P, w.B, w.Bt, false, s))) return rc;
        Bp = w.B;
        Bt = w.Bt;
    }
    if ((rc = dispatch_lw<Pointwise>(P.lw, P, w.A, w.At, Bp, Bt, s))) return rc;
    if ((rc = dispatch_lw<Transform>(P.lw, P, w.A, w.At, true, s))) return rc;
    hipLaunchKernelGGL(k_smul_decode, dim3((unsigned)((nw + kT - 1) / kT)), dim3(kT), 0, s, c, (long long)nw,
                       (const uint32_t*)w.A, P.n, P.W, P.s, w.gmask, w.pmask);
    if ((rc = launch_status())) return rc;
    return carry_resolve(c, (long long)nw, w.gmask, w.pmask, w.cin01, w.seg_gp, w.seg_cin, s);
}

int dkss_smul_forward(uint32_t* poly, uint32_t* tops, const uint32_t* a, size_t alen, size_t blen,
                      const dkss_smul_params* p, dkss_stream_t st) {
    clear_stale_hip_error();
    if (!poly || !tops || (alen && !a)) return DKSS_EINVAL;
    if (alen == 0 || blen == 0) return DKSS_ERANGE;
    SmulPlan P;
    int rc = smul_plan(alen, blen, p, &P);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)st;
    if ((rc = encode(P, poly, tops, a, alen, s))) return rc;
    return dispatch_lw<Transform>(P.lw, P, poly, tops, false, s);
}

}  // extern "C"
