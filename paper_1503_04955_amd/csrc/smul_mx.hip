// libdkss: SMUL's componentwise products (Step 5 of Sec. 2.9.3) on the matrix cores of gfx950.
//
// Element k of A becomes A_k B_k 2^(-log2 n) mod 2^K + 1 (K = 32 W bits, W = 64 lw limbs, lw <= 16),
// as k_smul_pointwise does on the vector units, with the 2K-bit product of the two factors (both
// below 2^K) computed from exact 8-bit integer products:
//
// The product is a convolution of the factors' N = 4W bytes.  With 64-byte blocks
// a = sum_i A_i z^i, b = sum_j B_j z^j (z = 2^512), the sums
//     C[r][k] = sum_i sum_(u < 64) A_i[r - u] B_(k-i)[u],   r < 128, k < 2 NB - 1,
// (A_i[x] = 0 outside 0 <= x < 64, B_j = 0 outside 0 <= j < NB) give column t = 64 k + r of the
// product from C[t mod 64][t div 64] + C[t mod 64 + 64][t div 64 - 1].  For fixed i the u-sum is a
// product of a 128 x 64 Toeplitz matrix of A_i's bytes with the 64 x (2 NB - 1) matrix of b's
// blocks: a dense contraction, done by v_mfma_i32_32x32x32_i8 (32 x 32 tiles, 32 bytes of the
// reduction per instruction).  The instruction takes signed bytes, so both factors enter as
// byte - 128 and the column sums are corrected with the factors' byte sums over each column's range:
//     sum a_x b_y = sum (a_x - 128)(b_y - 128) + 128 (sum a_x + sum b_y) - 16384 pairs,
// over the pairs x + y = t; prefix sums of the bytes give the ranges' sums.  Every column sum is
// below 4W 255^2 < 2^28, every partial sum of signed products below 2^26 in magnitude.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "../../include/dkss.h"
#include "hip_status.hpp"
#include "smul_ring.hpp"
#include "wave_carry.hpp"

namespace {

constexpr int kT = 256;                   // threads per workgroup: four wavefronts
constexpr int kMxMaxLw = 16;              // the products' LDS fits up to W = 1024 limbs

typedef int mx_v4i __attribute__((ext_vector_type(4)));
typedef int mx_v16i __attribute__((ext_vector_type(16)));

__host__ __device__ constexpr int mx_nb(int W) { return W / 16; }                 // 64-byte blocks
__host__ __device__ constexpr int mx_nct(int W) { return (2 * mx_nb(W) - 1 + 31) / 32; }   // 32-column tiles
__host__ __device__ constexpr int mx_pitch(int W) { return 32 * mx_nct(W) + 1; }  // int32 per row of C (odd)
// words of the padded, reversed first factor: per block 16 zero words, its 16 words byte-reversed
// in reverse order, 16 zero words; 4 more words of zeros at the end
__host__ __device__ constexpr int mx_apw(int W) { return 48 * mx_nb(W) + 4; }
__host__ __device__ constexpr size_t mx_al16(size_t x) { return (x + 15) & ~(size_t)15; }
// shared region: the padded first factor and the second factor's bytes while the products run,
// then the 64 x pitch column sums C, then the 2W word sums
__host__ __device__ constexpr size_t mx_region(int W) {
    return mx_al16(std::max(std::max((size_t)4 * mx_apw(W) + 4 * (size_t)W, (size_t)64 * mx_pitch(W) * 4),
                            (size_t)16 * W));
}
__host__ __device__ constexpr size_t mx_pref(int W) { return mx_al16((size_t)4 * (W + 1)); }
// LDS bytes: the factors (8W), the region, the word prefix sums of both factors' bytes, a 16-word
// scan scratch, the product's 2W words
__host__ __device__ constexpr size_t mx_lds_bytes(int W) {
    return (size_t)8 * W + mx_region(W) + 2 * mx_pref(W) + 64 + (size_t)8 * W;
}

// One wavefront: the 2W-word product P from its 64-bit word sums V (P = sum_w V_w 2^(32 w), each
// V_w below 2^53, so x_w = low(V_w) + high(V_(w-1)) < 2^33 carries one bit into the next word),
// into PW; then P = P_hi 2^K + P_lo = P_lo - P_hi (mod 2^K + 1) into R (V, PW and R in separate
// LDS).  Returns R's top.
__device__ __forceinline__ uint32_t mx_fold(const uint64_t* V, uint32_t* PW, uint32_t* R, int W) {
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
    return fw_norm(R, -(int)bo, W);
}

// Exclusive prefix over the workgroup of one value per thread (tmp: 4 words); also the total.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* tmp, uint32_t* total) {
    const int l = lane_id(), wv = (int)(threadIdx.x >> 6);
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (l >= d) x += y;
    }
    if (l == 63) tmp[wv] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int q = 0; q < kT / 64; ++q) {
        const uint32_t t = tmp[q];
        if (q < wv) before += t;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

__device__ __forceinline__ uint32_t mx_bytesum(uint32_t w) {
    return (w & 0xFFu) + ((w >> 8) & 0xFFu) + ((w >> 16) & 0xFFu) + (w >> 24);
}

// sum of the bytes x' < x of a factor (words X, word prefix sums PW of W + 1 entries), x <= 4W
__device__ __forceinline__ uint32_t mx_prefix(const uint32_t* X, const uint32_t* P, int x, int W) {
    const int w = x >> 2, e = x & 3;
    uint32_t s = P[w];
    if (e) s += mx_bytesum(X[w] & ((1u << (8 * e)) - 1u));
    (void)W;
    return s;
}

// One workgroup per element; B == A for a squaring; a factor equal to 2^K (= -1) makes the
// product the other factor's negation.
template <int LW>
__global__ __launch_bounds__(kT) void k_smul_pointwise_mx(uint32_t* Ap, uint32_t* At, const uint32_t* Bp,
                                                          const uint32_t* Bt, int log2n) {
    constexpr int W = 64 * LW;
    constexpr int K = 32 * W;
    constexpr int N = 4 * W;                     // bytes per factor
    constexpr int NB = mx_nb(W), KC = 2 * NB - 1, NCT = mx_nct(W), PITCH = mx_pitch(W);
    constexpr int APW = mx_apw(W);
    extern __shared__ uint4 smx[];
    unsigned char* const base = reinterpret_cast<unsigned char*>(smx);
    uint32_t* XA = reinterpret_cast<uint32_t*>(base);
    uint32_t* XB = XA + W;
    unsigned char* RG = base + 8 * W;
    uint32_t* AP = reinterpret_cast<uint32_t*>(RG);                       // APW words
    uint32_t* BS = reinterpret_cast<uint32_t*>(RG + 4 * APW);             // b's bytes, signed
    int* Cm = reinterpret_cast<int*>(RG);                                 // after the products
    uint64_t* V = reinterpret_cast<uint64_t*>(RG);                        // after the columns
    uint32_t* PA = reinterpret_cast<uint32_t*>(RG + mx_region(W));
    uint32_t* PB = reinterpret_cast<uint32_t*>(RG + mx_region(W) + mx_pref(W));
    uint32_t* TMP = reinterpret_cast<uint32_t*>(RG + mx_region(W) + 2 * mx_pref(W));
    uint32_t* PW = TMP + 16;
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
    uint32_t* R = XA;
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
        // the operands as byte - 128: the first factor padded and reversed per block (byte p of
        // block i's 192 bytes is A_i[127 - p] for 64 <= p < 128, zero elsewhere), the second
        // factor's bytes in order
        for (int d = threadIdx.x; d < APW; d += kT) {
            const int i = d / 48, m = d - 48 * i;
            uint32_t v = 0;
            if (i < NB && m >= 16 && m < 32) v = __builtin_bswap32(XA[16 * i + 31 - m]) ^ 0x80808080u;
            AP[d] = v;
        }
        for (int i = threadIdx.x; i < W; i += kT) BS[i] = XB[i] ^ 0x80808080u;
        // the factors' byte sums below each word: a scan over the workgroup, WT words per thread
        {
            constexpr int WT = (W + kT - 1) / kT;
            const int w0 = (int)threadIdx.x * WT;
            uint32_t sa = 0, sb = 0;
#pragma unroll
            for (int e = 0; e < WT; ++e) {
                if (w0 + e < W) {
                    sa += mx_bytesum(XA[w0 + e]);
                    sb += mx_bytesum(XB[w0 + e]);
                }
            }
            uint32_t ta, tb;
            uint32_t ea = block_excl_scan(sa, TMP, &ta);
            uint32_t eb = block_excl_scan(sb, TMP + 4, &tb);
#pragma unroll
            for (int e = 0; e < WT; ++e) {
                if (w0 + e < W) {
                    PA[w0 + e] = ea;
                    PB[w0 + e] = eb;
                    ea += mx_bytesum(XA[w0 + e]);
                    eb += mx_bytesum(XB[w0 + e]);
                }
            }
            if (threadIdx.x == kT - 1) {
                PA[W] = ta;
                PB[W] = tb;
            }
        }
        __syncthreads();
        // the products: wavefront wv accumulates NCT tiles (row tile rtl, column tile ct) of C
        const int wv = (int)(threadIdx.x >> 6), l = lane_id();
        mx_v16i acc[NCT];
#pragma unroll
        for (int q = 0; q < NCT; ++q)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[q][e] = 0;
        for (int i = 0; i < NB; ++i) {
#pragma unroll
            for (int ch = 0; ch < 2; ++ch) {
#pragma unroll
                for (int q = 0; q < NCT; ++q) {
                    const int t = wv + 4 * q;
                    const int rtl = t / NCT, ct = (t % NCT + rtl) % NCT;
                    // rows r < 32 meet bytes u <= r only, rows r >= 96 bytes u > r - 64 only
                    if ((rtl == 0 && ch == 1) || (rtl == 3 && ch == 0)) continue;
                    if (i < 32 * ct - NB + 1 || i > 32 * ct + 31) continue;
                    const int r = 32 * rtl + (l & 31);
                    const int u0 = 32 * ch + 16 * (l >> 5);
                    const int p = 192 * i + 127 - r + u0;        // A_i[r - u0 - e] at byte p + e
                    const uint32_t* src = AP + (p >> 2);
                    const int sh = p & 3;
                    const uint32_t w0 = src[0], w1 = src[1], w2 = src[2], w3 = src[3], w4 = src[4];
                    mx_v4i av, bv;
                    av[0] = (int)__builtin_amdgcn_alignbyte(w1, w0, sh);
                    av[1] = (int)__builtin_amdgcn_alignbyte(w2, w1, sh);
                    av[2] = (int)__builtin_amdgcn_alignbyte(w3, w2, sh);
                    av[3] = (int)__builtin_amdgcn_alignbyte(w4, w3, sh);
                    const int kk = 32 * ct + (l & 31), j = kk - i;
                    if (kk < KC && j >= 0 && j < NB) {
                        const uint4 q4 = *reinterpret_cast<const uint4*>(
                            reinterpret_cast<const unsigned char*>(BS) + 64 * j + u0);
                        bv[0] = (int)q4.x;
                        bv[1] = (int)q4.y;
                        bv[2] = (int)q4.z;
                        bv[3] = (int)q4.w;
                    } else {
                        bv[0] = bv[1] = bv[2] = bv[3] = 0;
                    }
                    acc[q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(av, bv, acc[q], 0, 0, 0);
                }
            }
        }
        __syncthreads();                                  // the operands are read: C takes the region
        // C'[r][k] = C[r][k] + C[r + 64][k - 1] (r < 64): the rows below 64 first, then the rows
        // above added one column on
#pragma unroll
        for (int ph = 0; ph < 2; ++ph) {
            if (ph == 0 && (int)threadIdx.x < 64) Cm[threadIdx.x * PITCH + 32 * NCT] = 0;
#pragma unroll
            for (int q = 0; q < NCT; ++q) {
                const int t = wv + 4 * q;
                const int rtl = t / NCT, ct = (t % NCT + rtl) % NCT;
                if ((rtl >= 2) != (ph == 1)) continue;
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int row = 32 * rtl + 8 * (e >> 2) + 4 * (l >> 5) + (e & 3);
                    const int col = 32 * ct + (l & 31);
                    if (ph == 0) Cm[row * PITCH + col] = acc[q][e];
                    else Cm[(row - 64) * PITCH + col + 1] += acc[q][e];
                }
            }
            __syncthreads();
        }
        // word sums V_w = sum_(e < 4) c_(4w + e) 2^(8e), c_t the corrected column sums
        constexpr int WPT = (2 * W + kT - 1) / kT;       // words per thread
        uint64_t vw[WPT];
#pragma unroll
        for (int g = 0; g < WPT; ++g) {
            const int w = (int)threadIdx.x + g * kT;
            uint64_t sum = 0;
            if (w < 2 * W) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int t = 4 * w + e;
                    if (t > 2 * N - 2) continue;
                    const long long m = Cm[(t & 63) * PITCH + (t >> 6)];
                    const int lo = t - N + 1 > 0 ? t - N + 1 : 0;
                    const int hi = t < N - 1 ? t : N - 1;
                    const long long sa = (long long)mx_prefix(XA, PA, hi + 1, W) - mx_prefix(XA, PA, lo, W);
                    const long long sb = (long long)mx_prefix(XB, PB, t - lo + 1, W) - mx_prefix(XB, PB, t - hi, W);
                    const long long c = m + 128 * (sa + sb) - 16384LL * (hi - lo + 1);
                    sum += (uint64_t)c << (8 * e);
                }
            }
            vw[g] = sum;
        }
        __syncthreads();                                  // C is read: V takes the region
#pragma unroll
        for (int g = 0; g < WPT; ++g) {
            const int w = (int)threadIdx.x + g * kT;
            if (w < 2 * W) V[w] = vw[g];
        }
        __syncthreads();
        if (wave0) rt = mx_fold(V, PW, R, W);
    }
    if (wave0) {
        // times 2^(-log2 n) = 2^(2K - log2 n) = -2^(K - log2 n)
        rt = fw_shift<LW>(R, rt, K - log2n);
        rt = fw_neg<LW>(R, rt);
        for (int i = lane_id(); i < W; i += 64) a[i] = R[i];
        if (lane_id() == 0) At[k] = rt;
    }
}

template <int LW>
int launch_mx(long long n, uint32_t* A, uint32_t* At, const uint32_t* B, const uint32_t* Bt, int log2n,
              hipStream_t s) {
    hipLaunchKernelGGL(k_smul_pointwise_mx<LW>, dim3((unsigned)n), dim3(kT), mx_lds_bytes(64 * LW), s, A, At, B, Bt,
                       log2n);
    return dkss::launch_status();
}

}  // namespace

namespace dkss {

bool smul_mx_supported(int lw) { return lw >= 1 && lw <= kMxMaxLw; }

int smul_pointwise_mx(int lw, long long n, uint32_t* A, uint32_t* At, const uint32_t* B, const uint32_t* Bt,
                      int log2n, hipStream_t s) {
    switch (lw) {
        case 1: return launch_mx<1>(n, A, At, B, Bt, log2n, s);
        case 2: return launch_mx<2>(n, A, At, B, Bt, log2n, s);
        case 4: return launch_mx<4>(n, A, At, B, Bt, log2n, s);
        case 8: return launch_mx<8>(n, A, At, B, Bt, log2n, s);
        case 16: return launch_mx<16>(n, A, At, B, Bt, log2n, s);
        default: return DKSS_ERANGE;
    }
}

}  // namespace dkss
