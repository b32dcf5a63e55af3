// libdkss: SMUL's componentwise products (Step 5 of Sec. 2.9.3) on the matrix cores of gfx950.
//
// Element k of A becomes A_k B_k 2^(-log2 n) mod 2^K + 1 (K = 32 W bits, W = 64 lw limbs, lw <= 16),
// as k_smul_pointwise does on the vector units, with the 2K-bit product of the two factors (both
// below 2^K) computed from exact 8-bit integer products:
//
// The product is a convolution of the factors' N = 4W bytes.  With column t = 32 T + r (r < 32) of
// the product and b's 32-byte groups b_g (g < NG = N / 32), the sums
//     C[r][T] = sum_d sum_(u < 32) a[32 d + r - u] b_(T - d)[u],   0 <= d <= NG,
// (a zero outside 0 <= x < N, b_g = 0 outside 0 <= g < NG) are column 32 T + r.  For fixed d the
// u-sum is the 32 x 32 Toeplitz matrix W_d[r][u] = a[32 d + r - u] of a 63-byte window of a times
// the 32 x (2 NG) matrix of b's groups shifted by d: a dense contraction, done by
// v_mfma_i32_32x32x32_i8 on 32 x 32 tiles of C (32 bytes of the reduction per instruction), each
// W_d loaded once and applied to every tile it meets, about (NG + 1)(NG / 16 + 1) instructions per
// element (640 at N = 4096, 1.25 N^2 byte products).  The instruction takes signed bytes, so both
// factors enter as byte - 128 and the column sums are corrected with the factors' byte sums over
// each column's range:
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

__host__ __device__ constexpr int mx_ng(int W) { return W / 8; }                 // 32-byte groups of b
__host__ __device__ constexpr int mx_nt(int W) { return (2 * mx_ng(W) + 31) / 32; }   // 32-column tiles of C
__host__ __device__ constexpr int mx_pitch(int W) { return 2 * mx_ng(W) + 1; }    // int32 per row of C (odd)
// words of one copy of the padded, reversed first factor (N + 64 bytes)
__host__ __device__ constexpr int mx_cw(int W) { return W + 16; }
__host__ __device__ constexpr size_t mx_al16(size_t x) { return (x + 15) & ~(size_t)15; }
// shared region: four copies of the padded first factor and the second factor's bytes while the
// products run, then the 32 x pitch column sums C, then the 2W word sums and the product's 2W
// words
__host__ __device__ constexpr size_t mx_region(int W) {
    return mx_al16(std::max(std::max((size_t)16 * mx_cw(W) + 4 * (size_t)W, (size_t)32 * mx_pitch(W) * 4),
                            (size_t)24 * W));
}
__host__ __device__ constexpr size_t mx_pref(int W) { return mx_al16((size_t)4 * (W + 1)); }
// LDS bytes: the factors (8W), the region, the word prefix sums of both factors' bytes, a 16-word
// scan scratch (under 50 KB at W = 1024: three workgroups per CU)
__host__ __device__ constexpr size_t mx_lds_bytes(int W) {
    return (size_t)8 * W + mx_region(W) + 2 * mx_pref(W) + 64;
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
__global__ __launch_bounds__(kT, 3) void k_smul_pointwise_mx(uint32_t* Ap, uint32_t* At, const uint32_t* Bp,
                                                          const uint32_t* Bt, int log2n) {
    constexpr int W = 64 * LW;
    constexpr int K = 32 * W;
    constexpr int N = 4 * W;                     // bytes per factor
    constexpr int NG = mx_ng(W), NT = mx_nt(W), PITCH = mx_pitch(W), CW = mx_cw(W);
    extern __shared__ uint4 smx[];
    unsigned char* const base = reinterpret_cast<unsigned char*>(smx);
    uint32_t* XA = reinterpret_cast<uint32_t*>(base);
    uint32_t* XB = XA + W;
    unsigned char* RG = base + 8 * W;
    uint32_t* AR = reinterpret_cast<uint32_t*>(RG);                       // 4 CW words
    uint32_t* BS = reinterpret_cast<uint32_t*>(RG + 16 * CW);             // b's bytes, signed
    int* Cm = reinterpret_cast<int*>(RG);                                 // after the products
    uint64_t* V = reinterpret_cast<uint64_t*>(RG);                        // after the columns
    uint32_t* PA = reinterpret_cast<uint32_t*>(RG + mx_region(W));
    uint32_t* PB = reinterpret_cast<uint32_t*>(RG + mx_region(W) + mx_pref(W));
    uint32_t* TMP = reinterpret_cast<uint32_t*>(RG + mx_region(W) + 2 * mx_pref(W));
    uint32_t* PW = reinterpret_cast<uint32_t*>(RG + 16 * (size_t)W);            // after the word sums
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
        // the operands as byte - 128: the first factor padded with 32 zero bytes on each side and
        // reversed, AR[i] = a[N + 31 - i] (zero outside a), in four copies shifted by c = 0..3
        // bytes (copy c, byte i: AR[i + c]) so that every lane's 16-byte run starts on a word; the
        // second factor's bytes in order
        for (int q = threadIdx.x; q < 4 * CW; q += kT) {
            const int c = q / CW, wi = q - c * CW;
            uint32_t v = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int x = N + 31 - 4 * wi - e - c;
                if (x >= 0 && x < N) v |= (((XA[x >> 2] >> (8 * (x & 3))) & 0xFFu) ^ 0x80u) << (8 * e);
            }
            AR[q] = v;
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
        // the products: wavefront wv takes d = wv, wv + 4, ... and all column tiles; lane (r, h)
        // holds W_d[r][16h .. 16h + 15] (bytes a[32d + r - 16h - e], a run of AR from
        // s = N + 31 - 32d - r + 16h, word-aligned in copy s mod 4) and, for tile ct, column
        // T = 32 ct + r of the shifted groups (b_(T - d) bytes 16h .. 16h + 15)
        const int wv = (int)(threadIdx.x >> 6), l = lane_id();
        const int r = l & 31, h = l >> 5;
        mx_v16i acc[NT];
#pragma unroll
        for (int q = 0; q < NT; ++q)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[q][e] = 0;
        for (int d = wv; d <= NG; d += 4) {
            const int sidx = N + 31 - 32 * d - r + 16 * h;
            const int c = sidx & 3;
            const uint32_t* src = AR + c * CW + ((sidx - c) >> 2);
            mx_v4i av;
            av[0] = (int)src[0];
            av[1] = (int)src[1];
            av[2] = (int)src[2];
            av[3] = (int)src[3];
#pragma unroll
            for (int ct = 0; ct < NT; ++ct) {
                if (32 * ct - d + 31 < 0 || 32 * ct - d >= NG) continue;     // no group of b meets it
                const int g = 32 * ct + r - d;
                mx_v4i bv;
                if (g >= 0 && g < NG) {
                    const uint4 q4 = *reinterpret_cast<const uint4*>(
                        reinterpret_cast<const unsigned char*>(BS) + 32 * g + 16 * h);
                    bv[0] = (int)q4.x;
                    bv[1] = (int)q4.y;
                    bv[2] = (int)q4.z;
                    bv[3] = (int)q4.w;
                } else {
                    bv[0] = bv[1] = bv[2] = bv[3] = 0;
                }
                acc[ct] = __builtin_amdgcn_mfma_i32_32x32x32_i8(av, bv, acc[ct], 0, 0, 0);
            }
        }
        __syncthreads();                                  // the operands are read: C takes the region
        for (int i = threadIdx.x; i < 32 * PITCH; i += kT) Cm[i] = 0;
        __syncthreads();
        // C[row][T] summed over the four wavefronts (row-major at an odd pitch: the lanes of one
        // add hit distinct banks)
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
            const int T = 32 * ct + r;
            if (T >= 2 * NG) continue;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int row = 8 * (e >> 2) + 4 * h + (e & 3);
                atomicAdd(&Cm[row * PITCH + T], acc[ct][e]);
            }
        }
        __syncthreads();
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
                    const long long m = Cm[(t & 31) * PITCH + (t >> 5)];
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
