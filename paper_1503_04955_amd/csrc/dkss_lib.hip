// libdkss: DKSS multiplication of large unsigned integers on one MI355X (gfx950).
//
// Pipeline of one product c = a*b (thesis Sec. 3.2, Steps 4-8), all on one HIP stream:
//   k_encode      Step 4 (Sec. 3.2.4): operand bits -> 2M elements of R, u bits per coefficient
//   k_dft         Step 5 (Sec. 3.2.5 i/iii): one FFT level = independent radix-r DFTs with root
//                 alpha^(2m/r) over columns of stride mu, staged in LDS; every butterfly
//                 multiplies by a power of alpha, i.e. rotates and negates coefficients
//   k_twiddle     Step 5 (Sec. 3.2.5 ii): the "bad multiplications" by rho^(base*l*v) between
//                 levels; rho^e = alpha^(e div mu_top) rho^(e mod mu_top) (Sec. 4.2), the alpha
//                 power folded into the product's indexing
//   k_pointwise   Step 6 (Sec. 3.2.6): componentwise products in R, scaled by (2M)^-1
//   inverse FFT   Step 7 (Sec. 3.2.7): the levels in reverse order with root rho^-1 (twiddles
//                 first, then DFTs with alpha^-1), which returns natural order directly
//   k_decode      Step 8 (Sec. 3.2.8): evaluate at alpha = 2^u, x = 2^(um/2); per 32-bit word
//                 the overlapping coefficient pieces are summed, leaving a 1-bit carry per word
//   k_carry_*     carry resolution: 64-word generate/propagate masks per wavefront (ballot),
//                 carries inside a wavefront by one 64-bit addition, a scan across wavefronts
//
// The forward transform runs the levels top-down (decimation in frequency: natural input,
// digit-reversed output); the inverse runs them bottom-up (decimation in time: digit-reversed
// input, natural output), so no reordering pass is needed between them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/dkss.h"
#include "kernels.hpp"
#include "planner.hpp"

using namespace dkss;

namespace {

constexpr int kThreads = 256;
constexpr int kTaskMax = 4;              // radix-2 butterfly tasks per thread per pass
constexpr uint64_t kDefaultCutoffBits = 2048;
constexpr size_t kSchoolbookMaxWords = 4096;   // alen + blen of the base case

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

__device__ __forceinline__ int bitrev(int x, int bits) {
    return bits ? (int)(__brev((unsigned)x) >> (32 - bits)) : 0;
}

// ---------------------------------------------------------------------------------------------
// Step 4: encode
// ---------------------------------------------------------------------------------------------

// poly: 2M elements x m coefficients x L limbs.  Coefficient k < m/2 of element i < M gets bits
// [u (i m/2 + k), u (i m/2 + k) + u) of a; all others are zero.
template <int L>
__global__ __launch_bounds__(kThreads) void k_encode(uint32_t* __restrict__ poly,
                                                     const uint32_t* __restrict__ a, long long alen,
                                                     long long M, int log2m, int u) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (2 * M) << log2m;
    if (t >= total) return;
    const int m = 1 << log2m;
    const long long i = t >> log2m;
    const int k = (int)(t & (m - 1));
    uint32_t out[L];
#pragma unroll
    for (int w = 0; w < L; ++w) out[w] = 0;
    if (i < M && k < m / 2) {
        const unsigned long long pos = ((unsigned long long)i * (m / 2) + k) * (unsigned)u;
#pragma unroll
        for (int w = 0; w < L; ++w) {
            const int nb = u - 32 * w;
            if (nb > 0) {
                const unsigned long long bit = pos + 32ull * w;
                const long long wi = (long long)(bit >> 5);
                const int sh = (int)(bit & 31);
                const uint64_t lo = wi < alen ? a[wi] : 0u;
                const uint64_t hi = wi + 1 < alen ? a[wi + 1] : 0u;
                uint32_t v = (uint32_t)(((hi << 32) | lo) >> sh);
                if (nb < 32) v &= (1u << nb) - 1u;
                out[w] = v;
            }
        }
    }
    uint32_t* dst = poly + (size_t)t * L;
#pragma unroll
    for (int w = 0; w < L; ++w) dst[w] = out[w];
}

// ---------------------------------------------------------------------------------------------
// Step 5: one FFT level of radix-r DFTs with root alpha^(+-2m/r)
// ---------------------------------------------------------------------------------------------

// Columns: the level has 2M/n_lvl blocks of n_lvl elements; within a block, column l < mu holds
// elements l, l + mu, ..., l + (r-1) mu.  A workgroup takes C consecutive columns, loads them
// into LDS in bit-reversed order and runs log2 r radix-2 decimation-in-time passes; the pass that
// merges halves of h points multiplies the odd half by alpha^((m/h) k), k < h (alpha^-... for the
// inverse).  Output v goes to element l + v mu.
template <int L>
__global__ __launch_bounds__(kThreads) void k_dft(uint32_t* __restrict__ poly, long long n_lvl,
                                                  long long mu, int log2r, int log2m, int C,
                                                  long long ncols, int inverse, QConst Q) {
    extern __shared__ uint32_t sm[];
    const int m = 1 << log2m, r = 1 << log2r;
    const int EW = m * L;
    const long long c0 = (long long)blockIdx.x * C;
    const int ncol = (int)min((long long)C, ncols - c0);
    const int total = ncol * r * EW;
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
        const int wk = t % EW;
        const int rest = t / EW;
        const int c = rest % ncol;
        const int j1 = rest / ncol;
        const long long col = c0 + c;
        const long long b = col / mu, l = col - b * mu;
        const long long el = b * n_lvl + (long long)j1 * mu + l;
        sm[(c * r + bitrev(j1, log2r)) * EW + wk] = poly[(size_t)el * EW + wk];
    }
    __syncthreads();
    const int half_r = r >> 1;
    const int tasks = ncol * half_r * m;
    for (int h = 1; h < r; h <<= 1) {
        uint32_t nx[kTaskMax][L], ny[kTaskMax][L];
        const int mh = m / h;
#pragma unroll
        for (int it = 0; it < kTaskMax; ++it) {
            const int t = threadIdx.x + it * kThreads;
            if (t < tasks) {
                const int jj = t & (m - 1);
                const int rest = t >> log2m;
                const int bf = rest % half_r;
                const int c = rest / half_r;
                const int kk = bf & (h - 1);
                const int xs = (bf - kk) * 2 + kk;
                const int ys = xs + h;
                int e = kk * mh;
                if (inverse) e = (2 * m - e) & (2 * m - 1);
                // (alpha^e y)_jj = +- y_idx, negated once per wrap past degree m-1
                int idx = jj - e;
                bool neg = false;
                if (idx < 0) {
                    idx += m;
                    neg = true;
                    if (idx < 0) {
                        idx += m;
                        neg = false;
                    }
                }
                const uint32_t* X = sm + (c * r + xs) * EW + jj * L;
                const uint32_t* Y = sm + (c * r + ys) * EW + idx * L;
                uint32_t xv[L], yv[L], s[L], d[L];
#pragma unroll
                for (int w = 0; w < L; ++w) {
                    xv[w] = X[w];
                    yv[w] = Y[w];
                }
                mod_add<L>(s, xv, yv, Q);
                mod_sub<L>(d, xv, yv, Q);
#pragma unroll
                for (int w = 0; w < L; ++w) {
                    nx[it][w] = neg ? d[w] : s[w];
                    ny[it][w] = neg ? s[w] : d[w];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kTaskMax; ++it) {
            const int t = threadIdx.x + it * kThreads;
            if (t < tasks) {
                const int jj = t & (m - 1);
                const int rest = t >> log2m;
                const int bf = rest % half_r;
                const int c = rest / half_r;
                const int kk = bf & (h - 1);
                const int xs = (bf - kk) * 2 + kk;
                const int ys = xs + h;
                uint32_t* X = sm + (c * r + xs) * EW + jj * L;
                uint32_t* Y = sm + (c * r + ys) * EW + jj * L;
#pragma unroll
                for (int w = 0; w < L; ++w) {
                    X[w] = nx[it][w];
                    Y[w] = ny[it][w];
                }
            }
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
        const int wk = t % EW;
        const int rest = t / EW;
        const int c = rest % ncol;
        const int v = rest / ncol;
        const long long col = c0 + c;
        const long long b = col / mu, l = col - b * mu;
        const long long el = b * n_lvl + (long long)v * mu + l;
        poly[(size_t)el * EW + wk] = sm[(c * r + v) * EW + wk];
    }
}

// ---------------------------------------------------------------------------------------------
// Step 5 ii: bad multiplications, element (block, v, l) *= rho^(+-base l v)
// ---------------------------------------------------------------------------------------------

// m threads per element, 256/m elements per workgroup.  LDS per element: the m digits-coefficients
// of the table entry rho^s (Montgomery form) and the 2m of the element's negacyclic extension.
template <int L>
__global__ __launch_bounds__(kThreads) void k_twiddle(uint32_t* __restrict__ poly,
                                                      const uint32_t* __restrict__ table,
                                                      long long twoM, long long n_lvl, long long mu,
                                                      long long base, long long mu_top, int log2m,
                                                      int inverse, QConst Q) {
    using G = Dig<L>;
    extern __shared__ uint32_t sm[];
    const int m = 1 << log2m;
    const int per = kThreads >> log2m;
    const int g = threadIdx.x >> log2m, j = threadIdx.x & (m - 1);
    uint32_t* T = sm + g * 3 * m * G::D;
    uint32_t* E = T + m * G::D;
    const long long p = (long long)blockIdx.x * per + g;
    long long e = 0;
    if (p < twoM) {
        const long long o = p % n_lvl;
        const long long v = o / mu, l = o - v * mu;
        e = base * l * v;                       // < base * n_lvl = 2M
        if (inverse && e) e = twoM - e;
    }
    const bool active = e != 0;
    int rot = 0;
    if (active) {
        rot = (int)(e / mu_top);
        const long long s = e - (long long)rot * mu_top;
        uint32_t x[L], nx[L];
        const uint32_t* src = poly + ((size_t)p * m + j) * L;
#pragma unroll
        for (int w = 0; w < L; ++w) x[w] = src[w];
        neg_q<L>(nx, x, Q);
        limbs_to_digits<L>(x, E + j * G::D);
        limbs_to_digits<L>(nx, E + (j + m) * G::D);
        const uint32_t* ts = table + ((size_t)s * m + j) * G::D;
#pragma unroll
        for (int y = 0; y < G::D; ++y) T[j * G::D + y] = ts[y];
    }
    __syncthreads();
    if (active) {
        uint32_t out[L];
        rprod_coeff<L>(T, E, log2m, j, rot, Q, out);
        uint32_t* dst = poly + ((size_t)p * m + j) * L;
#pragma unroll
        for (int w = 0; w < L; ++w) dst[w] = out[w];
    }
}

// ---------------------------------------------------------------------------------------------
// Step 6: componentwise products, A[i] = A[i] * B[i] (2M)^-1
// ---------------------------------------------------------------------------------------------

template <int L>
__global__ __launch_bounds__(kThreads) void k_pointwise(uint32_t* A, const uint32_t* B,
                                                        long long count, int log2m, QConst Q) {
    using G = Dig<L>;
    extern __shared__ uint32_t sm[];
    const int m = 1 << log2m;
    const int per = kThreads >> log2m;
    const int g = threadIdx.x >> log2m, j = threadIdx.x & (m - 1);
    uint32_t* T = sm + g * 3 * m * G::D;
    uint32_t* E = T + m * G::D;
    const long long p = (long long)blockIdx.x * per + g;
    const bool active = p < count;
    if (active) {
        uint32_t x[L], y[L], ny[L];
        const uint32_t* sa = A + ((size_t)p * m + j) * L;
        const uint32_t* sb = B + ((size_t)p * m + j) * L;
#pragma unroll
        for (int w = 0; w < L; ++w) {
            x[w] = sa[w];
            y[w] = sb[w];
        }
        neg_q<L>(ny, y, Q);
        limbs_to_digits<L>(x, T + j * G::D);
        limbs_to_digits<L>(y, E + j * G::D);
        limbs_to_digits<L>(ny, E + (j + m) * G::D);
    }
    __syncthreads();
    if (active) {
        uint32_t c[L], out[L];
        rprod_coeff<L>(T, E, log2m, j, 0, Q, c);     // (a*b)_j 2^-28K
        mont_scalar<L>(c, Q.kpw, Q, out);            // * (2M)^-1 2^28K
        uint32_t* dst = A + ((size_t)p * m + j) * L;
#pragma unroll
        for (int w = 0; w < L; ++w) dst[w] = out[w];
    }
}

// ---------------------------------------------------------------------------------------------
// Table of rho^s, s < mu_top, in Montgomery form, 28-bit digits.  One launch computes
// table[dst + j] = table[src + j] * table[mul] for j < cnt (all in Montgomery form).
// ---------------------------------------------------------------------------------------------

template <int L>
__global__ __launch_bounds__(kThreads) void k_table_mul(uint32_t* table, long long src, long long mul,
                                                        long long dst, long long cnt, int log2m,
                                                        QConst Q) {
    using G = Dig<L>;
    extern __shared__ uint32_t sm[];
    const int m = 1 << log2m;
    const int per = kThreads >> log2m;
    const int g = threadIdx.x >> log2m, j = threadIdx.x & (m - 1);
    uint32_t* T = sm + g * 3 * m * G::D;
    uint32_t* E = T + m * G::D;
    const long long jj = (long long)blockIdx.x * per + g;
    const bool active = jj < cnt;
    if (active) {
        const uint32_t* xs = table + ((size_t)(src + jj) * m + j) * G::D;
        const uint32_t* ts = table + ((size_t)mul * m + j) * G::D;
        uint32_t xd[G::D + 1], x[L], nx[L];
#pragma unroll
        for (int y = 0; y < G::D; ++y) {
            xd[y] = xs[y];
            T[j * G::D + y] = ts[y];
        }
        xd[G::D] = 0;
        digits_to_limbs<L>(xd, x);
        neg_q<L>(nx, x, Q);
#pragma unroll
        for (int y = 0; y < G::D; ++y) E[j * G::D + y] = xd[y];
        limbs_to_digits<L>(nx, E + (j + m) * G::D);
    }
    __syncthreads();
    if (active) {
        uint32_t out[L];
        rprod_coeff<L>(T, E, log2m, j, 0, Q, out);
        uint32_t od[G::D];
        limbs_to_digits<L>(out, od);
        uint32_t* dst_p = table + ((size_t)(dst + jj) * m + j) * G::D;
#pragma unroll
        for (int y = 0; y < G::D; ++y) dst_p[y] = od[y];
    }
}

// ---------------------------------------------------------------------------------------------
// Step 8: decode and carry
// ---------------------------------------------------------------------------------------------

// Sum of the 32-bit pieces that the coefficients c_(l,k) (value sum c_(l,k) 2^(u (k + l m/2)))
// put into output word w.  Coefficients are exact integers below 2^(32L).
template <int L>
__device__ __forceinline__ uint64_t word_sum(long long w, const uint32_t* __restrict__ poly,
                                             long long twoM, int log2m, int u) {
    const int m = 1 << log2m;
    const int hm = m >> 1;
    const long long lo_excl = 32 * w - 32 * L;            // piece iff u g > lo_excl
    const long long g_lo = lo_excl < 0 ? 0 : lo_excl / u + 1;
    const long long g_hi = (32 * w + 31) / u;
    uint64_t V = 0;
    for (long long g = g_lo; g <= g_hi; ++g) {
        const long long P = (long long)u * g;
        const long long off = 32 * w - P;                  // bit of the term at word w's bit 0
        const long long lmax = g / hm;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const long long l = lmax - t;
            if (l < 0 || l >= twoM) continue;
            const int k = (int)(g - l * hm);
            const uint32_t* T = poly + ((size_t)l * m + k) * L;
            uint32_t piece;
            if (off >= 0) {
                const int li = (int)(off >> 5), bs = (int)(off & 31);
                uint64_t v = T[li];
                if (li + 1 < L) v |= (uint64_t)T[li + 1] << 32;
                piece = (uint32_t)(v >> bs);
            } else {
                piece = T[0] << (int)(-off);
            }
            V += piece;
        }
    }
    return V;
}

// Per 256 output words: x_w = low(V_w) + high(V_(w-1)) < 2^32 + 2^5, so word w generates a carry
// (x_w >= 2^32) or propagates one (low 32 bits all ones), never both.  Writes the low 32 bits
// and the per-wavefront generate / propagate masks.
template <int L>
__global__ __launch_bounds__(kThreads) void k_decode(uint32_t* __restrict__ out, long long nw,
                                                     const uint32_t* __restrict__ poly,
                                                     long long twoM, int log2m, int u,
                                                     unsigned long long* __restrict__ gmask,
                                                     unsigned long long* __restrict__ pmask) {
    __shared__ uint32_t hiv[kThreads + 1];
    const long long w0 = (long long)blockIdx.x * kThreads;
    const long long w = w0 + threadIdx.x;
    const uint64_t V = w < nw ? word_sum<L>(w, poly, twoM, log2m, u) : 0;
    hiv[threadIdx.x + 1] = (uint32_t)(V >> 32);
    if (threadIdx.x == 0)
        hiv[0] = w0 > 0 ? (uint32_t)(word_sum<L>(w0 - 1, poly, twoM, log2m, u) >> 32) : 0u;
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

// carry out of a 64-word wavefront for a carry in c: the carry out of (G|P) + G + c
__device__ __forceinline__ void wave_fn(unsigned long long G, unsigned long long P, bool* g, bool* p) {
    const unsigned long long A = G | P;
    const unsigned long long s = A + G;
    const bool c0 = s < A;
    *g = c0;
    *p = c0 || s == ~0ull;
}

// Single workgroup: carry into every wavefront.  Each thread composes the carry functions
// c -> g | (p & c) of a contiguous run of wavefronts; thread 0 scans the 1024 compositions.
__global__ __launch_bounds__(1024) void k_carry_scan(const unsigned long long* __restrict__ gmask,
                                                     const unsigned long long* __restrict__ pmask,
                                                     unsigned char* __restrict__ cin,
                                                     long long nwaves) {
    __shared__ unsigned char ag[1024], ap[1024], ac[1024];
    const long long ch = (nwaves + 1023) / 1024;
    const long long s = threadIdx.x * ch;
    const long long e = min(s + ch, nwaves);
    bool fg = false, fp = true;
    for (long long k = s; k < e; ++k) {
        bool g, p;
        wave_fn(gmask[k], pmask[k], &g, &p);
        fg = g || (p && fg);
        fp = p && fp;
    }
    ag[threadIdx.x] = fg;
    ap[threadIdx.x] = fp;
    __syncthreads();
    if (threadIdx.x == 0) {
        bool c = false;
        for (int i = 0; i < 1024; ++i) {
            ac[i] = c;
            c = ag[i] || (ap[i] && c);
        }
    }
    __syncthreads();
    bool c = ac[threadIdx.x];
    for (long long k = s; k < e; ++k) {
        cin[k] = c;
        bool g, p;
        wave_fn(gmask[k], pmask[k], &g, &p);
        c = g || (p && c);
    }
}

// word w += carry into w: bit (w mod 64) of ((G|P) + G + cin) ^ (G|P) ^ G
__global__ __launch_bounds__(kThreads) void k_carry_apply(uint32_t* __restrict__ out, long long nw,
                                                          const unsigned long long* __restrict__ gmask,
                                                          const unsigned long long* __restrict__ pmask,
                                                          const unsigned char* __restrict__ cin) {
    const long long w = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nw) return;
    const long long wave = w >> 6;
    const unsigned long long G = gmask[wave], A = G | pmask[wave];
    const unsigned long long carries = (A + G + (unsigned long long)cin[wave]) ^ A ^ G;
    out[w] += (uint32_t)((carries >> (w & 63)) & 1);
}

// ---------------------------------------------------------------------------------------------
// Base case: schoolbook product (Sec. 2.3), one workgroup per product, alen + blen <= 4096
// ---------------------------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_schoolbook(uint32_t* __restrict__ c,
                                                         const uint32_t* __restrict__ a, long long alen,
                                                         const uint32_t* __restrict__ b, long long blen) {
    extern __shared__ uint32_t sv[];
    const long long n = alen + blen;
    for (long long w = threadIdx.x; w < n; w += blockDim.x) {
        uint64_t lo = 0, hi = 0;
        const long long i0 = w - blen + 1 > 0 ? w - blen + 1 : 0;
        const long long i1 = w < alen - 1 ? w : alen - 1;
        for (long long i = i0; i <= i1; ++i) {
            const uint64_t p = (uint64_t)a[i] * b[w - i];
            lo += (uint32_t)p;
            hi += p >> 32;
        }
        const uint64_t t = hi + (lo >> 32);
        sv[3 * w] = (uint32_t)lo;
        sv[3 * w + 1] = (uint32_t)t;
        sv[3 * w + 2] = (uint32_t)(t >> 32);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t carry = 0;
        for (long long w = 0; w < n; ++w) {
            uint64_t s = carry + sv[3 * w];
            if (w >= 1) s += sv[3 * (w - 1) + 1];
            if (w >= 2) s += sv[3 * (w - 2) + 2];
            c[w] = (uint32_t)s;
            carry = s >> 32;
        }
    }
}

__global__ void k_fill(uint32_t* __restrict__ p, long long n, uint32_t v) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------------------------
// Forward output in digit-reversed order -> natural order (dkss_forward only)
// ---------------------------------------------------------------------------------------------

struct LevelIdx {
    int n;
    int log2mu[8];
    int log2r[8];
    int shift[8];    // log2 of the product of the radices of the earlier levels
};

__global__ void k_unscramble(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src,
                             long long twoM, int EW, LevelIdx LI) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= twoM * EW) return;
    const long long pos = t / EW;
    const int wk = (int)(t - pos * EW);
    long long f = 0;
    for (int k = 0; k < LI.n; ++k) {
        const long long v = (pos >> LI.log2mu[k]) & ((1LL << LI.log2r[k]) - 1);
        f |= v << LI.shift[k];
    }
    dst[(size_t)f * EW + wk] = src[t];
}

// ---------------------------------------------------------------------------------------------
// Residues x mod q for one-word primes q < 2^62 (Montgomery arithmetic with R = 2^64)
// ---------------------------------------------------------------------------------------------

__device__ __forceinline__ uint64_t montmul64(uint64_t a, uint64_t b, uint64_t q, uint64_t qinv) {
    const uint64_t lo = a * b, hi = __umul64hi(a, b);
    const uint64_t mq = lo * qinv;                        // lo + mq*q = 0 mod 2^64
    const uint64_t mlo = mq * q, mhi = __umul64hi(mq, q);
    const uint64_t carry = (lo + mlo) < lo ? 1 : 0;
    uint64_t r = hi + mhi + carry;
    if (r >= q) r -= q;
    return r;
}

struct ResConst {
    uint64_t q, qinv;     // q and -q^-1 mod 2^64
    uint64_t w;           // 2^32 * 2^64 mod q  (multiplying by it = times 2^32)
    uint64_t chunk_pow[9];// 2^(32*64*2^k) * 2^64 mod q, k <= 8
};

// per workgroup: sum_{i in block} x_i 2^(32 (i - i0)) mod q over 256 chunks of 64 limbs
__global__ __launch_bounds__(kThreads) void k_residue_block(const uint32_t* __restrict__ x, long long n,
                                                            ResConst R, uint64_t* __restrict__ part) {
    __shared__ uint64_t rs[kThreads];
    const long long base = (long long)blockIdx.x * kThreads * 64 + (long long)threadIdx.x * 64;
    uint64_t r = 0;
    for (int i = 63; i >= 0; --i) {
        const long long k = base + i;
        r = montmul64(r, R.w, R.q, R.qinv);
        uint64_t xv = k < n ? x[k] : 0u;
        if (xv >= R.q) xv %= R.q;                // only for q below 2^32
        r += xv;
        if (r >= R.q) r -= R.q;
    }
    rs[threadIdx.x] = r;
    __syncthreads();
    int lvl = 0;
    for (int s = 1; s < kThreads; s <<= 1, ++lvl) {
        if ((threadIdx.x & (2 * s - 1)) == 0) {
            uint64_t v = rs[threadIdx.x] + montmul64(rs[threadIdx.x + s], R.chunk_pow[lvl], R.q, R.qinv);
            if (v >= R.q) v -= R.q;
            rs[threadIdx.x] = v;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = rs[0];
}

__global__ void k_residue_final(const uint64_t* __restrict__ part, long long nb, ResConst R,
                                uint64_t* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint64_t r = 0;
    for (long long b = nb - 1; b >= 0; --b) {
        r = montmul64(r, R.chunk_pow[8], R.q, R.qinv);
        r += part[b];
        if (r >= R.q) r -= R.q;
    }
    *out = r;
}

// ---------------------------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------------------------

// Event-based kernel timing (enabled per context).
struct Prof {
    bool on = false;
    struct Rec {
        int kind;
        hipEvent_t e0, e1;
        double bytes, ops;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    dkss_kernel_stats tot[DKSS_K_KINDS] = {};

    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    int drain() {
        int rc = DKSS_OK;
        for (Rec& r : pending) {
            float ms = 0.f;
            if (hipEventSynchronize(r.e1) != hipSuccess || hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess)
                rc = DKSS_EHIP;
            dkss_kernel_stats& t = tot[r.kind];
            t.launches += 1;
            t.total_ms += ms;
            t.alg_bytes += r.bytes;
            t.alg_ops += r.ops;
            pool.push_back(r.e0);
            pool.push_back(r.e1);
        }
        pending.clear();
        return rc;
    }
    ~Prof() {
        (void)drain();
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

// Brackets one kernel launch with events when profiling is on.
struct ProfScope {
    Prof* p;
    int kind;
    hipStream_t s;
    hipEvent_t e0 = nullptr;
    double bytes, ops;
    ProfScope(Prof* pp, int k, hipStream_t st, double b, double o) : p(pp), kind(k), s(st), bytes(b), ops(o) {
        if (p && p->on) {
            e0 = p->get();
            if (e0) (void)hipEventRecord(e0, s);
        }
    }
    ~ProfScope() {
        if (e0) {
            hipEvent_t e1 = p->get();
            if (e1) {
                (void)hipEventRecord(e1, s);
                p->pending.push_back({kind, e0, e1, bytes, ops});
            } else {
                p->pool.push_back(e0);
            }
        }
    }
};

struct Cached {
    Plan plan;                 // constants (parameters as resolved for the key)
    QConst Q;
    std::vector<uint32_t> table_host01;   // entries 0 and 1 of the table (digits)
    uint32_t* d_table = nullptr;
    long long table_count = 0;
    int D = 0;
};

// resolved per-call plan
struct Call {
    Plan P;                    // parameters + radices
    bool schoolbook = false;
    size_t alen = 0, blen = 0;
    Cached* C = nullptr;
    Prof* prof = nullptr;
};

int dig_D(int L) { return (32 * L + 27) / 28; }
int dig_K(int L) { return (32 * L + 6 + 27) / 28; }

}  // namespace

struct dkss_ctx {
    int policy = DKSS_POLICY_THESIS;
    std::map<std::string, std::unique_ptr<Cached>> cache;
    Prof prof;
};

namespace {

#define HIP_OK(expr)                                  \
    do {                                              \
        if ((expr) != hipSuccess) return DKSS_EHIP;   \
    } while (0)

// parameters for a product, from the policy or the caller
int resolve_params(dkss_ctx* ctx, size_t alen, size_t blen, const dkss_params* p, Call* out) {
    (void)ctx;
    out->alen = alen;
    out->blen = blen;
    const uint64_t N = 32ull * std::max(alen, blen);
    Plan& P = out->P;
    if (N == 0) return DKSS_OK;
    if (N > (1ull << 36)) return DKSS_ERANGE;
    if (p == nullptr) {
        int lM, lm, u, pb;
        if (!thesis_params(N, &lM, &lm, &u, &pb)) return DKSS_ERANGE;
        P.log2_M = lM;
        P.log2_m = lm;
        P.u = u;
        P.p_bits = pb;
        P.z = 1;
        P.cutoff_bits = kDefaultCutoffBits;
    } else {
        P.log2_M = (int)p->log2_M;
        P.log2_m = (int)p->log2_m;
        P.p_bits = (int)p->p_bits;
        P.z = (int)p->z;
        P.cutoff_bits = p->cutoff_bits;
        if (p->n_levels > 8) return DKSS_EINVAL;
        P.radix_log2.assign(p->radix_log2, p->radix_log2 + p->n_levels);
        if (P.log2_m < 1 || P.log2_M < P.log2_m || P.log2_M > 40 || P.z < 1 || P.p_bits < 2 ||
            P.p_bits > 512)
            return DKSS_ERANGE;
        const uint64_t Mm = 1ull << (P.log2_M + P.log2_m);
        P.u = p->u ? (int)p->u : (int)((2 * N + Mm - 1) / Mm);
    }
    if (P.log2_m < 1 || P.log2_m > 6 || P.log2_M < P.log2_m) return DKSS_ERANGE;
    // every operand fits: M blocks of u m/2 bits
    const unsigned __int128 cap = (unsigned __int128)(1ull << P.log2_M) * ((1u << P.log2_m) / 2) * (unsigned)P.u;
    const uint64_t minlen = 32ull * std::min(alen, blen);
    out->schoolbook = minlen <= P.cutoff_bits && alen + blen <= kSchoolbookMaxWords;
    if (out->schoolbook) return DKSS_OK;
    if (cap < N) return DKSS_ERANGE;
    return DKSS_OK;
}

// constants of the tuple (cached), then the level split
int plan_constants(dkss_ctx* ctx, Call* call) {
    Plan& P = call->P;
    std::string key = P.key();
    auto it = ctx->cache.find(key);
    if (it == ctx->cache.end()) {
        auto c = std::make_unique<Cached>();
        c->plan = P;
        if (!compute_constants(&c->plan)) return DKSS_ERANGE;
        if (c->plan.L > kMaxL) return DKSS_ERANGE;
        const int L = c->plan.L, D = dig_D(L), K = dig_K(L);
        c->D = D;
        const Plan& CP = c->plan;
        ModQ mq(CP.q);
        QConst& Q = c->Q;
        memset(&Q, 0, sizeof Q);
        for (int i = 0; i < L; ++i) Q.q[i] = CP.q.limb32(i);
        auto digits = [&](const Big& x, uint32_t* d) {
            for (int k = 0; k < D; ++k) {
                Big s = x.shr(28 * k);
                d[k] = (uint32_t)(s.w[0] & kMask28);
            }
        };
        digits(CP.q, Q.qd);
        // -q^-1 mod 2^28 by Newton iteration on the low word
        uint32_t q0 = (uint32_t)CP.q.w[0];
        uint32_t inv = q0;
        for (int i = 0; i < 5; ++i) inv *= 2u - q0 * inv;
        Q.qinv28 = (0u - inv) & kMask28;
        // R' = 2^(28K) mod q, R'^2 mod q, (2M)^-1 mod q
        Big Rm = mq.reduce(Big::of(1));
        for (int i = 0; i < 28 * K; ++i) Rm = mq.add(Rm, Rm);
        Big R2 = mq.mul(Rm, Rm);
        Big inv2M = mq.reduce(Big::of(1));
        for (int i = 0; i < CP.log2_M + 1; ++i) inv2M = mq.half(inv2M);
        digits(mq.mul(inv2M, R2), Q.kpw);
        // table entries 0 (one) and 1 (rho), Montgomery form
        const int m = CP.m();
        c->table_host01.assign((size_t)2 * m * D, 0u);
        digits(Rm, &c->table_host01[0]);
        for (int k = 0; k < m; ++k) digits(mq.mul(CP.rho[k], Rm), &c->table_host01[(size_t)(m + k) * D]);
        c->table_count = CP.mu_top();
        it = ctx->cache.emplace(key, std::move(c)).first;
    }
    call->C = it->second.get();
    const Plan& CP = call->C->plan;
    // copy the constants, keep the call's own u / cutoff / radices
    Plan merged = CP;
    merged.u = P.u;
    merged.cutoff_bits = P.cutoff_bits;
    merged.radix_log2 = P.radix_log2;
    if (merged.radix_log2.empty()) merged.radix_log2 = default_radices(CP.log2_M, CP.log2_m, CP.L);
    int sum = 0;
    const int cap = max_radix_log2(CP.log2_m, CP.L);
    for (int r : merged.radix_log2) {
        if (r < 1 || r > cap) return DKSS_ERANGE;
        sum += r;
    }
    if (sum != CP.log2_M + 1 || merged.radix_log2.size() > 8) return DKSS_ERANGE;
    // p^z >= Mm 2^(2u) with the call's u
    if (CP.q.bitlen() <= CP.log2_M + CP.log2_m + 2 * merged.u) return DKSS_ERANGE;
    P = merged;
    return DKSS_OK;
}

// launch helpers, dispatched on L
template <template <int> class F, typename... A>
int dispatch_L(int L, const A&... args) {
    switch (L) {
        case 1: return F<1>::run(args...);
        case 2: return F<2>::run(args...);
        case 3: return F<3>::run(args...);
        case 4: return F<4>::run(args...);
        case 5: return F<5>::run(args...);
        case 6: return F<6>::run(args...);
        case 7: return F<7>::run(args...);
        case 8: return F<8>::run(args...);
        default: return DKSS_ERANGE;
    }
}

size_t rprod_lds(int L) { return (size_t)kThreads * 3 * dig_D(L) * sizeof(uint32_t); }

template <int L>
struct TableBuild {
    // table[dst + j] = table[src + j] * table[mul], j < cnt
    static int launch(Cached* C, Prof* prof, hipStream_t s, long long src, long long mul,
                      long long dst, long long cnt) {
        const int m = C->plan.m();
        const int per = kThreads / m;
        const unsigned blocks = (unsigned)((cnt + per - 1) / per);
        ProfScope ps(prof, DKSS_K_TABLE, s, 2.0 * cnt * m * dig_D(L) * 4, (double)cnt * m * m * L * L);
        hipLaunchKernelGGL(k_table_mul<L>, dim3(blocks), dim3(kThreads), rprod_lds(L), s, C->d_table,
                           src, mul, dst, cnt, C->plan.log2_m, C->Q);
        return hipGetLastError() == hipSuccess ? DKSS_OK : DKSS_EHIP;
    }
    // entries 0 (one) and 1 (rho) are given; for n = 2, 4, ...: rho^n = rho^(n/2) rho^(n/2),
    // then rho^(n+j) = rho^j rho^n for 0 < j < n
    static int run(Cached* C, Prof* prof, hipStream_t s) {
        int rc;
        for (long long n = 2; n < C->table_count; n *= 2) {
            if ((rc = launch(C, prof, s, n / 2, n / 2, n, 1))) return rc;
            const long long cnt = std::min(n, C->table_count - n) - 1;
            if (cnt > 0 && (rc = launch(C, prof, s, 1, n, n + 1, cnt))) return rc;
        }
        return DKSS_OK;
    }
};

int ensure_table(Cached* C, Prof* prof, hipStream_t s) {
    if (C->d_table) return DKSS_OK;
    const int m = C->plan.m();
    const size_t entries = (size_t)std::max<long long>(C->table_count, 2);
    const size_t bytes = entries * m * C->D * sizeof(uint32_t);
    uint32_t* d = nullptr;
    HIP_OK(hipMalloc(&d, bytes));
    C->d_table = d;
    const size_t first = (size_t)std::min<long long>(C->table_count, 2) * m * C->D * sizeof(uint32_t);
    HIP_OK(hipMemcpyAsync(d, C->table_host01.data(), first, hipMemcpyHostToDevice, s));
    int rc = dispatch_L<TableBuild>(C->plan.L, C, prof, s);
    if (rc) return rc;
    HIP_OK(hipStreamSynchronize(s));
    return DKSS_OK;
}

struct Workspace {
    uint32_t* A;
    uint32_t* B;
    unsigned long long* gmask;
    unsigned long long* pmask;
    unsigned char* cin;
    size_t bytes;
};

size_t poly_words(const Plan& P) { return ((size_t)2 << P.log2_M) * P.m() * P.L; }

Workspace layout(const Call& c, char* base) {
    Workspace w{};
    const size_t S = poly_words(c.P) * 4;
    const size_t nw = c.alen + c.blen;
    const size_t nwaves = (nw + 63) / 64;
    size_t off = 0;
    w.A = (uint32_t*)(base + off);
    off += align256(S);
    w.B = (uint32_t*)(base + off);
    off += align256(S);
    w.gmask = (unsigned long long*)(base + off);
    off += align256(nwaves * 8);
    w.pmask = (unsigned long long*)(base + off);
    off += align256(nwaves * 8);
    w.cin = (unsigned char*)(base + off);
    off += align256(nwaves);
    w.bytes = off;
    return w;
}

template <int L>
struct Transform {
    // forward (inverse = 0) or inverse (inverse = 1) transform of poly in place
    static int run(const Call& c, uint32_t* poly, int inverse, hipStream_t s) {
        const Plan& P = c.P;
        const long long twoM = 2LL << P.log2_M;
        const int m = P.m();
        const int nl = (int)P.radix_log2.size();
        const QConst& Q = c.C->Q;
        long long n_lvl[8], mu[8], base[8];
        long long n = twoM;
        for (int k = 0; k < nl; ++k) {
            n_lvl[k] = n;
            mu[k] = n >> P.radix_log2[k];
            base[k] = twoM / n;
            n = mu[k];
        }
        auto dft = [&](int k) -> int {
            const int log2r = P.radix_log2[k];
            const int r = 1 << log2r;
            const long long ncols = twoM >> log2r;
            // columns per workgroup: <= kTaskMax*256 butterfly tasks, <= 64 KiB of LDS
            int C = std::max(1, (kTaskMax * kThreads) / ((r / 2) * m));
            const size_t colbytes = (size_t)r * m * L * 4;
            while (C > 1 && (size_t)C * colbytes > 65536) C /= 2;
            const unsigned blocks = (unsigned)((ncols + C - 1) / C);
            ProfScope ps(c.prof, DKSS_K_DFT, s, 2.0 * twoM * m * L * 4, 0.0);
            hipLaunchKernelGGL(k_dft<L>, dim3(blocks), dim3(kThreads), (size_t)C * colbytes, s, poly,
                               n_lvl[k], mu[k], log2r, P.log2_m, C, ncols, inverse, Q);
            return hipGetLastError() == hipSuccess ? DKSS_OK : DKSS_EHIP;
        };
        auto twiddle = [&](int k) -> int {
            const int per = kThreads / m;
            const unsigned blocks = (unsigned)((twoM + per - 1) / per);
            // products: elements with l != 0 and v != 0 in every block
            const double nprod = (double)(twoM / n_lvl[k]) * ((1LL << P.radix_log2[k]) - 1) * (mu[k] - 1);
            ProfScope ps(c.prof, DKSS_K_TWIDDLE, s, 2.0 * nprod * m * L * 4,
                         nprod * (double)m * m * L * L);
            hipLaunchKernelGGL(k_twiddle<L>, dim3(blocks), dim3(kThreads), rprod_lds(L), s, poly,
                               (const uint32_t*)c.C->d_table, twoM, n_lvl[k], mu[k], base[k],
                               c.C->table_count, P.log2_m, inverse, Q);
            return hipGetLastError() == hipSuccess ? DKSS_OK : DKSS_EHIP;
        };
        int rc;
        if (!inverse) {
            for (int k = 0; k < nl; ++k) {
                if ((rc = dft(k))) return rc;
                if (k + 1 < nl && (rc = twiddle(k))) return rc;
            }
        } else {
            for (int k = nl - 1; k >= 0; --k) {
                if (k + 1 < nl && (rc = twiddle(k))) return rc;
                if ((rc = dft(k))) return rc;
            }
        }
        return DKSS_OK;
    }
};

template <int L>
struct Encode {
    static int run(const Call& c, uint32_t* poly, const uint32_t* a, size_t alen, hipStream_t s) {
        const long long M = 1LL << c.P.log2_M;
        const long long total = (2 * M) << c.P.log2_m;
        const unsigned blocks = (unsigned)((total + kThreads - 1) / kThreads);
        ProfScope ps(c.prof, DKSS_K_ENCODE, s, 4.0 * alen + 4.0 * total * L, 0.0);
        hipLaunchKernelGGL(k_encode<L>, dim3(blocks), dim3(kThreads), 0, s, poly, a, (long long)alen, M,
                           c.P.log2_m, c.P.u);
        return hipGetLastError() == hipSuccess ? DKSS_OK : DKSS_EHIP;
    }
};

template <int L>
struct Pointwise {
    static int run(const Call& c, uint32_t* A, const uint32_t* B, hipStream_t s) {
        const long long count = 2LL << c.P.log2_M;
        const int per = kThreads / c.P.m();
        const unsigned blocks = (unsigned)((count + per - 1) / per);
        const int m = c.P.m();
        ProfScope ps(c.prof, DKSS_K_POINTWISE, s, 3.0 * count * m * L * 4,
                     (double)count * ((double)m * m * L * L + (double)m * L * L));
        hipLaunchKernelGGL(k_pointwise<L>, dim3(blocks), dim3(kThreads), rprod_lds(L), s, A, B, count,
                           c.P.log2_m, c.C->Q);
        return hipGetLastError() == hipSuccess ? DKSS_OK : DKSS_EHIP;
    }
};

template <int L>
struct Decode {
    static int run(const Call& c, uint32_t* out, const uint32_t* poly, const Workspace& w, hipStream_t s) {
        const long long nw = (long long)(c.alen + c.blen);
        const long long nwaves = (nw + 63) / 64;
        const unsigned blocks = (unsigned)((nw + kThreads - 1) / kThreads);
        const double S = (double)(2LL << c.P.log2_M) * c.P.m() * L * 4;
        {
            ProfScope ps(c.prof, DKSS_K_DECODE, s, S + 4.0 * nw + 16.0 * nwaves, 0.0);
            hipLaunchKernelGGL(k_decode<L>, dim3(blocks), dim3(kThreads), 0, s, out, nw, poly,
                               2LL << c.P.log2_M, c.P.log2_m, c.P.u, w.gmask, w.pmask);
        }
        HIP_OK(hipGetLastError());
        {
            ProfScope ps(c.prof, DKSS_K_CARRY_SCAN, s, 17.0 * nwaves, 0.0);
            hipLaunchKernelGGL(k_carry_scan, dim3(1), dim3(1024), 0, s, w.gmask, w.pmask, w.cin, nwaves);
        }
        HIP_OK(hipGetLastError());
        {
            ProfScope ps(c.prof, DKSS_K_CARRY_APPLY, s, 8.0 * nw + 17.0 * nwaves, 0.0);
            hipLaunchKernelGGL(k_carry_apply, dim3(blocks), dim3(kThreads), 0, s, out, nw, w.gmask,
                               w.pmask, w.cin);
        }
        HIP_OK(hipGetLastError());
        return DKSS_OK;
    }
};

int fill_zero(uint32_t* p, size_t n, hipStream_t s) {
    if (n == 0) return DKSS_OK;
    const unsigned blocks = (unsigned)((n + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(kThreads), 0, s, p, (long long)n, 0u);
    return hipGetLastError() == hipSuccess ? DKSS_OK : DKSS_EHIP;
}

bool overlaps(const void* x, size_t xb, const void* y, size_t yb) {
    const char* a = (const char*)x;
    const char* b = (const char*)y;
    return a < b + yb && b < a + xb;
}

int prepare_call(dkss_ctx* ctx, size_t alen, size_t blen, const dkss_params* p, Call* call) {
    call->prof = &ctx->prof;
    int rc = resolve_params(ctx, alen, blen, p, call);
    if (rc) return rc;
    if (alen == 0 || blen == 0 || call->schoolbook) return DKSS_OK;
    return plan_constants(ctx, call);
}

int run_mul(const Call& call, uint32_t* c, const uint32_t* a, size_t alen, const uint32_t* b,
            size_t blen, void* ws, size_t ws_bytes, hipStream_t s) {
    const size_t nw = alen + blen;
    if (alen == 0 || blen == 0) return fill_zero(c, nw, s);
    if (call.schoolbook) {
        ProfScope ps(call.prof, DKSS_K_SCHOOLBOOK, s, 4.0 * (alen + blen) * 2,
                     (double)alen * (double)blen);
        hipLaunchKernelGGL(k_schoolbook, dim3(1), dim3(kThreads), nw * 3 * sizeof(uint32_t), s, c, a,
                           (long long)alen, b, (long long)blen);
        return hipGetLastError() == hipSuccess ? DKSS_OK : DKSS_EHIP;
    }
    Workspace w = layout(call, (char*)ws);
    if (ws == nullptr || ((uintptr_t)ws & 255)) return DKSS_EINVAL;
    if (ws_bytes < w.bytes) return DKSS_ENOSPC;
    const bool squaring = (a == b && alen == blen);
    const int L = call.P.L;
    int rc;
    if ((rc = dispatch_L<Encode>(L, call, w.A, a, alen, s))) return rc;
    if ((rc = dispatch_L<Transform>(L, call, w.A, 0, s))) return rc;
    if (!squaring) {
        if ((rc = dispatch_L<Encode>(L, call, w.B, b, blen, s))) return rc;
        if ((rc = dispatch_L<Transform>(L, call, w.B, 0, s))) return rc;
    }
    if ((rc = dispatch_L<Pointwise>(L, call, w.A, squaring ? (const uint32_t*)w.A : w.B, s))) return rc;
    if ((rc = dispatch_L<Transform>(L, call, w.A, 1, s))) return rc;
    return dispatch_L<Decode>(L, call, c, (const uint32_t*)w.A, w, s);
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------------------------

extern "C" {

int dkss_ctx_create(dkss_ctx** out, int policy, const char* cache_dir) {
    (void)cache_dir;
    if (!out || (policy != DKSS_POLICY_THESIS && policy != DKSS_POLICY_TUNED)) return DKSS_EINVAL;
    dkss_ctx* c = new (std::nothrow) dkss_ctx();
    if (!c) return DKSS_EINVAL;
    c->policy = policy;
    *out = c;
    return DKSS_OK;
}

void dkss_ctx_destroy(dkss_ctx* ctx) {
    if (!ctx) return;
    for (auto& kv : ctx->cache)
        if (kv.second->d_table) (void)hipFree(kv.second->d_table);
    delete ctx;
}

int dkss_select_params(dkss_ctx* ctx, uint64_t a_bits, uint64_t b_bits, uint32_t batch,
                       dkss_params* out) {
    (void)batch;
    if (!ctx || !out) return DKSS_EINVAL;
    const uint64_t N = 32 * ((std::max(a_bits, b_bits) + 31) / 32);
    if (N == 0 || N > (1ull << 36)) return DKSS_ERANGE;
    int lM, lm, u, pb;
    if (!thesis_params(N, &lM, &lm, &u, &pb)) return DKSS_ERANGE;
    memset(out, 0, sizeof *out);
    out->log2_M = (uint32_t)lM;
    out->log2_m = (uint32_t)lm;
    out->u = (uint32_t)u;
    out->p_bits = (uint32_t)pb;
    out->z = 1;
    out->cutoff_bits = kDefaultCutoffBits;
    std::vector<int> r = default_radices(lM, lm, (pb + 31) / 32);
    out->n_levels = (uint32_t)r.size();
    for (size_t i = 0; i < r.size() && i < 8; ++i) out->radix_log2[i] = (uint32_t)r[i];
    return DKSS_OK;
}

int dkss_plan_info(dkss_ctx* ctx, size_t alen, size_t blen, const dkss_params* p, dkss_plan* out) {
    if (!ctx || !out) return DKSS_EINVAL;
    Call call;
    int rc = prepare_call(ctx, alen, blen, p, &call);
    if (rc) return rc;
    memset(out, 0, sizeof *out);
    const Plan& P = call.P;
    out->schoolbook = call.schoolbook ? 1 : 0;
    out->params.log2_M = (uint32_t)P.log2_M;
    out->params.log2_m = (uint32_t)P.log2_m;
    out->params.u = (uint32_t)P.u;
    out->params.p_bits = (uint32_t)P.p_bits;
    out->params.z = (uint32_t)P.z;
    out->params.cutoff_bits = P.cutoff_bits;
    out->params.n_levels = (uint32_t)P.radix_log2.size();
    for (size_t i = 0; i < P.radix_log2.size() && i < 8; ++i)
        out->params.radix_log2[i] = (uint32_t)P.radix_log2[i];
    if (call.C) {
        out->L = (uint32_t)P.L;
        out->q_bits = (uint32_t)P.q_bits;
        out->poly_bytes = poly_words(P) * 4;
        out->table_bytes = (uint64_t)std::max<long long>(call.C->table_count, 2) * P.m() * call.C->D * 4;
        for (int i = 0; i < P.L && i < 16; ++i) out->q[i] = P.q.limb32(i);
    }
    return DKSS_OK;
}

int dkss_workspace_bytes(dkss_ctx* ctx, size_t alen, size_t blen, const dkss_params* p, size_t* out) {
    if (!ctx || !out) return DKSS_EINVAL;
    Call call;
    int rc = prepare_call(ctx, alen, blen, p, &call);
    if (rc) return rc;
    if (alen == 0 || blen == 0 || call.schoolbook) {
        *out = 0;
        return DKSS_OK;
    }
    *out = layout(call, nullptr).bytes;
    return DKSS_OK;
}

int dkss_prepare(dkss_ctx* ctx, size_t alen, size_t blen, const dkss_params* p, dkss_stream_t s) {
    if (!ctx) return DKSS_EINVAL;
    Call call;
    int rc = prepare_call(ctx, alen, blen, p, &call);
    if (rc) return rc;
    if (!call.C) return DKSS_OK;
    return ensure_table(call.C, &ctx->prof, (hipStream_t)s);
}

int dkss_mul(dkss_ctx* ctx, uint32_t* c, const uint32_t* a, size_t alen, const uint32_t* b,
             size_t blen, const dkss_params* p, void* ws, size_t ws_bytes, dkss_stream_t s) {
    if (!ctx || !c || (alen && !a) || (blen && !b)) return DKSS_EINVAL;
    const size_t nw = alen + blen;
    if ((alen && overlaps(c, nw * 4, a, alen * 4)) || (blen && overlaps(c, nw * 4, b, blen * 4)))
        return DKSS_EINVAL;
    Call call;
    int rc = prepare_call(ctx, alen, blen, p, &call);
    if (rc) return rc;
    if (call.C && (rc = ensure_table(call.C, &ctx->prof, (hipStream_t)s))) return rc;
    return run_mul(call, c, a, alen, b, blen, ws, ws_bytes, (hipStream_t)s);
}

int dkss_batch_workspace_bytes(dkss_ctx* ctx, size_t count, const size_t* alen, const size_t* blen,
                               const dkss_params* p, size_t* out) {
    if (!ctx || !out || (count && (!alen || !blen))) return DKSS_EINVAL;
    size_t mx = 0;
    for (size_t i = 0; i < count; ++i) {
        size_t b = 0;
        int rc = dkss_workspace_bytes(ctx, alen[i], blen[i], p ? p + i : nullptr, &b);
        if (rc) return rc;
        mx = std::max(mx, b);
    }
    *out = mx;
    return DKSS_OK;
}

int dkss_mul_batch(dkss_ctx* ctx, size_t count, uint32_t* const* c, const uint32_t* const* a,
                   const size_t* alen, const uint32_t* const* b, const size_t* blen,
                   const dkss_params* p, void* ws, size_t ws_bytes, dkss_stream_t s) {
    if (!ctx || (count && (!c || !a || !alen || !b || !blen))) return DKSS_EINVAL;
    for (size_t i = 0; i < count; ++i) {
        int rc = dkss_mul(ctx, c[i], a[i], alen[i], b[i], blen[i], p ? p + i : nullptr, ws, ws_bytes, s);
        if (rc) return rc;
    }
    return DKSS_OK;
}

int dkss_forward(dkss_ctx* ctx, uint32_t* poly, const uint32_t* a, size_t alen, size_t blen,
                 const dkss_params* p, void* ws, size_t ws_bytes, dkss_stream_t s) {
    if (!ctx || !poly || !a || alen == 0 || blen == 0) return DKSS_EINVAL;
    Call call;
    int rc = prepare_call(ctx, alen, blen, p, &call);
    if (rc) return rc;
    if (call.schoolbook) return DKSS_ERANGE;
    if ((rc = ensure_table(call.C, &ctx->prof, (hipStream_t)s))) return rc;
    Workspace w = layout(call, (char*)ws);
    if (ws == nullptr || ((uintptr_t)ws & 255)) return DKSS_EINVAL;
    if (ws_bytes < w.bytes) return DKSS_ENOSPC;
    hipStream_t st = (hipStream_t)s;
    if ((rc = dispatch_L<Encode>(call.P.L, call, w.A, a, alen, st))) return rc;
    if ((rc = dispatch_L<Transform>(call.P.L, call, w.A, 0, st))) return rc;
    LevelIdx LI{};
    LI.n = (int)call.P.radix_log2.size();
    int nlog = call.P.log2_M + 1, shift = 0;
    for (int k = 0; k < LI.n; ++k) {
        nlog -= call.P.radix_log2[k];
        LI.log2mu[k] = nlog;
        LI.log2r[k] = call.P.radix_log2[k];
        LI.shift[k] = shift;
        shift += call.P.radix_log2[k];
    }
    const long long twoM = 2LL << call.P.log2_M;
    const int EW = call.P.m() * call.P.L;
    const long long total = twoM * EW;
    ProfScope ps(call.prof, DKSS_K_UNSCRAMBLE, st, 8.0 * total, 0.0);
    hipLaunchKernelGGL(k_unscramble, dim3((unsigned)((total + kThreads - 1) / kThreads)), dim3(kThreads),
                       0, st, poly, (const uint32_t*)w.A, twoM, EW, LI);
    return hipGetLastError() == hipSuccess ? DKSS_OK : DKSS_EHIP;
}

int dkss_residues(const uint32_t* x, size_t n, const uint64_t* primes_host, size_t count,
                  uint64_t* out, dkss_stream_t s) {
    if ((n && !x) || (count && (!primes_host || !out))) return DKSS_EINVAL;
    hipStream_t st = (hipStream_t)s;
    const long long per_block = (long long)kThreads * 64;
    const long long nb = std::max<long long>(1, ((long long)n + per_block - 1) / per_block);
    for (size_t j = 0; j < count; ++j) {
        const uint64_t q = primes_host[j];
        if (!(q & 1) || q < 3 || q >= (1ull << 62)) return DKSS_EINVAL;
    }
    if (count == 0) return DKSS_OK;
    uint64_t* part = nullptr;
    HIP_OK(hipMalloc((void**)&part, (size_t)nb * 8 * count));
    for (size_t j = 0; j < count; ++j) {
        const uint64_t q = primes_host[j];
        ResConst R{};
        R.q = q;
        uint64_t inv = q;
        for (int i = 0; i < 6; ++i) inv *= 2 - q * inv;
        R.qinv = 0 - inv;
        auto mulmod = [&](uint64_t a, uint64_t b) {
            return (uint64_t)(((unsigned __int128)a * b) % q);
        };
        const uint64_t r64 = (uint64_t)(((unsigned __int128)1 << 64) % q);   // 2^64 mod q
        R.w = mulmod((uint64_t)((1ull << 32) % q), r64);
        // chunk_pow[k] = 2^(32*64*2^k) mod q, Montgomery form
        uint64_t base = 1;
        for (int i = 0; i < 64; ++i) base = mulmod(base, (1ull << 32) % q);  // 2^(32*64)
        for (int k = 0; k <= 8; ++k) {
            R.chunk_pow[k] = mulmod(base, r64);
            base = mulmod(base, base);
        }
        hipLaunchKernelGGL(k_residue_block, dim3((unsigned)nb), dim3(kThreads), 0, st, x, (long long)n, R,
                           part + j * nb);
        hipLaunchKernelGGL(k_residue_final, dim3(1), dim3(64), 0, st, (const uint64_t*)(part + j * nb), nb, R,
                           out + j);
        if (hipGetLastError() != hipSuccess) {
            (void)hipStreamSynchronize(st);
            (void)hipFree(part);
            return DKSS_EHIP;
        }
    }
    const hipError_t e1 = hipStreamSynchronize(st);
    const hipError_t e2 = hipFree(part);
    return (e1 == hipSuccess && e2 == hipSuccess) ? DKSS_OK : DKSS_EHIP;
}

int dkss_profile_enable(dkss_ctx* ctx, int on) {
    if (!ctx) return DKSS_EINVAL;
    ctx->prof.on = on != 0;
    return DKSS_OK;
}

int dkss_profile_read(dkss_ctx* ctx, int kind, dkss_kernel_stats* out) {
    if (!ctx || !out || kind < 0 || kind >= DKSS_K_KINDS) return DKSS_EINVAL;
    int rc = ctx->prof.drain();
    *out = ctx->prof.tot[kind];
    return rc;
}

int dkss_profile_reset(dkss_ctx* ctx) {
    if (!ctx) return DKSS_EINVAL;
    int rc = ctx->prof.drain();
    for (auto& t : ctx->prof.tot) t = dkss_kernel_stats{};
    return rc;
}

const char* dkss_kernel_name(int kind) {
    static const char* names[DKSS_K_KINDS] = {"k_encode", "k_dft", "k_twiddle", "k_pointwise",
                                              "k_decode", "k_carry_scan", "k_carry_apply",
                                              "k_schoolbook", "k_table_mul", "k_unscramble"};
    if (kind < 0 || kind >= DKSS_K_KINDS) return nullptr;
    return names[kind];
}

const char* dkss_strerror(int code) {
    switch (code) {
        case DKSS_OK: return "ok";
        case DKSS_EINVAL: return "invalid argument";
        case DKSS_ENOSPC: return "workspace too small";
        case DKSS_ERANGE: return "size or parameters unsupported or infeasible";
        case DKSS_EHIP: return "HIP runtime error";
        case DKSS_ENOTIMPL: return "not implemented";
        default: return "unknown error";
    }
}

}  // extern "C"
