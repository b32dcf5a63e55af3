// libdkss: DKSS multiplication of large unsigned integers on one MI355X (gfx950).
//
// Pipeline of one product c = a*b (thesis Sec. 3.2, Steps 4-8), all on one HIP stream:
//   k_encode      Step 4 (Sec. 3.2.4): operand bits -> 2M elements of R, u bits per coefficient
//   k_level       Step 5 (Sec. 3.2.5 i/iii): one FFT level = independent radix-r DFTs with root
//                 alpha^(2m/r) over columns of stride mu, staged in LDS; every butterfly
//                 multiplies by a power of alpha, i.e. rotates and negates coefficients
//                 + (Sec. 3.2.5 ii) the "bad multiplications" by rho^(base*l*v) between
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
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/dkss.h"
#include "hip_status.hpp"
#include "kernels.hpp"
#include "planner.hpp"
#include "wave_carry.hpp"

using namespace dkss;

static thread_local int g_last_hip = 0;

int dkss::note_hip(hipError_t e) {
    if (e == hipSuccess) return DKSS_OK;
    g_last_hip = (int)e;
    return DKSS_EHIP;
}

namespace {

constexpr int kThreads = 256;

constexpr uint64_t kDefaultCutoffBits = 2048;
constexpr size_t kSchoolbookMaxWords = 4096;   // alen + blen of a schoolbook product (one workgroup)
constexpr int kMaxKaraDepth = 2;                // Karatsuba levels above the schoolbook leaves

// Karatsuba levels the base case needs for alen x blen limbs so that every leaf fits the
// schoolbook (0: none), or -1 beyond kMaxKaraDepth levels.  A level's largest sub-product is
// (h + 1) x (h + 1), h = ceil(max / 2).
inline int kara_depth(size_t alen, size_t blen) {
    size_t na = alen, nb = blen;
    for (int d = 0; d <= kMaxKaraDepth; ++d) {
        if (na + nb <= kSchoolbookMaxWords) return d;
        const size_t h = (std::max(na, nb) + 1) / 2;
        na = nb = h + 1;
    }
    return -1;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// A dispatch's work-items per grid dimension must fit in 32 bits.
inline bool grid_ok(size_t blocks, size_t threads = 256) { return blocks * threads < (1ull << 32); }

// Orders LDS accesses among the lanes of one wavefront (a wavefront's LDS operations are
// performed in issue order; this keeps the compiler from moving them across the point).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int bitrev(int x, int bits) {
    return bits ? (int)(__brev((unsigned)x) >> (32 - bits)) : 0;
}

// One product of a launch: operands, result, and its u (bits per inner coefficient).  Kernels
// that handle several products at once take the product index from blockIdx.y; their
// polynomials sit at a fixed stride in the workspace.
struct ProdDesc {
    uint32_t* c;
    const uint32_t* a;
    const uint32_t* b;
    long long alen, blen;
    int u;
    int pad;
};

// A single product by value, or a device array of many
struct ProdArgs {
    ProdDesc one;
    const ProdDesc* many;
    __device__ __forceinline__ ProdDesc get() const { return many ? many[blockIdx.y] : one; }
};

// ---------------------------------------------------------------------------------------------
// Step 4: encode
// ---------------------------------------------------------------------------------------------

// Coefficient k of element i as limbs: bits [u (i m/2 + k), u (i m/2 + k) + u) of a for k < m/2
// and i < M; zero otherwise.
template <int C>
__device__ __forceinline__ void encode_limbs(const uint32_t* __restrict__ a, long long alen, int u, long long i,
                                             int k, long long M, int log2m, uint32_t* out) {
    constexpr int L = fmt_L(C);
    const int hm = 1 << (log2m - 1);
#pragma unroll
    for (int w = 0; w < L; ++w) out[w] = 0;
    if (i < M && k < hm) {
        const unsigned long long pos = ((unsigned long long)i * hm + k) * (unsigned)u;
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
}

// poly: 2M elements x m coefficients x L limbs.
template <int C>
__global__ __launch_bounds__(kThreads) void k_encode(ProdArgs PA, int which, uint32_t* __restrict__ poly0,
                                                     long long stride, long long M, int log2m) {
    constexpr int L = fmt_L(C);
    const ProdDesc pd = PA.get();
    const uint32_t* __restrict__ a = which ? pd.b : pd.a;
    const long long alen = which ? pd.blen : pd.alen;
    const int u = pd.u;
    uint32_t* __restrict__ poly = poly0 + (size_t)blockIdx.y * stride;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (2 * M) << log2m;
    if (t >= total) return;
    const int m = 1 << log2m;
    const long long i = t >> log2m;
    const int k = (int)(t & (m - 1));
    uint32_t out[L];
    encode_limbs<C>(a, alen, u, i, k, M, log2m, out);
    uint32_t* dst = poly + (size_t)t * L;
#pragma unroll
    for (int w = 0; w < L; ++w) dst[w] = out[w];
}

// ---------------------------------------------------------------------------------------------
// Step 5: one FFT level (radix-r DFTs with root alpha^(+-2m/r)), with the twiddle products fused
// ---------------------------------------------------------------------------------------------

// The level has 2M/n_lvl blocks of n_lvl elements; within a block, column l < mu holds elements
// l, l + mu, ..., l + (r-1) mu.  A workgroup takes C = 2^log2C consecutive columns (C r
// elements) and
//   mode 0: loads them, runs the radix-r DFT, stores them;
//   mode 1 (forward): loads, DFT, then multiplies output v of column l by rho^(base l v) (the bad
//           multiplications of Sec. 3.2.5 ii) on its way back to HBM;
//   mode 2 (inverse): loads, multiplies input v by rho^-(base l v), runs the DFT with alpha^-1,
//           stores.
// The DFT works on 32-bit limbs (additions with the hardware carry): inputs in bit-reversed LDS
// slots, log2 r radix-2 decimation-in-time passes between the two halves of the workgroup's LDS;
// the pass merging halves of h points multiplies the odd half by alpha^((m/h) k), k < h
// (alpha^-((m/h) k) for the inverse).  Output v ends in slot v.  HBM holds limbs; products in R
// work on 28-bit digits, the columns converted in LDS between the two forms.  Twiddle
// products run in rounds of 256/m elements, one output coefficient per thread: the element's
// digits are read in place, the table entry rho^s (Montgomery form) is staged in the other half
// together with its negation, formed while staging.
struct LevelArgs {
    long long twoM, base, mu_top;
    int log2mut;                  // log2 mu_top
    int log2nl, log2mu, log2r, log2m, log2C;
    int mode, inverse;
    int half;                     // words of each of the two LDS halves
    int ew, sw;                   // LDS words per element in digits, per staged operand
};

// Position of element j of column c0 + c in the polynomial (positions stay below 2M < 2^32)
__device__ __forceinline__ long long level_pos(const LevelArgs& A, long long c0, int c, int j) {
    const uint32_t col = (uint32_t)c0 + (uint32_t)c;
    const uint32_t b = col >> A.log2mu, l = col & ((1u << A.log2mu) - 1u);
    return (long long)((b << A.log2nl) + ((uint32_t)j << A.log2mu) + l);
}

// Copies between the workgroup's C r elements in HBM (L limbs per residue) and LDS.  Element
// index e: column c fastest, then position j; LDS slot bitrev(j) on the way in, slot v on the
// way out.

// HBM limbs into LDS as digits, D words per residue (an inverse level's twiddles come first)
template <int C>
__device__ __forceinline__ void level_load_digits(uint32_t* cur, const uint32_t* __restrict__ poly,
                                                  const LevelArgs& A, long long c0) {
    constexpr int L = fmt_L(C);
    constexpr int D = Dig<C>::D;
    const int nel = 1 << (A.log2C + A.log2r);
    for (int t = threadIdx.x; t < (nel << A.log2m); t += kThreads) {
        const int e = t >> A.log2m, k = t & ((1 << A.log2m) - 1);
        const int c = e & ((1 << A.log2C) - 1), j = e >> A.log2C;
        const uint32_t* src = poly + (((size_t)level_pos(A, c0, c, j) << A.log2m) + k) * L;
        uint32_t x[L], dv[D];
#pragma unroll
        for (int w = 0; w < L; ++w) x[w] = src[w];
        limbs_to_digits<C>(x, dv);
        uint32_t* dst = cur + ((c << A.log2r) + bitrev(j, A.log2r)) * A.ew + k * D;
#pragma unroll
        for (int w = 0; w < D; ++w) dst[w] = dv[w];
    }
}

// HBM limbs into LDS limbs, LS words per residue (one coefficient per thread and step)
template <int C, int LS>
__device__ __forceinline__ void level_load_limbs(uint32_t* cur, const uint32_t* __restrict__ poly,
                                                 const LevelArgs& A, long long c0) {
    constexpr int L = fmt_L(C);
    const int nel = 1 << (A.log2C + A.log2r);
    for (int t = threadIdx.x; t < (nel << A.log2m); t += kThreads) {
        const int e = t >> A.log2m, k = t & ((1 << A.log2m) - 1);
        const int c = e & ((1 << A.log2C) - 1), j = e >> A.log2C;
        const uint32_t* src = poly + (((size_t)level_pos(A, c0, c, j) << A.log2m) + k) * L;
        uint32_t* dst = cur + ((((c << A.log2r) + bitrev(j, A.log2r)) << A.log2m) + k) * LS;
#pragma unroll
        for (int w = 0; w < L; ++w) dst[w] = src[w];
    }
}

// The top forward level's columns straight from the operand (Step 4 fused into the first level),
// with the DFT's first pass done on the way in.  At the top level position j of a column is
// element j mu + l, which is zero padding for j >= r/2 (elements M..2M-1, Sec. 3.2.4); the first
// decimation-in-time pass pairs slots 2k and 2k+1, holding positions bitrev(2k) < r/2 and
// bitrev(2k) + r/2, without rotation, so it leaves the element of position bitrev(2k) in both.
// Each element at j < r/2 is therefore written, as limbs, to slots bitrev(j) and bitrev(j) + 1,
// and the DFT starts at its second pass.
template <int C, int LS>
__device__ __forceinline__ void level_encode_in(uint32_t* cur, const uint32_t* __restrict__ a, long long alen,
                                                int u, long long M, const LevelArgs& A, long long c0) {
    constexpr int L = fmt_L(C);
    const int nel = 1 << (A.log2C + A.log2r - 1);        // the elements at j < r/2
    for (int t = threadIdx.x; t < (nel << A.log2m); t += kThreads) {
        const int e = t >> A.log2m, k = t & ((1 << A.log2m) - 1);
        const int c = e & ((1 << A.log2C) - 1), j = e >> A.log2C;
        uint32_t out[L];
        encode_limbs<C>(a, alen, u, level_pos(A, c0, c, j), k, M, A.log2m, out);
        const int slot = (c << A.log2r) + bitrev(j, A.log2r);
        uint32_t* d0 = cur + ((slot << A.log2m) + k) * LS;
        uint32_t* d1 = cur + (((slot + 1) << A.log2m) + k) * LS;
#pragma unroll
        for (int w = 0; w < L; ++w) {
            d0[w] = out[w];
            d1[w] = out[w];
        }
    }
}

// LDS limbs (slot v) out to HBM limbs (position v)
template <int C, int LS>
__device__ __forceinline__ void level_store_limbs(uint32_t* __restrict__ poly, const uint32_t* cur,
                                                  const LevelArgs& A, long long c0) {
    constexpr int L = fmt_L(C);
    const int nel = 1 << (A.log2C + A.log2r);
    for (int t = threadIdx.x; t < (nel << A.log2m); t += kThreads) {
        const int e = t >> A.log2m, k = t & ((1 << A.log2m) - 1);
        const int c = e & ((1 << A.log2C) - 1), v = e >> A.log2C;
        const uint32_t* src = cur + ((((c << A.log2r) + v) << A.log2m) + k) * LS;
        uint32_t* dst = poly + (((size_t)level_pos(A, c0, c, v) << A.log2m) + k) * L;
#pragma unroll
        for (int w = 0; w < L; ++w) dst[w] = src[w];
    }
}

// Within LDS: every coefficient from limbs to digits, same slot (then a barrier)
template <int C, int LS>
__device__ __forceinline__ void lds_to_digits(uint32_t* dg, const uint32_t* lb, const LevelArgs& A) {
    constexpr int L = fmt_L(C);
    constexpr int D = Dig<C>::D;
    const int n = 1 << (A.log2C + A.log2r + A.log2m);
    for (int t = threadIdx.x; t < n; t += kThreads) {
        uint32_t x[L], dv[D];
#pragma unroll
        for (int w = 0; w < L; ++w) x[w] = lb[t * LS + w];
        limbs_to_digits<C>(x, dv);
#pragma unroll
        for (int w = 0; w < D; ++w) dg[(t >> A.log2m) * A.ew + (t & ((1 << A.log2m) - 1)) * D + w] = dv[w];
    }
    __syncthreads();
}

// Within LDS: every coefficient from digits to limbs; the element in slot s of its column moves
// to slot bitrev(s) if perm (then a barrier)
template <int C, int LS>
__device__ __forceinline__ void lds_to_limbs(uint32_t* lb, const uint32_t* dg, const LevelArgs& A, bool perm) {
    constexpr int L = fmt_L(C);
    constexpr int D = Dig<C>::D;
    const int n = 1 << (A.log2C + A.log2r + A.log2m);
    for (int t = threadIdx.x; t < n; t += kThreads) {
        uint32_t dv[D], x[L];
#pragma unroll
        for (int w = 0; w < D; ++w) dv[w] = dg[(t >> A.log2m) * A.ew + (t & ((1 << A.log2m) - 1)) * D + w];
        digits_to_limbs<C>(dv, x);
        int to = t;
        if (perm) {
            const int k = t & ((1 << A.log2m) - 1);
            const int e = t >> A.log2m;
            const int c = e >> A.log2r, sl = e & ((1 << A.log2r) - 1);
            to = ((((c << A.log2r) + bitrev(sl, A.log2r))) << A.log2m) + k;
        }
#pragma unroll
        for (int w = 0; w < L; ++w) lb[to * LS + w] = x[w];
    }
    __syncthreads();
}

// A thread's operand for one round of products, fetched from HBM a round ahead (the load is
// issued before the preceding work and waited for at first use): coefficient j of the table
// entry rho^s (twiddles), or coefficient j of b (componentwise products).
template <int C>
struct Ahead {
    static constexpr int L = fmt_L(C);
    uint32_t v[Dig<C>::D];
    int rot;                      // the twiddle's power of alpha
    bool nz;                      // the element gets a product
};

// Twiddle of the element that this thread serves in the round starting at element r0.
template <int C>
__device__ __forceinline__ void tw_fetch(Ahead<C>& f, int r0, const uint32_t* __restrict__ table,
                                         const LevelArgs& A, long long c0) {
    constexpr int L = fmt_L(C);
    constexpr int D = Dig<C>::D;
    const int m = 1 << A.log2m;
    const int g = threadIdx.x >> A.log2m, j = threadIdx.x & (m - 1);
    const int el = r0 + g;
    f.nz = false;
    f.rot = 0;
    if (el >= (1 << (A.log2C + A.log2r))) return;
    // the round's elements go by LDS slot (consecutive slots: their residues fall on distinct
    // banks); a slot holds its own position after a DFT (mode 1), the bit-reversed one before
    // a DFT (mode 2)
    const int c = el >> A.log2r, slot = el & ((1 << A.log2r) - 1);
    const int v = A.mode == 2 ? bitrev(slot, A.log2r) : slot;
    const uint32_t l = ((uint32_t)c0 + (uint32_t)c) & ((1u << A.log2mu) - 1u);
    uint32_t e = (uint32_t)A.base * l * (uint32_t)v;    // < 2M < 2^32
    if (A.inverse && e) e = (uint32_t)A.twoM - e;
    if (!e) return;
    f.nz = true;
    f.rot = (int)(e >> A.log2mut);
    const uint32_t s = e & ((1u << A.log2mut) - 1u);
    const uint32_t* ts = table + (size_t)s * m * D;
#pragma unroll
    for (int y = 0; y < D; ++y) f.v[y] = ts[j * D + y];
}

// Twiddle products of all C r elements of the workgroup, in rounds of 256/m elements.  The
// element with position v in column c sits in LDS slot v (after the DFT, mode 1) or bitrev(v)
// (before it, mode 2).  Mode 1 writes results to HBM; mode 2 writes them back into the slot once
// the round's products (which read the slot) are done.  f holds round 0's twiddle on entry.
template <int C, int MODE, int FM>
__device__ __forceinline__ void level_twiddle(Ahead<C>& f, uint32_t* cur, uint32_t* RB, uint32_t* __restrict__ poly,
                                              const uint32_t* __restrict__ table, const LevelArgs& A,
                                              long long c0, const QConst& Q) {
    constexpr int L = fmt_L(C);
    constexpr int D = Dig<C>::D;
    const int m = 1 << A.log2m;
    const int EW = A.ew;                                // an element's digits in LDS
    const int per = kThreads >> A.log2m;
    const int g = threadIdx.x >> A.log2m, j = threadIdx.x & (m - 1);
    const int nel = 1 << (A.log2C + A.log2r);
    uint32_t* TP = RB + g * A.sw;
    // The m lanes of an element lie in one wavefront (m <= 64) and touch only that element's
    // column slot and staging area, so the rounds synchronize per wavefront.
    for (int r0 = 0; r0 < nel; r0 += per) {
        const int el = r0 + g;                          // (c, slot) with slot fastest
        const bool valid = el < nel;
        const int c = el >> A.log2r, slot = el & ((1 << A.log2r) - 1);
        const int v = MODE == 2 ? bitrev(slot, A.log2r) : slot;          // its position
        uint32_t* X = cur + ((c << A.log2r) + slot) * EW;
        const bool nz = f.nz;
        if (nz) {
            // the twiddle's extension to 2m entries: t_j and, m further on, q - t_j
            uint32_t nt[D];
            dneg_q<C>(nt, f.v, Q);
            uint32_t* t0 = TP + stage_pos(j, f.rot, A.log2m) * Dig<C>::DS;
            uint32_t* t1 = TP + stage_pos(j + m, f.rot, A.log2m) * Dig<C>::DS;
#pragma unroll
            for (int y = 0; y < D; ++y) {
                t0[y] = f.v[y];
                t1[y] = nt[y];
            }
        }
        if (r0 + per < nel) tw_fetch<C>(f, r0 + per, table, A, c0);     // next round's twiddle
        wave_sync();
        uint32_t out[D];                                // mode 1: L limbs; mode 2: D digits
        if (valid) {
            if (nz) {
                rprod_coeff<C, MODE == 1, FM>(TP, X, A.log2m, j, Q, out);
            } else if (MODE == 1) {
                digits_to_limbs<C>(X + j * D, out);
            }
            if (MODE == 1) {
                uint32_t* dst = poly + (((size_t)level_pos(A, c0, c, v) << A.log2m) + j) * L;
#pragma unroll
                for (int y = 0; y < L; ++y) dst[y] = out[y];
            }
        }
        wave_sync();
        if (MODE == 2 && valid && nz) {
#pragma unroll
            for (int y = 0; y < D; ++y) X[j * D + y] = out[y];
        }
    }
    if (MODE == 2) __syncthreads();
}

// log2 r radix-2 decimation-in-time passes over the workgroup's columns (limbs, LS words per
// coefficient), from cur into nxt and back (the buffers are swapped after each pass; on return
// cur holds the result).  Input: the element at position j of a column in slot bitrev(j);
// output: position v in slot v.  The pass merging halves of h points multiplies the odd half by
// alpha^((m/h) k) (alpha^-1 if inverse).  Passes before first_pass are taken as done.
template <int C, int LS>
__device__ __forceinline__ void dft_passes(uint32_t*& cur, uint32_t*& nxt, const LevelArgs& A, int inverse,
                                           const QConst& Q, int first_pass = 0) {
    constexpr int L = fmt_L(C);
    const int m = 1 << A.log2m, r = 1 << A.log2r;
    const int tasks = (1 << (A.log2C + A.log2r - 1)) << A.log2m;   // butterflies x coefficients
    // q's limbs in vector registers for all passes: an add or subtract with carry already reads
    // its carry from scalar registers and may read only one scalar operand
    uint32_t qv[L];
#pragma unroll
    for (int w = 0; w < L; ++w) asm volatile("v_mov_b32 %0, %1" : "=v"(qv[w]) : "s"(Q.ql[w]));
    for (int h = 1 << first_pass, lh = first_pass; h < r; h <<= 1, ++lh) {
        const int lmh = A.log2m - lh;                   // log2(m/h)
        for (int t = threadIdx.x; t < tasks; t += kThreads) {
            const int jj = t & (m - 1);
            const int rest = t >> A.log2m;
            const int bf = rest & ((r >> 1) - 1);
            const int c = rest >> (A.log2r - 1);
            const int kk = bf & (h - 1);
            const int xs = (bf << 1) - kk;
            const int e = kk << lmh;                    // alpha^e, alpha^-e if inverse
            // (alpha^(+-e) y)_jj = y_w for w = jj -+ e mod 2m below m, -y_(w-m) otherwise
            // (alpha^m = -1, alpha^2m = 1)
            const int w2 = (inverse ? jj + e : jj - e) & (2 * m - 1);
            const bool neg = (w2 & m) != 0;
            const int idx = w2 & (m - 1);
            // coefficient slots (element * m + coefficient), LS words each
            const int ex = ((c << A.log2r) + xs) << A.log2m;
            const int ey = ex + (h << A.log2m);
            const uint32_t* X = cur + (ex + jj) * LS;
            const uint32_t* Y = cur + (ey + idx) * LS;
            uint32_t xv[L], yv[L], sv[L], dv[L];
#pragma unroll
            for (int w = 0; w < L; ++w) {
                xv[w] = X[w];
                yv[w] = Y[w];
            }
            lmod_add<C>(sv, xv, yv, qv);
            lmod_sub<C>(dv, xv, yv, qv);
            // a negated y swaps the two outputs: chosen by address, not per limb
            uint32_t* PS = nxt + ((neg ? ey : ex) + jj) * LS;
            uint32_t* PD = nxt + ((neg ? ex : ey) + jj) * LS;
#pragma unroll
            for (int w = 0; w < L; ++w) PS[w] = sv[w];
#pragma unroll
            for (int w = 0; w < L; ++w) PD[w] = dv[w];
        }
        __syncthreads();
        uint32_t* tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
}

// Coefficient j of b for the element that this thread serves in the round starting at r0.
template <int C>
__device__ __forceinline__ void pw_fetch(Ahead<C>& f, int r0, const uint32_t* __restrict__ bpoly,
                                         const LevelArgs& A, long long c0) {
    constexpr int L = fmt_L(C);
    const int g = threadIdx.x >> A.log2m, j = threadIdx.x & ((1 << A.log2m) - 1);
    const int el = r0 + g;
    f.nz = el < (1 << (A.log2C + A.log2r));
    if (!f.nz || !bpoly) return;
    const int c = el >> A.log2r, v = el & ((1 << A.log2r) - 1);
    const uint32_t* src = bpoly + (((size_t)level_pos(A, c0, c, v) << A.log2m) + j) * L;
    uint32_t x[L];
#pragma unroll
    for (int y = 0; y < L; ++y) x[y] = src[y];
    limbs_to_digits<C>(x, f.v);
}

// Componentwise products of the bottom level (Step 6 fused between the last forward and the
// first inverse level): the element at position v of each column (slot v, after the forward
// DFT) becomes a_v * b_v * (2M)^-1, in place.  b_v is read from the transform of b at the same
// polynomial position (bpoly; f holds round 0's on entry), or is a_v itself for a squaring
// (bpoly NULL), and is staged with its negation, like a twiddle.  Rounds of 256/m elements,
// synchronized per wavefront as in level_twiddle.
template <int C, int FM>
__device__ __forceinline__ void level_pointwise(Ahead<C>& f, uint32_t* cur, uint32_t* RB,
                                                const uint32_t* __restrict__ bpoly, const LevelArgs& A,
                                                long long c0, const QConst& Q) {
    constexpr int L = fmt_L(C);
    constexpr int D = Dig<C>::D;
    const int m = 1 << A.log2m;
    const int EW = A.ew;                                // an element's digits in LDS
    const int per = kThreads >> A.log2m;
    const int g = threadIdx.x >> A.log2m, j = threadIdx.x & (m - 1);
    const int nel = 1 << (A.log2C + A.log2r);
    uint32_t* TP = RB + g * A.sw;
    for (int r0 = 0; r0 < nel; r0 += per) {
        const int el = r0 + g;
        const bool valid = el < nel;
        const int c = el >> A.log2r, v = el & ((1 << A.log2r) - 1);
        uint32_t* X = cur + ((c << A.log2r) + v) * EW;
        if (valid) {
            uint32_t bv[D], nb[D];
#pragma unroll
            for (int y = 0; y < D; ++y) bv[y] = bpoly ? f.v[y] : X[j * D + y];
            dneg_q<C>(nb, bv, Q);
            uint32_t* t0 = TP + stage_pos(j, 0, A.log2m) * Dig<C>::DS;
            uint32_t* t1 = TP + stage_pos(j + m, 0, A.log2m) * Dig<C>::DS;
#pragma unroll
            for (int y = 0; y < D; ++y) {
                t0[y] = bv[y];
                t1[y] = nb[y];
            }
        }
        if (r0 + per < nel) pw_fetch<C>(f, r0 + per, bpoly, A, c0);     // next round's b
        wave_sync();
        uint32_t out[D];
        if (valid) {
            uint32_t cv[D];
            rprod_coeff<C, false, FM>(TP, X, A.log2m, j, Q, cv);   // (a*b)_j 2^-28K
            mont_scalar<C>(cv, Q.kpw, Q, out);              // * (2M)^-1 2^28K
        }
        wave_sync();
        if (valid) {
#pragma unroll
            for (int y = 0; y < D; ++y) X[j * D + y] = out[y];
        }
    }
    __syncthreads();
}

// MODE 0: DFT only; 1: forward DFT, then twiddles on the way out; 2: twiddles, then inverse DFT;
// 3 (bottom level, no twiddles): forward DFT, componentwise products with bpoly, inverse DFT.
// ENC (top forward level): the columns are encoded from operand `which` of PA's product instead
// of being read from poly.  FM, FR > 0: the launch has log2 m = FM and radix 2^FR (the commonest
// shapes), given to the compiler so that the index arithmetic of the passes and rounds folds and
// the sum of the products in R unrolls; 0: taken from A (FM > 0 with FR = 0: m fixed, any radix).  LDS: two halves of A.half words; a DFT runs between them on limbs,
// products run on digits in one half with their operands staged in the other.
template <int C, int MODE, bool ENC, int FM, int FR>
__global__ __launch_bounds__(kThreads) void k_level(uint32_t* __restrict__ poly0, long long stride,
                                                    const uint32_t* __restrict__ table, LevelArgs A,
                                                    QConst Q, const uint32_t* __restrict__ bpoly0,
                                                    int squaring, ProdArgs PA, int which, long long M) {
    constexpr int L = fmt_L(C);
    A.mode = MODE;
    if (FM > 0) A.log2m = FM;
    if (FR > 0) A.log2r = FR;
    // words per limb-form residue in LDS: padded to an odd count, so that the lanes of a
    // butterfly pass or a conversion that read consecutive residues hit distinct banks
    constexpr int LS = Dig<C>::LS;
    uint32_t* __restrict__ poly = poly0 + (size_t)blockIdx.y * stride;
    extern __shared__ uint4 smv[];
    uint32_t* const H0 = reinterpret_cast<uint32_t*>(smv);
    uint32_t* const H1 = H0 + A.half;
    const long long c0 = (long long)blockIdx.x << A.log2C;
    const uint32_t* bpoly = (MODE == 3 && !squaring) ? bpoly0 + (size_t)blockIdx.y * stride : nullptr;
    Ahead<C> f;
    if (MODE == 2) {
        // twiddles on digits in H0 (operands staged in H1), then limbs in H1 for the DFT
        tw_fetch<C>(f, 0, table, A, c0);
        level_load_digits<C>(H0, poly, A, c0);
        __syncthreads();
        level_twiddle<C, 2, FM>(f, H0, H1, poly, table, A, c0, Q);
        lds_to_limbs<C, LS>(H1, H0, A, false);
        uint32_t* cur = H1;
        uint32_t* nxt = H0;
        dft_passes<C, LS>(cur, nxt, A, 1, Q);
        level_store_limbs<C, LS>(poly, cur, A, c0);
        return;
    }
    if (ENC) {
        const ProdDesc pd = PA.get();
        level_encode_in<C, LS>(H0, which ? pd.b : pd.a, which ? pd.blen : pd.alen, pd.u, M, A, c0);
    } else {
        level_load_limbs<C, LS>(H0, poly, A, c0);
    }
    // round 0's operand after the column loads, so that its latency hides behind the DFT
    if (MODE == 1) tw_fetch<C>(f, 0, table, A, c0);
    if (MODE == 3) pw_fetch<C>(f, 0, bpoly, A, c0);
    __syncthreads();
    uint32_t* cur = H0;
    uint32_t* nxt = H1;
    dft_passes<C, LS>(cur, nxt, A, MODE == 3 ? 0 : A.inverse, Q, ENC ? 1 : 0);   // ENC: pass 0 done
    if (MODE == 0) {
        level_store_limbs<C, LS>(poly, cur, A, c0);
        return;
    }
    // digits for the products in the other half; the staging takes the DFT's half
    uint32_t* dg = nxt;
    lds_to_digits<C, LS>(dg, cur, A);
    if (MODE == 1) {
        level_twiddle<C, 1, FM>(f, dg, cur, poly, table, A, c0, Q);
    } else {
        level_pointwise<C, FM>(f, dg, cur, bpoly, A, c0, Q);
        lds_to_limbs<C, LS>(cur, dg, A, true);          // slot v -> bitrev(v): the inverse DFT's input
        nxt = dg;
        dft_passes<C, LS>(cur, nxt, A, 1, Q);
        level_store_limbs<C, LS>(poly, cur, A, c0);
    }
}

// ---------------------------------------------------------------------------------------------
// Step 6: componentwise products, A[i] = A[i] * B[i] (2M)^-1
// ---------------------------------------------------------------------------------------------

// m threads per element, 256/m elements per workgroup; LDS per element: a and q - a (2m
// residues) and b (m residues), digits.
template <int C>
__global__ __launch_bounds__(kThreads) void k_pointwise(uint32_t* A0, const uint32_t* B0, long long stride,
                                                        long long count, int log2m, QConst Q) {
    constexpr int L = fmt_L(C);
    constexpr int D = Dig<C>::D;
    uint32_t* A = A0 + (size_t)blockIdx.y * stride;
    const uint32_t* B = B0 + (size_t)blockIdx.y * stride;
    extern __shared__ uint32_t sm[];
    const int m = 1 << log2m;
    const int per = kThreads >> log2m;
    const int g = threadIdx.x >> log2m, j = threadIdx.x & (m - 1);
    constexpr int DS = Dig<C>::DS;
    uint32_t* TP = sm + g * m * (2 * DS + D);
    uint32_t* X = TP + 2 * m * DS;
    const long long p = (long long)blockIdx.x * per + g;
    const bool active = p < count;
    if (active) {
        uint32_t la[L], lb[L], x[D], xb[D], nx[D];
        const uint32_t* sa = A + ((size_t)p * m + j) * L;
        const uint32_t* sb = B + ((size_t)p * m + j) * L;
#pragma unroll
        for (int w = 0; w < L; ++w) {
            la[w] = sa[w];
            lb[w] = sb[w];
        }
        limbs_to_digits<C>(la, x);
        limbs_to_digits<C>(lb, xb);
#pragma unroll
        for (int w = 0; w < D; ++w) X[j * D + w] = xb[w];
        dneg_q<C>(nx, x, Q);
#pragma unroll
        for (int w = 0; w < D; ++w) {
            TP[stage_pos(j, 0, log2m) * DS + w] = x[w];
            TP[stage_pos(j + m, 0, log2m) * DS + w] = nx[w];
        }
    }
    __syncthreads();
    if (active) {
        uint32_t c[D], out[D], lo[L];
        rprod_coeff<C>(TP, X, log2m, j, Q, c);        // (a*b)_j 2^-28K
        mont_scalar<C>(c, Q.kpw, Q, out);             // * (2M)^-1 2^28K
        digits_to_limbs<C>(out, lo);
        uint32_t* dst = A + ((size_t)p * m + j) * L;
#pragma unroll
        for (int w = 0; w < L; ++w) dst[w] = lo[w];
    }
}

// ---------------------------------------------------------------------------------------------
// Step 6 as the thesis writes it (Sec. 3.2.6): a product in R by Kronecker-Schoenhage
// substitution, the integer products by the library's own multiplication (recursively DKSS
// above the base-case cutoff)
// ---------------------------------------------------------------------------------------------

// Element p of each of the group's polynomials (m coefficients of L limbs, canonical) becomes
// the integer X_p = sum_j a_j 2^(slot j) of wks limbs; slot = 2 bits(q) + ceil(log2 m) holds any
// coefficient of the product polynomial (a sum of m products below q^2).  Since slot exceeds
// bits(q) + 32, a 32-bit window meets at most one coefficient.  One thread per limb.
template <int C>
__global__ __launch_bounds__(kThreads) void k_ks_pack(uint32_t* __restrict__ X, const uint32_t* __restrict__ A0,
                                                      long long stride, long long count, int log2m, int slot,
                                                      int wks) {
    constexpr int L = fmt_L(C);
    const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (t >= count * wks) return;
    const size_t y = blockIdx.y;
    const long long p = t / wks;
    const int w = (int)(t - p * wks);
    const int m = 1 << log2m;
    const uint32_t* A = A0 + y * stride + ((size_t)p << log2m) * L;
    const long long bit0 = 32LL * w;
    const int j = (int)(bit0 / slot);
    uint32_t v = 0;
    for (int jj = j; jj <= j + 1 && jj < m; ++jj) {
        const long long off = bit0 - (long long)slot * jj;     // bit of a_jj at the window's bit 0
        if (off >= 32 * L || off <= -32) continue;
        const uint32_t* cf = A + (size_t)jj * L;
        if (off >= 0) {
            const int q = (int)(off >> 5), b = (int)(off & 31);
            const uint32_t lo = cf[q];
            const uint32_t hi = q + 1 < L ? cf[q + 1] : 0u;
            v |= b ? (lo >> b) | (hi << (32 - b)) : lo;
        } else {
            v |= cf[0] << (int)(-off);
        }
    }
    X[y * (size_t)count * wks + t] = v;
}

// Coefficient j of element p: slots j and j + m of Z_p (the product X_p Y_p, 2 wks limbs) are
// the sums of the product polynomial's coefficients j and j + m, below m q^2 <= 64 q^2; each is
// reduced by Montgomery's method from its 28-bit digits, then c_j = (s_j - s_(j+m)) (2M)^-1
// (alpha^m = -1), written as limbs.  One thread per coefficient.
template <int C>
__global__ __launch_bounds__(kThreads) void k_ks_unpack(uint32_t* A0, long long stride,
                                                        const uint32_t* __restrict__ Z0, long long count,
                                                        int log2m, int slot, int wks, QConst Q) {
    constexpr int L = fmt_L(C);
    using G = Dig<C>;
    constexpr int D = G::D;
    const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
    const int m = 1 << log2m;
    if (t >= (count << log2m)) return;
    const size_t y = blockIdx.y;
    const long long p = t >> log2m;
    const int j = (int)(t & (m - 1));
    const uint32_t* Z = Z0 + (y * (size_t)count + p) * 2 * wks;
    const int zw = 2 * wks;
    auto reduce_slot = [&](int i, uint32_t* r) {
        uint64_t col[G::NC];
#pragma unroll
        for (int k = 0; k < G::NC; ++k) {
            const long long bit = (long long)slot * i + 28LL * k;
            uint32_t d = 0;
            if (28 * k < slot) {
                const long long q = bit >> 5;
                const int b = (int)(bit & 31);
                const uint32_t lo = q < zw ? Z[q] : 0u;
                const uint32_t hi = q + 1 < zw ? Z[q + 1] : 0u;
                d = (uint32_t)((((uint64_t)hi << 32) | lo) >> b) & kMask28;
                const int nb = slot - 28 * k;           // the slot's bits left
                if (nb < 28) d &= (1u << nb) - 1u;
            }
            col[k] = d;
        }
        redc_cols<C>(col, Q, r);
    };
    uint32_t r1[D], r2[D], c[D], out[D], lo[L];
    reduce_slot(j, r1);
    if (j + m < 2 * m - 1) {
        reduce_slot(j + m, r2);
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) r2[k] = 0;
    }
    dmod_sub<C>(c, r1, r2, Q);                     // (a*b)_j 2^-28K
    mont_scalar<C>(c, Q.kpw, Q, out);              // * (2M)^-1 2^28K
    digits_to_limbs<C>(out, lo);
    uint32_t* dst = A0 + y * stride + (((size_t)p << log2m) + j) * L;
#pragma unroll
    for (int k = 0; k < L; ++k) dst[k] = lo[k];
}

// descriptors of the integer products Z_i = X_i Y_i (Y = X for a squaring)
__global__ void k_ks_descs(ProdDesc* __restrict__ d, uint32_t* Z, const uint32_t* X, const uint32_t* Y,
                           long long n, int wks, int u) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    d[i] = ProdDesc{Z + (size_t)i * 2 * wks, X + (size_t)i * wks, Y + (size_t)i * wks, wks, wks, u, 0};
}

// ---------------------------------------------------------------------------------------------
// Table of rho^s, s < mu_top, Montgomery form: entry s = the m coefficients of rho^s as digit
// residues.  One launch computes table[dst + j] = table[src + j] * table[mul], j < cnt.
// ---------------------------------------------------------------------------------------------

// Words [first, first + count) of a table, count <= kPutWords, taken from the launch's arguments.
// Entries 0 and 1 of a table reach the device this way, so that building a table is a sequence
// of kernel launches on the caller's stream (no host buffer has to outlive the call, and a
// stream capture records the whole build).
constexpr int kPutWords = kThreads;
struct PutChunk {
    uint32_t w[kPutWords];
};

__global__ __launch_bounds__(kThreads) void k_table_put(uint32_t* __restrict__ table, PutChunk ch, long long first,
                                                        int count) {
    if ((int)threadIdx.x < count) table[first + threadIdx.x] = ch.w[threadIdx.x];
}

template <int C>
__global__ __launch_bounds__(kThreads) void k_table_mul(uint32_t* table, long long src, long long mul,
                                                        long long dst, long long cnt, int log2m,
                                                        QConst Q) {
    constexpr int L = fmt_L(C);
    constexpr int D = Dig<C>::D;
    extern __shared__ uint32_t sm[];
    const int m = 1 << log2m;
    const int per = kThreads >> log2m;
    const int g = threadIdx.x >> log2m, j = threadIdx.x & (m - 1);
    constexpr int DS = Dig<C>::DS;
    uint32_t* TP = sm + g * m * (2 * DS + D);
    uint32_t* X = TP + 2 * m * DS;
    const long long jj = (long long)blockIdx.x * per + g;
    const bool active = jj < cnt;
    if (active) {
        const uint32_t* xs = table + (size_t)(src + jj) * m * D;
        const uint32_t* ts = table + (size_t)mul * m * D;
        uint32_t tv[D], nt[D];
#pragma unroll
        for (int y = 0; y < D; ++y) tv[y] = ts[j * D + y];
        dneg_q<C>(nt, tv, Q);
#pragma unroll
        for (int y = 0; y < D; ++y) {
            X[j * D + y] = xs[j * D + y];
            TP[stage_pos(j, 0, log2m) * DS + y] = tv[y];
            TP[stage_pos(j + m, 0, log2m) * DS + y] = nt[y];
        }
    }
    __syncthreads();
    if (active) {
        uint32_t out[D];
        rprod_coeff<C>(TP, X, log2m, j, Q, out);
        uint32_t* dp = table + (size_t)(dst + jj) * m * D;
#pragma unroll
        for (int y = 0; y < D; ++y) dp[j * D + y] = out[y];
    }
}

// ---------------------------------------------------------------------------------------------
// Step 8: decode and carry
// ---------------------------------------------------------------------------------------------

// Sum of the 32-bit pieces that the coefficients c_(l,k) (value sum c_(l,k) 2^(u (k + l m/2)))
// put into output word w.  Coefficients are exact integers below q < 2^(32L), in L limbs.
// floor(x / u) for 0 <= x < 2^40 and 1 <= u < 2^20: a double-precision estimate, corrected by
// one step either way (the estimate is within 1 of the quotient)
__device__ __forceinline__ long long div_u(long long x, int u, double inv_u) {
    long long q = (long long)((double)x * inv_u);
    if (q * u > x) --q;
    else if ((q + 1) * u <= x) ++q;
    return q;
}

// poly holds the elements from lbase on (the whole polynomial: lbase 0).
template <int C>
__device__ __forceinline__ uint64_t word_sum(long long w, const uint32_t* __restrict__ poly, long long lbase,
                                             long long twoM, int log2m, int u) {
    constexpr int L = fmt_L(C);
    const int m = 1 << log2m;
    const int hm = m >> 1;
    const double inv_u = 1.0 / (double)u;
    const long long lo_excl = 32 * w - 32 * L;            // piece iff u g > lo_excl
    const long long g_lo = lo_excl < 0 ? 0 : div_u(lo_excl, u, inv_u) + 1;
    const long long g_hi = div_u(32 * w + 31, u, inv_u);
    uint64_t V = 0;
    for (long long g = g_lo; g <= g_hi; ++g) {
        const long long P = (long long)u * g;
        const long long off = 32 * w - P;                  // bit of the term at word w's bit 0
        const long long lmax = g >> (log2m - 1);          // g / (m/2)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const long long l = lmax - t;
            if (l < 0 || l >= twoM) continue;
            const int k = (int)(g - l * hm);
            const uint32_t* T = poly + ((size_t)(l - lbase) * m + k) * L;
            uint32_t piece;
            if (off >= 0) {
                const int o = (int)off;                 // below 32 L
                const int k0 = o >> 5, sh = o & 31;
                uint64_t v = T[k0];
                if (k0 + 1 < L) v |= (uint64_t)T[k0 + 1] << 32;
                piece = (uint32_t)(v >> sh);
            } else {
                piece = T[0] << (int)(-off);            // -32 < off < 0
            }
            V += piece;
        }
    }
    return V;
}

// Words of a position's aligned value: V_g < 2q < 2^(32L + 1) shifted left by up to 31 bits.
template <int C>
__host__ __device__ constexpr int pos_words() {
    return fmt_L(C) + 1;
}

// Position g = l m/2 + k (k < m/2) of the product's coefficient sequence: the value
// V_g = c_(l,k) + c_(l-1,k+m/2) (the upper half of element l-1 overlaps the lower half of element l,
// Sec. 3.2.8) starts at bit u g.  Writes V_g shifted left by (u g) mod 32 as pos_words() words,
// so that word i of it is bits [32 (W_g + i), 32 (W_g + i + 1)) of its contribution, W_g = u g div 32.
template <int C>
__device__ __forceinline__ void position_value(const uint32_t* __restrict__ poly, long long g, long long twoM,
                                               int log2m, int u, uint32_t* out) {
    constexpr int L = fmt_L(C);
    constexpr int NW = pos_words<C>();
    const int m = 1 << log2m, hm = m >> 1;
    const long long l = g >> (log2m - 1);
    const int k = (int)(g & (hm - 1));
    const bool has1 = l < twoM, has2 = l >= 1 && l - 1 < twoM;
    const size_t o1 = has1 ? ((size_t)l * m + k) * L : 0;
    const size_t o2 = has2 ? ((size_t)(l - 1) * m + k + hm) * L : 0;
    uint32_t v[L + 1];
    unsigned int carry = 0;
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const uint32_t x = has1 ? poly[o1 + i] : 0u;
        const uint32_t y = has2 ? poly[o2 + i] : 0u;
        v[i] = __builtin_addc(x, y, carry, &carry);
    }
    v[L] = carry;
    const int sh = (int)(((unsigned)u * (unsigned)g) & 31u);
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const uint32_t lo = w >= 1 ? v[w - 1] : 0u;
        out[w] = (uint32_t)(((((uint64_t)v[w] << 32) | lo) << sh) >> 32);
    }
}

// Sum of word w's 32-bit pieces from the positions in LDS (positions g_min .. g_max of the
// workgroup, pos_words() words each).
// floor(y / u) for 0 <= y < 2^22 and 1 <= u < 2^16: a single-precision estimate, corrected by
// one step either way (the estimate is within 1 of the quotient)
__device__ __forceinline__ int div_small(int y, int u, float inv_u) {
    int q = (int)((float)y * inv_u);
    if (q * u > y) --q;
    else if ((q + 1) * u <= y) ++q;
    return q;
}

// V_w from the aligned position values pv of positions g_min..g_max (LDS).  The quotients by u
// are taken relative to the workgroup's base bq (bq u is at most every numerator here, and the
// numerators exceed it by less than 2^15), so that they are small divisions; the bit offset u g
// of each position advances by u per step.
template <int C>
__device__ __forceinline__ uint64_t word_sum_tiled(long long w, const uint32_t* pv, long long g_min, long long g_max,
                                                   int u, long long bq, float inv_u) {
    constexpr int L = fmt_L(C);
    constexpr int NW = pos_words<C>();
    const long long B = bq * u;
    const long long lo_excl = 32 * w - (32 * L + 1);      // V_g reaches word w iff u g > lo_excl
    long long g = lo_excl < 0 ? 0 : bq + div_small((int)(lo_excl - B), u, inv_u) + 1;
    long long g_hi = bq + div_small((int)(32 * w + 31 - B), u, inv_u);
    if (g < g_min) g = g_min;
    if (g_hi > g_max) g_hi = g_max;
    uint64_t V = 0;
    long long ug = (long long)u * g;
    for (; g <= g_hi; ++g, ug += u) V += pv[(g - g_min) * NW + (w - (ug >> 5))];
    return V;
}

// Per 256 output words: x_w = low(V_w) + high(V_(w-1)) < 2^32 + 2^12, so word w generates a carry
// (x_w >= 2^32) or propagates one (low 32 bits all ones), never both.  Writes the low 32 bits
// and the per-wavefront generate / propagate masks.  TILED: the workgroup first writes the
// aligned values of the positions its words draw on into LDS (one position per thread and step),
// then sums each word from them; the host picks it when those positions fit.
template <int C, bool TILED>
__global__ __launch_bounds__(kThreads) void k_decode(ProdArgs PA, const uint32_t* __restrict__ poly0,
                                                     long long stride, long long twoM, int log2m,
                                                     unsigned long long* __restrict__ gmask0,
                                                     unsigned long long* __restrict__ pmask0,
                                                     long long wstride) {
    constexpr int L = fmt_L(C);
    constexpr int NW = pos_words<C>();
    __shared__ uint32_t hiv[kThreads + 1];
    extern __shared__ uint4 dsmv[];
    const ProdDesc pd = PA.get();
    uint32_t* __restrict__ out = pd.c;
    const long long nw = pd.alen + pd.blen;
    const int u = pd.u;
    const uint32_t* __restrict__ poly = poly0 + (size_t)blockIdx.y * stride;
    unsigned long long* __restrict__ gmask = gmask0 + (size_t)blockIdx.y * wstride;
    unsigned long long* __restrict__ pmask = pmask0 + (size_t)blockIdx.y * wstride;
    const long long w0 = (long long)blockIdx.x * kThreads;
    const long long w = w0 + threadIdx.x;
    uint64_t V = 0, Vprev = 0;
    if (TILED) {
        // positions reaching words w0 - 1 .. min(w0 + 255, nw - 1)
        uint32_t* pv = reinterpret_cast<uint32_t*>(dsmv);
        const double inv_u = 1.0 / (double)u;
        long long g_min = 0, g_max = -1;
        if (w0 < nw) {
            const long long wlo = w0 > 0 ? w0 - 1 : 0;
            const long long whi = (w0 + kThreads - 1 < nw ? w0 + kThreads : nw) - 1;
            const long long lo_excl = 32 * wlo - (32 * L + 1);
            g_min = lo_excl < 0 ? 0 : div_u(lo_excl, u, inv_u) + 1;
            g_max = div_u(32 * whi + 31, u, inv_u);
        }
        for (long long g = g_min + threadIdx.x; g <= g_max; g += kThreads)
            position_value<C>(poly, g, twoM, log2m, u, pv + (g - g_min) * NW);
        __syncthreads();
        const long long bq = g_min > 0 ? g_min - 1 : 0;    // floor(lo_excl(w0 - 1) / u)
        const float inv_uf = 1.0f / (float)u;
        if (w < nw) V = word_sum_tiled<C>(w, pv, g_min, g_max, u, bq, inv_uf);
        if (threadIdx.x == 0 && w0 > 0 && w0 < nw) Vprev = word_sum_tiled<C>(w0 - 1, pv, g_min, g_max, u, bq, inv_uf);
    } else {
        if (w < nw) V = word_sum<C>(w, poly, 0, twoM, log2m, u);
        if (threadIdx.x == 0 && w0 > 0 && w0 < nw) Vprev = word_sum<C>(w0 - 1, poly, 0, twoM, log2m, u);
    }
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

// carry out of a 64-word wavefront for a carry in c: the carry out of (G|P) + G + c
__device__ __forceinline__ void wave_fn(unsigned long long G, unsigned long long P, bool* g, bool* p) {
    const unsigned long long A = G | P;
    const unsigned long long s = A + G;
    const bool c0 = s < A;
    *g = c0;
    *p = c0 || s == ~0ull;
}

// Carry functions c -> g | (p & c) compose as (g2, p2) o (g1, p1) = (g2 | (p2 & g1), p2 & p1).
// Segments of 256 wavefronts (16384 words): one workgroup scans a segment's 256 functions in LDS
// and stores, per wavefront, its carry in for a segment carry in of 0 (bit 0) and of 1 (bit 1),
// plus the segment's composed function.
__global__ __launch_bounds__(kThreads) void k_carry_block(ProdArgs PA,
                                                          const unsigned long long* __restrict__ gmask0,
                                                          const unsigned long long* __restrict__ pmask0,
                                                          unsigned char* __restrict__ cin010,
                                                          unsigned char* __restrict__ seg_gp0,
                                                          long long wstride, long long sstride) {
    __shared__ unsigned char sg[kThreads], sp[kThreads];
    const ProdDesc pd = PA.get();
    const long long nwaves = (pd.alen + pd.blen + 63) / 64;
    const size_t y = blockIdx.y;
    const unsigned long long* __restrict__ gmask = gmask0 + y * wstride;
    const unsigned long long* __restrict__ pmask = pmask0 + y * wstride;
    unsigned char* __restrict__ cin01 = cin010 + y * wstride;
    unsigned char* __restrict__ seg_gp = seg_gp0 + y * sstride;
    const long long nseg = (nwaves + kThreads - 1) / kThreads;
    const long long k = (long long)blockIdx.x * kThreads + threadIdx.x;
    bool g = false, p = true;                 // identity beyond the last wavefront
    if (k < nwaves) wave_fn(gmask[k], pmask[k], &g, &p);
    sg[threadIdx.x] = g;
    sp[threadIdx.x] = p;
    __syncthreads();
    for (int d = 1; d < kThreads; d <<= 1) {
        bool ng = g, np = p;
        if ((int)threadIdx.x >= d) {
            const bool g1 = sg[threadIdx.x - d], p1 = sp[threadIdx.x - d];
            ng = g || (p && g1);
            np = p && p1;
        }
        __syncthreads();
        sg[threadIdx.x] = ng;
        sp[threadIdx.x] = np;
        g = ng;
        p = np;
        __syncthreads();
    }
    // exclusive prefix = inclusive value of the previous thread
    bool eg = false, ep = true;
    if (threadIdx.x > 0) {
        eg = sg[threadIdx.x - 1];
        ep = sp[threadIdx.x - 1];
    }
    if (k < nwaves) cin01[k] = (unsigned char)((eg ? 1 : 0) | ((eg || ep) ? 2 : 0));
    if (threadIdx.x == kThreads - 1 && (long long)blockIdx.x < nseg)
        seg_gp[blockIdx.x] = (unsigned char)((g ? 1 : 0) | (p ? 2 : 0));
}

// Single workgroup: carry into every segment (each thread composes a contiguous run of segments,
// thread 0 scans the 1024 compositions).
__global__ __launch_bounds__(1024) void k_carry_top(ProdArgs PA, const unsigned char* __restrict__ seg_gp0,
                                                    unsigned char* __restrict__ seg_cin0, long long sstride) {
    __shared__ unsigned char ag[1024], ap[1024], ac[1024];
    const ProdDesc pd = PA.get();
    const long long nseg = ((pd.alen + pd.blen + 63) / 64 + kThreads - 1) / kThreads;
    const unsigned char* __restrict__ seg_gp = seg_gp0 + (size_t)blockIdx.y * sstride;
    unsigned char* __restrict__ seg_cin = seg_cin0 + (size_t)blockIdx.y * sstride;
    const long long ch = (nseg + 1023) / 1024;
    const long long s = threadIdx.x * ch;
    const long long e = min(s + ch, nseg);
    bool fg = false, fp = true;
    for (long long k = s; k < e; ++k) {
        const bool g = seg_gp[k] & 1, p = (seg_gp[k] >> 1) & 1;
        fg = g || (p && fg);
        fp = p && fp;
    }
    // inclusive scan of the 1024 run compositions (Hillis-Steele), then shift for exclusive
    ag[threadIdx.x] = fg;
    ap[threadIdx.x] = fp;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        bool ng = fg, np = fp;
        if ((int)threadIdx.x >= d) {
            ng = fg || (fp && ag[threadIdx.x - d]);
            np = fp && ap[threadIdx.x - d];
        }
        __syncthreads();
        ag[threadIdx.x] = ng;
        ap[threadIdx.x] = np;
        fg = ng;
        fp = np;
        __syncthreads();
    }
    ac[threadIdx.x] = threadIdx.x ? ag[threadIdx.x - 1] : false;   // carry in: segment cin is 0
    __syncthreads();
    bool c = ac[threadIdx.x];
    for (long long k = s; k < e; ++k) {
        seg_cin[k] = c;
        const bool g = seg_gp[k] & 1, p = (seg_gp[k] >> 1) & 1;
        c = g || (p && c);
    }
}

// word w += carry into w: bit (w mod 64) of ((G|P) + G + c_in) ^ (G|P) ^ G
__global__ __launch_bounds__(kThreads) void k_carry_apply(ProdArgs PA,
                                                          const unsigned long long* __restrict__ gmask0,
                                                          const unsigned long long* __restrict__ pmask0,
                                                          const unsigned char* __restrict__ cin010,
                                                          const unsigned char* __restrict__ seg_cin0,
                                                          long long wstride, long long sstride) {
    const ProdDesc pd = PA.get();
    uint32_t* __restrict__ out = pd.c;
    const long long nw = pd.alen + pd.blen;
    const size_t y = blockIdx.y;
    const unsigned long long* __restrict__ gmask = gmask0 + y * wstride;
    const unsigned long long* __restrict__ pmask = pmask0 + y * wstride;
    const unsigned char* __restrict__ cin01 = cin010 + y * wstride;
    const unsigned char* __restrict__ seg_cin = seg_cin0 + y * sstride;
    // four consecutive words per thread, all in the same 64-word wavefront group
    const long long w = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (w >= nw) return;
    const long long wave = w >> 6;
    const int c = (cin01[wave] >> (seg_cin[wave >> 8] ? 1 : 0)) & 1;
    const unsigned long long G = gmask[wave], A = G | pmask[wave];
    const unsigned long long carries = (A + G + (unsigned long long)c) ^ A ^ G;
    const uint32_t bits = (uint32_t)(carries >> (w & 63)) & 0xFu;
    if (w + 4 <= nw && ((uintptr_t)(out + w) & 15) == 0) {
        uint4 v = *reinterpret_cast<const uint4*>(out + w);
        v.x += bits & 1u;
        v.y += (bits >> 1) & 1u;
        v.z += (bits >> 2) & 1u;
        v.w += (bits >> 3) & 1u;
        *reinterpret_cast<uint4*>(out + w) = v;
    } else {
        for (int k = 0; k < 4 && w + k < nw; ++k) out[w + k] += (bits >> k) & 1u;
    }
}

// ---------------------------------------------------------------------------------------------
// Base case: schoolbook product (Sec. 2.3), one workgroup per product, alen + blen <= 4096
// ---------------------------------------------------------------------------------------------

// LDS: a, a zero word, b, a zero word (at least 64 words), then the three 32-bit parts of every
// output column's sum; once the columns are summed, the first 256 bytes hold one carry function
// per thread.  Thread t sums columns 2t and 2t + 1, then 2t + 512 and 2t + 513, ...; each column
// total sum_i a_i b_(w-i) < 2^76 is kept as 64 + 32 bits (a carry count beside a 64-bit
// accumulator).
// The words x_w = col_w[0] + col_(w-1)[1] + col_(w-2)[2] < 3 2^32 then take carries of 0, 1 or 2:
// thread t owns the chunk of K consecutive words starting at t K, its carry out as a function of
// its carry in (three values of {0, 1, 2}) is composed across threads by a prefix scan, and each
// chunk is finished with its carry in.
__device__ __forceinline__ uint32_t chunk_carry(const uint32_t* col, long long w0, long long w1, uint32_t cin,
                                                uint32_t* __restrict__ out) {
    uint64_t carry = cin;
    for (long long w = w0; w < w1; ++w) {
        uint64_t x = carry + col[3 * w];
        if (w >= 1) x += col[3 * (w - 1) + 1];
        if (w >= 2) x += col[3 * (w - 2) + 2];
        if (out) out[w] = (uint32_t)x;
        carry = x >> 32;
    }
    return (uint32_t)carry;
}

__global__ __launch_bounds__(kThreads) void k_schoolbook(ProdArgs PA) {
    extern __shared__ uint32_t sv[];
    const ProdDesc pd = PA.get();
    const long long alen = pd.alen, blen = pd.blen;
    const long long n = alen + blen;
    // a, then b between two zero words (B[-1] = B[blen] = 0), then the columns
    uint32_t* const A = sv;
    uint32_t* const B = sv + alen + 1;
    uint32_t* const col = sv + (n + 2 > 64 ? n + 2 : 64);
    unsigned char* const fn = reinterpret_cast<unsigned char*>(sv);     // after the columns
    for (long long i = threadIdx.x; i < alen; i += kThreads) A[i] = pd.a[i];
    for (long long i = threadIdx.x; i < blen; i += kThreads) B[i] = pd.b[i];
    if (threadIdx.x == 0) {
        B[-1] = 0;
        B[blen] = 0;
    }
    __syncthreads();
    // two neighbouring columns w, w + 1 per thread: each a_i read once for both, and b's
    // words shared between them (b_(w+1-i) = b_(w-(i-1))); i runs over the union of the two
    // ranges, the zero words standing in for the terms one column does not have
    for (long long w = 2 * (long long)threadIdx.x; w < n; w += 2 * kThreads) {
        // four independent partial sums per column (terms i = i0 + 4 k + r), so that
        // consecutive multiply-adds do not wait on each other's accumulator
        uint64_t acc0[4] = {0, 0, 0, 0}, acc1[4] = {0, 0, 0, 0};
        uint32_t top0[4] = {0, 0, 0, 0}, top1[4] = {0, 0, 0, 0};
        const long long i0 = w - blen + 1 > 0 ? w - blen + 1 : 0;
        const long long i1 = w + 1 < alen - 1 ? w + 1 : alen - 1;
        long long i = i0;
        for (; i + 3 <= i1; i += 4) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint64_t a = A[i + r];
                const uint64_t s0 = a * B[w - i - r] + acc0[r];
                const uint64_t s1 = a * B[w + 1 - i - r] + acc1[r];
                top0[r] += s0 < acc0[r];
                top1[r] += s1 < acc1[r];
                acc0[r] = s0;
                acc1[r] = s1;
            }
        }
        for (int r = 0; i <= i1; ++i, ++r) {
            const uint64_t a = A[i];
            const uint64_t s0 = a * B[w - i] + acc0[r];
            const uint64_t s1 = a * B[w + 1 - i] + acc1[r];
            top0[r] += s0 < acc0[r];
            top1[r] += s1 < acc1[r];
            acc0[r] = s0;
            acc1[r] = s1;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint64_t* acc = h ? acc1 : acc0;
            const uint32_t* top = h ? top1 : top0;
            uint64_t sum = acc[0];
            uint32_t t = top[0];
#pragma unroll
            for (int r = 1; r < 4; ++r) {
                const uint64_t s2 = sum + acc[r];
                t += top[r] + (s2 < sum);
                sum = s2;
            }
            if (w + h < n) {
                col[3 * (w + h)] = (uint32_t)sum;
                col[3 * (w + h) + 1] = (uint32_t)(sum >> 32);
                col[3 * (w + h) + 2] = t;
            }
        }
    }
    __syncthreads();
    // carries: chunk t covers words [t K, min(n, (t+1) K))
    const long long K = (n + kThreads - 1) / kThreads;
    const long long w0 = threadIdx.x * K < n ? threadIdx.x * K : n;
    const long long w1 = w0 + K < n ? w0 + K : n;
    uint32_t f = 0;                                   // bits 2c..2c+1: carry out for carry in c
    for (uint32_t c = 0; c < 3; ++c) f |= chunk_carry(col, w0, w1, c, nullptr) << (2 * c);
    fn[threadIdx.x] = (unsigned char)f;
    __syncthreads();
    // inclusive scan of the carry functions: g = f_t o f_(t-1) o ... o f_0
    for (int d = 1; d < kThreads; d <<= 1) {
        const uint32_t mine = fn[threadIdx.x];
        const uint32_t prev = threadIdx.x >= d ? fn[threadIdx.x - d] : 0x24u;   // 0x24: identity
        __syncthreads();
        uint32_t comp = 0;
        for (uint32_t c = 0; c < 3; ++c) comp |= ((mine >> (2 * ((prev >> (2 * c)) & 3))) & 3) << (2 * c);
        fn[threadIdx.x] = (unsigned char)comp;
        __syncthreads();
    }
    const uint32_t cin = threadIdx.x ? fn[threadIdx.x - 1] & 3 : 0;
    chunk_carry(col, w0, w1, cin, pd.c);
}

// ---------------------------------------------------------------------------------------------
// Base case above the schoolbook's size: Karatsuba levels (Sec. 2.4) over schoolbook leaves
// ---------------------------------------------------------------------------------------------
// A product of a (na limbs) and b (nb limbs), n = max(na, nb), h = ceil(n / 2), a = a0 + a1 B^h,
// b = b0 + b1 B^h (B = 2^32; a0 = a's low min(h, na) limbs, a1 the rest, possibly empty):
// a b = P0 + (P1 - P0 - P2) B^h + P2 B^2h with P0 = a0 b0, P2 = a1 b1 and
// P1 = (a0 + a1)(b0 + b1).  One level's kernels: k_kara_eval writes a0 + a1 and b0 + b1 (h + 1
// limbs) into the product's slot and the three sub-products' descriptors; the sub-products run as
// a batch (the schoolbook, or another Karatsuba level); k_kara_combine assembles c.  One wavefront
// per product; carries cross a row of 64 limbs by mask addition (wave_carry.hpp).

// limbs of one level's slot for a product with half size h: a0 + a1, b0 + b1, P0, P2, P1
__host__ __device__ inline long long kara_slot_words(long long h) { return 8 * h + 8; }

__global__ __launch_bounds__(64) void k_kara_eval(ProdArgs PA, ProdDesc* __restrict__ child,
                                                  uint32_t* __restrict__ scratch, long long stride) {
    const ProdDesc pd = PA.get();
    const size_t y = blockIdx.y;
    const long long na = pd.alen, nb = pd.blen;
    const long long n = na > nb ? na : nb;
    const long long h = (n + 1) / 2;
    uint32_t* SA = scratch + y * stride;
    uint32_t* SB = SA + (h + 1);
    uint32_t* P0 = SB + (h + 1);
    uint32_t* P2 = P0 + 2 * h;
    uint32_t* P1 = P2 + 2 * h;
    const int l = wave_lane();
    // x0 + x1 for both operands, h limbs each plus the carry out as limb h
    for (int op = 0; op < 2; ++op) {
        const uint32_t* x = op ? pd.b : pd.a;
        const long long nx = op ? nb : na;
        uint32_t* S = op ? SB : SA;
        uint32_t c = 0;
        for (long long w0 = 0; w0 < h; w0 += 64) {
            const long long w = w0 + l;
            const uint32_t u = w < h && w < nx ? x[w] : 0u;
            const uint32_t v = w < h && h + w < nx ? x[h + w] : 0u;
            uint32_t t = u + v;
            const unsigned long long G = __ballot(t < u);
            // lanes past the last limb pass a carry on, so that it leaves the row's top lane
            const unsigned long long P = __ballot(w >= h || t == 0xFFFFFFFFu);
            t += lane_bit(row_carries(G, P, c, &c));
            if (w < h) S[w] = t;
        }
        if (l == 0) S[h] = c;
    }
    if (l == 0) {
        const long long a0 = na < h ? na : h, b0 = nb < h ? nb : h;
        const long long a1 = na > h ? na - h : 0, b1 = nb > h ? nb - h : 0;
        child[3 * y + 0] = ProdDesc{P0, pd.a, pd.b, a0, b0, 0, 0};
        child[3 * y + 1] = ProdDesc{P2, pd.a + h, pd.b + h, a1, b1, 0, 0};
        child[3 * y + 2] = ProdDesc{P1, SA, SB, h + 1, h + 1, 0, 0};
    }
}

__global__ __launch_bounds__(64) void k_kara_combine(ProdArgs PA, const ProdDesc* __restrict__ child) {
    const ProdDesc pd = PA.get();
    const size_t y = blockIdx.y;
    const long long nc = pd.alen + pd.blen;
    const long long na = pd.alen, nb = pd.blen;
    const long long n = na > nb ? na : nb;
    const long long h = (n + 1) / 2;
    const ProdDesc d0 = child[3 * y], d2 = child[3 * y + 1], d1 = child[3 * y + 2];
    const long long l0 = d0.alen + d0.blen, l2 = d2.alen + d2.blen, l1 = d1.alen + d1.blen;
    uint32_t* P0 = d0.c;
    uint32_t* P2 = d2.c;
    uint32_t* P1 = d1.c;
    uint32_t* c = pd.c;
    const int l = wave_lane();
    // T = P1 - P0 - P2 >= 0, in place of P1 (two subtractions with borrows)
    for (int pass = 0; pass < 2; ++pass) {
        const uint32_t* Q = pass ? P2 : P0;
        const long long lq = pass ? l2 : l0;
        uint32_t bo = 0;
        for (long long w0 = 0; w0 < l1; w0 += 64) {
            const long long w = w0 + l;
            const uint32_t x = w < l1 ? P1[w] : 0u;
            const uint32_t v = w < lq ? Q[w] : 0u;
            uint32_t d = x - v;
            const unsigned long long G = __ballot(x < v);
            const unsigned long long P = __ballot(w < l1 && d == 0u);
            d -= lane_bit(row_carries(G, P, bo, &bo));
            if (w < l1) P1[w] = d;
        }
    }
    // c = P0 + P2 B^2h (disjoint) + T B^h; the words above c's length are zero
    uint32_t cy = 0;
    for (long long w0 = 0; w0 < nc; w0 += 64) {
        const long long w = w0 + l;
        uint32_t base = 0;
        if (w < 2 * h) {
            base = w < l0 ? P0[w] : 0u;
        } else if (w - 2 * h < l2) {
            base = P2[w - 2 * h];
        }
        const uint32_t t = w >= h && w - h < l1 ? P1[w - h] : 0u;
        uint32_t s = base + t;
        const unsigned long long G = __ballot(w < nc && s < base);
        const unsigned long long P = __ballot(w < nc && s == 0xFFFFFFFFu);
        s += lane_bit(row_carries(G, P, cy, &cy));
        if (w < nc) c[w] = s;
    }
}

// Batch descriptors [first, first + count) from the launch's arguments (count <= kDescPerPut):
// a batch's descriptors reach the device as kernel launches on the caller's stream, without a
// staging buffer or a wait on the host.
constexpr int kDescPerPut = 40;
struct DescChunk {
    ProdDesc d[kDescPerPut];
};

__global__ void k_desc_put(ProdDesc* __restrict__ dst, DescChunk ch, long long first, int count) {
    if ((int)threadIdx.x < count) dst[first + threadIdx.x] = ch.d[threadIdx.x];
}

// c = 0 for products of the launch (alen + blen words each)
__global__ void k_zero_products(ProdArgs PA) {
    const ProdDesc pd = PA.get();
    const long long n = pd.alen + pd.blen;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        pd.c[i] = 0;
}

// ---------------------------------------------------------------------------------------------
// Forward output in digit-reversed order -> natural order, digits -> limbs (dkss_forward only)
// ---------------------------------------------------------------------------------------------

struct LevelIdx {
    int n;
    int log2mu[8];
    int log2r[8];
    int shift[8];    // log2 of the product of the radices of the earlier levels
};

// one thread per coefficient: position pos holds a(rho^f), f from the digits of pos
template <int C>
__global__ void k_unscramble(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src,
                             long long twoM, int log2m, LevelIdx LI) {
    constexpr int L = fmt_L(C);
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (twoM << log2m)) return;
    const long long pos = t >> log2m;
    const int k = (int)(t & ((1 << log2m) - 1));
    long long f = 0;
    for (int i = 0; i < LI.n; ++i) {
        const long long v = (pos >> LI.log2mu[i]) & ((1LL << LI.log2r[i]) - 1);
        f |= v << LI.shift[i];
    }
    uint32_t* o = dst + (((size_t)f << log2m) + k) * L;
#pragma unroll
    for (int w = 0; w < L; ++w) o[w] = src[(size_t)t * L + w];
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
    uint32_t* d_table = nullptr;          // the context's copy of the table, once built
    bool table_ready = false;             // d_table holds the finished table
    long long table_count = 0;
    int D = 0;
    // bytes of the table: max(table_count, 2) entries of m residues in D digits
    size_t table_bytes() const {
        return (size_t)std::max<long long>(table_count, 2) * plan.m() * D * sizeof(uint32_t);
    }
};

// resolved per-call plan
struct Call {
    Plan P;                    // parameters + radices
    bool schoolbook = false;
    int kara = 0;                     // Karatsuba levels of a base-case product
    size_t alen = 0, blen = 0;
    Cached* C = nullptr;
    const uint32_t* table = nullptr;  // the rho^s table the call's levels read
    Prof* prof = nullptr;
    long long dft_lds = 32768;
    bool overlap = false;
    bool fuse_pw = true;              // componentwise products fused into the bottom level
    hipStream_t aux = nullptr;        // second stream for the transform of b
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // Step 6 by Kronecker-Schoenhage (DKSS_OPT_STEP6_KS): slot bits, limbs per packed integer
    // and the plan of the integer products (recursively with its own Step 6)
    int ks_slot = 0, ks_wks = 0;
    std::shared_ptr<Call> ks_inner;
};

// 32-bit limbs of q = p^z for a prime of pb bits (q < 2^(z pb)); exact for z = 1 and z = 2
int tuple_limbs(int pb, int z) { return (z * pb + 31) / 32; }

}  // namespace

// Tuned choices: for log2(N) in [lo, hi), candidate index cand (see candidate_params).
// Optionally with the FFT level split and the LDS budget of the DFT-only levels.
constexpr int kCandThesis = -1;  // a table entry that names the thesis rule ("T")
constexpr int kMaxLanes = 8;     // concurrent streams of a batch's groups

struct TuneEntry {
    double lo, hi;
    int cand;                      // a candidate index, DKSS_CAND_SCHOOLBOOK or kCandThesis
    uint32_t batch = 1;            // the entry holds for batches of at least this many products
    std::vector<int> radices;      // empty: the library default
    long long dft_lds = 0;         // 0: the context's option
};

struct dkss_ctx {
    int policy = DKSS_POLICY_THESIS;
    std::vector<TuneEntry> tuning;
    // learned selector
    std::vector<float> mlp;             // weights (empty: none installed)
    float* d_mlp = nullptr;             // device copy, made at the first inference
    bool d_mlp_stale = true;
    hipStream_t mlp_stream = nullptr;   // private stream of the selector's inference
    float* h_io = nullptr;              // pinned features + predictions of io_cap samples
    float* d_io = nullptr;
    size_t io_cap = 0;
    std::map<std::tuple<size_t, size_t, uint32_t>, int> choices;   // (alen, blen, batch) -> choice
    std::map<std::string, std::unique_ptr<Cached>> cache;
    Prof prof;
    bool overlap = false;
    bool fuse_pw = true;
    long long dft_lds = 32768;
    hipStream_t aux = nullptr;          // made when DKSS_OPT_OVERLAP is first switched on
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // batches: groups spread over batch_lanes streams (the caller's and lane_s[0 .. lanes-2],
    // made by planning calls or the option), forked and joined with lane_ev
    bool step6_ks = false;              // Step 6 by Kronecker-Schoenhage substitution
    int batch_lanes = 4;
    int lanes_made = 1;                 // streams available: 1 + the internal ones made so far
    hipStream_t lane_s[kMaxLanes - 1] = {};
    hipEvent_t lane_ev[kMaxLanes] = {};
    ~dkss_ctx() {
        for (int i = 0; i < kMaxLanes; ++i)
            if (lane_ev[i]) (void)hipEventDestroy(lane_ev[i]);
        for (int i = 0; i < kMaxLanes - 1; ++i)
            if (lane_s[i]) (void)hipStreamDestroy(lane_s[i]);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (aux) (void)hipStreamDestroy(aux);
        if (mlp_stream) {
            (void)hipStreamSynchronize(mlp_stream);
            (void)hipStreamDestroy(mlp_stream);
        }
        if (d_mlp) (void)hipFree(d_mlp);
        if (d_io) (void)hipFree(d_io);
        if (h_io) (void)hipHostFree(h_io);
    }
};

namespace {

#define HIP_OK(expr)                                   \
    do {                                               \
        const hipError_t e_ = (expr);                  \
        if (e_ != hipSuccess) return note_hip(e_);     \
    } while (0)

// the context's policy: the tuned table's entry for N (in *te) if it has one, else the thesis
// rule.  Among the entries whose range holds N the one measured at the largest batch size not
// above `batch` wins.  A schoolbook entry sets *school and leaves the thesis tuple in place
// (the product falls back to it where the base case does not apply).
bool policy_tuple(const dkss_ctx* ctx, uint64_t N, uint32_t batch, int* lM, int* lm, int* u, int* pb,
                  int* z, const TuneEntry** te = nullptr, bool* school = nullptr) {
    if (te) *te = nullptr;
    if (school) *school = false;
    *z = 1;
    if (ctx && ctx->policy == DKSS_POLICY_TUNED) {
        const double lg = std::log2((double)N);
        const TuneEntry* hit = nullptr;
        for (const TuneEntry& t : ctx->tuning)
            if (t.batch <= batch && lg >= t.lo && lg < t.hi && (!hit || t.batch > hit->batch) &&
                (t.cand == DKSS_CAND_SCHOOLBOOK || t.cand == kCandThesis ||
                 candidate_params(N, t.cand, lM, lm, u, pb, z)))
                hit = &t;
        if (hit && hit->cand == kCandThesis) {
            // measured no faster than the rule: the rule, with its default level split
        } else if (hit && hit->cand == DKSS_CAND_SCHOOLBOOK) {
            if (school) *school = true;
        } else if (hit && candidate_params(N, hit->cand, lM, lm, u, pb, z)) {
            if (te) *te = hit;
            return true;
        }
    }
    *z = 1;
    return thesis_params(N, lM, lm, u, pb);
}

// ----- learned selector ------------------------------------------------------------------------

// Can the selector's output c run a product of alen x blen limbs?
bool learned_feasible(size_t alen, size_t blen, int c) {
    if (c == DKSS_CAND_SCHOOLBOOK) return kara_depth(alen, blen) >= 0;
    int lM, lm, u, pb, z;
    const uint64_t N = 32ull * std::max(alen, blen);
    return candidate_params(N, c, &lM, &lm, &u, &pb, &z) &&
           default_radices(lM, lm, tuple_limbs(pb, z)).size() <= 8;
}

int ensure_mlp_io(dkss_ctx* ctx, size_t n) {
    if (!ctx->mlp_stream) HIP_OK(hipStreamCreateWithFlags(&ctx->mlp_stream, hipStreamNonBlocking));
    if (!ctx->d_mlp) HIP_OK(hipMalloc((void**)&ctx->d_mlp, DKSS_MLP_NPARAM * sizeof(float)));
    if (ctx->d_mlp_stale) {
        HIP_OK(hipMemcpy(ctx->d_mlp, ctx->mlp.data(), DKSS_MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice));
        ctx->d_mlp_stale = false;
    }
    if (ctx->io_cap < n) {
        if (ctx->d_io) HIP_OK(hipFree(ctx->d_io));
        if (ctx->h_io) HIP_OK(hipHostFree(ctx->h_io));
        ctx->d_io = nullptr;
        ctx->h_io = nullptr;
        ctx->io_cap = 0;
        const size_t cap = std::max<size_t>(n, 256);
        const size_t bytes = cap * (DKSS_MLP_IN + DKSS_MLP_OUT) * sizeof(float);
        HIP_OK(hipMalloc((void**)&ctx->d_io, bytes));
        HIP_OK(hipHostMalloc((void**)&ctx->h_io, bytes, hipHostMallocDefault));
        ctx->io_cap = cap;
    }
    return DKSS_OK;
}

// The selector's choice for each product of alen[i] x blen[i] limbs in a batch of `batch`:
// a candidate index, DKSS_CAND_SCHOOLBOOK, or -1 (no weights, nothing feasible, empty operand).
// Shapes not seen before are evaluated together in one inference launch.
int learned_choices(dkss_ctx* ctx, size_t count, const size_t* alen, const size_t* blen, uint32_t batch,
                    int* out) {
    using Key = std::tuple<size_t, size_t, uint32_t>;
    for (size_t i = 0; i < count; ++i) out[i] = -1;
    if (ctx->mlp.empty() || batch == 0) return DKSS_OK;
    std::map<Key, size_t> fresh;               // unseen shape -> its row in the inference
    std::vector<size_t> rows;                  // product index of each row
    for (size_t i = 0; i < count; ++i) {
        if (alen[i] == 0 || blen[i] == 0) continue;
        const Key k{alen[i], blen[i], batch};
        if (ctx->choices.count(k) || fresh.count(k)) continue;
        fresh.emplace(k, rows.size());
        rows.push_back(i);
    }
    if (!rows.empty()) {
        const size_t n = rows.size();
        int rc = ensure_mlp_io(ctx, n);
        if (rc) return rc;
        float* hx = ctx->h_io;
        float* hy = ctx->h_io + n * DKSS_MLP_IN;
        for (size_t r = 0; r < n; ++r)
            dkss_mlp_features(32ull * alen[rows[r]], 32ull * blen[rows[r]], batch, hx + r * DKSS_MLP_IN);
        float* dx = ctx->d_io;
        float* dy = ctx->d_io + n * DKSS_MLP_IN;
        hipStream_t st = ctx->mlp_stream;
        HIP_OK(hipMemcpyAsync(dx, hx, n * DKSS_MLP_IN * sizeof(float), hipMemcpyHostToDevice, st));
        if ((rc = dkss_mlp_forward(ctx->d_mlp, dx, (int)n, dy, (dkss_stream_t)st))) return rc;
        HIP_OK(hipMemcpyAsync(hy, dy, n * DKSS_MLP_OUT * sizeof(float), hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        for (size_t r = 0; r < n; ++r) {
            const size_t i = rows[r];
            int best = -1;
            for (int c = 0; c < DKSS_MLP_OUT; ++c)
                if ((best < 0 || hy[r * DKSS_MLP_OUT + c] < hy[r * DKSS_MLP_OUT + best]) &&
                    learned_feasible(alen[i], blen[i], c))
                    best = c;
            ctx->choices[Key{alen[i], blen[i], batch}] = best;
        }
    }
    for (size_t i = 0; i < count; ++i)
        if (alen[i] && blen[i]) out[i] = ctx->choices[Key{alen[i], blen[i], batch}];
    return DKSS_OK;
}

// The choice cached for a shape by an earlier planning call (-1: none).  Products take the
// selector's choice from here only, so that they never wait for an inference.
int learned_lookup(const dkss_ctx* ctx, size_t alen, size_t blen, uint32_t batch) {
    const auto it = ctx->choices.find(std::make_tuple(alen, blen, batch));
    return it == ctx->choices.end() ? -1 : it->second;
}

// parameters for a product, from the policy or the caller.  choice: the learned selector's
// output for the product (-1: none, use the policy's tuple).
int resolve_params(dkss_ctx* ctx, size_t alen, size_t blen, const dkss_params* p, Call* out, int choice,
                   uint32_t batch) {
    out->alen = alen;
    out->blen = blen;
    const uint64_t N = 32ull * std::max(alen, blen);
    Plan& P = out->P;
    if (N == 0) return DKSS_OK;
    if (N > (1ull << 36)) return DKSS_ERANGE;
    if (p == nullptr) {
        int lM, lm, u, pb, z;
        P.cutoff_bits = kDefaultCutoffBits;
        const TuneEntry* te = nullptr;
        if (choice >= 0 && choice < kNumCandidates && candidate_params(N, choice, &lM, &lm, &u, &pb, &z)) {
            P.cutoff_bits = 0;
        } else {
            bool school = false;
            if (!policy_tuple(ctx, N, batch, &lM, &lm, &u, &pb, &z, &te, &school)) return DKSS_ERANGE;
            if (school || choice == DKSS_CAND_SCHOOLBOOK) P.cutoff_bits = UINT64_MAX;
        }
        if (te) {                      // the tuned level split and LDS budget, where recorded
            int sum = 0;
            bool fits = true;
            for (int r : te->radices) {
                sum += r;
                fits = fits && r <= max_radix_log2(lm, tuple_limbs(pb, z));
            }
            if (fits && sum == lM + 1) P.radix_log2 = te->radices;
            if (te->dft_lds) out->dft_lds = te->dft_lds;
        }
        P.log2_M = lM;
        P.log2_m = lm;
        P.u = u;
        P.p_bits = pb;
        P.z = z;
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
    out->kara = kara_depth(alen, blen);
    out->schoolbook = minlen <= P.cutoff_bits && out->kara >= 0;
    if (out->schoolbook) return DKSS_OK;
    out->kara = 0;
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
        // the tight format where q fits one digit fewer (not for one limb: no kernels for it)
        const int tight = fmt_code(c->plan.L, true);
        c->plan.fmt = fmt_code(c->plan.L, c->plan.L >= 2 && c->plan.q_bits <= fmt_qbits(tight));
        const int L = c->plan.L, D = fmt_D(c->plan.fmt), K = fmt_K(c->plan.fmt);
        c->D = D;
        const Plan& CP = c->plan;
        ModQ mq(CP.q);
        QConst& Q = c->Q;
        memset(&Q, 0, sizeof Q);
        auto digits = [&](const Big& x, uint32_t* d) {
            for (int k = 0; k < D; ++k) {
                Big s = x.shr(28 * k);
                d[k] = (uint32_t)(s.w[0] & kMask28);
            }
        };
        digits(CP.q, Q.qd);
        for (int k = 0; k < L; ++k) Q.ql[k] = (uint32_t)(CP.q.w[k / 2] >> (32 * (k % 2)));
        // -q^-1 mod 2^28 by Newton iteration on the low word
        uint32_t q0 = (uint32_t)CP.q.w[0];
        uint32_t inv = q0;
        for (int i = 0; i < 5; ++i) inv *= 2u - q0 * inv;
        Q.qinv28 = (0u - inv) & kMask28;
        // q = 1 + qd[e] 2^(28e) + qd[e+1] 2^(28(e+1)): the reduction's sparse steps
        if (Q.qd[0] == 1) {
            int e = 1;
            while (e < D && Q.qd[e] == 0) ++e;
            bool sparse = e < D;
            for (int k = e + 2; k < D; ++k) sparse = sparse && Q.qd[k] == 0;
            Q.se = sparse ? e : 0;
        }
        // R' = 2^(28K) mod q, R'^2 mod q, (2M)^-1 mod q
        Big Rm = mq.reduce(Big::of(1));
        for (int i = 0; i < 28 * K; ++i) Rm = mq.add(Rm, Rm);
        Big R2 = mq.mul(Rm, Rm);
        Big inv2M = mq.reduce(Big::of(1));
        for (int i = 0; i < CP.log2_M + 1; ++i) inv2M = mq.half(inv2M);
        digits(mq.mul(inv2M, R2), Q.kpw);
        // table entries 0 (one) and 1 (rho), Montgomery form
        const int m = CP.m();
        // entry = m residues (the kernels form the negations q - x when they stage an entry)
        c->table_host01.assign((size_t)2 * m * D, 0u);
        auto put = [&](int entry, int k, const Big& x) {
            digits(x, &c->table_host01[((size_t)entry * m + k) * D]);
        };
        for (int k = 0; k < m; ++k) {
            put(0, k, k == 0 ? Rm : Big());
            put(1, k, mq.mul(CP.rho[k], Rm));
        }
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

// launch helpers, dispatched on the residue format (limbs, tight digits)
template <template <int> class F, typename... A>
int dispatch_fmt(int fmt, const A&... args) {
    switch (fmt) {
        case 1: return F<1>::run(args...);
        case 2: return F<2>::run(args...);
        case 3: return F<3>::run(args...);
        case 4: return F<4>::run(args...);
        case 5: return F<5>::run(args...);
        case 6: return F<6>::run(args...);
        case 7: return F<7>::run(args...);
        case 8: return F<8>::run(args...);
        case 16 + 2: return F<16 + 2>::run(args...);
        case 16 + 3: return F<16 + 3>::run(args...);
        case 16 + 4: return F<16 + 4>::run(args...);
        case 16 + 5: return F<16 + 5>::run(args...);
        case 16 + 6: return F<16 + 6>::run(args...);
        case 16 + 7: return F<16 + 7>::run(args...);
        case 16 + 8: return F<16 + 8>::run(args...);
        default: return DKSS_ERANGE;
    }
}

// LDS of the R-product kernels: kThreads coefficient slots, 3 D digits each (T, x, q - x)
size_t rprod_lds(int fmt) { return (size_t)kThreads * (2 * (fmt_D(fmt) | 1) + fmt_D(fmt)) * sizeof(uint32_t); }

template <int C>
struct TableBuild {
    static constexpr int L = fmt_L(C);
    // tab[dst + j] = tab[src + j] * tab[mul], j < cnt
    static int launch(const Cached* tc, uint32_t* tab, Prof* prof, hipStream_t s, long long src, long long mul,
                      long long dst, long long cnt) {
        const int m = tc->plan.m();
        const int per = kThreads / m;
        const unsigned blocks = (unsigned)((cnt + per - 1) / per);
        ProfScope ps(prof, DKSS_K_TABLE, s, 2.0 * cnt * m * Dig<C>::D * 4, (double)cnt * m * m * L * L);
        hipLaunchKernelGGL(k_table_mul<C>, dim3(blocks), dim3(kThreads), rprod_lds(C), s, tab, src, mul, dst, cnt,
                           tc->plan.log2_m, tc->Q);
        return launch_status();
    }
    // The whole table into tab (tc->table_bytes() bytes), on stream s: entries 0 (one) and 1
    // (rho) from the host as launch arguments; then for n = 2, 4, ...: rho^n = rho^(n/2)
    // rho^(n/2), and rho^(n+j) = rho^j rho^n for 0 < j < n.
    static int run(const Cached* tc, uint32_t* tab, Prof* prof, hipStream_t s) {
        const size_t words01 = (size_t)std::min<long long>(tc->table_count, 2) * tc->plan.m() * tc->D;
        for (size_t off = 0; off < words01; off += kPutWords) {
            PutChunk ch;
            const int n = (int)std::min<size_t>(kPutWords, words01 - off);
            memcpy(ch.w, tc->table_host01.data() + off, (size_t)n * sizeof(uint32_t));
            hipLaunchKernelGGL(k_table_put, dim3(1), dim3(kThreads), 0, s, tab, ch, (long long)off, n);
        }
        int rc = launch_status();
        if (rc) return rc;
        for (long long n = 2; n < tc->table_count; n *= 2) {
            if ((rc = launch(tc, tab, prof, s, n / 2, n / 2, n, 1))) return rc;
            const long long cnt = std::min(n, tc->table_count - n) - 1;
            if (cnt > 0 && (rc = launch(tc, tab, prof, s, 1, n, n + 1, cnt))) return rc;
        }
        return DKSS_OK;
    }
};

// The context's own copy of a tuple's table (planning calls only: dkss_prepare, the batch
// preparation and graph creation).  Allocates it, builds it on s and waits for the build; only
// a finished table is marked ready, and on any failure the memory is released and the entry
// stays unbuilt.  Refused on a capturing stream: the build must really run before the table is
// used by later calls.
int ensure_table(Cached* C, Prof* prof, hipStream_t s) {
    if (C->table_ready) return DKSS_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_OK(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone) return DKSS_EINVAL;
    uint32_t* d = nullptr;
    HIP_OK(hipMalloc(&d, C->table_bytes()));
    int rc = dispatch_fmt<TableBuild>(C->plan.fmt, C, d, prof, s);
    if (!rc) rc = note_hip(hipStreamSynchronize(s));
    if (rc) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(d);
        return rc;
    }
    C->d_table = d;
    C->table_ready = true;
    return DKSS_OK;
}

// Workspace of one launch group: G products sharing a plan.  Polynomials at stride S words,
// carry state at strides wst (wavefronts) and sst (segments) of the longest product.
struct Workspace {
    uint32_t* A;
    uint32_t* B;
    size_t S;                          // words per polynomial
    unsigned long long* gmask;
    unsigned long long* pmask;
    unsigned char* cin01;
    unsigned char* seg_gp;
    unsigned char* seg_cin;
    uint32_t* tab;                     // room for the tuple's table (tab_bytes of layout), or NULL
    char* ks;                          // Step 6 by Kronecker-Schoenhage: its region, or NULL
    size_t wst, sst;
    size_t bytes;
};

// words of one polynomial in the workspace (digits) and in limb form (dkss_forward's output)
size_t poly_words(const Plan& P) { return ((size_t)2 << P.log2_M) * P.m() * P.L; }

// tab_bytes: room for a table after the group's buffers (0: none)
Workspace layout(const Plan& P, size_t G, size_t nw_max, bool need_b, char* base, size_t tab_bytes = 0) {
    Workspace w{};
    w.S = poly_words(P);
    const size_t nwaves = (nw_max + 63) / 64;
    const size_t nseg = (nwaves + kThreads - 1) / kThreads;
    w.wst = nwaves;
    w.sst = nseg;
    size_t off = 0;
    w.A = (uint32_t*)(base + off);
    off += align256(G * w.S * 4);
    w.B = (uint32_t*)(base + off);
    off += need_b ? align256(G * w.S * 4) : 0;
    w.gmask = (unsigned long long*)(base + off);
    off += align256(G * nwaves * 8);
    w.pmask = (unsigned long long*)(base + off);
    off += align256(G * nwaves * 8);
    w.cin01 = (unsigned char*)(base + off);
    off += align256(G * nwaves);
    w.seg_gp = (unsigned char*)(base + off);
    off += align256(G * nseg);
    w.seg_cin = (unsigned char*)(base + off);
    off += align256(G * nseg);
    w.tab = tab_bytes ? (uint32_t*)(base + off) : nullptr;
    off += align256(tab_bytes);
    w.ks = nullptr;
    w.bytes = off;
    return w;
}

// Bytes of the Kronecker-Schoenhage region of G products of call's plan: the packed factors
// (2M G integers of wks limbs each, twice), their products (2 wks limbs), the descriptors, and
// the integer products' own workspace (groups of at most 65535, one after another), with room
// for their table and, recursively, their own Step 6.
size_t ks_bytes(const Call& c, size_t G);

// layout() for a product run under call, with the Kronecker-Schoenhage region appended
Workspace layout_call(const Call& call, size_t G, size_t nw_max, bool need_b, char* base, size_t tab_bytes = 0) {
    Workspace w = layout(call.P, G, nw_max, need_b, base, tab_bytes);
    if (call.ks_inner) {
        w.ks = base ? base + w.bytes : nullptr;
        w.bytes += ks_bytes(call, G);
    }
    return w;
}

size_t ks_bytes(const Call& c, size_t G) {
    if (!c.ks_inner) return 0;
    const Call& in = *c.ks_inner;
    const size_t cnt = ((size_t)2 << c.P.log2_M) * G;
    const size_t wks = (size_t)c.ks_wks;
    size_t b = 2 * align256(cnt * wks * 4) + align256(cnt * 2 * wks * 4) + align256(cnt * sizeof(ProdDesc));
    if (!in.schoolbook) {
        const size_t Gi = std::min<size_t>(cnt, 65535);
        b += layout_call(in, Gi, 2 * wks, true, nullptr, in.C->table_bytes()).bytes;
    }
    return b;
}

template <int C>
struct Transform {
    static constexpr int L = fmt_L(C);
    // Forward (inverse = 0) or inverse (inverse = 1) transform of G polynomials in place.
    // fused (forward): the bottom level also multiplies componentwise by bpoly (poly itself if
    // squaring, (2M)^-1 included) and runs the bottom inverse level, so the inverse transform
    // that follows starts one level up (fused = 1 there too).
    // enc (forward): the top level encodes operand `which` of the products in *enc itself (Step 4
    // fused in; in_words: operand limbs read, for the byte count).
    static int run(const Call& c, uint32_t* poly, size_t stride, unsigned G, int inverse, hipStream_t s,
                   int fused = 0, const uint32_t* bpoly = nullptr, int squaring = 0,
                   const ProdArgs* enc = nullptr, int which = 0, double in_words = 0.0) {
        const Plan& P = c.P;
        const long long twoM = 2LL << P.log2_M;
        if (twoM > (1LL << 31)) return DKSS_ERANGE;     // the kernels index positions in 32 bits
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
        // one launch per level: the DFT with the following (forward) or preceding (inverse)
        // twiddle products fused in
        auto level = [&](int k, bool tw) -> int {
            const int log2r = P.radix_log2[k];
            const int r = 1 << log2r;
            const long long ncols = twoM >> log2r;
            constexpr int D = Dig<C>::D;
            const bool pw = fused && !inverse && k == nl - 1;     // fused componentwise products
            // columns per workgroup: two LDS halves of C columns (limbs; digits too where the
            // products run) within the budget, at most ncols; one column on twiddle levels
            const size_t colbytes = (size_t)r * (pw ? elem_words(m, D) : m * Dig<C>::LS) * 4;
            int log2C = 0;
            while (!tw && (2 * colbytes << (log2C + 1)) <= (size_t)c.dft_lds &&
                   (1LL << (log2C + 1)) <= ncols)
                ++log2C;
            LevelArgs A{};
            A.twoM = twoM;
            A.base = base[k];
            A.mu_top = c.C->table_count;
            while ((1LL << A.log2mut) < A.mu_top) ++A.log2mut;
            A.log2r = log2r;
            A.log2m = P.log2_m;
            A.log2C = log2C;
            while ((1LL << A.log2nl) < n_lvl[k]) ++A.log2nl;
            while ((1LL << A.log2mu) < mu[k]) ++A.log2mu;
            A.mode = pw ? 3 : tw ? (inverse ? 2 : 1) : 0;
            A.inverse = inverse;
            // two halves: each holds the columns in limbs (DFT) and, where products run, the
            // columns in digits and the staging of 256/m operands of 2m residues
            A.ew = elem_words(m, D);
            A.sw = stage_words(m, Dig<C>::DS);
            const size_t ncl = ((size_t)r << log2C) * m * Dig<C>::LS;
            const size_t ncd = ((size_t)r << log2C) * A.ew;
            const size_t rb_words = (size_t)(kThreads / m) * A.sw;
            size_t half = ncl;
            if (tw || pw) half = std::max(half, std::max(ncd, rb_words));
            half = (half + 3) & ~(size_t)3;                       // 16-byte aligned halves
            A.half = (int)half;
            const size_t lds = 2 * half * 4;
            if (!grid_ok((size_t)(ncols >> log2C))) return DKSS_ERANGE;
            const unsigned blocks = (unsigned)(ncols >> log2C);
            const double nprod = tw ? (double)(twoM / n_lvl[k]) * (r - 1) * (mu[k] - 1) : 0.0;
            const uint32_t* tab = c.table;
            const bool ec = enc && !inverse && k == 0;         // encode fused into the top level
            const ProdArgs PA = ec ? *enc : ProdArgs{};
            const long long M = twoM / 2;
            const double Sb = (double)G * twoM * m * L * 4;   // one polynomial set, limb form
            const double in_b = ec ? Sb + 4.0 * in_words : 2.0 * Sb;   // bytes: read + write
            const uint32_t* bp = pw ? bpoly : nullptr;
            const int sq = pw ? squaring : 0;
#define DKSS_LEVEL_AT(MD, EC, FM, FR)                                                                \
    hipLaunchKernelGGL((k_level<C, MD, EC, FM, FR>), dim3(blocks, G), dim3(kThreads), lds, s, poly,     \
                       (long long)stride, tab, A, Q, bp, sq, PA, which, M)
#define DKSS_LEVEL(MD, EC)                                                                          \
    do {                                                                                            \
        if (A.log2m == 4 && A.log2r == 5) DKSS_LEVEL_AT(MD, EC, 4, 5);                              \
        else if (A.log2m == 5 && A.log2r == 5) DKSS_LEVEL_AT(MD, EC, 5, 5);                         \
        else if (A.log2m == 5 && A.log2r == 6) DKSS_LEVEL_AT(MD, EC, 5, 6);                         \
        else if (A.log2m == 4) DKSS_LEVEL_AT(MD, EC, 4, 0);                                         \
        else if (A.log2m == 5) DKSS_LEVEL_AT(MD, EC, 5, 0);                                         \
        else DKSS_LEVEL_AT(MD, EC, 0, 0);                                                           \
    } while (0)
            if (pw) {
                // algorithmic work: a and b read, the product written; 2M products in R and
                // 2M m scalar products for the (2M)^-1
                ProfScope ps(c.prof, DKSS_K_POINTWISE, s, ec ? Sb + 4.0 * in_words + Sb : 3.0 * Sb,
                             (double)G * twoM * ((double)m * m * L * L + (double)m * L * L));
                if (ec) DKSS_LEVEL(3, true);
                else DKSS_LEVEL(3, false);
                return launch_status();
            }
            ProfScope ps(c.prof, tw ? (inverse ? DKSS_K_TWIDDLE_INV : DKSS_K_TWIDDLE) : DKSS_K_DFT, s, in_b,
                         (double)G * nprod * (double)m * m * L * L);
            if (A.mode == 0) {
                if (ec) DKSS_LEVEL(0, true);
                else DKSS_LEVEL(0, false);
            } else if (A.mode == 1) {
                if (ec) DKSS_LEVEL(1, true);
                else DKSS_LEVEL(1, false);
            } else {
                DKSS_LEVEL(2, false);
            }
#undef DKSS_LEVEL
#undef DKSS_LEVEL_AT
            return launch_status();
        };
        int rc;
        if (!inverse) {
            for (int k = 0; k < nl; ++k)
                if ((rc = level(k, k + 1 < nl))) return rc;
        } else {
            for (int k = nl - 1 - (fused ? 1 : 0); k >= 0; --k)
                if ((rc = level(k, k + 1 < nl))) return rc;
        }
        return DKSS_OK;
    }
};

template <int C>
struct Encode {
    static constexpr int L = fmt_L(C);
    // operand a (which = 0) or b (which = 1) of each product into poly + y * stride
    static int run(const Call& c, const ProdArgs& PA, unsigned G, int which, uint32_t* poly, size_t stride,
                   double in_words, hipStream_t s) {
        const long long M = 1LL << c.P.log2_M;
        const long long total = (2 * M) << c.P.log2_m;
        if (!grid_ok((size_t)((total + kThreads - 1) / kThreads))) return DKSS_ERANGE;
        const unsigned blocks = (unsigned)((total + kThreads - 1) / kThreads);
        ProfScope ps(c.prof, DKSS_K_ENCODE, s, 4.0 * in_words + 4.0 * G * total * L, 0.0);
        hipLaunchKernelGGL(k_encode<C>, dim3(blocks, G), dim3(kThreads), 0, s, PA, which, poly,
                           (long long)stride, M, c.P.log2_m);
        return launch_status();
    }
};

template <int C>
struct Pointwise {
    static constexpr int L = fmt_L(C);
    static int run(const Call& c, uint32_t* A, const uint32_t* B, size_t stride, unsigned G, hipStream_t s) {
        const long long count = 2LL << c.P.log2_M;
        const int per = kThreads / c.P.m();
        if (!grid_ok((size_t)((count + per - 1) / per))) return DKSS_ERANGE;
        const unsigned blocks = (unsigned)((count + per - 1) / per);
        const int m = c.P.m();
        ProfScope ps(c.prof, DKSS_K_POINTWISE, s, 3.0 * G * count * m * L * 4,
                     (double)G * count * ((double)m * m * L * L + (double)m * L * L));
        hipLaunchKernelGGL(k_pointwise<C>, dim3(blocks, G), dim3(kThreads), rprod_lds(C), s, A, B,
                           (long long)stride, count, c.P.log2_m, c.C->Q);
        return launch_status();
    }
};

template <int C>
struct Decode {
    static constexpr int L = fmt_L(C);
    // u_min: the smallest u of the products (it bounds the elements one workgroup reads)
    static int run(const Call& c, const ProdArgs& PA, unsigned G, size_t nw_max, double out_words,
                   const Workspace& w, hipStream_t s, int u_min) {
        const long long nwaves = ((long long)nw_max + 63) / 64;
        if (!grid_ok((size_t)((nw_max + kThreads - 1) / kThreads))) return DKSS_ERANGE;
        const unsigned blocks = (unsigned)((nw_max + kThreads - 1) / kThreads);
        const double S = (double)G * (2LL << c.P.log2_M) * c.P.m() * L * 4;
        const long long nseg = (nwaves + kThreads - 1) / kThreads;
        {
            ProfScope ps(c.prof, DKSS_K_DECODE, s, S + 4.0 * out_words, 0.0);
            // positions per workgroup: the values reaching 257 words start within
            // 32*257 + 32L + 1 bits, (32*257 + 32L + 1)/u + 2 positions of pos_words() words each
            const long long gspan = (32LL * (kThreads + 1) + 32 * L + 1) / std::max(u_min, 1) + 2;
            const long long tile_words = gspan * pos_words<C>();
            if (u_min >= 1 && tile_words * 4 <= 32768)
                hipLaunchKernelGGL((k_decode<C, true>), dim3(blocks, G), dim3(kThreads), tile_words * 4, s, PA,
                                   (const uint32_t*)w.A, (long long)w.S, 2LL << c.P.log2_M, c.P.log2_m,
                                   w.gmask, w.pmask, (long long)w.wst);
            else
                hipLaunchKernelGGL((k_decode<C, false>), dim3(blocks, G), dim3(kThreads), 0, s, PA,
                                   (const uint32_t*)w.A, (long long)w.S, 2LL << c.P.log2_M, c.P.log2_m,
                                   w.gmask, w.pmask, (long long)w.wst);
        }
        if (int rc_ = launch_status()) return rc_;
        {
            ProfScope ps(c.prof, DKSS_K_CARRY_SCAN, s, 17.0 * G * nwaves, 0.0);
            hipLaunchKernelGGL(k_carry_block, dim3((unsigned)nseg, G), dim3(kThreads), 0, s, PA, w.gmask,
                               w.pmask, w.cin01, w.seg_gp, (long long)w.wst, (long long)w.sst);
            hipLaunchKernelGGL(k_carry_top, dim3(1, G), dim3(1024), 0, s, PA, w.seg_gp, w.seg_cin,
                               (long long)w.sst);
        }
        if (int rc_ = launch_status()) return rc_;
        {
            ProfScope ps(c.prof, DKSS_K_CARRY_APPLY, s, 8.0 * out_words, 0.0);
            const unsigned blocks4 = (unsigned)((nw_max + 4 * kThreads - 1) / (4 * kThreads));
            hipLaunchKernelGGL(k_carry_apply, dim3(blocks4, G), dim3(kThreads), 0, s, PA, w.gmask, w.pmask,
                               w.cin01, w.seg_cin, (long long)w.wst, (long long)w.sst);
        }
        if (int rc_ = launch_status()) return rc_;
        return DKSS_OK;
    }
};

}  // namespace

// Carry resolution of a product whose words and per-wavefront generate/propagate masks were
// written under k_decode's contract (word w = low 32 bits of its sum plus the high part of the
// previous word's, a 1-bit carry left); used by the SMUL decode too.
int dkss::carry_resolve(uint32_t* c, long long nw, unsigned long long* gmask, unsigned long long* pmask,
                        unsigned char* cin01, unsigned char* seg_gp, unsigned char* seg_cin, hipStream_t s) {
    if (nw <= 0) return DKSS_OK;
    const long long nwaves = (nw + 63) / 64;
    const long long nseg = (nwaves + kThreads - 1) / kThreads;
    if (nseg > (1LL << 31)) return DKSS_ERANGE;
    ProdArgs PA{};
    PA.one = ProdDesc{c, nullptr, nullptr, nw, 0, 0, 0};
    hipLaunchKernelGGL(k_carry_block, dim3((unsigned)nseg, 1), dim3(kThreads), 0, s, PA, gmask, pmask, cin01,
                       seg_gp, nwaves, nseg);
    hipLaunchKernelGGL(k_carry_top, dim3(1, 1), dim3(1024), 0, s, PA, seg_gp, seg_cin, nseg);
    const unsigned blocks4 = (unsigned)((nw + 4 * kThreads - 1) / (4 * kThreads));
    hipLaunchKernelGGL(k_carry_apply, dim3(blocks4, 1), dim3(kThreads), 0, s, PA, gmask, pmask, cin01, seg_cin,
                       nwaves, nseg);
    return launch_status();
}

namespace {

template <int C>
struct Unscramble {
    static constexpr int L = fmt_L(C);
    static int run(const Call& c, uint32_t* poly, const uint32_t* src, const LevelIdx& LI, hipStream_t s) {
        const long long twoM = 2LL << c.P.log2_M;
        const long long total = twoM << c.P.log2_m;
        ProfScope ps(c.prof, DKSS_K_UNSCRAMBLE, s, (4.0 * L + 4.0 * Dig<C>::D) * total, 0.0);
        hipLaunchKernelGGL(k_unscramble<C>, dim3((unsigned)((total + kThreads - 1) / kThreads)), dim3(kThreads),
                           0, s, poly, src, twoM, c.P.log2_m, LI);
        return launch_status();
    }
};

bool overlaps(const void* x, size_t xb, const void* y, size_t yb) {
    const char* a = (const char*)x;
    const char* b = (const char*)y;
    return a < b + yb && b < a + xb;
}

// batch: the product's batch size, the learned selector's third input.  infer: a planning call
// may run the selector's inference for a shape it has not seen (and cache the choice); products
// (infer false) only look the choice up and otherwise take the policy's fallback, the thesis rule.
int prepare_call(dkss_ctx* ctx, size_t alen, size_t blen, const dkss_params* p, Call* call,
                 uint32_t batch, bool infer) {
    call->prof = &ctx->prof;
    call->dft_lds = ctx->dft_lds;          // a tuned entry may override it in resolve_params
    call->overlap = ctx->overlap;
    call->fuse_pw = ctx->fuse_pw;
    int choice = -1;
    if (!p && ctx->policy == DKSS_POLICY_LEARNED) {
        if (infer) {
            int rc = learned_choices(ctx, 1, &alen, &blen, batch, &choice);
            if (rc) return rc;
        } else {
            choice = learned_lookup(ctx, alen, blen, batch);
        }
    }
    int rc = resolve_params(ctx, alen, blen, p, call, choice, batch);
    if (rc) return rc;
    if (alen == 0 || blen == 0 || call->schoolbook) return DKSS_OK;
    if ((rc = plan_constants(ctx, call))) return rc;
    if (ctx->step6_ks) {
        // the packed integers and their products' plan (the policy's, without a tuple of the
        // caller's: that belongs to the outer product)
        const int m = call->P.m();
        call->ks_slot = 2 * call->P.q_bits + call->P.log2_m;
        call->ks_wks = (int)(((long long)m * call->ks_slot + 31) / 32);
        call->ks_inner = std::make_shared<Call>();
        const size_t cnt = (size_t)2 << call->P.log2_M;
        rc = prepare_call(ctx, (size_t)call->ks_wks, (size_t)call->ks_wks, nullptr, call->ks_inner.get(),
                          (uint32_t)std::min<size_t>(cnt, UINT32_MAX), infer);
        if (rc) return rc;
    }
    return DKSS_OK;
}

int run_group(const Call& call, const ProdArgs& PA, unsigned G, size_t nw_max, double in_a, double in_b,
              double out_w, bool squaring, const Workspace& w, hipStream_t s, int u_min);
int launch_schoolbook(const Call& call, const ProdArgs& PA, unsigned G, size_t nw_max, double ops,
                      hipStream_t s);

template <int C>
struct KsPack {
    static constexpr int L = fmt_L(C);
    static int run(const Call& c, uint32_t* X, const uint32_t* A, size_t stride, unsigned G, hipStream_t s) {
        const long long count = 2LL << c.P.log2_M;
        const long long total = count * c.ks_wks;
        if (!grid_ok((size_t)((total + kThreads - 1) / kThreads))) return DKSS_ERANGE;
        hipLaunchKernelGGL(k_ks_pack<C>, dim3((unsigned)((total + kThreads - 1) / kThreads), G), dim3(kThreads), 0, s,
                           X, A, (long long)stride, count, c.P.log2_m, c.ks_slot, c.ks_wks);
        return launch_status();
    }
};

template <int C>
struct KsUnpack {
    static constexpr int L = fmt_L(C);
    static int run(const Call& c, uint32_t* A, const uint32_t* Z, size_t stride, unsigned G, hipStream_t s) {
        const long long count = 2LL << c.P.log2_M;
        const long long total = count << c.P.log2_m;
        if (!grid_ok((size_t)((total + kThreads - 1) / kThreads))) return DKSS_ERANGE;
        hipLaunchKernelGGL(k_ks_unpack<C>, dim3((unsigned)((total + kThreads - 1) / kThreads), G), dim3(kThreads), 0,
                           s, A, (long long)stride, Z, count, c.P.log2_m, c.ks_slot, c.ks_wks, c.C->Q);
        return launch_status();
    }
};

// Step 6 by Kronecker-Schoenhage substitution (Sec. 3.2.6) for G products: pack every element
// of A and B into integers, multiply them pairwise with the library's own multiplication under
// the inner plan (the schoolbook base case or DKSS, whose Step 6 recurses the same way), unpack,
// fold alpha^m = -1 and reduce mod q, scaled by (2M)^-1, into A.  B == nullptr: a squaring.
int ks_pointwise(const Call& c, uint32_t* A, const uint32_t* B, size_t stride, unsigned G, char* ks, hipStream_t s) {
    const Call& in = *c.ks_inner;
    const size_t cnt = ((size_t)2 << c.P.log2_M) * G;
    const size_t wks = (size_t)c.ks_wks;
    uint32_t* X = (uint32_t*)ks;
    uint32_t* Y = (uint32_t*)(ks + align256(cnt * wks * 4));
    uint32_t* Z = (uint32_t*)(ks + 2 * align256(cnt * wks * 4));
    ProdDesc* d = (ProdDesc*)(ks + 2 * align256(cnt * wks * 4) + align256(cnt * 2 * wks * 4));
    char* iws = (char*)d + align256(cnt * sizeof(ProdDesc));
    int rc;
    if ((rc = dispatch_fmt<KsPack>(c.P.fmt, c, X, A, stride, G, s))) return rc;
    if (B && (rc = dispatch_fmt<KsPack>(c.P.fmt, c, Y, B, stride, G, s))) return rc;
    hipLaunchKernelGGL(k_ks_descs, dim3((unsigned)((cnt + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, d, Z, X,
                       B ? (const uint32_t*)Y : (const uint32_t*)X, (long long)cnt, (int)wks, in.P.u);
    if ((rc = launch_status())) return rc;
    Call ic = in;
    ic.prof = c.prof;
    ic.aux = nullptr;
    if (!ic.schoolbook) {
        const size_t Gmax = std::min<size_t>(cnt, 65535);
        Workspace iw = layout_call(ic, Gmax, 2 * wks, true, iws, ic.C->table_bytes());
        ic.table = ic.C->table_ready ? ic.C->d_table : iw.tab;
        if (!ic.C->table_ready && (rc = dispatch_fmt<TableBuild>(ic.P.fmt, ic.C, iw.tab, c.prof, s))) return rc;
        for (size_t g0 = 0; g0 < cnt; g0 += 65535) {
            const unsigned Gi = (unsigned)std::min<size_t>(65535, cnt - g0);
            ProdArgs PA{};
            PA.many = d + g0;
            rc = run_group(ic, PA, Gi, 2 * wks, (double)Gi * wks, (double)Gi * wks, (double)Gi * 2 * wks, !B,
                           iw, s, ic.P.u);
            if (rc) return rc;
        }
    } else {
        if (ic.kara) return DKSS_ERANGE;           // packed integers stay within the schoolbook
        for (size_t g0 = 0; g0 < cnt; g0 += 65535) {
            const unsigned Gi = (unsigned)std::min<size_t>(65535, cnt - g0);
            ProdArgs PA{};
            PA.many = d + g0;
            if ((rc = launch_schoolbook(ic, PA, Gi, 2 * wks, (double)Gi * wks * wks, s))) return rc;
        }
    }
    return dispatch_fmt<KsUnpack>(c.P.fmt, c, A, Z, stride, G, s);
}

// The DKSS pipeline (Steps 4-8) for G products sharing call's plan, described by PA; the
// workspace w holds their polynomials at stride w.S.  With squaring, b is not transformed.
int run_group(const Call& call, const ProdArgs& PA, unsigned G, size_t nw_max, double in_a, double in_b,
              double out_w, bool squaring, const Workspace& w, hipStream_t s, int u_min) {
    const int fmt = call.P.fmt;
    int rc;
    // the transform of b on the auxiliary stream (forked from s, joined back before the products)
    const bool fork = !squaring && call.aux;
    hipStream_t sb = fork ? call.aux : s;
    if (fork) {
        HIP_OK(hipEventRecord(call.ev_fork, s));
        HIP_OK(hipStreamWaitEvent(sb, call.ev_fork, 0));
    }
    // the encoding of each operand runs inside the top level of its transform
    if (!squaring && (rc = dispatch_fmt<Transform>(fmt, call, w.B, w.S, G, 0, sb, 0, nullptr, 0, &PA, 1, in_b)))
        return rc;
    // the componentwise products run inside the bottom level of a's transform (one launch for
    // the last forward level, the products and the first inverse level) unless b is still being
    // transformed on the other stream
    const int fz = (call.fuse_pw && !fork && !call.ks_inner) ? 1 : 0;
    const uint32_t* bp = squaring ? (const uint32_t*)w.A : w.B;
    if ((rc = dispatch_fmt<Transform>(fmt, call, w.A, w.S, G, 0, s, fz, squaring ? nullptr : bp,
                                    squaring ? 1 : 0, &PA, 0, in_a)))
        return rc;
    if (fork) {
        HIP_OK(hipEventRecord(call.ev_join, sb));
        HIP_OK(hipStreamWaitEvent(s, call.ev_join, 0));
    }
    if (call.ks_inner) {
        if ((rc = ks_pointwise(call, w.A, squaring ? nullptr : bp, w.S, G, w.ks, s))) return rc;
    } else if (!fz && (rc = dispatch_fmt<Pointwise>(fmt, call, w.A, bp, w.S, G, s))) {
        return rc;
    }
    if ((rc = dispatch_fmt<Transform>(fmt, call, w.A, w.S, G, 1, s, fz))) return rc;
    return dispatch_fmt<Decode>(fmt, call, PA, G, nw_max, out_w, w, s, u_min);
}

int launch_zero(const ProdArgs& PA, unsigned G, size_t nw_max, hipStream_t s) {
    if (nw_max == 0) return DKSS_OK;
    const unsigned blocks = (unsigned)std::min<size_t>((nw_max + kThreads - 1) / kThreads, 4096);
    hipLaunchKernelGGL(k_zero_products, dim3(blocks, G), dim3(kThreads), 0, s, PA);
    return launch_status();
}

int launch_schoolbook(const Call& call, const ProdArgs& PA, unsigned G, size_t nw_max, double ops,
                      hipStream_t s) {
    ProfScope ps(call.prof, DKSS_K_SCHOOLBOOK, s, 8.0 * G * nw_max, ops);
    const size_t lds = (std::max<size_t>(nw_max + 2, 64) + 3 * nw_max) * sizeof(uint32_t);   // 64 KiB + 8 B at most
    hipLaunchKernelGGL(k_schoolbook, dim3(1, G), dim3(kThreads), lds, s, PA);
    return launch_status();
}

// Workspace of the base case's Karatsuba levels for G products whose longer operand has at most
// n_max limbs: per level, a slot per parent and three sub-product descriptors per parent.
size_t kara_bytes(int depth, size_t G, size_t n_max) {
    size_t bytes = 0, parents = G, n = n_max;
    for (int lv = 0; lv < depth; ++lv) {
        const size_t h = (n + 1) / 2;
        bytes += align256(parents * (size_t)kara_slot_words((long long)h) * 4) + align256(3 * parents * sizeof(ProdDesc));
        parents *= 3;
        n = h + 1;
    }
    return bytes;
}

// The base case of G products: the schoolbook (one workgroup per product), or depth Karatsuba
// levels (k_kara_eval level by level, the schoolbook on the 3^depth G leaves, k_kara_combine back
// up) in ws.
int launch_base(const Call& call, const ProdArgs& PA, unsigned G, size_t nw_max, size_t n_max, double ops,
                char* ws, hipStream_t s) {
    const int depth = call.kara;
    if (depth == 0) return launch_schoolbook(call, PA, G, nw_max, ops, s);
    if (!ws) return DKSS_ENOSPC;
    ProdArgs lvl[kMaxKaraDepth + 1];
    long long stride[kMaxKaraDepth];
    size_t parents = G, n = n_max, off = 0;
    lvl[0] = PA;
    {
        ProfScope ps(call.prof, DKSS_K_SCHOOLBOOK, s, 0.0, 0.0);
        for (int lv = 0; lv < depth; ++lv) {
            const size_t h = (n + 1) / 2;
            stride[lv] = kara_slot_words((long long)h);
            uint32_t* scratch = (uint32_t*)(ws + off);
            off += align256(parents * (size_t)stride[lv] * 4);
            ProdDesc* child = (ProdDesc*)(ws + off);
            off += align256(3 * parents * sizeof(ProdDesc));
            hipLaunchKernelGGL(k_kara_eval, dim3(1, (unsigned)parents), dim3(64), 0, s, lvl[lv], child, scratch,
                               stride[lv]);
            lvl[lv + 1] = ProdArgs{};
            lvl[lv + 1].many = child;
            parents *= 3;
            n = h + 1;
        }
        if (int rc_ = launch_status()) return rc_;
    }
    int rc = launch_schoolbook(call, lvl[depth], (unsigned)parents, 2 * n, ops, s);
    if (rc) return rc;
    ProfScope ps(call.prof, DKSS_K_SCHOOLBOOK, s, 0.0, 0.0);
    for (int lv = depth - 1; lv >= 0; --lv) {
        parents /= 3;
        hipLaunchKernelGGL(k_kara_combine, dim3(1, (unsigned)parents), dim3(64), 0, s, lvl[lv], lvl[lv + 1].many);
    }
    return launch_status();
}

// The table a product reads: the context's copy when a planning call has built it, else a copy
// built on the stream into the workspace's table room (w.tab), part of this call's work.
int use_table(Call* call, const Workspace& w, hipStream_t s) {
    if (call->C->table_ready) {
        call->table = call->C->d_table;
        return DKSS_OK;
    }
    if (!w.tab) return DKSS_ENOSPC;
    call->table = w.tab;
    return dispatch_fmt<TableBuild>(call->P.fmt, call->C, w.tab, call->prof, s);
}

int run_mul(Call call, uint32_t* c, const uint32_t* a, size_t alen, const uint32_t* b, size_t blen,
            void* ws, size_t ws_bytes, hipStream_t s) {
    const size_t nw = alen + blen;
    ProdArgs PA{};
    PA.one = ProdDesc{c, a, b, (long long)alen, (long long)blen, call.P.u, 0};
    PA.many = nullptr;
    if (alen == 0 || blen == 0) return launch_zero(PA, 1, nw, s);
    if (call.schoolbook) {
        if (call.kara) {
            if (ws == nullptr || ((uintptr_t)ws & 255)) return DKSS_EINVAL;
            if (ws_bytes < kara_bytes(call.kara, 1, std::max(alen, blen))) return DKSS_ENOSPC;
        }
        return launch_base(call, PA, 1, nw, std::max(alen, blen), (double)alen * (double)blen, (char*)ws, s);
    }
    const bool squaring = (a == b && alen == blen);
    if (ws == nullptr || ((uintptr_t)ws & 255)) return DKSS_EINVAL;
    Workspace w = layout_call(call, 1, nw, !squaring, (char*)ws, call.C->table_ready ? 0 : call.C->table_bytes());
    if (ws_bytes < w.bytes) return DKSS_ENOSPC;
    int rc = use_table(&call, w, s);
    if (rc) return rc;
    return run_group(call, PA, 1, nw, (double)alen, (double)blen, (double)nw, squaring, w, s, call.P.u);
}

// A batch, planned: products grouped by plan (zero products, schoolbook products, and one group
// per DKSS parameter tuple and level split), in the order of `order`.
struct BatchPlan {
    struct Grp {
        int kind;                  // 0 zero, 1 base case (schoolbook, Karatsuba levels), 2 DKSS
        size_t first, count;       // range in order
        size_t nw_max;
        size_t n_max = 0;          // the longest operand
        int u_min = 0;             // smallest u of the group's products
        double in_a, in_b, out_w, ops;
        Call call;
    };
    std::vector<Grp> groups;
    std::vector<size_t> order;
    std::vector<Call> calls;
    // the distinct tuples of the DKSS groups, each with room for its table after the
    // descriptors (used when the context has not built that table)
    std::vector<std::pair<Cached*, size_t>> tabs;
    size_t desc_bytes = 0, tab_bytes = 0, ws_bytes = 0;
    // groups spread over lanes (streams), each lane with its own workspace slice
    int lanes = 1;
    std::vector<int> lane_of;          // per group
    std::vector<size_t> lane_off;      // per lane: its slice's offset after descriptors and tables
};

constexpr size_t kMaxGroup = 65535;     // gridDim.y

// infer: as in prepare_call (planning calls run one inference for every new shape)
int plan_batch(dkss_ctx* ctx, size_t count, const size_t* alen, const size_t* blen,
               const dkss_params* p, BatchPlan* B, bool infer) {
    const int lanes = std::max(1, std::min(ctx->batch_lanes, kMaxLanes));
    B->calls.assign(count, Call());
    std::map<std::string, std::vector<size_t>> by_key;
    const uint32_t batch = (uint32_t)std::min<size_t>(count, UINT32_MAX);
    if (infer && !p && ctx->policy == DKSS_POLICY_LEARNED) {
        std::vector<int> ch(count);
        int rc = learned_choices(ctx, count, alen, blen, batch, ch.data());
        if (rc) return rc;
    }
    for (size_t i = 0; i < count; ++i) {
        int rc = prepare_call(ctx, alen[i], blen[i], p ? p + i : nullptr, &B->calls[i], batch, false);
        if (rc) return rc;
        const Call& c = B->calls[i];
        std::string key;
        if (alen[i] == 0 || blen[i] == 0) {
            key = "0";
        } else if (c.schoolbook) {
            key = "1" + std::to_string(c.kara);
        } else {
            key = "2" + c.P.key() + "_r";
            for (int r : c.P.radix_log2) key += std::to_string(r) + ".";
        }
        by_key[key].push_back(i);
    }
    B->desc_bytes = align256(count * sizeof(ProdDesc));
    std::vector<size_t> gws;           // workspace bytes of each group
    for (auto& kv : by_key) {
        const std::vector<size_t>& idx = kv.second;
        // a Karatsuba group's leaves (3^depth per product) share one launch's grid
        size_t cap = kMaxGroup;
        if (kv.first[0] == '1')
            for (int d = 0; d < B->calls[idx[0]].kara; ++d) cap /= 3;
        for (size_t off = 0; off < idx.size(); off += cap) {
            BatchPlan::Grp g{};
            g.kind = kv.first[0] - '0';
            g.first = B->order.size();
            g.count = std::min(cap, idx.size() - off);
            g.call = B->calls[idx[off]];
            for (size_t k = off; k < off + g.count; ++k) {
                const size_t i = idx[k];
                B->order.push_back(i);
                g.nw_max = std::max(g.nw_max, alen[i] + blen[i]);
                g.n_max = std::max(g.n_max, std::max(alen[i], blen[i]));
                const int ui = B->calls[i].P.u;
                g.u_min = g.u_min ? std::min(g.u_min, ui) : ui;
                g.in_a += (double)alen[i];
                g.in_b += (double)blen[i];
                g.out_w += (double)(alen[i] + blen[i]);
                g.ops += (double)alen[i] * (double)blen[i];
            }
            gws.push_back(g.kind == 1 ? kara_bytes(g.call.kara, g.count, g.n_max) : 0);
            if (g.kind == 2) {
                gws.back() = layout_call(g.call, g.count, g.nw_max, true, nullptr).bytes;
                bool seen = false;
                for (const auto& t : B->tabs) seen = seen || t.first == g.call.C;
                if (!seen) {
                    B->tabs.emplace_back(g.call.C, B->tab_bytes);
                    B->tab_bytes += align256(g.call.C->table_bytes());
                }
            }
            B->groups.push_back(g);
        }
    }
    // groups to lanes, largest modelled work first, each to the lane with the least so far
    // (work ~ the group's operand words times its transform length's log, schoolbook ~ words^2)
    const size_t ng = B->groups.size();
    B->lanes = (int)std::min<size_t>((size_t)lanes, std::max<size_t>(ng, 1));
    std::vector<double> work(ng);
    for (size_t i = 0; i < ng; ++i) {
        const BatchPlan::Grp& g = B->groups[i];
        work[i] = g.kind == 2 ? (double)gws[i] * (double)(g.call.P.log2_M + 1)
                              : g.kind == 1 ? g.ops : g.out_w;
    }
    std::vector<size_t> by_work(ng);
    for (size_t i = 0; i < ng; ++i) by_work[i] = i;
    std::stable_sort(by_work.begin(), by_work.end(), [&](size_t x, size_t y) { return work[x] > work[y]; });
    std::vector<double> load(B->lanes, 0.0);
    std::vector<size_t> lane_ws(B->lanes, 0);
    B->lane_of.assign(ng, 0);
    for (size_t i : by_work) {
        const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        B->lane_of[i] = l;
        load[l] += work[i];
        lane_ws[l] = std::max(lane_ws[l], gws[i]);
    }
    B->lane_off.assign(B->lanes, 0);
    size_t off = 0;
    for (int l = 0; l < B->lanes; ++l) {
        B->lane_off[l] = off;
        off += align256(lane_ws[l]);
    }
    B->ws_bytes = B->desc_bytes + B->tab_bytes + off;
    return DKSS_OK;
}

// The batch's descriptors, in group order, to d_desc on stream s.
int put_descs(const BatchPlan& B, size_t count, uint32_t* const* c, const uint32_t* const* a, const size_t* alen,
              const uint32_t* const* b, const size_t* blen, ProdDesc* d_desc, hipStream_t s) {
    for (size_t k0 = 0; k0 < count; k0 += kDescPerPut) {
        DescChunk ch;
        const int n = (int)std::min<size_t>(kDescPerPut, count - k0);
        for (int j = 0; j < n; ++j) {
            const size_t i = B.order[k0 + j];
            ch.d[j] = ProdDesc{c[i], a[i], b[i], (long long)alen[i], (long long)blen[i], B.calls[i].P.u, 0};
        }
        hipLaunchKernelGGL(k_desc_put, dim3(1), dim3(64), 0, s, d_desc, ch, (long long)k0, n);
    }
    return launch_status();
}


}  // namespace

// ---------------------------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------------------------

static int scratch_address(void** out);

extern "C" {

static int ensure_aux(dkss_ctx* ctx) {
    if (ctx->aux) return DKSS_OK;
    // default priority (same as any caller stream), non-blocking with respect to the null stream
    HIP_OK(hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
    HIP_OK(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
    HIP_OK(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
    return DKSS_OK;
}

// The batch lanes' streams and events (planning calls and the option; never a product call).
static int ensure_lanes(dkss_ctx* ctx) {
    const int want = std::max(1, std::min(ctx->batch_lanes, kMaxLanes));
    if (want > 1 && !ctx->lane_ev[0]) HIP_OK(hipEventCreateWithFlags(&ctx->lane_ev[0], hipEventDisableTiming));
    while (ctx->lanes_made < want) {
        const int l = ctx->lanes_made;
        // default priority (same as any caller stream)
        HIP_OK(hipStreamCreateWithFlags(&ctx->lane_s[l - 1], hipStreamNonBlocking));
        HIP_OK(hipEventCreateWithFlags(&ctx->lane_ev[l], hipEventDisableTiming));
        ctx->lanes_made = l + 1;
    }
    return DKSS_OK;
}

int dkss_set_option(dkss_ctx* ctx, int option, long long value) {
    if (!ctx) return DKSS_EINVAL;
    switch (option) {
        case DKSS_OPT_OVERLAP:
            if (value) {
                const int rc = ensure_aux(ctx);      // the second stream, made here and not in a product
                if (rc) return rc;
            }
            ctx->overlap = value != 0;
            return DKSS_OK;
        case DKSS_OPT_FUSE_PW:
            ctx->fuse_pw = value != 0;
            return DKSS_OK;
        case DKSS_OPT_STEP6_KS:
            ctx->step6_ks = value != 0;
            return DKSS_OK;
        case DKSS_OPT_BATCH_LANES:
            if (value < 1 || value > kMaxLanes) return DKSS_EINVAL;
            ctx->batch_lanes = (int)value;
            return ensure_lanes(ctx);
        case DKSS_OPT_DFT_LDS:
            if (value < 16384 || value > 163840) return DKSS_EINVAL;
            ctx->dft_lds = value;
            return DKSS_OK;
        default:
            return DKSS_EINVAL;
    }
}

// The tuning table: text lines "lo hi cand" (log2 N range, candidate index, S or
// DKSS_CAND_SCHOOLBOOK for the base case, T for the thesis rule); '#' comments; a line "@batch B" starts the entries measured at B
// products per batch.
static void load_tuning(dkss_ctx* c, const char* dir) {
    if (!dir) return;
    std::string path = std::string(dir) + "/dkss_tuning.txt";
    FILE* f = fopen(path.c_str(), "r");
    if (!f) return;
    // "lo hi cand [radices|-] [dft_lds]", radices as log2 values joined by '.', e.g. 5.5.5.5
    char line[256];
    uint32_t batch = 1;
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        unsigned long b = 0;
        if (sscanf(line, "@batch %lu", &b) == 1) {
            batch = (uint32_t)std::min<unsigned long>(std::max<unsigned long>(b, 1), UINT32_MAX);
            continue;
        }
        TuneEntry e{};
        e.batch = batch;
        char rad[64] = "-", cs[16] = "";
        long long lds = 0;
        const int n = sscanf(line, "%lf %lf %15s %63s %lld", &e.lo, &e.hi, cs, rad, &lds);
        if (n < 3) continue;
        if (strcmp(cs, "T") == 0) {
            e.cand = kCandThesis;
        } else {
            char* end = nullptr;
            const long v = strtol(cs, &end, 10);
            if (strcmp(cs, "S") == 0) {
                e.cand = DKSS_CAND_SCHOOLBOOK;
            } else {
                if (end == cs || *end || v < 0 || (v >= kNumCandidates && v != DKSS_CAND_SCHOOLBOOK)) continue;
                e.cand = (int)v;
            }
        }
        if (n >= 4 && rad[0] != '-' && rad[0] != '#') {
            bool ok = true;
            for (char* t = rad; *t && ok;) {
                char* end = nullptr;
                const long r = strtol(t, &end, 10);
                ok = end != t && r >= 1 && r <= 7 && e.radices.size() < 8;
                if (ok) e.radices.push_back((int)r);
                t = (end && *end == '.') ? end + 1 : end;
                if (end && *end && *end != '.') ok = false;
            }
            if (!ok) e.radices.clear();
        }
        if (n >= 5 && lds >= 16384 && lds <= 163840) e.dft_lds = lds;
        c->tuning.push_back(e);
    }
    fclose(f);
}

int dkss_ctx_create(dkss_ctx** out, int policy, const char* cache_dir) {
    if (!out || (policy != DKSS_POLICY_THESIS && policy != DKSS_POLICY_TUNED && policy != DKSS_POLICY_LEARNED))
        return DKSS_EINVAL;
    dkss_ctx* c = new (std::nothrow) dkss_ctx();
    if (!c) return DKSS_EINVAL;
    c->policy = policy;
    load_tuning(c, cache_dir);
    {
        // set-up of the allocation-free entry point for the current device; without a device
        // (or on failure) its first call does it
        int ndev = 0;
        void* ptr = nullptr;
        if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) (void)scratch_address(&ptr);
        clear_stale_hip_error();
    }
    if (cache_dir && policy == DKSS_POLICY_LEARNED) {
        std::vector<float> w(DKSS_MLP_NPARAM);
        if (dkss_mlp_load((std::string(cache_dir) + "/dkss_mlp.txt").c_str(), w.data()) == DKSS_OK)
            c->mlp = std::move(w);
    }
    *out = c;
    return DKSS_OK;
}

int dkss_set_mlp(dkss_ctx* ctx, const float* params) {
    if (!ctx) return DKSS_EINVAL;
    if (params) {
        for (int i = 0; i < DKSS_MLP_NPARAM; ++i)
            if (!std::isfinite(params[i])) return DKSS_EINVAL;
        ctx->mlp.assign(params, params + DKSS_MLP_NPARAM);
    } else {
        ctx->mlp.clear();
    }
    ctx->d_mlp_stale = true;
    ctx->choices.clear();
    return DKSS_OK;
}

int dkss_mlp_load(const char* path, float* params) {
    if (!path || !params) return DKSS_EINVAL;
    FILE* f = fopen(path, "r");
    if (!f) return DKSS_EINVAL;
    char line[256];
    int in = 0, hid = 0, outn = 0, got = 0;
    bool header = false;
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        if (!header) {
            header = sscanf(line, "%d %d %d", &in, &hid, &outn) == 3;
            if (!header || in != DKSS_MLP_IN || hid != DKSS_MLP_HID || outn != DKSS_MLP_OUT) break;
            continue;
        }
        float v;
        if (got >= DKSS_MLP_NPARAM || sscanf(line, "%f", &v) != 1 || !std::isfinite(v)) {
            got = -1;
            break;
        }
        params[got++] = v;
    }
    fclose(f);
    return header && got == DKSS_MLP_NPARAM ? DKSS_OK : DKSS_EINVAL;
}

int dkss_mlp_features(uint64_t a_bits, uint64_t b_bits, uint32_t batch, float* out) {
    if (!out || batch == 0) return DKSS_EINVAL;
    const double la = 32.0 * (double)std::max<uint64_t>(1, (a_bits + 31) / 32);
    const double lb = 32.0 * (double)std::max<uint64_t>(1, (b_bits + 31) / 32);
    out[0] = (float)((std::log2(std::max(la, lb)) - 21.0) / 9.0);
    out[1] = (float)((std::log2(std::min(la, lb)) - 21.0) / 9.0);
    out[2] = (float)(std::log2((double)batch) / 12.0);
    return DKSS_OK;
}

int dkss_mlp_choose(dkss_ctx* ctx, uint64_t a_bits, uint64_t b_bits, uint32_t batch, int* cand) {
    if (!ctx || !cand || batch == 0) return DKSS_EINVAL;
    const size_t alen = (size_t)((a_bits + 31) / 32), blen = (size_t)((b_bits + 31) / 32);
    if (alen == 0 || blen == 0 || 32ull * std::max(alen, blen) > (1ull << 36)) return DKSS_ERANGE;
    return learned_choices(ctx, 1, &alen, &blen, batch, cand);
}

static_assert(DKSS_NCAND == kNumCandidates, "candidate count");

int dkss_candidates(dkss_ctx* ctx, uint64_t a_bits, uint64_t b_bits, dkss_params* out, int* valid) {
    if (!ctx || !out || !valid) return DKSS_EINVAL;
    const uint64_t N = 32 * ((std::max(a_bits, b_bits) + 31) / 32);
    if (N == 0 || N > (1ull << 36)) return DKSS_ERANGE;
    for (int c = 0; c < DKSS_NCAND; ++c) {
        int lM = 0, lm = 0, u = 0, pb = 0, z = 1;
        memset(&out[c], 0, sizeof out[c]);
        valid[c] = candidate_params(N, c, &lM, &lm, &u, &pb, &z) ? 1 : 0;
        if (!valid[c]) continue;
        out[c].log2_M = (uint32_t)lM;
        out[c].log2_m = (uint32_t)lm;
        out[c].u = (uint32_t)u;
        out[c].p_bits = (uint32_t)pb;
        out[c].z = (uint32_t)z;
        std::vector<int> r = default_radices(lM, lm, tuple_limbs(pb, z));
        if (r.size() > 8) {           // more FFT levels than a plan holds
            valid[c] = 0;
            continue;
        }
        out[c].n_levels = (uint32_t)r.size();
        for (size_t i = 0; i < r.size(); ++i) out[c].radix_log2[i] = (uint32_t)r[i];
    }
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
    if (!ctx || !out) return DKSS_EINVAL;
    const uint64_t N = 32 * ((std::max(a_bits, b_bits) + 31) / 32);
    if (N == 0 || N > (1ull << 36)) return DKSS_ERANGE;
    int choice = -1;
    if (ctx->policy == DKSS_POLICY_LEARNED) {
        const size_t alen = (size_t)((a_bits + 31) / 32), blen = (size_t)((b_bits + 31) / 32);
        int rc = learned_choices(ctx, 1, &alen, &blen, batch ? batch : 1, &choice);
        if (rc) return rc;
    }
    int lM, lm, u, pb, z;
    uint64_t cutoff = kDefaultCutoffBits;
    const TuneEntry* te = nullptr;
    if (choice >= 0 && choice < kNumCandidates && candidate_params(N, choice, &lM, &lm, &u, &pb, &z)) {
        cutoff = 0;
    } else {
        bool school = false;
        if (!policy_tuple(ctx, N, batch ? batch : 1, &lM, &lm, &u, &pb, &z, &te, &school)) return DKSS_ERANGE;
        if (school || choice == DKSS_CAND_SCHOOLBOOK) cutoff = UINT64_MAX;
    }
    memset(out, 0, sizeof *out);
    out->log2_M = (uint32_t)lM;
    out->log2_m = (uint32_t)lm;
    out->u = (uint32_t)u;
    out->p_bits = (uint32_t)pb;
    out->z = (uint32_t)z;
    out->cutoff_bits = cutoff;
    std::vector<int> r = default_radices(lM, lm, tuple_limbs(pb, z));
    if (te && !te->radices.empty()) {
        int sum = 0;
        bool fits = true;
        for (int x : te->radices) {
            sum += x;
            fits = fits && x <= max_radix_log2(lm, tuple_limbs(pb, z));
        }
        if (fits && sum == lM + 1) r = te->radices;
    }
    out->n_levels = (uint32_t)r.size();
    for (size_t i = 0; i < r.size() && i < 8; ++i) out->radix_log2[i] = (uint32_t)r[i];
    return DKSS_OK;
}

int dkss_plan_info(dkss_ctx* ctx, size_t alen, size_t blen, const dkss_params* p, dkss_plan* out) {
    if (!ctx || !out) return DKSS_EINVAL;
    Call call;
    int rc = prepare_call(ctx, alen, blen, p, &call, 1, true);
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
        out->table_bytes = call.C->table_bytes();
        for (int i = 0; i < P.L && i < 16; ++i) out->q[i] = P.q.limb32(i);
        out->digits = (uint32_t)fmt_D(P.fmt);
    }
    return DKSS_OK;
}

int dkss_workspace_bytes(dkss_ctx* ctx, size_t alen, size_t blen, const dkss_params* p, size_t* out) {
    if (!ctx || !out) return DKSS_EINVAL;
    Call call;
    int rc = prepare_call(ctx, alen, blen, p, &call, 1, true);
    if (rc) return rc;
    if (alen == 0 || blen == 0 || call.schoolbook) {
        *out = call.schoolbook ? kara_bytes(call.kara, 1, std::max(alen, blen)) : 0;
        return DKSS_OK;
    }
    // room for the table too: a product whose tuple the context has not prepared builds its
    // table in the workspace
    *out = layout_call(call, 1, alen + blen, true, nullptr, call.C->table_bytes()).bytes;
    return DKSS_OK;
}

// the tables of the integer products of a Kronecker-Schoenhage Step 6, level by level
static int ensure_inner_tables(const Call& c, Prof* prof, hipStream_t s) {
    for (const Call* in = c.ks_inner.get(); in && !in->schoolbook && in->C; in = in->ks_inner.get()) {
        const int rc = ensure_table(in->C, prof, s);
        if (rc) return rc;
    }
    return DKSS_OK;
}

int dkss_prepare(dkss_ctx* ctx, size_t alen, size_t blen, const dkss_params* p, dkss_stream_t s) {
    clear_stale_hip_error();
    if (!ctx) return DKSS_EINVAL;
    Call call;
    int rc = prepare_call(ctx, alen, blen, p, &call, 1, true);
    if (rc) return rc;
    if (!call.C) return DKSS_OK;
    if ((rc = ensure_table(call.C, &ctx->prof, (hipStream_t)s))) return rc;
    return ensure_inner_tables(call, &ctx->prof, (hipStream_t)s);
}

// The product path of dkss_mul on a workspace (also the allocation-free entry point's).
static int mul_on(dkss_ctx* ctx, uint32_t* c, const uint32_t* a, size_t alen, const uint32_t* b, size_t blen,
                  const dkss_params* p, void* ws, size_t ws_bytes, hipStream_t s) {
    if (!ctx || !c || (alen && !a) || (blen && !b)) return DKSS_EINVAL;
    const size_t nw = alen + blen;
    if ((alen && overlaps(c, nw * 4, a, alen * 4)) || (blen && overlaps(c, nw * 4, b, blen * 4)))
        return DKSS_EINVAL;
    Call call;
    int rc = prepare_call(ctx, alen, blen, p, &call, 1, false);
    if (rc) return rc;
    if (call.C && ctx->overlap && ctx->aux) {
        call.aux = ctx->aux;
        call.ev_fork = ctx->ev_fork;
        call.ev_join = ctx->ev_join;
    }
    return run_mul(call, c, a, alen, b, blen, ws, ws_bytes, s);
}

int dkss_mul(dkss_ctx* ctx, uint32_t* c, const uint32_t* a, size_t alen, const uint32_t* b,
             size_t blen, const dkss_params* p, void* ws, size_t ws_bytes, dkss_stream_t s) {
    clear_stale_hip_error();
    return mul_on(ctx, c, a, alen, b, blen, p, ws, ws_bytes, (hipStream_t)s);
}

}  // extern "C"

// ----- allocation-free products: one fixed scratch per device ----------------------------------
// dkss_mul_noalloc places the workspace of dkss_mul's kernels in this array instead of a caller
// buffer.  Every device the library runs on holds its own copy, at its own address, until the
// process ends.  In host code the name `scratch` is only a host-side stand-in: kernels receive
// the device address that hipGetSymbolAddress returns for the current device.
__device__ __align__(256) unsigned char scratch[DKSS_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices];     // device address of `scratch` per device, or null
}  // namespace

// The current device's scratch address, looked up once per device with that device current.
static int scratch_address(void** out) {
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return DKSS_ERANGE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* ptr = nullptr;
        HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr || ((uintptr_t)ptr & 255)) return DKSS_EHIP;
        g_scratch_addr[dev] = ptr;
    }
    *out = g_scratch_addr[dev];
    return DKSS_OK;
}

extern "C" {

int dkss_mul_noalloc(dkss_ctx* ctx, uint32_t* c, const uint32_t* a, size_t alen, const uint32_t* b,
                     size_t blen, const dkss_params* p, dkss_stream_t s) {
    clear_stale_hip_error();
    if (!ctx) return DKSS_EINVAL;
    void* ws = nullptr;
    int rc = scratch_address(&ws);
    if (rc) return rc;
    rc = mul_on(ctx, c, a, alen, b, blen, p, ws, DKSS_NOALLOC_SCRATCH_BYTES, (hipStream_t)s);
    return rc == DKSS_ENOSPC ? DKSS_ETOOBIG : rc;
}

int dkss_batch_workspace_bytes(dkss_ctx* ctx, size_t count, const size_t* alen, const size_t* blen,
                               const dkss_params* p, size_t* out) {
    if (!ctx || !out || (count && (!alen || !blen))) return DKSS_EINVAL;
    BatchPlan B;
    int rc = plan_batch(ctx, count, alen, blen, p, &B, true);
    if (rc) return rc;
    *out = count ? B.ws_bytes : 0;
    return ensure_lanes(ctx);
}

int dkss_batch_prepare(dkss_ctx* ctx, size_t count, const size_t* alen, const size_t* blen,
                       const dkss_params* p, dkss_stream_t s) {
    clear_stale_hip_error();
    if (!ctx || (count && (!alen || !blen))) return DKSS_EINVAL;
    BatchPlan B;
    int rc = plan_batch(ctx, count, alen, blen, p, &B, true);
    if (rc) return rc;
    if ((rc = ensure_lanes(ctx))) return rc;
    for (const auto& t : B.tabs)
        if ((rc = ensure_table(t.first, &ctx->prof, (hipStream_t)s))) return rc;
    for (const auto& g : B.groups)
        if (g.kind == 2 && (rc = ensure_inner_tables(g.call, &ctx->prof, (hipStream_t)s))) return rc;
    return DKSS_OK;
}

static int check_batch_args(size_t count, uint32_t* const* c, const uint32_t* const* a, const size_t* alen,
                            const uint32_t* const* b, const size_t* blen) {
    if (count && (!c || !a || !alen || !b || !blen)) return DKSS_EINVAL;
    for (size_t i = 0; i < count; ++i) {
        const size_t nw = alen[i] + blen[i];
        if (!c[i] || (alen[i] && !a[i]) || (blen[i] && !b[i])) return DKSS_EINVAL;
        if ((alen[i] && overlaps(c[i], nw * 4, a[i], alen[i] * 4)) ||
            (blen[i] && overlaps(c[i], nw * 4, b[i], blen[i] * 4)))
            return DKSS_EINVAL;
    }
    return DKSS_OK;
}

// The launches of a planned batch whose descriptors sit at the start of ws.  Tuples whose table
// the context has not built get one in the workspace's table room first.  prof: NULL inside a
// graph capture (no timing events there).
static int enqueue_batch(const dkss_ctx* ctx, const BatchPlan& B, void* ws, Prof* prof, hipStream_t st) {
    ProdDesc* d_desc = (ProdDesc*)ws;
    char* tws = (char*)ws + B.desc_bytes;
    char* gws = tws + B.tab_bytes;
    std::map<const Cached*, const uint32_t*> table;
    for (const auto& t : B.tabs) {
        if (t.first->table_ready) {
            table[t.first] = t.first->d_table;
            continue;
        }
        uint32_t* dst = (uint32_t*)(tws + t.second);
        int rc = dispatch_fmt<TableBuild>(t.first->plan.fmt, t.first, dst, prof, st);
        if (rc) return rc;
        table[t.first] = dst;
    }
    // lane 0 is the caller's stream; the others fork from it after the tables and join back at
    // the end (without the context's lane streams every lane runs on the caller's stream)
    const int nl = ctx->lanes_made >= B.lanes ? B.lanes : 1;
    hipStream_t ls[kMaxLanes];
    ls[0] = st;
    for (int l = 1; l < B.lanes; ++l) ls[l] = nl > 1 ? ctx->lane_s[l - 1] : st;
    if (nl > 1) {
        HIP_OK(hipEventRecord(ctx->lane_ev[0], st));
        for (int l = 1; l < nl; ++l) HIP_OK(hipStreamWaitEvent(ls[l], ctx->lane_ev[0], 0));
    }
    int rc_all = DKSS_OK;
    for (size_t gi = 0; gi < B.groups.size() && !rc_all; ++gi) {
        const BatchPlan::Grp& g = B.groups[gi];
        const int lane = B.lane_of[gi];
        hipStream_t gst = ls[lane];
        char* lws = gws + B.lane_off[lane];
        ProdArgs PA{};
        PA.many = d_desc + g.first;
        const unsigned G = (unsigned)g.count;
        Call call = g.call;
        call.prof = prof;
        call.aux = nullptr;                // groups are wide enough to fill the GPU on one stream
        if (g.kind == 2) call.table = table[g.call.C];
        int rc;
        if (g.kind == 0) {
            rc = launch_zero(PA, G, g.nw_max, gst);
        } else if (g.kind == 1) {
            rc = launch_base(call, PA, G, g.nw_max, g.n_max, g.ops, lws, gst);
        } else {
            Workspace w = layout_call(call, G, g.nw_max, true, lws);
            rc = run_group(call, PA, G, g.nw_max, g.in_a, g.in_b, g.out_w, false, w, gst, g.u_min);
        }
        rc_all = rc;
    }
    // the join is enqueued also after an error, so that no lane stream is left forked from a
    // capture
    if (nl > 1) {
        for (int l = 1; l < nl; ++l) {
            const int rc1 = note_hip(hipEventRecord(ctx->lane_ev[l], ls[l]));
            const int rc2 = note_hip(hipStreamWaitEvent(st, ctx->lane_ev[l], 0));
            if (!rc_all) rc_all = rc1 ? rc1 : rc2;
        }
    }
    return rc_all;
}

int dkss_mul_batch(dkss_ctx* ctx, size_t count, uint32_t* const* c, const uint32_t* const* a,
                   const size_t* alen, const uint32_t* const* b, const size_t* blen,
                   const dkss_params* p, void* ws, size_t ws_bytes, dkss_stream_t s) {
    clear_stale_hip_error();
    if (!ctx) return DKSS_EINVAL;
    int rc = check_batch_args(count, c, a, alen, b, blen);
    if (rc) return rc;
    if (count == 0) return DKSS_OK;
    BatchPlan B;
    if ((rc = plan_batch(ctx, count, alen, blen, p, &B, false))) return rc;
    if (ws == nullptr || ((uintptr_t)ws & 255)) return DKSS_EINVAL;
    if (ws_bytes < B.ws_bytes) return DKSS_ENOSPC;
    hipStream_t st = (hipStream_t)s;
    if ((rc = put_descs(B, count, c, a, alen, b, blen, (ProdDesc*)ws, st))) return rc;
    return enqueue_batch(ctx, B, ws, &ctx->prof, st);
}

}  // extern "C"

struct dkss_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    size_t count = 0, launches = 0;
    ~dkss_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

extern "C" {

int dkss_batch_graph_create(dkss_ctx* ctx, size_t count, uint32_t* const* c, const uint32_t* const* a,
                            const size_t* alen, const uint32_t* const* b, const size_t* blen,
                            const dkss_params* p, void* ws, size_t ws_bytes, dkss_graph** out) {
    clear_stale_hip_error();
    if (!ctx || !out) return DKSS_EINVAL;
    *out = nullptr;
    int rc = check_batch_args(count, c, a, alen, b, blen);
    if (rc) return rc;
    if (count == 0) return DKSS_EINVAL;
    BatchPlan B;
    if ((rc = plan_batch(ctx, count, alen, blen, p, &B, true))) return rc;
    if (ws == nullptr || ((uintptr_t)ws & 255)) return DKSS_EINVAL;
    if (ws_bytes < B.ws_bytes) return DKSS_ENOSPC;
    if ((rc = ensure_lanes(ctx))) return rc;
    hipStream_t cs = nullptr;
    HIP_OK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    std::unique_ptr<dkss_graph> G(new (std::nothrow) dkss_graph());
    rc = G ? DKSS_OK : DKSS_EINVAL;
    // tables and descriptors are written once, before the capture; the graph holds the
    // products' kernels only
    for (size_t k = 0; !rc && k < B.tabs.size(); ++k) rc = ensure_table(B.tabs[k].first, nullptr, cs);
    for (size_t k = 0; !rc && k < B.groups.size(); ++k)
        if (B.groups[k].kind == 2) rc = ensure_inner_tables(B.groups[k].call, nullptr, cs);
    if (!rc) rc = put_descs(B, count, c, a, alen, b, blen, (ProdDesc*)ws, cs);
    if (!rc) rc = note_hip(hipStreamSynchronize(cs));
    if (!rc) {
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = DKSS_EHIP;
        } else {
            rc = enqueue_batch(ctx, B, ws, nullptr, cs);
            hipGraph_t graph = nullptr;      // the capture is always ended, also after an error
            const hipError_t e = hipStreamEndCapture(cs, &graph);
            G->graph = graph;
            if (!rc && (e != hipSuccess || !graph)) rc = DKSS_EHIP;
        }
    }
    if (!rc && hipGraphInstantiate(&G->exec, G->graph, nullptr, nullptr, 0) != hipSuccess) rc = DKSS_EHIP;
    if (!rc) {
        size_t nodes = 0;
        if (hipGraphGetNodes(G->graph, nullptr, &nodes) != hipSuccess) rc = DKSS_EHIP;
        G->launches = nodes;
        G->count = count;
    }
    (void)hipStreamDestroy(cs);
    if (rc) return rc;
    *out = G.release();
    return DKSS_OK;
}

int dkss_graph_launch(dkss_graph* g, dkss_stream_t s) {
    clear_stale_hip_error();
    if (!g || !g->exec) return DKSS_EINVAL;
    return hipGraphLaunch(g->exec, (hipStream_t)s) == hipSuccess ? DKSS_OK : DKSS_EHIP;
}

int dkss_graph_info(const dkss_graph* g, size_t* products, size_t* kernels) {
    if (!g || !products || !kernels) return DKSS_EINVAL;
    *products = g->count;
    *kernels = g->launches;
    return DKSS_OK;
}

void dkss_graph_destroy(dkss_graph* g) { delete g; }

int dkss_forward(dkss_ctx* ctx, uint32_t* poly, const uint32_t* a, size_t alen, size_t blen,
                 const dkss_params* p, void* ws, size_t ws_bytes, dkss_stream_t s) {
    clear_stale_hip_error();
    if (!ctx || !poly || !a || alen == 0 || blen == 0) return DKSS_EINVAL;
    Call call;
    int rc = prepare_call(ctx, alen, blen, p, &call, 1, false);
    if (rc) return rc;
    if (call.schoolbook) return DKSS_ERANGE;
    if (ws == nullptr || ((uintptr_t)ws & 255)) return DKSS_EINVAL;
    Workspace w = layout(call.P, 1, alen + blen, true, (char*)ws, call.C->table_ready ? 0 : call.C->table_bytes());
    if (ws_bytes < w.bytes) return DKSS_ENOSPC;
    hipStream_t st = (hipStream_t)s;
    if ((rc = use_table(&call, w, st))) return rc;
    ProdArgs PA{};
    PA.one = ProdDesc{nullptr, a, a, (long long)alen, (long long)blen, call.P.u, 0};
    if ((rc = dispatch_fmt<Encode>(call.P.fmt, call, PA, 1u, 0, w.A, w.S, (double)alen, st))) return rc;
    if ((rc = dispatch_fmt<Transform>(call.P.fmt, call, w.A, w.S, 1u, 0, st))) return rc;
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
    return dispatch_fmt<Unscramble>(call.P.fmt, call, poly, (const uint32_t*)w.A, LI, st);
}

int dkss_residues(const uint32_t* x, size_t n, const uint64_t* primes_host, size_t count,
                  uint64_t* out, dkss_stream_t s) {
    clear_stale_hip_error();
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
        if (launch_status() != DKSS_OK) {
            (void)hipStreamSynchronize(st);
            (void)hipFree(part);
            return DKSS_EHIP;
        }
    }
    const hipError_t e1 = hipStreamSynchronize(st);
    const hipError_t e2 = hipFree(part);
    return note_hip(e1 != hipSuccess ? e1 : e2);
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
                                              "k_schoolbook", "k_table_mul", "k_unscramble",
                                              "k_twiddle_inv"};
    if (kind < 0 || kind >= DKSS_K_KINDS) return nullptr;
    return names[kind];
}

}  // extern "C"

// The VALU rate of the multiply-add the products in R are built from: every thread runs eight
// independent chains of v_mad_u64_u32 (64-bit accumulators, as the column sums use them).
constexpr int kProbeChains = 8;
constexpr int kProbeSteps = 4096;
__global__ __launch_bounds__(kThreads) void k_probe_mad(uint64_t* out, uint32_t seed) {
    uint64_t acc[kProbeChains];
    uint32_t x = seed ^ (uint32_t)(blockIdx.x * kThreads + threadIdx.x);
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) acc[c] = x + c;
    for (int i = 0; i < kProbeSteps; ++i) {
#pragma unroll
        for (int c = 0; c < kProbeChains; ++c) acc[c] = (uint64_t)(uint32_t)acc[c] * (x + (uint32_t)c) + acc[c];
    }
    uint64_t r = 0;
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) r ^= acc[c];
    if (r == 0x5EED5EED5EED5EEDull) out[0] = r;          // keeps the chains alive
}

extern "C" {

int dkss_probe_mad_rate(double* mads_per_s, dkss_stream_t st) {
    clear_stale_hip_error();
    if (!mads_per_s) return DKSS_EINVAL;
    hipStream_t s = (hipStream_t)st;
    int dev = 0, cus = 0;
    HIP_OK(hipGetDevice(&dev));
    HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const unsigned blocks = (unsigned)std::max(cus, 1) * 16;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_OK(hipEventCreate(&e0));
    int rc = note_hip(hipEventCreate(&e1));
    float ms = 0.0f;
    if (!rc) {
        hipLaunchKernelGGL(k_probe_mad, dim3(blocks), dim3(kThreads), 0, s, (uint64_t*)nullptr, 1u);   // warm-up
        rc = note_hip(hipEventRecord(e0, s));
        if (!rc) hipLaunchKernelGGL(k_probe_mad, dim3(blocks), dim3(kThreads), 0, s, (uint64_t*)nullptr, 2u);
        if (!rc) rc = launch_status();
        if (!rc) rc = note_hip(hipEventRecord(e1, s));
        if (!rc) rc = note_hip(hipEventSynchronize(e1));
        if (!rc) rc = note_hip(hipEventElapsedTime(&ms, e0, e1));
    }
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc) return rc;
    const double mads = (double)blocks * kThreads * kProbeSteps * kProbeChains;
    *mads_per_s = ms > 0.0f ? mads / (ms * 1e-3) : 0.0;
    return DKSS_OK;
}

int dkss_last_hip_error(void) { return g_last_hip; }

const char* dkss_hip_error_string(int code) { return hipGetErrorString((hipError_t)code); }

const char* dkss_strerror(int code) {
    switch (code) {
        case DKSS_OK: return "ok";
        case DKSS_EINVAL: return "invalid argument";
        case DKSS_ENOSPC: return "workspace too small";
        case DKSS_ERANGE: return "size or parameters unsupported or infeasible";
        case DKSS_EHIP: return "HIP runtime error";
        case DKSS_ENOTIMPL: return "not implemented";
        case DKSS_ETOOBIG: return "product needs more than the allocation-free entry point's fixed scratch";
        default: return "unknown error";
    }
}

}  // extern "C"
