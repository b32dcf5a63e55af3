// libdkss: the bad multiplications of the FFT levels (Sec. 3.2.5 ii: the products of the
// elements by the twiddle factors rho^s alpha^r) in two forms, for an A/B measurement of the
// vector units against the matrix cores of gfx950.
//
// A group is one twiddle t in R = (Z/qZ)[alpha]/(alpha^m + 1), m = 16, and 32 elements x_n with
// powers r_n of alpha: the elements of a transform whose twiddles share one table index s.  Both
// forms give, canonical in [0, q),
//     y_n = t alpha^(r_n) x_n 2^(-28K) mod q   (K: the Montgomery digit steps of the format),
// so they agree bit for bit.
//  - k_tw_valu (form 1): the product of the level kernels.  m lanes per element, one output
//    coefficient each: m D^2 products of 28-bit digits into 64-bit columns and Montgomery's
//    reduction (rprod_coeff), the twiddle staged rotated by alpha^(r_n) for every element.
//  - k_tw_mx (form 2): the 32 products of a group as one dense contraction on the matrix cores.
//    With T the negacyclic extension of t (T_w = t_w, T_(w+m) = q - t_w for w < m), coefficient
//    j of t x_n is the residue of c_j = sum_k x_k T_((j - k) mod 2m), a sum of non-negative terms
//    below m q^2.  Every residue is split into P = 4D digits of 7 bits (each 28-bit digit into
//    four), so that
//        c_j = sum_e 2^(7e) S_n[j][e],   S_n[j][e] = sum_k sum_a X_n[k][a] T7[(j - k) mod 2m][e - a]
//    (T7 zero outside 0 <= e - a < P).  With e = 2E + eps and a = 2A + eta (eps, eta < 2), the
//    32 x 32 block of S over rows (eps, j) and columns n is the sum over A of the matrices
//        Toep(E - A)[(eps, j)][(eta, k)] = T7[(j - k) mod 2m][2(E - A) + eps - eta]
//    times X(A)[(eta, k)][n] = X_n[k][2A + eta]: one v_mfma_i32_32x32x32_i8 per pair (E, A) with
//    0 <= E - A <= P/2, (P/2)(P/2 + 1) per group, against m^2 D^2 digit products per element on
//    the vector units.  Seven-bit digits are non-negative as the instruction's signed bytes, and
//    every S is below m P 127^2 < 2^31.  The S of coefficient j of element n enter the 64-bit
//    columns of the digit form (column e div 4, shifted by 7 (e mod 4)), the same Montgomery
//    reduction gives the residue, and the power of alpha is applied to the reduced coefficients.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>

#include "../../include/dkss.h"
#include "hip_status.hpp"
#include "kernels.hpp"

namespace {

using namespace dkss;

constexpr int kT = 256;          // threads per workgroup: four wavefronts
constexpr int kLog2m = 4;        // the products in R of m = 16 coefficients
constexpr int kM = 1 << kLog2m;
constexpr int kGroup = 32;       // elements per twiddle: the columns of one MFMA tile

typedef int tw_v4i __attribute__((ext_vector_type(4)));
typedef int tw_v16i __attribute__((ext_vector_type(16)));

__device__ __forceinline__ void tw_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ----- form 1: the vector units ------------------------------------------------------------

// One workgroup per group, in two rounds of 16 elements (m lanes each), as the level kernels'
// rounds: the element's digits and its rotated twiddle staged in LDS, one coefficient per lane.
template <int C>
__global__ __launch_bounds__(kT) void k_tw_valu(const uint32_t* __restrict__ t, const uint32_t* __restrict__ x,
                                                const uint32_t* __restrict__ r, uint32_t* __restrict__ y,
                                                QConst Q) {
    constexpr int L = fmt_L(C);
    using G = Dig<C>;
    constexpr int D = G::D;
    constexpr int SW = stage_words(kM, G::DS), EW = elem_words(kM, D);
    constexpr int PER = kT / kM;
    __shared__ uint32_t TS[PER * SW];
    __shared__ uint32_t XS[PER * EW];
    const long long g = blockIdx.x;
    const int e = (int)threadIdx.x >> kLog2m, j = (int)threadIdx.x & (kM - 1);
    uint32_t tl[L], tv[D], nt[D];
    const uint32_t* tp = t + ((size_t)g * kM + j) * L;
#pragma unroll
    for (int w = 0; w < L; ++w) tl[w] = tp[w];
    limbs_to_digits<C>(tl, tv);
    dneg_q<C>(nt, tv, Q);
    uint32_t* TP = TS + e * SW;
    uint32_t* X = XS + e * EW;
    for (int rd = 0; rd < kGroup / PER; ++rd) {
        const size_t n = (size_t)g * kGroup + rd * PER + e;
        const int rot = (int)(r[n] & (2 * kM - 1));
        uint32_t xl[L], xd[D];
        const uint32_t* xp = x + (n * kM + j) * L;
#pragma unroll
        for (int w = 0; w < L; ++w) xl[w] = xp[w];
        limbs_to_digits<C>(xl, xd);
#pragma unroll
        for (int k = 0; k < D; ++k) X[j * D + k] = xd[k];
        uint32_t* t0 = TP + stage_pos(j, rot, kLog2m) * G::DS;
        uint32_t* t1 = TP + stage_pos(j + kM, rot, kLog2m) * G::DS;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            t0[k] = tv[k];
            t1[k] = nt[k];
        }
        tw_wave_sync();
        uint32_t out[L];
        rprod_coeff<C, true, kLog2m>(TP, X, kLog2m, j, Q, out);
        uint32_t* yp = y + (n * kM + j) * L;
#pragma unroll
        for (int w = 0; w < L; ++w) yp[w] = out[w];
        tw_wave_sync();
    }
}

// ----- form 2: the matrix cores ------------------------------------------------------------

template <int C>
struct MxShape {
    static constexpr int D = Dig<C>::D;
    static constexpr int P = 4 * D;                // 7-bit digits per residue
    static constexpr int H = P / 2;                // digit pairs A < H; E - A runs over 0 .. H
    static constexpr int NCOL = 2 * D;             // 64-bit columns of a coefficient's sum
    static constexpr int XS = P + 1;               // 16-byte rows per element in X7 (odd)
    static constexpr int X7_BYTES = kGroup * XS * 16;
    static constexpr int AZ_BYTES = (P + 3) * 16 * 16;
    static constexpr int T7_BYTES = 2 * kM * P;
    static constexpr int CP = kM + 1;              // 64-bit words per element in a column block
    static constexpr int COL_BYTES = NCOL * kGroup * CP * 8;
    static constexpr int OPS_BYTES = X7_BYTES + AZ_BYTES + T7_BYTES;
    static constexpr int LDS = COL_BYTES > OPS_BYTES ? COL_BYTES : OPS_BYTES;
    static_assert(Dig<C>::NC >= NCOL, "the Montgomery columns hold the product's columns");
    static_assert(LDS <= 65536, "static LDS");
};

// The four 7-bit digits of a 28-bit digit, one per byte.
__device__ __forceinline__ uint32_t tw_pack7(uint32_t d) {
    return (d & 127u) | ((d >> 7) & 127u) << 8 | ((d >> 14) & 127u) << 16 | ((d >> 21) & 127u) << 24;
}

// Wavefront WV: the tiles E = 2c and 2c + 1 for the columns c = WV, WV + 4, ... below NCOL
// (which balances the products over the four wavefronts), then their 64-bit columns into COL.
//  X7: element n, digit a: 16 bytes (k = 0 .. 15) at 16 (n XS + a).
//  AZ: row dl = delta + 1 (delta in -1 .. P + 1), 16 runs of 16 bytes; run cr holds
//      T7[(15 - cr - b) mod 2m][delta] at byte b (zero outside 0 <= delta < P), so that lane
//      (eps, j, eta) finds its 16 bytes of Toep(d), k = 0 .. 15, as run 15 - j of row
//      2d + eps - eta + 1.
template <int C, int WV>
__device__ __forceinline__ void mx_wave(const unsigned char* lds, uint64_t* COL) {
    using S = MxShape<C>;
    constexpr int NCW = (S::NCOL - WV + 3) / 4;
    constexpr int NT = 2 * NCW;
    const int l = (int)threadIdx.x & 63;
    const int n = l & 31, eta = l >> 5, eps = (l & 31) >> 4, jr = l & 15;
    const unsigned char* X7 = lds;
    const unsigned char* AZ = lds + S::X7_BYTES;
    tw_v4i bop[S::H];
#pragma unroll
    for (int A = 0; A < S::H; ++A) {
        const uint4 v = *reinterpret_cast<const uint4*>(X7 + (n * S::XS + 2 * A + eta) * 16);
        bop[A][0] = (int)v.x;
        bop[A][1] = (int)v.y;
        bop[A][2] = (int)v.z;
        bop[A][3] = (int)v.w;
    }
    tw_v16i acc[NT];
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[ti][i] = 0;
#pragma unroll
    for (int d = 0; d <= S::H; ++d) {
        bool used = false;
#pragma unroll
        for (int ti = 0; ti < NT; ++ti) {
            const int E = 2 * (WV + 4 * (ti >> 1)) + (ti & 1);
            used = used || (E - d >= 0 && E - d < S::H);
        }
        if (!used) continue;
        const int dl = 2 * d + eps - eta + 1;
        const uint4 v = *reinterpret_cast<const uint4*>(AZ + (dl * 16 + 15 - jr) * 16);
        tw_v4i aop;
        aop[0] = (int)v.x;
        aop[1] = (int)v.y;
        aop[2] = (int)v.z;
        aop[3] = (int)v.w;
#pragma unroll
        for (int ti = 0; ti < NT; ++ti) {
            const int E = 2 * (WV + 4 * (ti >> 1)) + (ti & 1);
            const int A = E - d;
            if (A >= 0 && A < S::H) acc[ti] = __builtin_amdgcn_mfma_i32_32x32x32_i8(aop, bop[A], acc[ti], 0, 0, 0);
        }
    }
    __syncthreads();                     // every wavefront has its operands: COL takes the region
    // acc[ti][i]: row 8 (i div 4) + 4 eta + (i mod 4) = 16 eps + j of the tile, column n
#pragma unroll
    for (int cc = 0; cc < NCW; ++cc) {
        const int c = WV + 4 * cc;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int j = 8 * (i >> 2) + 4 * eta + (i & 3);
            const uint64_t v = (uint64_t)(uint32_t)acc[2 * cc][i] +
                               ((uint64_t)(uint32_t)acc[2 * cc][i + 8] << 7) +
                               ((uint64_t)(uint32_t)acc[2 * cc + 1][i] << 14) +
                               ((uint64_t)(uint32_t)acc[2 * cc + 1][i + 8] << 21);
            COL[(c * kGroup + n) * S::CP + j] = v;
        }
    }
}

// Persistent: workgroup b takes the groups b, b + gridDim.x, ...; the next group's elements and
// twiddle are loaded into registers while the current group's products run.  The contraction
// forms t x_n; the power of alpha is applied to the reduced coefficients on the way out
// (coefficient j of alpha^r z is z_u for u = (j - r) mod 2m < m, q - z_(u - m) otherwise, 0 for
// a zero coefficient), so the loads do not wait for r.
template <int C>
__global__ __launch_bounds__(kT, 2) void k_tw_mx(const uint32_t* __restrict__ t, const uint32_t* __restrict__ x,
                                              const uint32_t* __restrict__ r, uint32_t* __restrict__ y,
                                              long long groups, QConst Q) {
    constexpr int L = fmt_L(C);
    using S = MxShape<C>;
    constexpr int D = S::D, P = S::P;
    __shared__ __align__(16) unsigned char lds[S::LDS];
    unsigned char* X7 = lds;
    uint32_t* AZ = reinterpret_cast<uint32_t*>(lds + S::X7_BYTES);
    uint32_t* T7 = reinterpret_cast<uint32_t*>(lds + S::X7_BYTES + S::AZ_BYTES);
    uint64_t* COL = reinterpret_cast<uint64_t*>(lds);
    const int tid = (int)threadIdx.x;
    const bool xs = tid < 4 * kGroup;                           // thread (n, kq): 4 coefficients
    const bool ts = !xs && tid < 4 * kGroup + kM;               // thread w: t_w
    // registers of the next group: coefficients 4 kq .. 4 kq + 3 of x_n (4L words, 16-byte
    // aligned), or t_w; the powers of alpha of elements tid / 16 and tid / 16 + 16
    uint32_t nxw[4 * L];
    uint32_t nr[2];
    auto fetch = [&](long long g) {
        if (xs) {
            const uint4* src = reinterpret_cast<const uint4*>(x + ((size_t)g * kGroup * kM + 4 * tid) * L);
#pragma unroll
            for (int k = 0; k < L; ++k) {
                const uint4 v = src[k];
                nxw[4 * k] = v.x;
                nxw[4 * k + 1] = v.y;
                nxw[4 * k + 2] = v.z;
                nxw[4 * k + 3] = v.w;
            }
        } else if (ts) {
            const uint32_t* src = t + ((size_t)g * kM + (tid - 4 * kGroup)) * L;
#pragma unroll
            for (int k = 0; k < L; ++k) nxw[k] = src[k];
        }
        nr[0] = r[(size_t)g * kGroup + (tid >> 4)];
        nr[1] = r[(size_t)g * kGroup + (tid >> 4) + 16];
    };
    long long g = blockIdx.x;
    if (g < groups) fetch(g);
    for (; g < groups; g += gridDim.x) {
        const uint32_t rot[2] = {nr[0] & (2 * kM - 1), nr[1] & (2 * kM - 1)};
        if (xs) {
            const int n = tid >> 2, kq = tid & 3;
            uint32_t dig[4][D];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) limbs_to_digits<C>(nxw + kk * L, dig[kk]);
            uint32_t* dst = reinterpret_cast<uint32_t*>(X7 + n * S::XS * 16) + kq;
#pragma unroll
            for (int a = 0; a < P; ++a) {
                const int sh = 7 * (a & 3);
                uint32_t w = 0;
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) w |= ((dig[kk][a >> 2] >> sh) & 127u) << (8 * kk);
                dst[4 * a] = w;
            }
        } else if (ts) {
            // the twiddle's rows w and w + m of T7: t_w and q - t_w, P bytes each
            const int w = tid - 4 * kGroup;
            uint32_t td[D], nd[D];
            limbs_to_digits<C>(nxw, td);
            dneg_q<C>(nd, td, Q);
#pragma unroll
            for (int k = 0; k < D; ++k) {
                T7[w * D + k] = tw_pack7(td[k]);
                T7[(w + kM) * D + k] = tw_pack7(nd[k]);
            }
        }
        __syncthreads();
        {
            const unsigned char* T7b = reinterpret_cast<const unsigned char*>(T7);
            for (int wi = tid; wi < (P + 3) * 64; wi += kT) {
                const int dl = wi >> 6, cr = (wi >> 2) & 15, bq = wi & 3;
                const int delta = dl - 1;
                uint32_t v = 0;
                if (delta >= 0 && delta < P) {
#pragma unroll
                    for (int bb = 0; bb < 4; ++bb) {
                        const int w = (15 - cr - 4 * bq - bb) & (2 * kM - 1);
                        v |= (uint32_t)T7b[w * P + delta] << (8 * bb);
                    }
                }
                AZ[wi] = v;
            }
        }
        __syncthreads();
        if (g + gridDim.x < groups) fetch(g + gridDim.x);         // in flight during the products
        switch (tid >> 6) {
            case 0: mx_wave<C, 0>(lds, COL); break;
            case 1: mx_wave<C, 1>(lds, COL); break;
            case 2: mx_wave<C, 2>(lds, COL); break;
            default: mx_wave<C, 3>(lds, COL); break;
        }
        __syncthreads();
        // thread (n, j) for n = tid / 16 and tid / 16 + 16: coefficient u mod m of t x_n from its
        // columns by Montgomery, then alpha^r: L limbs out at coefficient j
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int n = (tid >> 4) + 16 * h, j = tid & 15;
            const int u = (j - (int)rot[h]) & (2 * kM - 1);
            const int src = u & (kM - 1);
            uint64_t col[Dig<C>::NC];
#pragma unroll
            for (int c = 0; c < Dig<C>::NC; ++c)
                col[c] = c < S::NCOL ? COL[(c * kGroup + n) * S::CP + src] : 0ull;
            uint32_t out[L];
            redc_cols_limbs<C>(col, Q, out);
            if (u >= kM) {
                uint32_t nz = 0;
#pragma unroll
                for (int w = 0; w < L; ++w) nz |= out[w];
                unsigned int b = 0;
#pragma unroll
                for (int w = 0; w < L; ++w) out[w] = nz ? __builtin_subc(Q.ql[w], out[w], b, &b) : 0u;
            }
            uint32_t* yp = y + (((size_t)g * kGroup + n) * kM + j) * L;
#pragma unroll
            for (int w = 0; w < L; ++w) yp[w] = out[w];
        }
        __syncthreads();                                          // COL is read: X7 takes the region
    }
}

// Constants of the modulus q (L limbs) for format C, as the library's plans hold them.
void tw_qconst(const uint32_t* q, int L, int C, QConst* Q) {
    memset(Q, 0, sizeof *Q);
    const int D = fmt_D(C);
    for (int k = 0; k < D && k < kMaxD + 2; ++k) {
        uint32_t v = 0;
        for (int b = 0; b < 28; ++b) {
            const int bit = 28 * k + b;
            if (bit < 32 * L && ((q[bit >> 5] >> (bit & 31)) & 1u)) v |= 1u << b;
        }
        Q->qd[k] = v;
    }
    for (int k = 0; k < L; ++k) Q->ql[k] = q[k];
    uint32_t inv = q[0];
    for (int i = 0; i < 5; ++i) inv *= 2u - q[0] * inv;     // q^-1 mod 2^32 by Newton's iteration
    Q->qinv28 = (0u - inv) & kMask28;
    if (Q->qd[0] == 1) {
        int e = 1;
        while (e < D && Q->qd[e] == 0) ++e;
        bool sparse = e < D;
        for (int k = e + 2; k < D; ++k) sparse = sparse && Q->qd[k] == 0;
        Q->se = sparse ? e : 0;
    }
}

// compute units of the current device (the persistent grid: two workgroups per CU)
int tw_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 256;
    return cus;
}

template <int C>
int tw_launch(int form, size_t groups, const uint32_t* t, const uint32_t* x, const uint32_t* r, uint32_t* y,
              const QConst& Q, hipStream_t s) {
    if (form == 1)
        hipLaunchKernelGGL(k_tw_valu<C>, dim3((unsigned)groups), dim3(kT), 0, s, t, x, r, y, Q);
    else
        hipLaunchKernelGGL(k_tw_mx<C>, dim3((unsigned)std::min<size_t>(groups, (size_t)tw_cus() * 2)), dim3(kT), 0, s,
                           t, x, r, y, (long long)groups, Q);
    return launch_status();
}

}  // namespace

extern "C" int dkss_probe_twiddle_products(int form, const uint32_t* q, uint32_t L, uint32_t log2_m,
                                           size_t groups, const uint32_t* t, const uint32_t* x,
                                           const uint32_t* r, uint32_t* y, dkss_stream_t st) {
    using namespace dkss;
    clear_stale_hip_error();
    if ((form != 1 && form != 2) || !q) return DKSS_EINVAL;
    if (log2_m != (uint32_t)kLog2m || L < 3 || L > 6) return DKSS_ERANGE;
    if (!(q[0] & 1u) || q[L - 1] == 0) return DKSS_EINVAL;          // odd, exactly L limbs
    if (groups == 0) return DKSS_OK;
    if (!t || !x || !r || !y || ((uintptr_t)x & 15)) return DKSS_EINVAL;
    if (groups > 0x7fffffffu) return DKSS_ERANGE;
    int qbits = 32 * (int)L;
    while (!((q[(qbits - 1) >> 5] >> ((qbits - 1) & 31)) & 1u)) --qbits;
    const int tight = fmt_code((int)L, true);
    const int C = fmt_code((int)L, qbits <= fmt_qbits(tight));
    QConst Q;
    tw_qconst(q, (int)L, C, &Q);
    hipStream_t s = (hipStream_t)st;
    switch (C) {
        case 3: return tw_launch<3>(form, groups, t, x, r, y, Q, s);
        case 4: return tw_launch<4>(form, groups, t, x, r, y, Q, s);
        case 5: return tw_launch<5>(form, groups, t, x, r, y, Q, s);
        case 6: return tw_launch<6>(form, groups, t, x, r, y, Q, s);
        case 19: return tw_launch<19>(form, groups, t, x, r, y, Q, s);
        case 20: return tw_launch<20>(form, groups, t, x, r, y, Q, s);
        case 21: return tw_launch<21>(form, groups, t, x, r, y, Q, s);
        case 22: return tw_launch<22>(form, groups, t, x, r, y, Q, s);
        default: return DKSS_ERANGE;
    }
}
