/*
 * CPU oracle for DKSS multiplication -- test infrastructure, not product code.
 *
 * Plain, slow and obviously correct C for what the GPU path computes, following the thesis
 * (C. Lueders, "Fast Multiplication of Large Integers: Implementation and Analysis of the DKSS
 * Algorithm", arXiv 1503.04955).  Only the test suite, __graft_entry__.smoke() and bench.py's
 * cpu_baseline leg may load this library.  It shares no code with the GPU path.
 *
 * Numbers are little-endian arrays of uint32 limbs (Sec. 2.1).  Inside the ring code a residue
 * mod q = p^z is held in 64-bit words (unsigned __int128 for products); polynomials cross the
 * interface as uint32 limbs, element-major: element i, inner coefficient k, limb w at
 * ((i*m + k)*L32 + w).
 *
 * Contents
 *   or_schoolbook       Sec. 2.3 (OMUL): c = a*b, word products with carries
 *   or_residue          a mod q for a one-word q (product checks by residues)
 *   ring arithmetic     R = (Z/qZ)[alpha]/(alpha^m + 1), Sec. 3.2: add, sub, rotation by a power
 *                       of alpha (Sec. 3.2.5 i), product by its definition (negacyclic convolution)
 *   or_encode           Sec. 3.2.4 (Step 4)
 *   or_fft              Sec. 3.2.5: inner DFTs, bad multiplications, outer DFTs by recursion
 *   or_pointwise        Sec. 3.2.6 (Step 6)
 *   or_decode           Sec. 3.2.8 with Sec. 2.7 (reversed order, 1/2M, evaluation, carries)
 *   or_dkss_mul         Steps 4-8 for given parameters and rho
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#define MAXW 8          /* 64-bit words per residue: q < 2^512 */
#define MAXX (4 * MAXW)   /* longest number reduced mod q, in 64-bit words */
#define MAXM 128        /* largest inner degree bound m */

/* ------------------------------------------------------------------------------------------ */
/* Sec. 2.3 OMUL: schoolbook multiplication                                                   */
/* ------------------------------------------------------------------------------------------ */

/* c[0 .. alen+blen) = a * b.  Row i adds a[i]*b into c at offset i, carrying as it goes. */
void or_schoolbook(uint32_t* c, const uint32_t* a, size_t alen, const uint32_t* b, size_t blen)
{
    memset(c, 0, (alen + blen) * sizeof(uint32_t));
    for (size_t i = 0; i < alen; ++i) {
        uint64_t carry = 0;
        for (size_t j = 0; j < blen; ++j) {
            uint64_t t = (uint64_t)a[i] * b[j] + c[i + j] + carry;
            c[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
        c[i + blen] = (uint32_t)carry;
    }
}

/* a mod q for a one-word modulus (Horner from the most significant limb). */
uint64_t or_residue(const uint32_t* a, size_t n, uint64_t q)
{
    u128 r = 0;
    for (size_t i = n; i-- > 0;)
        r = ((r << 32) | a[i]) % q;
    return (uint64_t)r;
}

/* ------------------------------------------------------------------------------------------ */
/* Residues mod q in W 64-bit words                                                           */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
    int W;                  /* 64-bit words per residue */
    int m;                  /* inner degree bound */
    uint64_t q[MAXW];
} ring_t;

static int cmp_w(const uint64_t* x, const uint64_t* y, int W)
{
    for (int i = W - 1; i >= 0; --i) {
        if (x[i] != y[i])
            return x[i] < y[i] ? -1 : 1;
    }
    return 0;
}

/* r = x + y mod q, inputs in [0, q) */
static void mod_add(uint64_t* r, const uint64_t* x, const uint64_t* y, const ring_t* R)
{
    uint64_t s[MAXW + 1];
    u128 c = 0;
    for (int i = 0; i < R->W; ++i) {
        c += (u128)x[i] + y[i];
        s[i] = (uint64_t)c;
        c >>= 64;
    }
    s[R->W] = (uint64_t)c;
    if (s[R->W] || cmp_w(s, R->q, R->W) >= 0) {
        u128 b = 0;
        for (int i = 0; i < R->W; ++i) {
            u128 t = (u128)s[i] - R->q[i] - b;
            s[i] = (uint64_t)t;
            b = (t >> 64) & 1;
        }
    }
    memcpy(r, s, R->W * sizeof(uint64_t));
}

/* r = x - y mod q, inputs in [0, q) */
static void mod_sub(uint64_t* r, const uint64_t* x, const uint64_t* y, const ring_t* R)
{
    uint64_t s[MAXW];
    u128 b = 0;
    for (int i = 0; i < R->W; ++i) {
        u128 t = (u128)x[i] - y[i] - b;
        s[i] = (uint64_t)t;
        b = (t >> 64) & 1;
    }
    if (b) {
        u128 c = 0;
        for (int i = 0; i < R->W; ++i) {
            c += (u128)s[i] + R->q[i];
            s[i] = (uint64_t)c;
            c >>= 64;
        }
    }
    memcpy(r, s, R->W * sizeof(uint64_t));
}

/* Remainder of the n-word number x by q: long division with base 2^64 digits, one quotient
 * digit at a time from the top, each estimated from the top two words of the running remainder
 * against the normalized top word of q and corrected downward (Knuth, TAOCP Vol. 2, 4.3.1,
 * Algorithm D).  r gets W words. */
static void mod_reduce(uint64_t* r, const uint64_t* x, int n, const ring_t* R)
{
    int W = R->W;
    while (W > 1 && R->q[W - 1] == 0)
        --W;
    /* normalize: shift q and x left so the top word of q has its high bit set */
    int s = __builtin_clzll(R->q[W - 1]);
    uint64_t v[MAXW];
    uint64_t u[MAXX + 1];
    if (n > MAXX)
        abort();
    memset(u, 0, sizeof u);
    for (int i = W - 1; i >= 0; --i)
        v[i] = (R->q[i] << s) | (s && i ? R->q[i - 1] >> (64 - s) : 0);
    u[n] = s ? x[n - 1] >> (64 - s) : 0;
    for (int i = n - 1; i >= 0; --i)
        u[i] = (x[i] << s) | (s && i ? x[i - 1] >> (64 - s) : 0);
    if (n >= W) {
        for (int j = n - W; j >= 0; --j) {
            /* estimate qhat = floor((u[j+W]*B + u[j+W-1]) / v[W-1]), then correct */
            u128 num = ((u128)u[j + W] << 64) | u[j + W - 1];
            u128 qhat = num / v[W - 1];
            u128 rhat = num % v[W - 1];
            while (qhat >> 64 ||
                   (W >= 2 && qhat * v[W - 2] > ((rhat << 64) | u[j + W - 2]))) {
                qhat -= 1;
                rhat += v[W - 1];
                if (rhat >> 64)
                    break;
            }
            /* u[j .. j+W] -= qhat * v */
            u128 borrow = 0, carry = 0;
            for (int i = 0; i < W; ++i) {
                u128 p = qhat * v[i] + carry;
                carry = p >> 64;
                u128 t = (u128)u[i + j] - (uint64_t)p - borrow;
                u[i + j] = (uint64_t)t;
                borrow = (t >> 64) & 1;
            }
            u128 t = (u128)u[j + W] - (uint64_t)carry - borrow;
            u[j + W] = (uint64_t)t;
            if ((t >> 64) & 1) {            /* qhat one too large: add v back */
                u128 c = 0;
                for (int i = 0; i < W; ++i) {
                    c += (u128)u[i + j] + v[i];
                    u[i + j] = (uint64_t)c;
                    c >>= 64;
                }
                u[j + W] += (uint64_t)c;
            }
        }
    }
    /* unnormalize the remainder (low W words of u) */
    memset(r, 0, R->W * sizeof(uint64_t));
    for (int i = 0; i < W; ++i)
        r[i] = (u[i] >> s) | (s ? u[i + 1] << (64 - s) : 0);
}

/* r = x mod q for an n-word number, exported for the tests of this routine */
void or_mod_reduce(uint64_t* r, const uint64_t* x, int n, const uint64_t* q, int W)
{
    ring_t R;
    memset(&R, 0, sizeof R);
    R.W = W;
    memcpy(R.q, q, W * sizeof(uint64_t));
    mod_reduce(r, x, n, &R);
}

/* ------------------------------------------------------------------------------------------ */
/* The ring R = P[alpha]/(alpha^m + 1), P = Z/qZ (Sec. 3.2).  An element is m residues.      */
/* ------------------------------------------------------------------------------------------ */

#define EL(R) ((size_t)(R)->m * (R)->W)       /* 64-bit words per element of R */

static void r_add(uint64_t* r, const uint64_t* x, const uint64_t* y, const ring_t* R)
{
    for (int k = 0; k < R->m; ++k)
        mod_add(r + k * R->W, x + k * R->W, y + k * R->W, R);
}

static void r_sub(uint64_t* r, const uint64_t* x, const uint64_t* y, const ring_t* R)
{
    for (int k = 0; k < R->m; ++k)
        mod_sub(r + k * R->W, x + k * R->W, y + k * R->W, R);
}

/* r = alpha^e * x.  alpha^m = -1, so a coefficient moved past degree m - 1 wraps around to the
 * bottom with its sign changed (Sec. 3.2.5 i); e is taken mod 2m.  r must not alias x. */
static void r_mul_alpha_pow(uint64_t* r, const uint64_t* x, long e, const ring_t* R)
{
    int m = R->m, W = R->W;
    long e2 = ((e % (2 * m)) + 2 * m) % (2 * m);
    uint64_t zero[MAXW] = {0};
    for (int k = 0; k < m; ++k) {
        long t = k + e2;            /* x_k alpha^k alpha^e2 = x_k alpha^t */
        int neg = 0;
        while (t >= m) {
            t -= m;
            neg ^= 1;
        }
        if (neg)
            mod_sub(r + t * W, zero, x + k * W, R);
        else
            memcpy(r + t * W, x + k * W, W * sizeof(uint64_t));
    }
}

/* r = x * y in R by the definition of the product in P[alpha]/(alpha^m + 1):
 * c_j = sum_{i+k=j} x_i y_k - sum_{i+k=j+m} x_i y_k  (mod q).  r may alias x or y. */
static void r_mul(uint64_t* r, const uint64_t* x, const uint64_t* y, const ring_t* R)
{
    int m = R->m, W = R->W;
    int AW = 2 * W + 2;                      /* exact sums of up to m products of W-word numbers */
    uint64_t out[MAXM * MAXW];
    if (m > MAXM)
        abort();
    uint64_t pos[2 * MAXW + 2], neg[2 * MAXW + 2], rp[MAXW], rn[MAXW];
    for (int j = 0; j < m; ++j) {
        memset(pos, 0, sizeof pos);
        memset(neg, 0, sizeof neg);
        for (int i = 0; i < m; ++i) {
            int k = j - i;
            uint64_t* acc = pos;
            if (k < 0) {
                k += m;
                acc = neg;
            }
            const uint64_t* a = x + i * W;
            const uint64_t* b = y + k * W;
            for (int s = 0; s < W; ++s) {
                u128 carry = 0;
                for (int t = 0; t < W; ++t) {
                    u128 p = (u128)a[s] * b[t] + acc[s + t] + carry;
                    acc[s + t] = (uint64_t)p;
                    carry = p >> 64;
                }
                for (int t = s + W; carry && t < AW; ++t) {
                    u128 p = (u128)acc[t] + carry;
                    acc[t] = (uint64_t)p;
                    carry = p >> 64;
                }
            }
        }
        mod_reduce(rp, pos, AW, R);
        mod_reduce(rn, neg, AW, R);
        mod_sub(out + j * W, rp, rn, R);
    }
    memcpy(r, out, EL(R) * sizeof(uint64_t));
}

/* ------------------------------------------------------------------------------------------ */
/* Conversions between uint32-limb polynomials and 64-bit residues                             */
/* ------------------------------------------------------------------------------------------ */

static void load_coeff(uint64_t* r, const uint32_t* src, int L32, int W)
{
    for (int i = 0; i < W; ++i) {
        uint64_t lo = 2 * i < L32 ? src[2 * i] : 0;
        uint64_t hi = 2 * i + 1 < L32 ? src[2 * i + 1] : 0;
        r[i] = lo | (hi << 32);
    }
}

static void store_coeff(uint32_t* dst, const uint64_t* r, int L32)
{
    for (int w = 0; w < L32; ++w)
        dst[w] = (uint32_t)(r[w / 2] >> (32 * (w % 2)));
}

static void init_ring(ring_t* R, const uint32_t* q32, int L32, int m)
{
    memset(R, 0, sizeof *R);
    R->W = (L32 + 1) / 2;
    R->m = m;
    load_coeff(R->q, q32, L32, R->W);
}

static uint64_t* load_poly(const uint32_t* src, size_t count, const ring_t* R, int L32)
{
    uint64_t* p = (uint64_t*)malloc(count * EL(R) * sizeof(uint64_t));
    for (size_t c = 0; c < count * R->m; ++c)
        load_coeff(p + c * R->W, src + c * L32, L32, R->W);
    return p;
}

static void store_poly(uint32_t* dst, const uint64_t* p, size_t count, const ring_t* R, int L32)
{
    for (size_t c = 0; c < count * R->m; ++c)
        store_coeff(dst + c * L32, p + c * R->W, L32);
}

/* exported ring product for the tests: r = x*y in R, elements as uint32 limbs */
void or_ring_mul(uint32_t* r, const uint32_t* x, const uint32_t* y, int m, int L32,
                 const uint32_t* q32)
{
    ring_t R;
    init_ring(&R, q32, L32, m);
    uint64_t* a = load_poly(x, 1, &R, L32);
    uint64_t* b = load_poly(y, 1, &R, L32);
    r_mul(a, a, b, &R);
    store_poly(r, a, 1, &R, L32);
    free(a);
    free(b);
}

/* exported rotation for the tests: r = alpha^e * x */
void or_ring_rotate(uint32_t* r, const uint32_t* x, long e, int m, int L32, const uint32_t* q32)
{
    ring_t R;
    init_ring(&R, q32, L32, m);
    uint64_t* a = load_poly(x, 1, &R, L32);
    uint64_t* b = load_poly(x, 1, &R, L32);
    r_mul_alpha_pow(b, a, e, &R);
    store_poly(r, b, 1, &R, L32);
    free(a);
    free(b);
}

/* ------------------------------------------------------------------------------------------ */
/* Sec. 3.2.4 (Step 4): encode an integer as a polynomial over R                               */
/* ------------------------------------------------------------------------------------------ */

/* bits [pos, pos + len) of the little-endian number a (zero beyond its end), len <= 64 */
static uint64_t get_bits(const uint32_t* a, size_t alen, uint64_t pos, int len)
{
    uint64_t v = 0;
    for (int b = 0; b < len; ++b) {
        uint64_t bit = pos + b;
        uint64_t w = bit / 32;
        if (w < alen && (a[w] >> (bit % 32)) & 1)
            v |= (uint64_t)1 << b;
    }
    return v;
}

/* poly gets 2M elements.  Outer coefficient i < M holds bits [i*u*m/2, (i+1)*u*m/2) of a,
 * split into inner coefficients k < m/2 of u bits each (little-endian bit order); the upper
 * m/2 inner coefficients and the upper M outer coefficients are zero. */
void or_encode(uint32_t* poly, const uint32_t* a, size_t alen, long M, int m, int L32, int u)
{
    memset(poly, 0, (size_t)2 * M * m * L32 * sizeof(uint32_t));
    for (long i = 0; i < M; ++i) {
        for (int k = 0; k < m / 2; ++k) {
            uint64_t base = ((uint64_t)i * (m / 2) + k) * (uint64_t)u;
            uint32_t* dst = poly + ((size_t)i * m + k) * L32;
            for (int b = 0; b < u; b += 32) {
                int len = u - b < 32 ? u - b : 32;
                dst[b / 32] = (uint32_t)get_bits(a, alen, base + b, len);
            }
        }
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Sec. 3.2.5: FFT of length 2M over R with root rho                                           */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
    ring_t R;
    long M2;                 /* FFT length 2M */
    long mu_top;             /* 2M / 2m */
    uint64_t* rho_pow;       /* rho^s, s < mu_top (Sec. 4.2: rho^i = alpha^(i / mu) rho^(i mod mu)) */
} fft_t;

static unsigned bit_rev(unsigned x, int bits)
{
    unsigned r = 0;
    for (int i = 0; i < bits; ++i)
        r |= ((x >> i) & 1u) << (bits - 1 - i);
    return r;
}

/* Length-n DFT of e[0..n) with root alpha^(2m/n) (n a power of two, n <= 2m): the input is put
 * in bit-reversed order, then radix-2 decimation in time, in place (Sec. 2.6).  In the pass
 * that merges halves of length h, butterfly k multiplies the odd part by the (2h)-th root of
 * unity to the k-th power, alpha^((2m/2h) k), a rotation. */
static void inner_dft(uint64_t* e, long n, const ring_t* R)
{
    size_t EW = EL(R);
    int bits = 0;
    while ((1L << bits) < n)
        ++bits;
    uint64_t* tmp = (uint64_t*)malloc(n * EW * sizeof(uint64_t));
    for (long j = 0; j < n; ++j)
        memcpy(tmp + bit_rev((unsigned)j, bits) * EW, e + j * EW, EW * sizeof(uint64_t));
    uint64_t* t = (uint64_t*)malloc(EW * sizeof(uint64_t));
    for (long h = 1; h < n; h *= 2) {
        long step = (2L * R->m) / (2 * h);           /* alpha^step is a primitive 2h-th root */
        for (long g = 0; g < n; g += 2 * h) {
            for (long k = 0; k < h; ++k) {
                uint64_t* x = tmp + (g + k) * EW;
                uint64_t* y = tmp + (g + k + h) * EW;
                r_mul_alpha_pow(t, y, step * k, R);
                r_sub(y, x, t, R);
                r_add(x, x, t, R);
            }
        }
    }
    memcpy(e, tmp, n * EW * sizeof(uint64_t));
    free(t);
    free(tmp);
}

/* rho^e for any e (taken mod 2M): alpha^(e / mu_top) * rho^(e mod mu_top) */
static void rho_power(uint64_t* r, const fft_t* F, long e)
{
    e %= F->M2;
    if (e < 0)
        e += F->M2;
    r_mul_alpha_pow(r, F->rho_pow + (e % F->mu_top) * EL(&F->R), e / F->mu_top, &F->R);
}

/* In place: a[i] <- sum_j a[j] w^(i j) for i < n, w = rho^base, n * base = 2M.
 * n > 2m: write the input as 2m rows of mu = n/2m columns; e_l(y) = sum_j a[j mu + l] y^j;
 * abar_(v,l) = e_l(alpha^v) by inner DFTs; bad multiplications abar_(v,l) *= w^(v l); for each
 * row v an outer DFT of length mu with root w^(2m), by recursion; a[2m f + v] = result_v[f].
 * n <= 2m: an inner DFT with root alpha^(2m/n) directly. */
static void fft_rec(uint64_t* a, long n, long base, const fft_t* F)
{
    const ring_t* R = &F->R;
    long m2 = 2L * R->m;
    size_t EW = EL(R);
    if (n <= m2) {
        inner_dft(a, n, R);
        return;
    }
    long mu = n / m2;
    uint64_t* abar = (uint64_t*)malloc(n * EW * sizeof(uint64_t));
    uint64_t* e = (uint64_t*)malloc(m2 * EW * sizeof(uint64_t));
    uint64_t* tw = (uint64_t*)malloc(EW * sizeof(uint64_t));
    /* (i) inner DFTs */
    for (long l = 0; l < mu; ++l) {
        for (long j = 0; j < m2; ++j)
            memcpy(e + j * EW, a + (j * mu + l) * EW, EW * sizeof(uint64_t));
        inner_dft(e, m2, R);
        for (long v = 0; v < m2; ++v)
            memcpy(abar + (v * mu + l) * EW, e + v * EW, EW * sizeof(uint64_t));
    }
    for (long v = 0; v < m2; ++v) {
        /* (ii) bad multiplications: abar_(v,l) *= w^(v l) = rho^(base v l) */
        for (long l = 1; l < mu; ++l) {
            rho_power(tw, F, base * v * l);
            r_mul(abar + (v * mu + l) * EW, abar + (v * mu + l) * EW, tw, R);
        }
        /* (iii) outer DFT of row v with root w^(2m) */
        fft_rec(abar + v * mu * EW, mu, base * m2, F);
        for (long f = 0; f < mu; ++f)
            memcpy(a + (f * m2 + v) * EW, abar + (v * mu + f) * EW, EW * sizeof(uint64_t));
    }
    free(tw);
    free(e);
    free(abar);
}

static void fft_init(fft_t* F, const uint32_t* rho32, long M2, int m, int L32, const uint32_t* q32)
{
    init_ring(&F->R, q32, L32, m);
    F->M2 = M2;
    F->mu_top = M2 / (2L * m);
    if (F->mu_top < 1)
        F->mu_top = 1;
    size_t EW = EL(&F->R);
    /* rho^0 = 1, rho^s = rho^(s-1) * rho (Sec. 4.2 precomputes the powers below mu) */
    F->rho_pow = (uint64_t*)calloc(F->mu_top * EW, sizeof(uint64_t));
    F->rho_pow[0] = 1;
    uint64_t* rho = load_poly(rho32, 1, &F->R, L32);
    for (long s = 1; s < F->mu_top; ++s)
        r_mul(F->rho_pow + s * EW, F->rho_pow + (s - 1) * EW, rho, &F->R);
    free(rho);
}

/* Forward transform in place: poly[i] <- a(rho^i), i < 2M, natural order.  rho holds the m
 * coefficients of the principal 2M-th root of unity with rho^(2M/2m) = alpha. */
void or_fft(uint32_t* poly, long M2, int m, int L32, const uint32_t* q32, const uint32_t* rho32)
{
    fft_t F;
    fft_init(&F, rho32, M2, m, L32, q32);
    uint64_t* a = load_poly(poly, M2, &F.R, L32);
    fft_rec(a, M2, 1, &F);
    store_poly(poly, a, M2, &F.R, L32);
    free(a);
    free(F.rho_pow);
}

/* Table rho^s, s < count, as uint32-limb elements (for tests of the power trick) */
void or_rho_powers(uint32_t* out, long count, int m, int L32, const uint32_t* q32,
                   const uint32_t* rho32)
{
    fft_t F;
    fft_init(&F, rho32, 2L * m * count, m, L32, q32);
    store_poly(out, F.rho_pow, count, &F.R, L32);
    free(F.rho_pow);
}

/* ------------------------------------------------------------------------------------------ */
/* Sec. 3.2.6 (Step 6): componentwise products                                                 */
/* ------------------------------------------------------------------------------------------ */

void or_pointwise(uint32_t* c, const uint32_t* a, const uint32_t* b, long count, int m, int L32,
                  const uint32_t* q32)
{
    ring_t R;
    init_ring(&R, q32, L32, m);
    uint64_t* x = load_poly(a, count, &R, L32);
    uint64_t* y = load_poly(b, count, &R, L32);
    for (long i = 0; i < count; ++i)
        r_mul(x + i * EL(&R), x + i * EL(&R), y + i * EL(&R), &R);
    store_poly(c, x, count, &R, L32);
    free(x);
    free(y);
}

/* ------------------------------------------------------------------------------------------ */
/* Sec. 3.2.8 (Step 8) with Sec. 2.7: decode and carry                                         */
/* ------------------------------------------------------------------------------------------ */

/* cc = forward transform of the pointwise products.  By Sec. 2.7 the coefficient l of the
 * product polynomial is c_l = (2M)^(-1) cc_((-l) mod 2M); its inner coefficients are exact
 * integers below q.  Evaluate at alpha = 2^u, x = 2^(u m / 2): add c_(l,k) at bit position
 * u (k + l m/2) into out[0 .. outlen).  Returns 0, or -1 if a bit lands beyond outlen. */
int or_decode(uint32_t* out, size_t outlen, const uint32_t* cc, long M2, int m, int L32, int u,
              const uint32_t* q32, const uint32_t* inv2M32)
{
    ring_t R;
    init_ring(&R, q32, L32, m);
    memset(out, 0, outlen * sizeof(uint32_t));
    uint64_t inv[MAXW], x[MAXW], wide[2 * MAXW], c[MAXW];
    load_coeff(inv, inv2M32, L32, R.W);
    int bad = 0;
    for (long l = 0; l < M2; ++l) {
        long src = (M2 - l) % M2;
        for (int k = 0; k < m; ++k) {
            load_coeff(x, cc + ((size_t)src * m + k) * L32, L32, R.W);
            /* c = inv * x mod q */
            memset(wide, 0, sizeof wide);
            for (int s = 0; s < R.W; ++s) {
                u128 carry = 0;
                for (int t = 0; t < R.W; ++t) {
                    u128 p = (u128)inv[s] * x[t] + wide[s + t] + carry;
                    wide[s + t] = (uint64_t)p;
                    carry = p >> 64;
                }
                wide[s + R.W] = (uint64_t)carry;
            }
            mod_reduce(c, wide, 2 * R.W, &R);
            /* add c at bit position u*(k + l*m/2) */
            uint64_t pos = (uint64_t)u * ((uint64_t)k + (uint64_t)l * (m / 2));
            size_t w0 = pos / 32;
            int sh = (int)(pos % 32);
            u128 carry = 0;
            for (size_t w = w0, i = 0;; ++w, ++i) {
                uint64_t piece = 0;           /* bits [32 i - sh, 32 i - sh + 32) of c */
                long lo = 32L * (long)i - sh;
                for (int b = 0; b < 32; ++b) {
                    long bit = lo + b;
                    if (bit >= 0 && bit < 64L * R.W && (c[bit / 64] >> (bit % 64)) & 1)
                        piece |= (uint64_t)1 << b;
                }
                int more = lo + 32 < 64L * R.W;
                if (!piece && !carry && !more)
                    break;
                if (w >= outlen) {
                    if (piece || carry)
                        bad = 1;
                    break;
                }
                carry += (u128)out[w] + piece;
                out[w] = (uint32_t)carry;
                carry >>= 32;
            }
        }
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Steps 4-8 for given parameters                                                              */
/* ------------------------------------------------------------------------------------------ */

/* c[0 .. alen+blen) = a*b by DKSS with FFT length 2M = M2, degree bound m, u bits per inner
 * coefficient, modulus q (L32 limbs), root rho (m coefficients) and inv2M = (2M)^(-1) mod q.
 * Returns 0 or -1 (decoded bits beyond alen+blen limbs: parameters too small). */
int or_dkss_mul(uint32_t* c, const uint32_t* a, size_t alen, const uint32_t* b, size_t blen,
                long M2, int m, int L32, int u, const uint32_t* q32, const uint32_t* rho32,
                const uint32_t* inv2M32)
{
    size_t words = (size_t)M2 * m * L32;
    uint32_t* pa = (uint32_t*)malloc(words * sizeof(uint32_t));
    uint32_t* pb = (uint32_t*)malloc(words * sizeof(uint32_t));
    or_encode(pa, a, alen, M2 / 2, m, L32, u);
    or_encode(pb, b, blen, M2 / 2, m, L32, u);
    or_fft(pa, M2, m, L32, q32, rho32);
    or_fft(pb, M2, m, L32, q32, rho32);
    or_pointwise(pa, pa, pb, M2, m, L32, q32);
    or_fft(pa, M2, m, L32, q32, rho32);
    int rc = or_decode(c, alen + blen, pa, M2, m, L32, u, q32, inv2M32);
    free(pa);
    free(pb);
    return rc;
}
