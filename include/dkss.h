/*
 * dkss.h -- C ABI of libdkss, DKSS multiplication of large unsigned integers on one AMD
 * Instinct MI355X (gfx950).
 *
 * The method is the one analysed in C. Lueders, "Fast Multiplication of Large Integers:
 * Implementation and Analysis of the DKSS Algorithm" (arXiv 1503.04955), Chapter 3: encode both
 * operands as polynomials over R = (Z/p^zZ)[alpha]/(alpha^m + 1) (Sec. 3.2.4), transform with a
 * length-2M FFT whose inner 2m-point DFTs multiply by powers of alpha and whose outer stages
 * multiply by powers of rho (Sec. 3.2.5), multiply componentwise in R (Sec. 3.2.6), transform
 * back (Sec. 3.2.7) and recover the integer with carries (Sec. 3.2.8).
 *
 * Conventions for every entry point
 *  - Integers are arrays of uint32_t limbs, least significant limb first (Sec. 2.1), with the
 *    length passed separately.  Operands need not be normalized (high zero limbs are allowed).
 *  - Pointers named a, b, c, x, ws are DEVICE pointers; pointers to parameter structs, length
 *    arrays and result scalars are HOST pointers.  The caller owns all memory and keeps it
 *    alive until the stream has finished the call.  The library never frees caller memory.
 *  - Work is enqueued asynchronously on the given HIP stream (NULL = the null stream).  Argument
 *    and feasibility errors are returned synchronously; device faults surface as DKSS_EHIP from
 *    a later call or from the caller's own synchronization.
 *  - A context is not thread-safe: use one per host thread or lock around it.
 *  - Return value: DKSS_OK (0) or a negative DKSS_E* code; dkss_strerror() names it.
 */
#ifndef DKSS_H
#define DKSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* dkss_stream_t;   /* hipStream_t */
typedef struct dkss_ctx dkss_ctx;

enum {
    DKSS_OK = 0,
    DKSS_EINVAL = -1,     /* null pointer, overlapping output, bad enum or struct contents */
    DKSS_ENOSPC = -2,     /* workspace smaller than dkss_workspace_bytes() */
    DKSS_ERANGE = -3,     /* size or parameter tuple unsupported or infeasible */
    DKSS_EHIP = -4,       /* a HIP runtime call failed */
    DKSS_ENOTIMPL = -5,
    DKSS_ETOOBIG = -6     /* dkss_mul_noalloc: the product needs more than its fixed scratch */
};

/* Parameter policy of a context. */
enum {
    DKSS_POLICY_THESIS = 0,   /* the thesis's rule, Sec. 4.1 (with Sec. 3.2 Steps 1-2) */
    DKSS_POLICY_TUNED = 1,    /* measured plans from the context's tuning table, else THESIS */
    DKSS_POLICY_LEARNED = 2   /* the learned selector's choice (dkss_set_mlp / dkss_mlp.txt),
                               * else THESIS */
};

/*
 * One parameter tuple (Sec. 3.2 Steps 1-2): FFT length 2M = 2^(log2_M+1), inner degree bound
 * m = 2^log2_m, u input bits per inner coefficient, prime p of p_bits bits (h*2^n + 1 with the
 * smallest odd h, Sec. 4.6) and modulus p^z.  Products with min(alen, blen)*32 <= cutoff_bits
 * use the schoolbook base case instead.  radix_log2[i] (i < n_levels) optionally fixes the FFT
 * level split: 2M = prod 2^radix_log2[i], each radix at most 2m; n_levels = 0 lets the library
 * choose (levels of radix 2m, then the remainder, as in the thesis's recursion, Sec. 4.2).
 * A struct whose u is 0 asks for u = ceil(2N / Mm).
 */
typedef struct {
    uint32_t log2_M;
    uint32_t log2_m;
    uint32_t u;
    uint32_t p_bits;
    uint32_t z;
    uint32_t n_levels;
    uint32_t radix_log2[8];
    uint64_t cutoff_bits;
} dkss_params;

/* Derived facts of a plan (for reporting and tests). */
typedef struct {
    dkss_params params;
    uint32_t L;               /* uint32 limbs per inner coefficient (ceil(bits(p^z)/32)) */
    uint32_t q_bits;          /* bits of p^z */
    uint32_t schoolbook;      /* 1 if the product goes to the schoolbook base case */
    uint32_t squaring;        /* filled by dkss_plan_info only when a == b was indicated */
    uint64_t poly_bytes;      /* S = 2M * m * L * 4, one polynomial */
    uint64_t table_bytes;     /* device table of rho^s, s < 2M/2m */
    uint32_t q[16];           /* p^z, L limbs */
    uint32_t digits;          /* 28-bit digits per residue in the products in R: ceil((32L+1)/28),
                                 or one fewer when q < 2^(28 digits - 1) (L >= 2) */
} dkss_plan;

/* Create a context with the given policy.  cache_dir may be NULL; a TUNED context reads
 * cache_dir/dkss_tuning.txt and a LEARNED one cache_dir/dkss_mlp.txt (dkss_mlp_load) when they
 * exist.  The tuning table is text: lines "lo hi cand [radices] [dft_lds]" (a log2 N range; a
 * candidate index of dkss_candidates, S or DKSS_CAND_SCHOOLBOOK for the base case, or T for the
 * thesis rule; a level split such as 5.5.4; a DFT LDS budget in bytes), '#' comments, and
 * "@batch B" lines: the entries after one hold for batches of at least B products (before the
 * first, B = 1); a product takes the entry of the largest such B whose range holds its N.
 * Allocates nothing on the device until a parameter tuple is first prepared or the selector's
 * first inference.  Errors: DKSS_EINVAL. */
int dkss_ctx_create(dkss_ctx** out, int policy, const char* cache_dir);

/* Release the context and the device tables it owns.  Safe on NULL. */
void dkss_ctx_destroy(dkss_ctx* ctx);

/* Parameters the context's policy picks for operands of a_bits and b_bits bits in a batch of
 * `batch` products.  N = max(a_bits, b_bits) rounded up to whole limbs (the thesis assumes equal
 * lengths, Sec. 3.2).  A LEARNED choice of a candidate sets cutoff_bits 0; a LEARNED or TUNED
 * choice of the schoolbook sets cutoff_bits UINT64_MAX (with the thesis rule's tuple).  Errors: DKSS_EINVAL
 * (null), DKSS_ERANGE (N = 0 or beyond 2^36 bits), DKSS_EHIP (learned inference). */
int dkss_select_params(dkss_ctx* ctx, uint64_t a_bits, uint64_t b_bits, uint32_t batch,
                       dkss_params* out);

/*
 * Candidate parameter tuples for operands of a_bits x b_bits bits (N = the longer, in whole
 * limbs), the search space of the tuner and of the learned selector.  t_min is the smallest
 * log2(Mm) whose u = ceil(2N/Mm) admits a prime modulus of at most 256 bits; M = Mm/m >= m.
 *   c = t_off * 6 + (log2_m - 1) < 18, t_off in 0..2, log2_m in 1..6: Mm = 2^(t_min + t_off),
 *       z = 1, p of the fewest whole 32-bit limbs with p > Mm 2^(2u) (Sec. 3.2.2), or, where
 *       a modulus of that size fits one 28-bit digit fewer than the limbs take, p of 28 D - 1
 *       bits for the fewest such D (the products in R then run on D digits, dkss_plan.digits);
 *   c = 18 + (log2_m - 1) < 24: Mm = 2^t_min, z = 2 (q = p^2, the lift of Sec. 3.2.3), p of the
 *       fewest bits with p^2 > Mm 2^(2u) (Sec. 3.2 Step 2).
 * out[c] is filled for every c < DKSS_NCAND; valid[c] = 1 where the tuple is feasible.  The
 * radices are the library default, cutoff_bits 0.  Errors: DKSS_EINVAL, DKSS_ERANGE.
 */
enum { DKSS_NCAND = 24 };
int dkss_candidates(dkss_ctx* ctx, uint64_t a_bits, uint64_t b_bits, dkss_params* out,
                    int* valid);

/* Plan facts for a product of alen x blen limbs under params p (NULL = the policy). */
int dkss_plan_info(dkss_ctx* ctx, size_t alen, size_t blen, const dkss_params* p, dkss_plan* out);

/* Workspace bytes dkss_mul needs for alen x blen limbs under params p (NULL = the policy),
 * including room for the tuple's table of rho^s (used only while the context has not prepared
 * that table, see dkss_prepare).  A planning call: under DKSS_POLICY_LEARNED it runs the
 * selector's inference for a shape not seen before and waits for it (as dkss_mlp_choose), so
 * that the products of that shape find the choice cached. */
int dkss_workspace_bytes(dkss_ctx* ctx, size_t alen, size_t blen, const dkss_params* p,
                         size_t* out);

/* Build (if not yet built) and keep in ctx the device table of params p for operands of alen x
 * blen limbs: rho^s for s below 2M/2m, Sec. 4.2 (and, under DKSS_POLICY_LEARNED, the selector's
 * choice for the shape).  A planning call: allocates device memory, runs the build on s and
 * waits for it; the table counts as built only once the build has finished, and a failed build
 * leaves nothing behind.  Refused (DKSS_EINVAL) while s is capturing.  Without it, every product
 * of the tuple rebuilds the table in its workspace (correct, slower).  Errors: DKSS_EINVAL,
 * DKSS_ERANGE, DKSS_EHIP. */
int dkss_prepare(dkss_ctx* ctx, size_t alen, size_t blen, const dkss_params* p, dkss_stream_t s);

/*
 * c[0 .. alen+blen) = a * b (Sec. 3.2, Steps 4-8).  Every limb of c is written, high zeros
 * included.  a == b with alen == blen is a squaring (one forward transform).  alen or blen of 0
 * gives c = 0.  c must not overlap a or b (DKSS_EINVAL).  ws must hold at least
 * dkss_workspace_bytes() bytes of device memory, 256-byte aligned (DKSS_ENOSPC / DKSS_EINVAL).
 * p = NULL uses the context's policy; under DKSS_POLICY_LEARNED the product takes the choice a
 * planning call (dkss_workspace_bytes, dkss_prepare, dkss_select_params, dkss_plan_info,
 * dkss_mlp_choose) cached for the shape with batch 1, and the thesis rule when there is none; a
 * TUNED context looks its table up with batch 1 (dkss_mul_batch: batch = count).
 * The call allocates no memory and never waits on the host: all of its work, including the
 * tuple's table when dkss_prepare has not built it (then in ws), is enqueued on s, so it may be
 * recorded by a stream capture.
 * Errors: DKSS_EINVAL, DKSS_ENOSPC, DKSS_ERANGE (p^z below
 * Mm 2^(2u), 2M not dividing p - 1, M < m, m < 2, capacity M*m/2*u below 32*max(alen, blen),
 * unsupported limb count, a transform length 2M above 2^31, a kernel grid of 2^32 work-items
 * or more: operands beyond about 2^35 bits, or a level split with very small radices),
 * DKSS_EHIP.
 */
int dkss_mul(dkss_ctx* ctx, uint32_t* c, const uint32_t* a, size_t alen, const uint32_t* b,
             size_t blen, const dkss_params* p, void* ws, size_t ws_bytes, dkss_stream_t s);

/*
 * Schoenhage-Strassen multiplication, the thesis's SMUL (Sec. 2.9), in its outermost form for the
 * full product (Sec. 2.9.3 with its optimizations): both operands cut into n = 2^log2_n
 * coefficients of s bits, a cyclic FFT of length n over Z/(2^K + 1)Z with root omega = 2^(2K/n)
 * (n | 2K; every multiplication by a root is a cyclic shift), componentwise products in that ring,
 * the inverse FFT and the coefficients added up with carries.  K = 2048 lw bits (lw = 1, 2, 4,
 * ..., 32).  The thesis's comparison method for DKSS; it needs no context.
 */
typedef struct {
    uint32_t log2_n;      /* FFT length n = 2^log2_n (0 = chosen by the library) */
    uint32_t lw;          /* K = 2048 lw bits per ring element (0 = chosen) */
    uint32_t s;           /* output: bits per input coefficient, ceil(32 (alen + blen) / n) */
    uint32_t K;           /* output: ring exponent */
    uint32_t n_levels;    /* output: LDS-staged FFT levels per transform */
    uint32_t products;    /* componentwise products (Step 5): 1 schoolbook of 28-bit digits on the
                             vector units, 2 exact 8-bit products on the matrix cores (lw <= 16);
                             0 = chosen by the modelled cost; output: the form used */
} dkss_smul_params;

/* The library's choice of (log2_n, lw, products) for alen x blen limbs (a modelled cost over the
 * feasible pairs: na + nb - 1 <= n coefficients, min(na, nb) (2^s - 1)^2 < 2^K, n | 2K; the
 * matrix-core products wherever lw <= 16 allows them, at half the digit form's cost).  All zero when
 * alen or blen is 0.  Errors: DKSS_EINVAL (null), DKSS_ERANGE (no feasible pair). */
int dkss_smul_select(size_t alen, size_t blen, dkss_smul_params* out);

/* Workspace bytes of dkss_smul under p (NULL or zero fields = the library's choice). */
int dkss_smul_workspace_bytes(size_t alen, size_t blen, const dkss_smul_params* p, size_t* out);

/* c[0 .. alen+blen) = a * b by SMUL (Sec. 2.9.3, Steps 1, 3-7, 9-10 of the outermost form), all
 * enqueued on s; conventions as dkss_mul (device pointers, c not overlapping a or b, a == b with
 * alen == blen a squaring with one forward transform, ws of dkss_smul_workspace_bytes() bytes,
 * 256-byte aligned).  Allocates nothing and does not wait.  Errors: DKSS_EINVAL, DKSS_ENOSPC,
 * DKSS_ERANGE (the given (log2_n, lw) infeasible, or none), DKSS_EHIP. */
int dkss_smul(uint32_t* c, const uint32_t* a, size_t alen, const uint32_t* b, size_t blen,
              const dkss_smul_params* p, void* ws, size_t ws_bytes, dkss_stream_t s);

/* The forward transform of SMUL for the operand a of an alen x blen product under p: Step 1
 * (n coefficients of s bits) and Steps 3-4 (evaluation at omega^i), in bit-reversed order: poly
 * (n x 64 lw limbs, device) element bitrev(i) holds a(omega^i) mod 2^K + 1 below 2^K and
 * tops[bitrev(i)] (n words, device) is 1 exactly when that value is 2^K.  Errors: as dkss_smul. */
int dkss_smul_forward(uint32_t* poly, uint32_t* tops, const uint32_t* a, size_t alen, size_t blen,
                      const dkss_smul_params* p, dkss_stream_t s);

/* Measured rate of the 32 x 32 -> 64-bit multiply-add (v_mad_u64_u32, the instruction of the
 * products in R) on the current device, in lane operations per second: 16 workgroups of 256
 * threads per CU, eight independent chains per thread, timed with events on s after a warm-up
 * launch.  A diagnostic: it waits for its launches.  Errors: DKSS_EINVAL, DKSS_EHIP. */
int dkss_probe_mad_rate(double* mads_per_s, dkss_stream_t s);

/* The bad multiplications of the FFT levels (Sec. 3.2.5 ii: the products by rho^s alpha^r) in
 * two forms, for an A/B measurement of the vector units against the matrix cores.  For
 * g < groups and n < 32, with m = 2^log2_m coefficients (log2_m must be 4):
 *     y[g][n] = t[g] * alpha^(r[g][n] mod 2m) * x[g][n] * 2^(-28 K) mod q   in R,
 * K the Montgomery digit steps of q's residue format (as dkss_plan.digits: K = ceil((qb + 6) / 28),
 * qb = 28 digits - 1 for a tight format, else 32 L), every coefficient canonical in [0, q): the
 * 32 elements of a group share one twiddle, as the elements of a transform whose twiddles have
 * the same table index s do.  form 1: 28-bit digit products on the vector units, one lane per
 * output coefficient (the level kernels' product); form 2: the group's 32 products as one
 * contraction of 7-bit digits by v_mfma_i32_32x32x32_i8.  Both give the same words.
 * q: HOST, L limbs (3 <= L <= 6, odd, top limb not zero).  t: DEVICE, groups x m residues of L
 * limbs; x, y: DEVICE, groups x 32 x m residues of L limbs (residues canonical, x 16-byte
 * aligned, y not overlapping t, x or r); r: DEVICE, groups x 32 words.  Enqueued on s; allocates
 * nothing and does not wait.  Errors: DKSS_EINVAL (form not 1 or 2, null pointer, x not aligned,
 * q even or not L limbs),
 * DKSS_ERANGE (log2_m, L or groups >= 2^31 unsupported), DKSS_EHIP. */
int dkss_probe_twiddle_products(int form, const uint32_t* q, uint32_t L, uint32_t log2_m, size_t groups,
                                const uint32_t* t, const uint32_t* x, const uint32_t* r, uint32_t* y,
                                dkss_stream_t s);

/* Bytes of the fixed device scratch of dkss_mul_noalloc (one copy per device). */
#define DKSS_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/*
 * dkss_mul without a workspace argument, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and result as dkss_mul, with the workspace placed in a scratch array of
 * DKSS_NOALLOC_SCRATCH_BYTES bytes that the library holds in device memory on every device it
 * runs on, until the process ends.  The call allocates nothing (no hipMalloc, no library
 * allocation) and does not wait; the scratch's device address for the current device is looked
 * up by dkss_ctx_create or by the first call on that device.  Products whose workspace
 * (dkss_workspace_bytes, which includes room for the tuple's table unless dkss_prepare has built
 * it) exceeds the scratch are refused with DKSS_ETOOBIG: about 2^24 bits per operand under the
 * thesis rule, 2^25 under the tuned table.  Nothing in the scratch needs to start at zero, and a
 * call keeps no state there for the next one.  Every call on one device shares that device's
 * scratch: calls that overlap in time on one device (several streams, several host threads,
 * several contexts) race and give wrong products; serialize them.
 * Errors: as dkss_mul (except DKSS_ENOSPC), DKSS_ETOOBIG.
 */
int dkss_mul_noalloc(dkss_ctx* ctx, uint32_t* c, const uint32_t* a, size_t alen, const uint32_t* b,
                     size_t blen, const dkss_params* p, dkss_stream_t s);

/*
 * count independent products c[i] = a[i] * b[i] (each as in dkss_mul).  The arrays of
 * pointers and lengths are HOST arrays of device pointers.  p is NULL (policy per product) or
 * an array of count tuples.  Products that share a parameter tuple run together in the same
 * kernel launches.  The workspace must hold dkss_batch_workspace_bytes().  Like dkss_mul it
 * allocates nothing and does not wait: the product descriptors reach the start of ws through
 * small kernel launches on s, and tables not built by a planning call are built in ws.
 */
int dkss_mul_batch(dkss_ctx* ctx, size_t count, uint32_t* const* c, const uint32_t* const* a,
                   const size_t* alen, const uint32_t* const* b, const size_t* blen,
                   const dkss_params* p, void* ws, size_t ws_bytes, dkss_stream_t s);

/* Workspace bytes for dkss_mul_batch with the same arguments (descriptors, room for the table
 * of every tuple the batch uses, the largest group's buffers).  A planning call like
 * dkss_workspace_bytes: the selector's inference for the batch's new shapes runs here. */
int dkss_batch_workspace_bytes(dkss_ctx* ctx, size_t count, const size_t* alen,
                               const size_t* blen, const dkss_params* p, size_t* out);

/* dkss_prepare for every parameter tuple a batch with these lengths uses (a planning call:
 * allocates, builds on s, waits).  Without it, dkss_mul_batch builds the tables it lacks in its
 * workspace on every call.  Errors: as dkss_prepare. */
int dkss_batch_prepare(dkss_ctx* ctx, size_t count, const size_t* alen, const size_t* blen,
                       const dkss_params* p, dkss_stream_t s);

/*
 * A batch (as in dkss_mul_batch) planned once and captured into a HIP graph; every
 * dkss_graph_launch recomputes all count products with one graph launch, reading the operands
 * and writing the results at the same device addresses.  At creation the library plans the
 * batch, builds the tables it needs in the context (as dkss_batch_prepare), writes the product
 * descriptors to the start of ws (on a stream of its own, waiting for them) and captures the
 * products' kernels; nothing else enters the graph.  The caller keeps ws, every operand and result buffer and the context alive and ws
 * otherwise unused until dkss_graph_destroy; launches of one graph must not overlap in time
 * (they share ws).  Profiling does not see graph launches.  count must be at least 1.
 * Errors: as dkss_mul_batch, DKSS_EHIP (capture or instantiation failed).
 */
typedef struct dkss_graph dkss_graph;
int dkss_batch_graph_create(dkss_ctx* ctx, size_t count, uint32_t* const* c,
                            const uint32_t* const* a, const size_t* alen, const uint32_t* const* b,
                            const size_t* blen, const dkss_params* p, void* ws, size_t ws_bytes,
                            dkss_graph** out);
/* Enqueue the graph on stream s.  Errors: DKSS_EINVAL, DKSS_EHIP. */
int dkss_graph_launch(dkss_graph* g, dkss_stream_t s);
/* Products in the graph and kernel nodes captured.  Errors: DKSS_EINVAL. */
int dkss_graph_info(const dkss_graph* g, size_t* products, size_t* kernels);
/* Release the graph (not the buffers).  Safe on NULL.  The caller makes sure no launch of it
 * is still pending. */
void dkss_graph_destroy(dkss_graph* g);

/*
 * Forward transform only (Steps 4-5): encode a into 2M elements of R and transform them with
 * root rho; poly receives a(rho^i) for i < 2M in natural order, element-major (element i, inner
 * coefficient k, limb w at ((i*m + k)*L + w)), canonical residues in [0, p^z).  poly holds
 * poly_bytes of dkss_plan; ws holds dkss_workspace_bytes().  For checking intermediates.
 */
int dkss_forward(dkss_ctx* ctx, uint32_t* poly, const uint32_t* a, size_t alen, size_t blen,
                 const dkss_params* p, void* ws, size_t ws_bytes, dkss_stream_t s);

/* Residues x mod primes[j] for j < count (each prime odd, below 2^62), written to the DEVICE
 * array out[count].  For checking products of any size by c = a*b mod q. */
int dkss_residues(const uint32_t* x, size_t n, const uint64_t* primes_host, size_t count,
                  uint64_t* out, dkss_stream_t s);

/*
 * Kernel timing.  With profiling on, every kernel launch a context makes is bracketed by two HIP
 * events recorded on the launch's stream, and the launch's algorithmic work is noted: bytes that
 * the step must move (each input read once, each output written once) and, for the products in
 * R, 32x32-bit multiply-adds of the schoolbook product (m^2 L^2 per product in R).  The figures
 * are summed per kernel kind.  dkss_profile_read synchronizes on the recorded events.
 * FFT levels: DKSS_K_DFT a level without twiddles (kernel k_level<L, 0>), DKSS_K_TWIDDLE a
 * forward level with its rho twiddles (k_level<L, 1>), DKSS_K_TWIDDLE_INV an inverse level with
 * its twiddles (k_level<L, 2>).  DKSS_K_POINTWISE: the componentwise products, as k_pointwise<L>
 * or, fused (DKSS_OPT_FUSE_PW), as k_level<L, 3> together with the bottom forward and inverse
 * DFTs (its bytes and operations are those of the products).
 */
enum {
    DKSS_K_ENCODE = 0, DKSS_K_DFT, DKSS_K_TWIDDLE, DKSS_K_POINTWISE, DKSS_K_DECODE,
    DKSS_K_CARRY_SCAN, DKSS_K_CARRY_APPLY, DKSS_K_SCHOOLBOOK, DKSS_K_TABLE, DKSS_K_UNSCRAMBLE,
    DKSS_K_TWIDDLE_INV, DKSS_K_KINDS
};

typedef struct {
    uint64_t launches;
    double total_ms;        /* sum of event-measured launch durations */
    double alg_bytes;       /* algorithmic bytes, summed over launches */
    double alg_ops;         /* algorithmic 32-bit multiply-adds, summed over launches */
} dkss_kernel_stats;

/* Turn profiling on (1) or off (0).  Errors: DKSS_EINVAL. */
int dkss_profile_enable(dkss_ctx* ctx, int on);
/* Totals of kernel kind `kind` (DKSS_K_*) since the last reset.  Errors: DKSS_EINVAL, DKSS_EHIP. */
int dkss_profile_read(dkss_ctx* ctx, int kind, dkss_kernel_stats* out);
/* Clear the totals (waits for pending events first). */
int dkss_profile_reset(dkss_ctx* ctx);
/* Name of a kernel kind, e.g. "k_twiddle"; NULL for an unknown kind. */
const char* dkss_kernel_name(int kind);

/*
 * Context options (tuning knobs; none changes any result bit).
 *  DKSS_OPT_OVERLAP      1: the forward transform of b runs on a second, internal stream of
 *                        the context (created when the option is first set to 1), forked from
 *                        and joined back to the caller's stream with events, so it overlaps
 *                        the transform of a; 0 (default): one stream.
 *  DKSS_OPT_DFT_LDS      LDS bytes an FFT-level workgroup may stage (default 32768; 16384 to
 *                        163840): more columns per workgroup versus more workgroups per CU.
 *  DKSS_OPT_FUSE_PW      1 (default): the componentwise products (Step 6) run inside the
 *                        bottom FFT level, which then also runs the bottom level of the inverse
 *                        transform (one launch instead of three); 0: separate launches.  Not
 *                        fused while DKSS_OPT_OVERLAP transforms b on the second stream.
 *  DKSS_OPT_BATCH_LANES  1..8 (default 4): a batch's launch groups (one per parameter tuple)
 *                        are spread over this many streams, the largest modelled work first,
 *                        each group to the least loaded one, every stream with its own
 *                        workspace slice (dkss_batch_workspace_bytes grows accordingly), so that
 *                        independent groups overlap; the extra streams of the context are made
 *                        by this option or by a planning call (dkss_batch_workspace_bytes,
 *                        dkss_batch_prepare, dkss_batch_graph_create), forked from and joined
 *                        back to the caller's stream with events, and a captured batch graph
 *                        holds them as parallel branches.  Without them (no planning call yet)
 *                        the groups run on the caller's stream.
 *  DKSS_OPT_STEP6_KS     1: the componentwise products in R (Step 6) as Sec. 3.2.6 writes them:
 *                        each element packed into one integer by Kronecker-Schoenhage
 *                        substitution (slots of 2 bits(q) + log2 m bits), the 2M integer
 *                        products of a polynomial pair computed by the library itself under the
 *                        context's policy (the schoolbook base case, or DKSS, whose own Step 6
 *                        recurses the same way), the slots unpacked, alpha^m = -1 folded and
 *                        reduced mod q.  Exact like the default (direct negacyclic products) and
 *                        much slower; dkss_workspace_bytes and dkss_batch_workspace_bytes grow
 *                        by the packed integers and the inner products' workspace, and the
 *                        planning calls also build the inner products' tables.  0 (default).
 */
enum { DKSS_OPT_OVERLAP = 0, DKSS_OPT_DFT_LDS = 1, DKSS_OPT_FUSE_PW = 2, DKSS_OPT_BATCH_LANES = 3,
       DKSS_OPT_STEP6_KS = 4 };
int dkss_set_option(dkss_ctx* ctx, int option, long long value);

/*
 * Learned parameter selector.  The thesis leaves the choice of parameters open beyond its
 * asymptotic rule (Sec. 3.2 Steps 1-2, Sec. 4.1, and its outlook, Chapter 5); this selector
 * predicts, for each candidate of dkss_candidates and for the schoolbook base case, the log of
 * the run time per product, and the LEARNED policy takes the feasible candidate of least
 * predicted time.  The network is an FP32 multilayer perceptron
 *     h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3
 * with DKSS_MLP_IN inputs, two hidden layers of DKSS_MLP_HID units and DKSS_MLP_OUT outputs:
 * output c < DKSS_NCAND is candidate c, output DKSS_CAND_SCHOOLBOOK the schoolbook product.
 * Parameters are one float array of DKSS_MLP_NPARAM entries in the order
 *     W1[HID][IN], b1[HID], W2[HID][HID], b2[HID], W3[OUT][HID], b3[OUT]   (row-major).
 * Training minimizes sum_n sum_k mask[n][k] (y[n][k] - t[n][k])^2 / mask_sum with Adam.
 */
enum {
    DKSS_MLP_IN = 3,
    DKSS_MLP_HID = 64,
    DKSS_MLP_OUT = DKSS_NCAND + 1,
    DKSS_CAND_SCHOOLBOOK = DKSS_NCAND,
    DKSS_MLP_NPARAM = DKSS_MLP_HID * DKSS_MLP_IN + DKSS_MLP_HID + DKSS_MLP_HID * DKSS_MLP_HID +
                      DKSS_MLP_HID + DKSS_MLP_OUT * DKSS_MLP_HID + DKSS_MLP_OUT
};

/* Selector inputs for a product of a_bits x b_bits bits in a batch of `batch` products (HOST
 * out[DKSS_MLP_IN]): (log2(longer) - 21) / 9, (log2(shorter) - 21) / 9, log2(batch) / 12, with
 * bit counts rounded up to whole limbs and at least one limb.  Errors: DKSS_EINVAL (null,
 * batch 0). */
int dkss_mlp_features(uint64_t a_bits, uint64_t b_bits, uint32_t batch, float* out);

/* Forward pass: y[n][DKSS_MLP_OUT] from x[n][DKSS_MLP_IN] (all DEVICE pointers).  One wavefront
 * per sample.  Errors: DKSS_EINVAL (null, n <= 0), DKSS_EHIP. */
int dkss_mlp_forward(const float* params, const float* x, int n, float* y, dkss_stream_t s);

/* Floats of the `work` buffer dkss_mlp_loss_grad needs for n samples: n * (DKSS_MLP_NPARAM + 1). */
size_t dkss_mlp_work_floats(int n);

/* Loss and its gradient (all DEVICE pointers): x[n][IN], targets t[n][OUT], mask[n][OUT]
 * (weights, usually 0/1: which targets were measured), mask_sum > 0 the normalizer.  Writes
 * grad[DKSS_MLP_NPARAM] and loss[1].  Per-sample gradients go to work and are summed in sample
 * order, so the result does not depend on scheduling.  Errors: DKSS_EINVAL, DKSS_EHIP. */
int dkss_mlp_loss_grad(const float* params, const float* x, const float* t, const float* mask, int n,
                       float mask_sum, float* grad, float* loss, float* work, dkss_stream_t s);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8; step counts from 1) on DEVICE arrays of
 * DKSS_MLP_NPARAM floats: m1, m2 are the moment estimates, zero before step 1.
 * Errors: DKSS_EINVAL, DKSS_EHIP. */
int dkss_mlp_adam(float* params, const float* grad, float* m1, float* m2, int step, float lr,
                  dkss_stream_t s);

/* Install selector weights (HOST array of DKSS_MLP_NPARAM finite floats, copied) in the
 * context; NULL removes them.  Clears the context's cache of choices; the device copy is made at
 * the next inference.  Errors: DKSS_EINVAL (null context, a non-finite weight). */
int dkss_set_mlp(dkss_ctx* ctx, const float* params);

/* Read weights from a text file (a header line "IN HID OUT" after '#' comments, then
 * DKSS_MLP_NPARAM numbers) into params (HOST).  Errors: DKSS_EINVAL (unreadable or malformed). */
int dkss_mlp_load(const char* path, float* params);

/*
 * The learned selector's choice for a product of a_bits x b_bits bits in a batch of `batch`:
 * *cand = c < DKSS_NCAND (candidate c), DKSS_CAND_SCHOOLBOOK, or -1 when the context has no
 * weights or no output is feasible (the thesis rule then applies).  Feasible: candidates that
 * dkss_candidates marks valid; the schoolbook when both operands together have at most 4096
 * limbs.  Inference runs dkss_mlp_forward on a stream private to the context and waits for it;
 * choices are cached per (limbs of a, limbs of b, batch), where the products look them up.  Errors: DKSS_EINVAL, DKSS_ERANGE,
 * DKSS_EHIP.
 */
int dkss_mlp_choose(dkss_ctx* ctx, uint64_t a_bits, uint64_t b_bits, uint32_t batch, int* cand);

/* Static description of an error code. */
const char* dkss_strerror(int code);

/* The hipError_t of the last failed HIP call made by the library on this host thread (0 if
 * none): the detail behind a DKSS_EHIP.  Entry points that launch kernels first discard a
 * pending error left by earlier, unrelated HIP calls of the thread, so a DKSS_EHIP names the
 * library's own call. */
int dkss_last_hip_error(void);
/* HIP's description of a hipError_t code. */
const char* dkss_hip_error_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* DKSS_H */
