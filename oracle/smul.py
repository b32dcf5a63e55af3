"""Schoenhage-Strassen multiplication modulo 2^N + 1 (the thesis's SMUL, Sec. 2.9), in Python
integers (oracle; test infrastructure, not product code).

Only the test suite, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline leg may use
this module.  Every element of the ring R = Z/(2^K + 1)Z is a Python int in [0, 2^K]; every
operation is its plain definition (shifts and ``%``), so that each step can be read against the
thesis.  It shares no code with the GPU library and never imports it.

Contents (thesis C. Lueders, arXiv 1503.04955, Sec. 2.9)
  fermat_shift     multiplication by a power of 2 in R (the "cyclic shift" of Sec. 2.9)
  roots            omega = 2^(2K/n) (and theta = 2^(K/n)), Sec. 2.9 first part and 2.9.2
  split / join     Step 1 (cut into n coefficients of s bits) and Step 10 (add up with carries)
  transform        Steps 3-4 / 6-7: evaluation at the powers of a root (radix 2, Sec. 2.6)
  smul_mod         the whole procedure of Sec. 2.9.3: a*b mod 2^N + 1 by a negacyclic
                   (weighted) convolution, Steps 1-11
  outer_params     the outermost SMUL's parameters (Sec. 2.9.3, optimizations: cyclic, n | 2K)
  smul_full        the outermost SMUL: the full product a*b by a cyclic convolution
"""
import math


def fermat_shift(x, t, K):
    """x * 2^t mod 2^K + 1 for any integer t (Sec. 2.9: 2 has order 2K in R, so a multiplication
    by a root of unity is a shift followed by a reduction).  By the definition of the residue."""
    F = (1 << K) + 1
    return (x << (t % (2 * K))) % F


def omega_shift(n, K):
    """Shift count of omega = 2^(2K/n), a primitive n-th root of unity in R when n | 2K
    (Sec. 2.9: 2 is a primitive 2K-th root of unity)."""
    assert (2 * K) % n == 0
    return 2 * K // n


def theta_shift(n, K):
    """Shift count of theta = 2^(K/n): theta^n = 2^K = -1 and theta^2 = omega (the weight of
    Sec. 2.9.2, Eq. (weightcoeff)); needs n | K."""
    assert K % n == 0
    return K // n


def split(x, s, n):
    """Step 1: n coefficients of s bits each, least significant first (zero beyond x)."""
    mask = (1 << s) - 1
    return [(x >> (s * i)) & mask for i in range(n)]


def join(coeffs, s):
    """Step 10: sum of c_k 2^(s k) (Python ints: carries and signs are exact)."""
    return sum(c << (s * k) for k, c in enumerate(coeffs))


def _bitrev(i, bits):
    r = 0
    for _ in range(bits):
        r = (r << 1) | (i & 1)
        i >>= 1
    return r


def transform(a, w_shift, K):
    """Evaluation of a(x) = sum a_j x^j at x = w^i for i < n, where w = 2^w_shift is a primitive
    n-th root of unity in R: result[i] = a(w^i) (Steps 3-4 and 6-7 of Sec. 2.9.3).

    Radix-2 decimation in time on the bit-reversed ("shuffled") input, Sec. 2.6: after the pass
    with half length h, position b + i of every block of 2h positions holds e(w'^i) + w'^i o(w'^i)
    and position b + i + h holds e(w'^i) - w'^i o(w'^i), where w' = w^(n/2h) is a primitive
    2h-th root and e, o are the halves evaluated by the previous passes."""
    n = len(a)
    F = (1 << K) + 1
    bits = n.bit_length() - 1
    assert 1 << bits == n
    v = [a[_bitrev(i, bits)] % F for i in range(n)]
    h = 1
    while h < n:
        step = w_shift * (n // (2 * h))           # w' = w^(n/2h) as a shift count
        for b in range(0, n, 2 * h):
            for i in range(h):
                e = v[b + i]
                o = fermat_shift(v[b + i + h], step * i, K)
                v[b + i] = (e + o) % F
                v[b + i + h] = (e - o) % F
        h *= 2
    return v


def smul_mod(a, b, N, log2_n, K=None):
    """a * b mod 2^N + 1 by the procedure of Sec. 2.9.3 (Steps 1-11), for 0 <= a, b <= 2^N.

    n = 2^log2_n is the FFT length, s = ceil(N/n) the coefficient bits, and K a multiple of n
    (Eq. (reqnthroot) with the weight theta = sqrt(omega)) with K >= log2_n + 2s + 1
    (Eq. (reqm2s)); K = None takes the smallest such K.  N must equal s*n, as in the recursive
    use where N is the caller's K."""
    n = 1 << log2_n
    s = -(-N // n)
    assert s * n == N, "N must be a multiple of the FFT length"
    if K is None:
        need = log2_n + 2 * s + 1
        K = -(-need // n) * n
    assert K % n == 0 and K >= log2_n + 2 * s + 1
    F = (1 << K) + 1
    FN = (1 << N) + 1
    # inputs equal to 2^N (= -1 mod 2^N + 1) need N + 1 bits: their top coefficient is split off
    # into coefficient n, which wraps onto coefficient 0 with a minus sign (x^n = -1)
    def coeffs(x):
        c = split(x % (1 << N), s, n)
        if x >> N:
            c[0] -= x >> N
        return c
    ta, tb = theta_shift(n, K), omega_shift(n, K)
    # Step 2: weights theta^i (negacyclic convolution, Sec. 2.9.2)
    wa = [fermat_shift(c % F, ta * i, K) for i, c in enumerate(coeffs(a))]
    wb = [fermat_shift(c % F, ta * i, K) for i, c in enumerate(coeffs(b))]
    # Steps 3-4: evaluate; Step 5: pointwise products in R
    fa = transform(wa, tb, K)
    fb = transform(wb, tb, K)
    fc = [(x * y) % F for x, y in zip(fa, fb)]
    # Steps 6-7: evaluate at the inverse root omega^-1 = 2^(2K - 2K/n)
    cc = transform(fc, 2 * K - tb, K)
    # Steps 8-9: counterweights theta^-k and 1/n = 2^-log2_n, both shifts
    out = []
    for k, c in enumerate(cc):
        c = fermat_shift(c, -ta * k - log2_n, K)
        # c is the negacyclic sum, in [-n 2^(2s), n 2^(2s)]: residues above 2^(K-1) are negative
        out.append(c - F if c > F // 2 else c)
    # Steps 10-11: add up with carries (signed coefficients), reduce mod 2^N + 1
    return join(out, s) % FN


def outer_params(alen_bits, blen_bits, log2_n, word=32):
    """Parameters of the outermost SMUL for the full product (Sec. 2.9.3, optimizations: no
    weights, a cyclic convolution whose sums stay nonnegative, n | 2K): s = ceil((bits(a) +
    bits(b)) / n) bits per coefficient, and K the smallest multiple of lcm(word, n/2) with
    2^K > min(na, nb) (2^s - 1)^2, na and nb the coefficient counts of a and b (the largest
    convolution sum).  Returns (s, K) or None if the product does not fit n coefficients."""
    n = 1 << log2_n
    s = -(-(alen_bits + blen_bits) // n)
    na = max(1, -(-alen_bits // s))
    nb = max(1, -(-blen_bits // s))
    if na + nb - 1 > n:
        return None
    bound = min(na, nb) * ((1 << s) - 1) ** 2
    unit = math.lcm(word, max(1, n // 2))
    K = unit
    while (1 << K) <= bound:
        K += unit
    return s, K


def smul_full(a, b, log2_n, s=None, K=None):
    """The full product a * b by the outermost SMUL (Sec. 2.9.3 with its optimizations): split
    into s-bit coefficients, evaluate at the powers of omega = 2^(2K/n), multiply pointwise in R,
    evaluate at omega^-1, scale by 1/n, add up.  Every convolution sum is the exact coefficient
    of the product polynomial (nonnegative and below 2^K), so no weights, signs or final
    reduction are needed.  s, K default to outer_params."""
    n = 1 << log2_n
    if s is None or K is None:
        p = outer_params(max(a.bit_length(), 1), max(b.bit_length(), 1), log2_n)
        assert p is not None
        s, K = p
    F = (1 << K) + 1
    w = omega_shift(n, K)
    fa = transform(split(a, s, n), w, K)
    fb = transform(split(b, s, n), w, K)
    fc = [(x * y) % F for x, y in zip(fa, fb)]
    cc = transform(fc, 2 * K - w, K)
    return join([fermat_shift(c, -log2_n, K) for c in cc], s)


def forward(a, s, log2_n, K):
    """The outermost SMUL's forward transform of a: split into n = 2^log2_n coefficients of s
    bits (Step 1) and evaluate at the powers of omega (Step 4), natural order."""
    n = 1 << log2_n
    return transform(split(a, s, n), omega_shift(n, K), K)
