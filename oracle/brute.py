"""Tiny brute-force references in Python integers (oracle; test infrastructure).

Only the test suite may use these.  They are slow by design and serve to pin the C oracle on
small inputs: every function is a textbook definition, not an algorithm from the thesis.
"""


def ring_mul(x, y, q):
    """Product in (Z/qZ)[alpha]/(alpha^m + 1) by the definition: multiply as polynomials, then
    replace alpha^(m+j) by -alpha^j."""
    m = len(x)
    full = [0] * (2 * m)
    for i in range(m):
        for k in range(m):
            full[i + k] += x[i] * y[k]
    return [(full[j] - full[j + m]) % q for j in range(m)]


def ring_pow(x, e, q):
    m = len(x)
    r = [1] + [0] * (m - 1)
    b = list(x)
    while e:
        if e & 1:
            r = ring_mul(r, b, q)
        b = ring_mul(b, b, q)
        e >>= 1
    return r


def ring_mul_ks(x, y, q):
    """Product in R by Kronecker-Schoenhage substitution (thesis Sec. 3.2.6): pack the m
    coefficients into one integer with 2d + ceil(log2 m) bits per slot, multiply the integers,
    unpack the 2m - 1 product coefficients, fold alpha^m = -1 and reduce mod q."""
    m = len(x)
    d = q.bit_length()
    slot = 2 * d + max(1, (m - 1).bit_length())
    X = sum(c << (slot * i) for i, c in enumerate(x))
    Y = sum(c << (slot * i) for i, c in enumerate(y))
    Z = X * Y
    mask = (1 << slot) - 1
    coef = [(Z >> (slot * i)) & mask for i in range(2 * m)]
    return [(coef[j] - coef[j + m]) % q for j in range(m)]


def alpha_pow(e, m, q):
    """alpha^e as an element of R"""
    e %= 2 * m
    r = [0] * m
    if e < m:
        r[e] = 1
    else:
        r[e - m] = q - 1
    return r


def naive_dft(a, root, q):
    """hat a_i = sum_j a_j root^(i j) over R, by the definition (O(n^2) ring products)."""
    n = len(a)
    m = len(root)
    pw = [[1] + [0] * (m - 1)]
    for _ in range(1, n):
        pw.append(ring_mul(pw[-1], root, q))
    out = []
    for i in range(n):
        acc = [0] * m
        for j in range(n):
            t = ring_mul(a[j], pw[(i * j) % n], q)
            acc = [(s + v) % q for s, v in zip(acc, t)]
        out.append(acc)
    return out


def encode(x, M, m, u):
    """Sec. 3.2.4 written on a Python int: 2M outer coefficients, each m inner coefficients,
    lower m/2 inner coefficients of the lower M outer ones get successive u-bit blocks."""
    out = []
    mask = (1 << u) - 1
    for i in range(2 * M):
        el = [0] * m
        if i < M:
            for k in range(m // 2):
                el[k] = (x >> (u * (k + i * (m // 2)))) & mask
        out.append(el)
    return out


def poly_product_over_Z(a, b):
    """Product of two polynomials in Z[alpha][x] (no reduction anywhere): coefficient lists of
    coefficient lists; the inner degree grows to 2m - 1."""
    m = len(a[0])
    out = [[0] * (2 * m - 1) for _ in range(len(a) + len(b) - 1)]
    for i, ai in enumerate(a):
        for j, bj in enumerate(b):
            for s, x in enumerate(ai):
                if x:
                    for t, y in enumerate(bj):
                        out[i + j][s + t] += x * y
    return out
