"""The library's digit arithmetic (paper_1503_04955_amd/csrc/kernels.hpp, compiled for the host)
against Python integers: modular add/sub/negation, one coefficient of a product in R with a
rotation by alpha^r (Sec. 3.2.5, the bad multiplications with the power trick of Sec. 4.2),
Montgomery scaling, limb conversion; random odd moduli and moduli p = h 2^n + 1."""
import ctypes
import os
import random
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def da(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("da") / "digit_arith.so")
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = os.path.join(HERE, "host_shim", "digit_arith.cpp")
    res = subprocess.run([hipcc, "-O1", "-std=c++17", "-fPIC", "-shared", "-o", out, src],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    lib = ctypes.CDLL(out)
    P = ctypes.POINTER(ctypes.c_uint32)
    lib.da_run.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_uint32, P, P,
                           ctypes.c_int, ctypes.c_int, ctypes.c_int, P]
    return lib


def digits(x, D):
    return [(x >> (28 * k)) & ((1 << 28) - 1) for k in range(D)]


def value(ds):
    return sum(int(v) << (28 * k) for k, v in enumerate(ds))


def arr(vals, n=None):
    n = n or len(vals)
    a = (ctypes.c_uint32 * n)()
    for i, v in enumerate(vals):
        a[i] = v
    return a


def moduli(L, rng):
    """Moduli q with ceil(bits(q)/32) = L: a random odd one and, where n >= 28, p = h 2^n + 1
    with a small h (mostly zero 28-bit digits: the reduction's sparse steps when the high digit
    sits where the library expects it, its general steps otherwise)."""
    bits = 32 * L
    out = [rng.getrandbits(bits) | (1 << (bits - 1)) | 1]
    for h in (3, 13, 27, 81):
        n = bits - h.bit_length()
        if n >= 28:
            out.append(h * (1 << n) + 1)
    return out


def staged(vals, D, DS):
    """Residues at the staging stride DS (>= D words); the padding words hold a value that would
    spoil any product that read them."""
    out = []
    for v in vals:
        out += digits(v, D) + [0x0FFFFFFF] * (DS - D)
    return out


def call(da, L, op, q, a, b, D, log2m=1, j=0, r=0, n_out=None):
    K = da.da_K(L)
    qinv = (-pow(q, -1, 1 << 28)) % (1 << 28)
    out = (ctypes.c_uint32 * (n_out or D))()
    da.da_run(L, op, arr(digits(q, D)), qinv, a, b, log2m, j, r, out)
    return out, K


@pytest.mark.parametrize("L", [1, 2, 3, 4, 5, 6, 7, 8])
def test_add_sub_neg(da, L):
    rng = random.Random(100 + L)
    D = da.da_D(L)
    assert (1 << (28 * D)) > 2 * (1 << (32 * L))
    for q in moduli(L, rng):
        for _ in range(40):
            x, y = rng.randrange(q), rng.randrange(q)
            o, _ = call(da, L, 0, q, arr(digits(x, D)), arr(digits(y, D)), D)
            assert value(o) == (x + y) % q
            o, _ = call(da, L, 1, q, arr(digits(x, D)), arr(digits(y, D)), D)
            assert value(o) == (x - y) % q
            o, _ = call(da, L, 2, q, arr(digits(x, D)), arr(digits(0, D)), D)
            assert value(o) == q - x


@pytest.mark.parametrize("L", [1, 2, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("log2m", [1, 3, 4])
def test_ring_product_coefficient(da, L, log2m):
    """Coefficient j of t * alpha^r * x in R = (Z/q)[alpha]/(alpha^m + 1), times 2^(-28K), with t
    given as its negacyclic extension (t, q - t) at the staging stride and x as m residues."""
    rng = random.Random(1000 * L + log2m)
    D = da.da_D(L)
    m = 1 << log2m
    for q in moduli(L, rng):
        K = da.da_K(L)
        Rinv = pow(1 << (28 * K), -1, q)
        for _ in range(6):
            t = [rng.randrange(q) for _ in range(m)]
            x = [rng.randrange(q) for _ in range(m)]
            if rng.random() < 0.3:
                t[rng.randrange(m)] = 0
                x[rng.randrange(m)] = q - 1
            TP = staged(t + [(q - v) if v else q for v in t], D, da.da_DS(L))
            X = [d for v in x for d in digits(v, D)]
            r = rng.randrange(2 * m)
            # alpha^r x, negacyclic
            ax = [0] * m
            for i in range(m):
                k = i + r
                sgn = -1 if (k // m) % 2 else 1
                ax[k % m] = (ax[k % m] + sgn * x[i]) % q
            for j in range(m):
                want = sum(t[i] * ax[(j - i) % m] * (1 if j >= i else -1) for i in range(m)) % q
                o, _ = call(da, L, 3, q, arr(TP), arr(X), D, log2m, j, r)
                assert value(o) == want * Rinv % q, (q, j, r)
                o, _ = call(da, L, 9, q, arr(TP), arr(X), D, log2m, j, r, n_out=L)
                assert sum(int(o[w]) << (32 * w) for w in range(L)) == want * Rinv % q, (q, j, r)


@pytest.mark.parametrize("L", [1, 2, 3, 4, 5, 6, 7, 8])
def test_sparse_reduction_is_exercised(da, L):
    """The thesis's kind of prime, p = h 2^n + 1 with n >= 28 and a small h, takes the sparse
    Montgomery steps (two digit products per step) at every L, and a random odd modulus the
    general ones; the products above check both against Python integers."""
    D = da.da_D(L)
    bits = 32 * L
    h = 13 if L != 1 else 3
    p = h * (1 << (bits - h.bit_length())) + 1
    assert da.da_sparse(L, arr(digits(p, D))) == 1
    q = random.Random(L).getrandbits(bits) | (1 << (bits - 1)) | 1
    assert da.da_sparse(L, arr(digits(q, D))) == 0


@pytest.mark.parametrize("L", [2, 5, 6, 8])
def test_montgomery_scalar_and_limbs(da, L):
    rng = random.Random(7 + L)
    D = da.da_D(L)
    for q in moduli(L, rng):
        K = da.da_K(L)
        Rinv = pow(1 << (28 * K), -1, q)
        for _ in range(30):
            x, k = rng.randrange(q), rng.randrange(q)
            o, _ = call(da, L, 4, q, arr(digits(x, D)), arr(digits(k, D)), D)
            assert value(o) == x * k * Rinv % q
            o, _ = call(da, L, 5, q, arr(digits(x, D)), arr(digits(0, D)), D, n_out=L)
            assert sum(int(o[w]) << (32 * w) for w in range(L)) == x


@pytest.mark.parametrize("L,log2m", [(1, 6), (2, 6), (5, 5), (6, 4), (6, 5), (6, 6), (7, 6), (8, 6)])
def test_ring_product_coefficient_extreme_digits(da, L, log2m):
    """Largest canonical digits: q = 2^(32L) - 1 (every 28-bit digit of q - 1 at or near its
    maximum) and t_i = x_i = q - 1 for every i, with no wrap (j = m - 1, r = 0), so that every
    column receives the most and the largest digit products; for degrees m up to 64."""
    D = da.da_D(L)
    m = 1 << log2m
    q = (1 << (32 * L)) - 1
    K = da.da_K(L)
    Rinv = pow(1 << (28 * K), -1, q)
    v = q - 1
    DS = da.da_DS(L)
    TP = staged([v] * m + [1] * m, D, DS)
    X = digits(v, D) * m
    o, _ = call(da, L, 3, q, arr(TP), arr(X), D, log2m, m - 1, 0)
    assert value(o) == m * v * v % q * Rinv % q
    o, _ = call(da, L, 9, q, arr(TP), arr(X), D, log2m, m - 1, 0, n_out=L)
    assert sum(int(o[w]) << (32 * w) for w in range(L)) == m * v * v % q * Rinv % q
    # and with every term wrapped (negated): r = m gives x_(j-i-m) = -x_(j-i)
    TPn = staged([1] * m + [v] * m, D, DS)
    o, _ = call(da, L, 3, q, arr(TPn), arr(X), D, log2m, m - 1, m)
    assert value(o) == m * v * v % q * Rinv % q



@pytest.mark.parametrize("L", [1, 2, 3, 4, 5, 6, 7, 8])
def test_product_lds_layout_is_bank_conflict_free(da, L):
    """The LDS layout of the products in R.  Staging: for every rotation r the staged positions
    of the 2m operand entries are a permutation; for every term k and digit y the 64 lanes of a
    wavefront (64/m elements of m lanes) read 64 distinct banks of 4 bytes (and 32 distinct
    banks modulo 32 in each half), whatever the elements' rotations.  Digits: the elements'
    broadcast reads of x_k (1, 2 or 4 words) fall on disjoint banks wherever there are enough
    banks for them."""
    D, DS = da.da_D(L), da.da_DS(L)
    width = 4 if D % 4 == 0 else 2 if D % 2 == 0 else 1
    for log2m in range(1, 7):
        m = 1 << log2m
        sw, ew = da.da_stage_words(m, L), da.da_elem_words(m, L)
        assert sw >= 2 * m * DS and ew >= m * D and ew % width == 0
        for r in range(2 * m):
            assert sorted(da.da_stage_pos(i, r, log2m) for i in range(2 * m)) == list(range(2 * m))
        n = 64 // m
        lanes = [(g, j) for g in range(n) for j in range(m)]
        for k in range(m):
            assert all(1 <= j + m - k < 2 * m for _, j in lanes)
            for y in range(D):
                words = [g * sw + (j + m - k) * DS + y for g, j in lanes]
                assert len({w % 64 for w in words}) == 64, (m, k, y)
                for h in (words[:32], words[32:]):
                    assert len({w % 32 for w in h}) == 32, (m, k, y)
            for banks, groups in ((64, range(n)), (32, range(n // 2)), (32, range(n // 2, n))):
                if len(groups) * width > banks or len(groups) < 2:
                    continue
                used = [(g * ew + k * D + y) % banks for g in groups for y in range(width)]
                assert len(set(used)) == len(used), (m, k, banks)


def limbs(x, L):
    return [(x >> (32 * k)) & 0xFFFFFFFF for k in range(L)]


@pytest.mark.parametrize("L", [1, 2, 3, 4, 5, 6, 7, 8])
def test_limb_add_sub_and_conversions(da, L):
    """The FFT passes' arithmetic on 32-bit limbs (add/sub with carry chains) and the conversions
    between limbs and 28-bit digits; moduli up to 32L bits, including q = 2^(32L) - 1 where the
    sum of two residues carries out of the top limb."""
    rng = random.Random(300 + L)
    D = da.da_D(L)
    qs = moduli(L, rng) + [(1 << (32 * L)) - 1]
    for q in qs:
        for _ in range(60):
            x, y = rng.randrange(q), rng.randrange(q)
            if rng.random() < 0.2:
                x, y = q - 1, q - 1 - rng.randrange(3)
            o, _ = call(da, L, 6, q, arr(limbs(x, L)), arr(limbs(y, L)), D, n_out=L)
            assert sum(int(o[w]) << (32 * w) for w in range(L)) == (x + y) % q
            o, _ = call(da, L, 7, q, arr(limbs(x, L)), arr(limbs(y, L)), D, n_out=L)
            assert sum(int(o[w]) << (32 * w) for w in range(L)) == (x - y) % q
            o, _ = call(da, L, 8, q, arr(limbs(x, L)), arr(limbs(0, L)), D, n_out=D)
            assert [o[k] for k in range(D)] == digits(x, D)
