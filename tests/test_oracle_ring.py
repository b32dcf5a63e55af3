"""Pins of the C oracle's modular and ring arithmetic, FFT, encode/decode and the whole DKSS
pipeline against textbook definitions written in Python integers (oracle.brute)."""
import random

import numpy as np
import pytest

import seeded_inputs as SI
from oracle import brute
from oracle import coracle as C
from oracle import params as P

# moduli of 1..4 64-bit words, including the thesis primes and a prime power (z > 1)
QS = [193, 3 * 2 ** 30 + 1, 27 * 2 ** 59 + 1, 81 * 2 ** 121 + 1, 13 * 2 ** 188 + 1,
      (3 * 2 ** 30 + 1) ** 4, 2 ** 255 - 19]


def _lw(q):
    return -(-q.bit_length() // 32)


@pytest.mark.parametrize("q", QS)
def test_mod_reduce_matches_python(q):
    rng = random.Random(q & 0xFFFF)
    W = -(-q.bit_length() // 64)
    vals = [0, 1, q - 1, q, q + 1, q * q - 1, (1 << (64 * 4 * W)) - 1]
    vals += [rng.getrandbits(rng.randint(1, 64 * 4 * W)) for _ in range(300)]
    vals += [rng.randrange(q) * q + rng.randrange(3) for _ in range(50)]
    for x in vals:
        assert C.mod_reduce(x, q) == x % q, x


@pytest.mark.parametrize("q", QS)
@pytest.mark.parametrize("m", [2, 4, 16, 32])
def test_ring_mul_matches_definition_and_ks(q, m):
    rng = random.Random(q * 31 + m)
    L = _lw(q)
    edge = [0, 1, q - 1]
    for trial in range(4):
        x = [rng.choice(edge) if trial == 0 else rng.randrange(q) for _ in range(m)]
        y = [rng.choice(edge) if trial == 1 else rng.randrange(q) for _ in range(m)]
        ref = brute.ring_mul(x, y, q)
        assert C.ring_mul(x, y, m, L, q) == ref
        assert brute.ring_mul_ks(x, y, q) == ref
        assert C.ring_mul(y, x, m, L, q) == ref          # commutative


@pytest.mark.parametrize("q", [193, 81 * 2 ** 121 + 1, (3 * 2 ** 30 + 1) ** 4])
@pytest.mark.parametrize("m", [2, 8, 16])
def test_rotation_is_product_with_monomial(q, m):
    rng = random.Random(m + q % 1000)
    L = _lw(q)
    x = [rng.randrange(q) for _ in range(m)]
    x[0] = 0                                          # a zero coefficient must stay 0 when negated
    for e in list(range(0, 2 * m + 3)) + [-1, -m - 1, 5 * m + 1]:
        assert C.ring_rotate(x, e, m, L, q) == brute.ring_mul(x, brute.alpha_pow(e, m, q), q)


def _setup(log2_M, log2_m, p, z):
    h, n = p - 1, 0
    while h % 2 == 0:
        h //= 2
        n += 1
    q = p ** z
    g = P.generator(p, h, n)
    om = P.principal_root(P.hensel_lift(g, p, z), p, z, log2_M)
    M, m = 1 << log2_M, 1 << log2_m
    return q, P.rho_lagrange(om, m, M // m, q), M, m


FFT_CASES = [
    (1, 1, 17, 3),          # 2M = 4 = 2m: only the base case
    (2, 2, 17, 3),          # 2M = 8 = 2m
    (3, 2, 97, 2),          # 2M = 16 = 2m * 2
    (4, 2, 193, 1),         # 2M = 32 = (2m)^2 * 2: two levels + base case
    (5, 2, 193, 2),         # 2M = 64 = (2m)^3
    (5, 3, 3 * 2 ** 30 + 1, 2),
    (6, 2, 3 * 2 ** 30 + 1, 1),
]


@pytest.mark.parametrize("log2_M,log2_m,p,z", FFT_CASES)
def test_fft_matches_naive_dft(log2_M, log2_m, p, z):
    q, rho, M, m = _setup(log2_M, log2_m, p, z)
    L = _lw(q)
    rng = random.Random(log2_M * 7 + log2_m)
    a = [[rng.randrange(q) for _ in range(m)] for _ in range(2 * M)]
    flat = np.concatenate([C.coeffs_to_limbs(e, L) for e in a])
    got = C.limbs_to_coeffs(C.fft(flat, 2 * M, m, L, q, rho), L)
    ref = brute.naive_dft(a, rho, q)
    assert [got[i * m:(i + 1) * m] for i in range(2 * M)] == ref


@pytest.mark.parametrize("log2_M,log2_m,p,z", FFT_CASES)
def test_fft_twice_is_scaled_reversal(log2_M, log2_m, p, z):
    """DFT(DFT(a))_l = 2M a_((-l) mod 2M) (Sec. 2.7)."""
    q, rho, M, m = _setup(log2_M, log2_m, p, z)
    L = _lw(q)
    rng = random.Random(log2_M * 5 + log2_m)
    a = [[rng.randrange(q) for _ in range(m)] for _ in range(2 * M)]
    flat = np.concatenate([C.coeffs_to_limbs(e, L) for e in a])
    twice = C.limbs_to_coeffs(C.fft(C.fft(flat, 2 * M, m, L, q, rho), 2 * M, m, L, q, rho), L)
    for l in range(2 * M):
        assert twice[l * m:(l + 1) * m] == [(2 * M * c) % q for c in a[(-l) % (2 * M)]]


def test_rho_power_table():
    q, rho, M, m = _setup(5, 2, 193, 2)
    L = _lw(q)
    tab = C.limbs_to_coeffs(C.rho_powers(M // m, m, L, q, rho), L)
    for s in range(M // m):
        assert tab[s * m:(s + 1) * m] == brute.ring_pow(rho, s, q)


@pytest.mark.parametrize("M,m,u", [(4, 4, 5), (8, 2, 32), (8, 4, 57), (4, 8, 64), (16, 4, 20)])
def test_encode_matches_definition(M, m, u):
    rng = random.Random(M * m + u)
    nbits = M * m // 2 * u
    for x in [rng.getrandbits(nbits), (1 << nbits) - 1, 1, 0, 1 << (nbits - 1)]:
        n = max(1, -(-nbits // 32))
        L = max(1, -(-u // 32))
        got = C.limbs_to_coeffs(C.encode(C.to_limbs(x, n), M, m, L, u), L)
        ref = brute.encode(x, M, m, u)
        assert [got[i * m:(i + 1) * m] for i in range(2 * M)] == ref


def test_product_coefficients_are_exact():
    """After the inverse transform and 1/2M, each inner coefficient equals the coefficient of the
    product of the encoded polynomials over Z[alpha][x] (no wrap, all below q; Sec. 3.2.2)."""
    pr = P.Params(N=256, log2_M=3, log2_m=2, u=16, p_bits=40, z=1)
    S = P.setup(pr)
    q, M, m, u, L = S.q, pr.M, pr.m, pr.u, S.L
    rng = random.Random(5)
    x, y = rng.getrandbits(256), rng.getrandbits(256)
    ea, eb = brute.encode(x, M, m, u), brute.encode(y, M, m, u)
    fa = C.fft(np.concatenate([C.coeffs_to_limbs(e, L) for e in ea]), 2 * M, m, L, q, S.rho)
    fb = C.fft(np.concatenate([C.coeffs_to_limbs(e, L) for e in eb]), 2 * M, m, L, q, S.rho)
    cc = C.limbs_to_coeffs(C.fft(C.pointwise(fa, fb, 2 * M, m, L, q), 2 * M, m, L, q, S.rho), L)
    inv = pow(2 * M, -1, q)
    exact = brute.poly_product_over_Z([e[:m] for e in ea[:M]], [e[:m] for e in eb[:M]])
    for l in range(2 * M):
        got = [inv * c % q for c in cc[((-l) % (2 * M)) * m:((-l) % (2 * M) + 1) * m]]
        want = (exact[l] + [0] * m)[:m] if l < len(exact) else [0] * m
        assert all(v == 0 for v in (exact[l][m:] if l < len(exact) else []))
        assert got == want


def test_schoolbook_matches_python():
    rng = random.Random(1)
    for alen, blen in [(1, 1), (1, 7), (13, 5), (64, 64), (100, 3)]:
        a = SI.limbs(rng.getrandbits(32), alen)
        b = SI.limbs(rng.getrandbits(32), blen)
        c = C.schoolbook(a, b)
        assert C.from_limbs(c) == C.from_limbs(a) * C.from_limbs(b)
    c = C.schoolbook(SI.all_ones(40), SI.all_ones(40))
    assert C.from_limbs(c) == (2 ** 1280 - 1) ** 2


def test_residue_matches_python():
    a = SI.limbs(3, 1000)
    x = C.from_limbs(a)
    for q in [3, 2 ** 61 - 1, 2305843009213693951, 1000000007]:
        assert C.residue(a, q) == x % q


SMALL_MUL = [(1, 1), (2, 1), (7, 7), (64, 64), (256, 32), (300, 299), (1024, 128)]


@pytest.mark.parametrize("alen,blen", SMALL_MUL)
def test_dkss_mul_matches_python(alen, blen):
    a, b = SI.operand_pair(alen * 1000 + blen, alen, blen)
    c = C.dkss_mul(a, b)
    assert C.from_limbs(c) == C.from_limbs(a) * C.from_limbs(b)


@pytest.mark.parametrize("kind", ["ones", "pow2", "square", "zero_high"])
def test_dkss_mul_edge_operands(kind):
    n = 512
    if kind == "ones":
        a, b = SI.all_ones(n), SI.all_ones(n)
    elif kind == "pow2":
        a, b = SI.power_of_two(n * 32 - 1, n), SI.power_of_two(77, n)
    elif kind == "square":
        a = SI.limbs(9, n)
        b = a
    else:
        a, b = SI.operand_pair(4, n, n)
        a[n // 2:] = 0
    c = C.dkss_mul(a, b)
    assert C.from_limbs(c) == C.from_limbs(a) * C.from_limbs(b)


def test_dkss_mul_favorable_length_all_ones():
    """3648 64-bit words (7296 limbs): u = 57 and Mm 2^(2u) = 2^127 meets the bound exactly."""
    a = SI.all_ones(7296)
    c = C.dkss_mul(a, a)
    assert np.array_equal(c, C.schoolbook(a, a))


@pytest.mark.parametrize("log2_M,log2_m,u,p_bits,z", [(4, 2, 8, 32, 1), (4, 3, 12, 32, 2),
                                                      (5, 2, 24, 32, 4), (3, 3, 40, 64, 2)])
def test_dkss_mul_other_moduli(log2_M, log2_m, u, p_bits, z):
    """z > 1 (Hensel-lifted roots) and non-rule parameter tuples give the same exact product."""
    pr = P.Params(N=0, log2_M=log2_M, log2_m=log2_m, u=u, p_bits=p_bits, z=z)
    S = P.setup(pr)
    cap = pr.M * pr.m // 2 * u // 32
    a, b = SI.operand_pair(u, cap, max(1, cap // 3))
    c = C.dkss_mul(a, b, S)
    assert C.from_limbs(c) == C.from_limbs(a) * C.from_limbs(b)


def _planted_setup(good, p_bits):
    """Steps 2-3 of Sec. 3.2 for good's M, m, u but a prime of p_bits bits, without the check
    p^z >= Mm 2^(2u): the mistake a wrong parameter tuple would make."""
    prm = P.Params(N=good.N, log2_M=good.log2_M, log2_m=good.log2_m, u=good.u, p_bits=p_bits, z=1)
    p, h, n = P.proth_prime(p_bits, prm.log2_M + 1)
    zeta = P.generator(p, h, n)
    omega = P.principal_root(P.hensel_lift(zeta, p, 1), p, 1, prm.log2_M)
    rho = P.rho_lagrange(omega, prm.m, prm.mu, p)
    return P.Setup(params=prm, p=p, h=h, n=n, q=p, zeta=zeta, zeta_z=zeta, omega=omega, rho=rho)


def test_residue_check_catches_planted_mistakes():
    """The verifier's check (residues modulo 61-bit primes, as dkss_residues computes them on the
    GPU) accepts the exact product and rejects: the product of a DKSS run whose modulus is below
    the bound of Sec. 3.2.2 (coefficient sums wrap), and single-limb corruptions of the exact
    product."""
    alen = blen = 256
    a, b = SI.all_ones(alen), SI.all_ones(blen)
    exact = C.schoolbook(a, b)
    rng = random.Random(77)
    primes = []
    while len(primes) < 8:
        q = rng.getrandbits(61) | (1 << 60) | 1
        if all(pow(w, q - 1, q) == 1 for w in (2, 3, 5, 7, 11, 13)):
            primes.append(q)

    def passes(c):
        return all(C.residue(c, q) == C.residue(a, q) * C.residue(b, q) % q for q in primes)

    assert passes(exact)
    good = P.thesis_rule(32 * alen)
    bad = _planted_setup(good, good.p_bits // 2)
    assert bad.q < 1 << (good.log2_M + good.log2_m + 2 * good.u)
    wrong = C.dkss_mul(a, b, setup=bad)
    assert not np.array_equal(wrong, exact) and not passes(wrong)
    for _ in range(20):
        c = exact.copy()
        i = rng.randrange(len(c))
        c[i] ^= np.uint32(1 << rng.randrange(32))
        assert not passes(c), i
