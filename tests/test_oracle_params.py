"""Pins of the oracle's parameter rule and ring constants (oracle.params) against the thesis's
printed numbers and against number-theoretic facts."""
import math
import random

import pytest

from conftest import golden_rows
from oracle import brute
from oracle import params as P


def _mr_probable_prime(n, bases=(2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)):
    """Miller-Rabin, independent of the oracle's Proth test."""
    if n < 2:
        return False
    for b in bases:
        if n % b == 0:
            return n == b
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in bases:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def _memory_model(pr):
    """DKSS_MUL memory as the thesis's allocation pattern implies (Sec. 4.2 listing, Sec. 4.5):
    two polynomials of 2M elements, the mu precomputed rho powers, per recursion level of the
    FFT a temporary of (2M' + 2m + 1) elements, the base case's one element, plus one element."""
    E = pr.m * pr.p_bits // 8
    total = 2 * (2 * pr.M * E) + pr.mu * E
    n = 2 * pr.M
    while n > 2 * pr.m:
        total += n * E + 2 * pr.m * E + E
        n //= 2 * pr.m
    return total + E + E


@pytest.mark.parametrize("row", golden_rows("favorable_lengths.txt"), ids=lambda r: r[0])
def test_rule_reproduces_memory_table(row):
    words, mem = int(row[0]), int(row[1])
    pr = P.thesis_rule(64 * words)
    assert _memory_model(pr) == mem
    # at the favorable lengths the encoding fills every coefficient exactly
    assert pr.M * pr.m * pr.u // 2 == 64 * words


@pytest.mark.parametrize("row", golden_rows("profiled_lengths.txt"), ids=lambda r: r[0])
def test_rule_matches_profiled_m_and_coefficient_words(row):
    words, m, wpc = map(int, row)
    pr = P.thesis_rule(64 * words)
    assert pr.m == m
    assert pr.p_bits // 64 == wpc


@pytest.mark.parametrize("N", [32, 64, 1000, 2 ** 12, 2 ** 18, 2 ** 18 + 32, 233472, 2 ** 24,
                               2 ** 28, 2 ** 30, 2 ** 34])
def test_rule_is_feasible(N):
    pr = P.thesis_rule(N)
    assert pr.m >= 2 and pr.M >= pr.m
    assert pr.M * pr.m * pr.u >= 2 * N                       # capacity (Sec. 3.2 Step 2)
    assert pr.log2_M + pr.log2_m + 2 * pr.u <= pr.p_bits - 1  # p^z >= Mm 2^(2u), p >= 2^(b-1)
    assert pr.p_bits % 64 == 0


def test_rule_stair_step():
    """One limb past a favorable length needs about twice the coefficients (Sec. 4.5)."""
    a = P.thesis_rule(64 * 3648)
    b = P.thesis_rule(64 * 3648 + 32)
    assert (b.M * b.m) == 2 * (a.M * a.m) or b.u > a.u


@pytest.mark.parametrize("row", golden_rows("qmul_primes.txt"), ids=lambda r: r[0])
def test_qmul_table_primes_generators_roots(row):
    bits, p, h, n, g, lg, w = map(int, row)
    assert p == h * 2 ** n + 1 and p.bit_length() == bits
    assert P.is_prime_proth(h, n)
    assert P.generator(p, h, n) == g
    assert pow(g, (p - 1) >> lg, p) == w
    assert pow(w, 1 << lg, p) == 1 and pow(w, 1 << (lg - 1), p) == p - 1


@pytest.mark.parametrize("bits", range(3, 25))
def test_proth_search_matches_trial_division(bits):
    """Smallest odd h such that h*2^n + 1 (n = bits - bitlen(h)) is prime, by trial division."""
    h = 1
    while True:
        n = bits - h.bit_length()
        if n < 1:
            pytest.skip("no such prime")
        cand = h * 2 ** n + 1
        if all(cand % d for d in range(2, math.isqrt(cand) + 1)):
            break
        h += 2
    assert P.proth_prime(bits) == (cand, h, n)


@pytest.mark.parametrize("bits,expect_h", [(64, 27), (128, 81), (192, 13), (256, None)])
def test_proth_large(bits, expect_h):
    p, h, n = P.proth_prime(bits)
    if expect_h is not None:
        assert h == expect_h
    assert p.bit_length() == bits and n == bits - h.bit_length()
    assert _mr_probable_prime(p)
    for hh in range(1, h, 2):
        nn = bits - hh.bit_length()
        assert not _mr_probable_prime(hh * 2 ** nn + 1)


@pytest.mark.parametrize("p,z", [(17, 3), (193, 2), (3 * 2 ** 30 + 1, 4), (97, 5)])
def test_hensel_lift(p, z):
    h = p - 1
    n = 0
    while h % 2 == 0:
        h //= 2
        n += 1
    g = P.generator(p, h, n)
    q = p ** z
    zz = P.hensel_lift(g, p, z)
    assert zz % p == g
    assert pow(zz, p - 1, q) == 1
    # the unique (p-1)-th root of unity above g is g^(p^(z-1)) (Teichmueller lift)
    assert zz == pow(g, p ** (z - 1), q)


def _small_setup(log2_M, log2_m, p, z):
    h, n = p - 1, 0
    while h % 2 == 0:
        h //= 2
        n += 1
    q = p ** z
    g = P.generator(p, h, n)
    om = P.principal_root(P.hensel_lift(g, p, z), p, z, log2_M)
    M, m = 1 << log2_M, 1 << log2_m
    rho = P.rho_lagrange(om, m, M // m, q)
    return q, om, rho, M, m


@pytest.mark.parametrize("log2_M,log2_m,p,z", [(3, 2, 17, 3), (4, 2, 97, 2), (4, 3, 193, 1),
                                               (5, 2, 193, 2), (6, 3, 3 * 2 ** 30 + 1, 2)])
def test_omega_and_rho(log2_M, log2_m, p, z):
    q, om, rho, M, m = _small_setup(log2_M, log2_m, p, z)
    n2 = 2 * M
    assert pow(om, n2, q) == 1 and pow(om, M, q) == q - 1
    for j in range(1, n2):                      # principal (Sec. 3.2.2 definition)
        assert sum(pow(om, i * j, q) for i in range(n2)) % q == 0
    mu = M // m
    one = [1] + [0] * (m - 1)
    assert brute.ring_pow(rho, mu, q) == brute.alpha_pow(1, m, q)    # rho^(2M/2m) = alpha
    assert brute.ring_pow(rho, M, q) == [(q - 1)] + [0] * (m - 1)
    assert brute.ring_pow(rho, n2, q) == one
    for j in range(1, n2):                      # principal in R
        acc = [0] * m
        for i in range(n2):
            acc = [(a + b) % q for a, b in zip(acc, brute.ring_pow(rho, i * j, q))]
        assert acc == [0] * m
    # inverse negacyclic transform of (omega, omega^3, ..., omega^(2m-1))
    gam = pow(om, mu, q)
    inv_m = pow(m, -1, q)
    closed = [inv_m * sum(pow(om, 2 * t + 1, q) * pow(gam, -(2 * t + 1) * k, q)
                          for t in range(m)) % q for k in range(m)]
    assert rho == closed


def test_setup_thesis_prime():
    S = P.setup(P.thesis_rule(2 ** 18))
    assert S.p == 81 * 2 ** 121 + 1 and S.zeta == 5 and S.q == S.p
    S = P.setup(P.thesis_rule(2 ** 28))
    assert S.p == 13 * 2 ** 188 + 1 and S.zeta == 3


def test_setup_rejects_infeasible():
    pr = P.thesis_rule(2 ** 18)
    pr.u += 40
    with pytest.raises(ValueError):
        P.setup(pr)
