"""Pins of the SMUL oracle (oracle/smul.py, thesis Sec. 2.9) against what the mathematics fixes:
the order of 2 modulo 2^K + 1, principal roots and the invertibility conditions of Sec. 2.9.1
by brute force, the transform against the naive DFT, the inverse, the convolution theorem and
the negacyclic weighting of Sec. 2.9.2 against convolutions by their definitions, and whole
products against Python's integer multiplication (a*b and a*b mod 2^N + 1)."""
import math
import random

import pytest

import seeded_inputs as SI
from oracle import smul as S


def _naive_dft(a, w_shift, K):
    F = (1 << K) + 1
    n = len(a)
    w = pow(2, w_shift, F)
    return [sum(a[j] * pow(w, i * j, F) for j in range(n)) % F for i in range(n)]


def _cyclic(a, b, F):
    n = len(a)
    return [sum(a[i] * b[(k - i) % n] for i in range(n)) % F for k in range(n)]


def _negacyclic(a, b):
    n = len(a)
    out = []
    for k in range(n):
        v = 0
        for i in range(n):
            j = k - i
            v += a[i] * b[j] if j >= 0 else -a[i] * b[j + n]
        out.append(v)
    return out


@pytest.mark.parametrize("K", [1, 2, 3, 5, 8, 12, 16, 24])
def test_two_has_order_2K(K):
    """Sec. 2.9: 2^K = -1 and 2 is a primitive 2K-th root of unity mod 2^K + 1."""
    F = (1 << K) + 1
    assert S.fermat_shift(1, K, K) == F - 1
    order = next(e for e in range(1, 4 * K + 1) if pow(2, e, F) == 1)
    assert order == 2 * K


@pytest.mark.parametrize("K,n", [(8, 2), (8, 4), (8, 16), (12, 8), (12, 24 // 3), (24, 16), (32, 64), (20, 8)])
def test_omega_principal_and_invertible(K, n):
    """omega = 2^(2K/n) is a principal n-th root (omega^(n/2) = -1, power sums vanish), and the
    conditions of Sec. 2.9.1 hold by brute force: omega^j - 1 (0 < j < n) and n are units."""
    F = (1 << K) + 1
    w = pow(2, S.omega_shift(n, K), F)
    assert pow(w, n, F) == 1 and pow(w, n // 2, F) == F - 1
    for j in range(1, n):
        assert sum(pow(w, i * j, F) for i in range(n)) % F == 0
        assert math.gcd((pow(w, j, F) - 1) % F, F) == 1
    assert math.gcd(n, F) == 1


def test_fermat_shift_inverse_and_composition():
    rng = random.Random(5)
    for K in (7, 32, 100, 2048):
        F = (1 << K) + 1
        for _ in range(20):
            x = rng.randrange(F)
            t, u = rng.randrange(2 * K), rng.randrange(2 * K)
            assert S.fermat_shift(S.fermat_shift(x, t, K), 2 * K - t, K) == x
            assert S.fermat_shift(S.fermat_shift(x, t, K), u, K) == S.fermat_shift(x, t + u, K)
            assert S.fermat_shift(x, t, K) == x * (1 << t) % F


@pytest.mark.parametrize("K,log2_n", [(8, 3), (16, 4), (64, 5), (96, 6), (2048, 4)])
def test_transform_is_the_dft_and_inverts(K, log2_n):
    """transform(a)[i] = sum_j a_j omega^(ij) (definition); the transform at omega^-1 of the
    transform is n times the input (Sec. 2.7)."""
    n = 1 << log2_n
    F = (1 << K) + 1
    rng = random.Random(K + log2_n)
    a = [rng.randrange(F) for _ in range(n)]
    a[0] = F - 1                                 # the value 2^K
    w = S.omega_shift(n, K)
    fa = S.transform(a, w, K)
    assert fa == _naive_dft(a, w, K)
    back = S.transform(fa, 2 * K - w, K)
    assert back == [x * n % F for x in a]


@pytest.mark.parametrize("K,log2_n", [(16, 3), (40, 3), (64, 4)])
def test_convolution_theorem(K, log2_n):
    """The transform of the cyclic convolution (Eq. (cycconv)) is the pointwise product of the
    transforms."""
    n = 1 << log2_n
    F = (1 << K) + 1
    rng = random.Random(3 * K)
    a = [rng.randrange(F) for _ in range(n)]
    b = [rng.randrange(F) for _ in range(n)]
    w = S.omega_shift(n, K)
    lhs = S.transform(_cyclic(a, b, F), w, K)
    rhs = [x * y % F for x, y in zip(S.transform(a, w, K), S.transform(b, w, K))]
    assert lhs == rhs


@pytest.mark.parametrize("K,log2_n", [(16, 2), (32, 3), (64, 4)])
def test_weights_give_the_negacyclic_convolution(K, log2_n):
    """Sec. 2.9.2, Eq. (weightresult): weighting by theta^i, convolving cyclically and
    counterweighting by theta^-k gives the negacyclic convolution (Eq. (ncycconv))."""
    n = 1 << log2_n
    F = (1 << K) + 1
    rng = random.Random(K * 7 + log2_n)
    s = (K - log2_n - 1) // 2
    a = [rng.randrange(1 << s) for _ in range(n)]
    b = [rng.randrange(1 << s) for _ in range(n)]
    th = S.theta_shift(n, K)
    assert S.fermat_shift(1, th * n, K) == F - 1           # theta^n = -1
    wa = [S.fermat_shift(x, th * i, K) for i, x in enumerate(a)]
    wb = [S.fermat_shift(x, th * i, K) for i, x in enumerate(b)]
    cyc = _cyclic(wa, wb, F)
    got = [S.fermat_shift(c, -th * k, K) for k, c in enumerate(cyc)]
    want = [v % F for v in _negacyclic(a, b)]
    assert got == want


MOD_CASES = [(64, 2), (64, 4), (256, 4), (1024, 5), (4096, 6), (6144, 6)]


@pytest.mark.parametrize("N,log2_n", MOD_CASES)
def test_smul_mod_matches_python(N, log2_n):
    """The whole procedure (Steps 1-11) gives a*b mod 2^N + 1, including the operand 2^N."""
    rng = random.Random(N + 97 * log2_n)
    FN = (1 << N) + 1
    vals = [0, 1, 2, FN - 2, FN - 1, (1 << N) - 1, 1 << (N // 2)]
    pairs = [(x, y) for x in vals for y in vals[:4]]
    pairs += [(rng.randrange(FN), rng.randrange(FN)) for _ in range(12)]
    for a, b in pairs:
        assert S.smul_mod(a, b, N, log2_n) == a * b % FN, (a, b)


def _rand_int(rng, bits):
    return rng.getrandbits(bits) | (1 << (bits - 1))


@pytest.mark.parametrize("bits", [64, 1000, 8192, 32768])
def test_smul_full_matches_python(bits):
    """The outermost SMUL gives the full product a*b at every feasible FFT length, for random
    operands, all-ones (the largest convolution sums), powers of two, 8:1 lengths and squares."""
    rng = random.Random(bits)
    ops = [(_rand_int(rng, bits), _rand_int(rng, bits)),
           ((1 << bits) - 1, (1 << bits) - 1),
           (1 << (bits - 1), 1 << (bits // 3)),
           (_rand_int(rng, bits), _rand_int(rng, max(8, bits // 8))),
           ((1 << bits) - 1, (1 << max(8, bits // 8)) - 1)]
    x = _rand_int(rng, bits)
    ops.append((x, x))
    for log2_n in range(1, 12):
        for a, b in ops:
            p = S.outer_params(a.bit_length(), b.bit_length(), log2_n)
            if p is None:
                continue
            assert S.smul_full(a, b, log2_n) == a * b, (bits, log2_n)


def test_outer_params_bound_is_tight_enough():
    """The chosen K holds the largest sum of the all-ones operands, and K is a multiple of the
    word and of n/2 (n | 2K)."""
    for bits in (100, 4096, 65536):
        for log2_n in range(2, 14):
            p = S.outer_params(bits, bits, log2_n)
            if p is None:
                continue
            s, K = p
            n = 1 << log2_n
            assert K % 32 == 0 and (2 * K) % n == 0
            na = -(-bits // s)
            assert na * ((1 << s) - 1) ** 2 < (1 << K)


def test_smul_full_on_seeded_limbs():
    """Operands from the seeded splitmix64 stream (as the GPU tests draw them)."""
    a_l, b_l = SI.operand_pair(SI.SEED_BASE + 900, 300, 257)
    a = int.from_bytes(a_l.astype("<u4").tobytes(), "little")
    b = int.from_bytes(b_l.astype("<u4").tobytes(), "little")
    for log2_n in (5, 6, 7, 8):
        assert S.smul_full(a, b, log2_n) == a * b
