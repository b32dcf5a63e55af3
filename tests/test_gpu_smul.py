"""GPU parity tests of SMUL (Schoenhage-Strassen multiplication, thesis Sec. 2.9) through the C ABI
against the SMUL oracle (oracle/smul.py) and Python integers: the forward transform element by
element (natural order, values in [0, 2^K], including the value 2^K), products bit-exact at many
(FFT length, ring size) pairs and edge operands, the 2^24-bit product against the oracle's SMUL
at the same parameters, and the 2^28-bit products against the stored digests of the oracle's
DKSS products (a product is the same integer whichever method computes it)."""
import numpy as np
import pytest

import seeded_inputs as SI
from conftest import golden_rows, host_residues, primes61, residues_agree, sha256_limbs
from oracle import coracle as C
from oracle import smul as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1503_04955_amd as dk
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dk.lib()
    return dk, torch


def _int(limbs):
    return int.from_bytes(np.ascontiguousarray(limbs, dtype=np.uint32).astype("<u4").tobytes(), "little")


def _limbs(x, n):
    return np.frombuffer(x.to_bytes(4 * n, "little"), dtype=np.uint32)


def _bitrev(i, bits):
    r = 0
    for _ in range(bits):
        r = (r << 1) | (i & 1)
        i >>= 1
    return r


def _feasible(alen, blen, log2_n, lw):
    """The library's feasibility rule, restated: s = ceil(32 (alen + blen) / n), na + nb - 1 <= n,
    2s + ceil(log2 min(na, nb)) <= K = 2048 lw, n | 2K."""
    n, K = 1 << log2_n, 2048 * lw
    if (2 * K) % n:
        return None
    s = -(-32 * (alen + blen) // n)
    if s > K:
        return None
    na, nb = max(1, -(-32 * alen // s)), max(1, -(-32 * blen // s))
    if na + nb - 1 > n:
        return None
    lg = (min(na, nb) - 1).bit_length()
    if 2 * s + lg > K:
        return None
    return s, K


def _smul(env, a, b, params=None, square=False):
    dk, torch = env
    da = dk.to_device(a)
    db = da if square else dk.to_device(b)
    c = dk.smul(da, db, params=params)
    torch.cuda.synchronize()
    return dk.to_host(c)


FWD = [  # (alen, blen, log2_n, lw)
    (64, 64, 4, 1), (64, 64, 6, 1), (64, 64, 8, 1), (300, 200, 10, 1), (300, 200, 9, 2),
    (1000, 900, 11, 4), (2000, 100, 12, 2), (40, 40, 3, 8),
]


@pytest.mark.parametrize("case", FWD, ids=lambda c: "%dx%d_n%d_lw%d" % c)
def test_smul_forward_matches_oracle(env, case):
    """The forward transform (bit-reversed on the device) equals the oracle's evaluation at the
    powers of omega = 2^(2K/n), element by element, with tops marking the value 2^K."""
    dk, torch = env
    alen, blen, log2_n, lw = case
    s, K = _feasible(alen, blen, log2_n, lw)
    a = SI.limbs(SI.SEED_BASE + 700 + log2_n, alen)
    poly, tops = dk.smul_forward(dk.to_device(a), alen, blen, dk.SmulParams.make(log2_n, lw))
    torch.cuda.synchronize()
    P = poly.cpu().numpy().view(np.uint32)
    T = tops.cpu().numpy()
    want = S.forward(_int(a), s, log2_n, K)
    for i in range(1 << log2_n):
        j = _bitrev(i, log2_n)
        got = (int(T[j]) << K) + _int(P[j])
        assert got == want[i], (i, j)


def test_smul_forward_value_two_to_the_K(env):
    """An operand whose two lowest coefficients are x and x + 1 evaluates to x - (x + 1) = -1 =
    2^K at omega^(n/2): the transform marks it with its top."""
    dk, torch = env
    alen, blen, log2_n, lw = 64, 64, 6, 1
    s, K = _feasible(alen, blen, log2_n, lw)
    x = 123456789
    v = x + ((x + 1) << s)
    a = _limbs(v, alen)
    poly, tops = dk.smul_forward(dk.to_device(a), alen, blen, dk.SmulParams.make(log2_n, lw))
    torch.cuda.synchronize()
    T = tops.cpu().numpy()
    want = S.forward(v, s, log2_n, K)
    assert want[1 << (log2_n - 1)] == 1 << K
    j = _bitrev(1 << (log2_n - 1), log2_n)
    assert T[j] == 1 and not poly.cpu().numpy()[j].any()


MUL = [  # (alen, blen, log2_n or 0, lw or 0)
    (1, 1, 0, 0), (2, 3, 0, 0), (17, 33, 0, 0), (100, 100, 0, 0), (257, 31, 0, 0),
    (1000, 1000, 0, 0), (4096, 4096, 0, 0), (8192, 8192, 0, 0), (20000, 3000, 0, 0),
    (64, 64, 4, 1), (64, 64, 7, 1), (64, 64, 8, 2), (500, 500, 6, 4), (500, 500, 5, 8),
    (3000, 3000, 9, 8), (3000, 3000, 8, 16), (3000, 3000, 7, 32), (12000, 11000, 10, 16),
]


@pytest.mark.parametrize("case", MUL, ids=lambda c: "%dx%d_n%d_lw%d" % c)
def test_smul_products_match_oracle(env, case):
    dk, torch = env
    alen, blen, log2_n, lw = case
    params = dk.SmulParams.make(log2_n, lw) if log2_n else None
    if log2_n:
        assert _feasible(alen, blen, log2_n, lw)
    a, b = SI.operand_pair(SI.SEED_BASE + 710 + alen, alen, blen)
    got = _smul(env, a, b, params)
    assert np.array_equal(got, C.schoolbook(a, b))


PRODUCTS = [  # (alen, blen, log2_n, lw): rings where both forms of the componentwise products run
    (64, 64, 4, 1), (300, 200, 9, 2), (500, 500, 6, 4), (3000, 3000, 9, 8), (3000, 3000, 8, 16),
    (12000, 11000, 10, 16), (20000, 3000, 11, 8),
]


@pytest.mark.parametrize("products", [1, 2])
@pytest.mark.parametrize("case", PRODUCTS, ids=lambda c: "%dx%d_n%d_lw%d" % c)
def test_smul_componentwise_products_both_forms(env, case, products):
    """The componentwise products by 28-bit digits on the vector units (1) and by exact 8-bit
    products on the matrix cores (2) give the product bit for bit: random and all-ones factors
    (every byte column at its largest sum) against the oracle's schoolbook."""
    dk, torch = env
    alen, blen, log2_n, lw = case
    params = dk.SmulParams.make(log2_n, lw, products)
    a, b = SI.operand_pair(SI.SEED_BASE + 740 + alen, alen, blen)
    got = _smul(env, a, b, params)
    assert np.array_equal(got, C.schoolbook(a, b))
    ones_a = np.full(alen, 0xFFFFFFFF, dtype=np.uint32)
    ones_b = np.full(blen, 0xFFFFFFFF, dtype=np.uint32)
    assert _int(_smul(env, ones_a, ones_b, params)) == _int(ones_a) * _int(ones_b)
    assert _int(_smul(env, ones_a, ones_a, params, square=True)) == _int(ones_a) ** 2


def test_smul_products_form_reported(env):
    """The parameters report the form of the products: the library's choice at 2^24 and 2^28 bits
    is the matrix cores (the faster form there), and asking for them beyond lw = 16 is refused."""
    dk, torch = env
    for n in (1 << 19, 1 << 23):
        p = dk.smul_select(n, n)
        assert p.products == 2 and p.lw <= 16, n
    a = dk.to_device(SI.limbs(SI.SEED_BASE + 750, 4096))
    with pytest.raises(dk.DkssError) as e:
        dk.smul(a, a, params=dk.SmulParams.make(0, 32, 2))
    assert e.value.code == dk.ERANGE


@pytest.mark.parametrize("n", [64, 3000, 32768])
@pytest.mark.parametrize("kind", ["ones", "ones_unbalanced", "pow2", "square", "coeff_minus_one"])
def test_smul_edge_operands(env, n, kind):
    """All-ones factors (the largest convolution sums), 8:1 all-ones, powers of two, a squaring
    (one transform), and operands whose transforms hold the value 2^K (componentwise products of
    -1 with -1 and with other values)."""
    dk, torch = env
    square = False
    if kind == "ones":
        x, y, na, nb = (1 << (32 * n)) - 1, (1 << (32 * n)) - 1, n, n
    elif kind == "ones_unbalanced":
        nb = max(1, n // 8)
        x, y, na = (1 << (32 * n)) - 1, (1 << (32 * nb)) - 1, n
    elif kind == "pow2":
        nb = max(1, n // 3)
        x, y, na = 1 << (32 * n - 1), 1 << (16 * nb + 5), n
    elif kind == "square":
        na = nb = n
        x = _int(SI.limbs(SI.SEED_BASE + 720 + n, n))
        y = x
        square = True
    else:
        # the library's ring, an FFT length at which two coefficients fit the operand
        na = nb = n
        sel = dk.smul_select(na, nb)
        lg = next(g for g in range(2, 25) if _feasible(na, nb, g, sel.lw) and
                  _feasible(na, nb, g, sel.lw)[0] * 2 + 4 <= 32 * n)
        params = dk.SmulParams.make(lg, sel.lw)
        s = _feasible(na, nb, lg, sel.lw)[0]
        x = 5 + (6 << s)
        y = 7 + (8 << s)
    a, b = _limbs(x, na), _limbs(y, nb)
    got = _smul(env, a, b, params=params if kind == "coeff_minus_one" else None, square=square)
    assert _int(got) == x * y
    if kind == "coeff_minus_one":
        assert _int(_smul(env, a, a, params=params, square=True)) == x * x


def test_smul_zero_lengths(env):
    dk, torch = env
    a = dk.to_device(SI.limbs(SI.SEED_BASE + 730, 5))
    b = torch.empty(0, dtype=torch.int32, device="cuda")
    out = torch.full((5,), -1, dtype=torch.int32, device="cuda")
    dk.smul(a, b, out=out, ws=torch.empty(256, dtype=torch.uint8, device="cuda"))
    torch.cuda.synchronize()
    assert bool((out == 0).all())


def test_smul_rejects_infeasible_params(env):
    dk, torch = env
    a = dk.to_device(SI.limbs(SI.SEED_BASE + 731, 100))
    with pytest.raises(dk.DkssError) as e:
        dk.smul(a, a, params=dk.SmulParams.make(2, 1))      # 4 coefficients cannot hold 6400 bits
    assert e.value.code == dk.ERANGE


def test_smul_2e24_matches_oracle_smul(env):
    """The 2^24-bit product at the library's parameters equals the oracle's SMUL at the same
    (n, s, K), and residues mod 8 primes."""
    dk, torch = env
    n = 1 << 19
    a, b = SI.operand_pair(SI.SEED_BASE + 1, n, n)
    p = dk.smul_select(n, n)
    print("2^24 smul params", p.as_dict(), flush=True)
    got = _smul(env, a, b)
    want = S.smul_full(_int(a), _int(b), p.log2_n, s=p.s, K=p.K)
    assert _int(got) == want
    qs = primes61(24, 8)
    ra, rb, rc = host_residues([a, b, got], qs)
    assert residues_agree(ra, rb, rc, qs)


@pytest.mark.parametrize("name", ["2p28_random", "2p28_square", "2p28_unbalanced"])
def test_smul_2e28_matches_stored_products(env, name):
    """2^28-bit products by SMUL equal the stored SHA-256 of the CPU oracle's DKSS products of the
    same operands (one integer, whichever method computes it), and residues mod 4 primes."""
    rows = {r[0]: r for r in golden_rows("dkss_digests.txt")}
    _, seed, alen, blen, square, want = rows[name]
    seed, alen, blen, square = int(seed), int(alen), int(blen), int(square)
    if square:
        a = SI.limbs(seed, alen)
        b = a
    else:
        a, b = SI.operand_pair(seed, alen, blen)
    print("smul case", name, flush=True)
    got = _smul(env, a, b, square=bool(square))
    assert sha256_limbs(got) == want
    qs = primes61(28, 4)
    ra, rb, rc = host_residues([a, b, got], qs)
    assert residues_agree(ra, rb, rc, qs)
