"""The bad multiplications in two forms (dkss_probe_twiddle_products): products by one twiddle t
of the 32 elements of a group, each with its own power of alpha, on the vector units (form 1) and
as one contraction of 7-bit digits on the matrix cores (form 2).  Both forms are compared word by
word with each other and, on samples, with the oracle's product in R (thesis Sec. 3.2.5 ii,
y = t alpha^r x) scaled by 2^(-28K) mod q, for every residue format of 3 to 6 limbs (tight and
whole-limb), with random odd moduli (the dense Montgomery steps) and the moduli of the library's
2^28-bit plans (primes h 2^n + 1: the sparse steps)."""
import numpy as np
import pytest

import seeded_inputs as SI
from oracle import coracle as C

pytestmark = pytest.mark.gpu

M = 16
GROUP = 32


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1503_04955_amd as dk
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dk.lib()
    return dk, torch


def _montgomery_steps(q, L):
    """K of q's residue format: the tight format (one 28-bit digit fewer than 32 L bits need) when
    q < 2^(28 D - 1), D = floor(32 L / 28); then K = ceil((qb + 6) / 28)."""
    d_tight = (32 * L) // 28
    qb = 28 * d_tight - 1 if q.bit_length() <= 28 * d_tight - 1 else 32 * L
    return (qb + 6 + 27) // 28


def _residues(seed, count, q, L):
    """count residues below 2^(bits(q) - 1) <= q from seeded words, as a (count, L) array."""
    w = SI.limbs(seed, count * L).reshape(count, L).copy()
    top = q.bit_length() - 1 - 32 * (L - 1)
    w[:, L - 1] &= np.uint32((1 << top) - 1) if top < 32 else np.uint32(0xFFFFFFFF)
    return w


def _int(row):
    return sum(int(v) << (32 * k) for k, v in enumerate(row))


def _random_q(seed, L, bits):
    w = SI.limbs(seed, L).copy()
    q = _int(w) & ((1 << bits) - 1)
    return q | (1 << (bits - 1)) | 1


def _case(dk, torch, q, L, groups, seed, edges=True):
    t = _residues(seed, groups * M, q, L)
    x = _residues(seed + 1, groups * GROUP * M, q, L)
    r = (SI.limbs(seed + 2, groups * GROUP) % (4 * M)).astype(np.uint32)   # taken mod 2m
    if edges:
        qm1 = np.array([(q - 1) >> (32 * k) & 0xFFFFFFFF for k in range(L)], np.uint32)
        x[0:M] = 0                                  # element 0: zero (its wrapped terms are q)
        x[M:2 * M] = qm1                            # element 1: q - 1 everywhere
        x[2 * M + 3] = 0
        t[0] = 0                                    # a zero coefficient of group 0's twiddle
        t[1] = qm1
        r[0:4] = [0, 16, 31, 32]
        if groups > 1:
            t[M:2 * M] = 0                          # group 1: the zero twiddle
    dev = lambda a: torch.from_numpy(a.view(np.int32)).cuda()
    tt, xx, rr = dev(t), dev(x), dev(r)
    ys = []
    for form in (1, 2):
        y = torch.full((groups * GROUP * M * L,), -1, dtype=torch.int32, device="cuda")
        dk.probe_twiddle_products(form, q, L, groups, tt, xx, rr, y)
        torch.cuda.synchronize()
        ys.append(y.cpu().numpy().view(np.uint32).reshape(groups, GROUP, M, L))
    return t.reshape(groups, M, L), x.reshape(groups, GROUP, M, L), r.reshape(groups, GROUP), ys


def _expect(t, x, rot, q, L):
    """oracle: alpha^rot (t x) in R, each coefficient times 2^(-28K) mod q"""
    K = _montgomery_steps(q, L)
    scale = pow(2, -28 * K, q)
    tv = [_int(c) for c in t]
    xv = [_int(c) for c in x]
    prod = C.ring_rotate(C.ring_mul(tv, xv, M, L, q), rot, M, L, q)
    return [v * scale % q for v in prod]


FORMATS = [(3, 83), (3, 96), (4, 111), (4, 128), (5, 139), (5, 160), (6, 167), (6, 192)]


@pytest.mark.parametrize("L,bits", FORMATS)
def test_twiddle_forms_random_modulus(env, L, bits):
    dk, torch = env
    q = _random_q(SI.SEED_BASE + 800 + bits, L, bits)
    t, x, r, (y1, y2) = _case(dk, torch, q, L, 3, SI.SEED_BASE + 810 + bits)
    assert np.array_equal(y1, y2)
    for g in range(3):
        for n in range(GROUP):
            got = [_int(c) for c in y2[g, n]]
            assert got == _expect(t[g], x[g, n], int(r[g, n]) % (2 * M), q, L), (g, n)


@pytest.mark.parametrize("policy", ["thesis", "learned"])
def test_twiddle_forms_plan_moduli(env, policy):
    """The moduli of the 2^28-bit plans (the sparse Montgomery steps), 2048 groups: the two forms
    equal everywhere, the oracle on a sample of elements."""
    dk, torch = env
    ctx = dk.Context(dk.POLICY_THESIS if policy == "thesis" else dk.POLICY_LEARNED)
    n = 1 << 23
    plan = ctx.plan_info(n, n)
    L = plan.L
    if plan.params.log2_m != 4 or L < 3 or L > 6:
        pytest.skip("plan outside the probe's shapes")
    q = _int(plan.q[:L])
    groups = 2048
    t, x, r, (y1, y2) = _case(dk, torch, q, L, groups, SI.SEED_BASE + 830 + L)
    assert np.array_equal(y1, y2)
    rng = np.random.default_rng(5)
    for g, e in [(0, 0), (0, 1), (1, 5), (groups - 1, GROUP - 1)] + \
            [(int(a), int(b)) for a, b in zip(rng.integers(0, groups, 12), rng.integers(0, GROUP, 12))]:
        got = [_int(c) for c in y2[g, e]]
        assert got == _expect(t[g], x[g, e], int(r[g, e]) % (2 * M), q, L), (g, e)


def test_twiddle_forms_errors(env):
    dk, torch = env
    q = _random_q(SI.SEED_BASE + 850, 4, 128)
    z = torch.zeros(GROUP * M * 4, dtype=torch.int32, device="cuda")
    for form, L, log2m, code in [(3, 4, 4, dk.EINVAL), (1, 7, 4, dk.ERANGE), (2, 4, 5, dk.ERANGE)]:
        with pytest.raises(dk.DkssError) as e:
            dk.probe_twiddle_products(form, q, L, 1, z, z, z, z, log2_m=log2m)
        assert e.value.code == code
    with pytest.raises(dk.DkssError) as e:
        dk.probe_twiddle_products(1, q - 1, 4, 1, z, z, z, z)            # even modulus
    assert e.value.code == dk.EINVAL
    dk.probe_twiddle_products(2, q, 4, 0, None, None, None, None)        # no groups: nothing to do
