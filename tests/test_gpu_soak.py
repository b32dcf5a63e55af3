"""Soak test: Lucas-Lehmer runs whose every squaring is a DKSS product on the GPU.

s_0 = 4, s_(k+1) = s_k^2 - 2 mod 2^p - 1; for an odd prime p, 2^p - 1 is prime iff s_(p-2) = 0
(Lucas-Lehmer).  The squarings (p up to 4423 bits, a few thousand each) go through dkss_mul with
a == b; the reduction mod 2^p - 1 and the subtraction are done on the host with Python integers.
Exponents: 4253 and 4423 give Mersenne primes (published), 4259 and 4271 are primes p with
2^p - 1 composite, whose final residue is also computed entirely on the host and compared.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _limbs(x, n):
    return np.frombuffer(x.to_bytes(4 * n, "little"), dtype=np.uint32).copy()


def _value(a):
    return int.from_bytes(np.ascontiguousarray(a, dtype=np.uint32).tobytes(), "little")


def _lucas_lehmer_gpu(dk, torch, ctx, p):
    mp = (1 << p) - 1
    n = (p + 31) // 32
    s = 4
    for _ in range(p - 2):
        d = dk.to_device(_limbs(s, n))
        sq = _value(dk.to_host(ctx.mul(d, d)))
        s = (sq - 2) % mp
    return s


def _lucas_lehmer_host(p):
    mp = (1 << p) - 1
    s = 4
    for _ in range(p - 2):
        s = (s * s - 2) % mp
    return s


@pytest.mark.parametrize("p,prime", [(4253, True), (4259, False), (4423, True), (4271, False)])
def test_lucas_lehmer_squarings(p, prime):
    import torch
    import paper_1503_04955_amd as dk
    ctx = dk.Context()
    plan = ctx.plan_info((p + 31) // 32, (p + 31) // 32)
    assert not plan.schoolbook                 # the squarings take the DKSS path
    s = _lucas_lehmer_gpu(dk, torch, ctx, p)
    assert (s == 0) == prime
    if not prime:
        assert s == _lucas_lehmer_host(p)
