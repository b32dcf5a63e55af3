"""Property tests (Hypothesis, derandomized so every run draws the same cases): products of
random lengths from 1 to 2^16 limbs, random length ratios, squarings (a == b), under the
thesis rule and the learned selector, against the oracle's schoolbook product where that is
cheap and against residues modulo 61-bit primes computed by the oracle otherwise."""
import random

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import seeded_inputs as SI
from oracle import coracle as C

pytestmark = pytest.mark.gpu

PRIMES = []


def _primes():
    if not PRIMES:
        rng = random.Random(4242)
        while len(PRIMES) < 4:
            q = rng.getrandbits(61) | (1 << 60) | 1
            if all(pow(b, q - 1, q) == 1 for b in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)):
                PRIMES.append(q)
    return PRIMES


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1503_04955_amd as dk
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dk.lib()
    return dk, torch, {"thesis": dk.Context(), "learned": dk.Context(dk.POLICY_LEARNED)}


def _check(a, b, c):
    if len(a) * len(b) <= 1 << 24:
        assert np.array_equal(c, C.schoolbook(a, b)), (len(a), len(b))
    else:
        for q in _primes():
            assert C.residue(c, q) == C.residue(a, q) * C.residue(b, q) % q, (len(a), len(b), q)


@settings(max_examples=40, derandomize=True, deadline=None)
@given(log2_alen=st.floats(0.0, 16.0), ratio=st.floats(1.0, 64.0), square=st.booleans(),
       swap=st.booleans(), learned=st.booleans(), seed=st.integers(0, 2 ** 31 - 1))
def test_random_lengths_and_ratios(env, log2_alen, ratio, square, swap, learned, seed):
    dk, torch, ctxs = env
    alen = max(1, int(round(2.0 ** log2_alen)))
    blen = alen if square else max(1, int(round(alen / ratio)))
    a, b = SI.operand_pair(seed, alen, blen)
    if swap:
        a, b = b, a
    ctx = ctxs["learned" if learned else "thesis"]
    da = dk.to_device(a)
    db = da if square else dk.to_device(b)
    c = ctx.mul(da, db)
    torch.cuda.synchronize()
    _check(a, a if square else b, dk.to_host(c))
