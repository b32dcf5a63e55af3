"""GPU test of dkss_mul_noalloc, the entry point that allocates nothing (its workspace is the
library's fixed scratch in device memory): its products equal dkss_mul's, bit for bit, on calls
in a row whose sizes shrink (the scratch keeps the previous call's contents), and a product too
large for the scratch is refused before anything is launched."""
import numpy as np
import pytest

import seeded_inputs as SI
from oracle import coracle as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1503_04955_amd as dk
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dk.lib()
    return dk, torch


# (seed, alen, blen, squaring): a 2^24-bit product first, then smaller ones in the same scratch
CALLS = [
    (SI.SEED_BASE + 101, 1 << 19, 1 << 19, False),     # 2^24 x 2^24 bits
    (SI.SEED_BASE + 102, 8192, 3001, False),           # 2^18 bits x a ragged length
    (SI.SEED_BASE + 103, 40000, 40000, True),          # a squaring (one polynomial)
    (SI.SEED_BASE + 104, 3000, 700, False),            # a DKSS product just above the base case
]


@pytest.mark.parametrize("prepared", [False, True], ids=["table_in_scratch", "prepared_table"])
def test_noalloc_equals_dkss_mul(env, prepared):
    """Calls in a row, each checked against dkss_mul on the same operands (and the small ones
    against the oracle's schoolbook).  Without preparation the tuple's table is built in the
    scratch by the call itself; with it the context's copy is read."""
    dk, torch = env
    ctx_ref = dk.Context()
    ctx = dk.Context()
    for seed, alen, blen, square in CALLS:
        print("noalloc case", seed, alen, blen, square, "prepared" if prepared else "unprepared", flush=True)
        if square:
            a = SI.limbs(seed, alen)
            b = a
        else:
            a, b = SI.operand_pair(seed, alen, blen)
        da = dk.to_device(a)
        db = da if square else dk.to_device(b)
        want = dk.to_host(ctx_ref.mul(da, db))
        if prepared:
            ctx.prepare(alen, blen)
        out = torch.full((alen + blen,), 0x5A5A5A5A, dtype=torch.int32, device=da.device)
        ctx.mul_noalloc(da, db, out)
        torch.cuda.synchronize()
        got = dk.to_host(out)
        assert np.array_equal(got, want), (seed, alen, blen)
        if alen * blen <= 1 << 27:
            assert np.array_equal(got, C.schoolbook(a, b)), (seed, alen, blen)


def test_noalloc_refuses_products_beyond_the_scratch(env):
    """A 2^26-bit product under the thesis rule needs about 260 MiB of workspace: refused with
    DKSS_ETOOBIG, the output untouched."""
    dk, torch = env
    ctx = dk.Context()
    n = 1 << 21
    assert ctx.workspace_bytes(n, n) > dk.NOALLOC_SCRATCH_BYTES
    a = torch.ones(n, dtype=torch.int32, device="cuda")
    out = torch.full((2 * n,), 7, dtype=torch.int32, device="cuda")
    with pytest.raises(dk.DkssError) as e:
        ctx.mul_noalloc(a, a, out)
    assert e.value.code == dk.ETOOBIG
    torch.cuda.synchronize()
    assert bool((out == 7).all())


def test_noalloc_zero_length(env):
    """An empty operand gives a zero product (no workspace needed)."""
    dk, torch = env
    ctx = dk.Context()
    a = dk.to_device(SI.limbs(SI.SEED_BASE + 105, 5))
    b = torch.empty(0, dtype=torch.int32, device="cuda")
    out = torch.full((5,), -1, dtype=torch.int32, device="cuda")
    ctx.mul_noalloc(a, b, out)
    torch.cuda.synchronize()
    assert bool((out == 0).all())
