"""GPU parity tests: the HIP path through the C ABI against the CPU oracle, bit-exact.

Every product is exact integer arithmetic, so the bar is bit-exact equality: against the
oracle's schoolbook product (small and mid sizes), the oracle's DKSS (2^24 bits), and residues
modulo seeded random 61-bit primes computed by the oracle on the host (2^28 bits).  Intermediate
parity: the GPU forward transform (natural order) against the oracle's FFT over R.
"""
import random

import numpy as np
import pytest

import seeded_inputs as SI
from conftest import golden_rows, host_residues, primes61, residues_agree, sha256_limbs
from oracle import coracle as C
from oracle import params as OP

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1503_04955_amd as dk
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dk.lib()
    return dk, torch, dk.Context()


def _gpu_mul(env, a, b, params=None, square=False):
    dk, torch, ctx = env
    da = dk.to_device(a)
    db = da if square else dk.to_device(b)
    c = ctx.mul(da, db, params=params)
    torch.cuda.synchronize()
    return dk.to_host(c)


def _primes61(seed, count):
    return primes61(seed, count)


def _residue_check(a, b, c, primes):
    for q in primes:
        assert C.residue(c, q) == C.residue(a, q) * C.residue(b, q) % q, q


def _params(dk, log2_M, log2_m, u=0, p_bits=128, z=1, radices=None):
    return dk.Params.make(log2_M, log2_m, u, p_bits, z, radices=radices, cutoff_bits=0)


# ---- intermediate: the forward transform ------------------------------------------------------

FWD = [  # (log2_M, log2_m, u, p_bits, z, radices, alen)
    (3, 2, 16, 64, 1, None, 4),              # 2M = 16 = 2m*2
    (4, 2, 20, 64, 1, None, 8),              # 2M = 32: radices 8, 4
    (5, 3, 24, 128, 1, None, 16),            # 2M = 64 = (2m)^2
    (5, 2, 24, 32, 4, None, 16),             # z = 4, q = p^4 with a 32-bit p
    (6, 2, 24, 64, 1, [1, 2, 3, 1], 24),     # forced split including radix 2
    (9, 4, 32, 128, 1, None, 256),           # C1-like ring, 2M = 1024 = 32 * 32
    (7, 3, 40, 192, 1, None, 64),            # L = 6
    # tight formats: q < 2^(28 D - 1), one 28-bit digit fewer than the limbs take
    (4, 2, 20, 55, 1, None, 8),              # L = 2, D = 2
    (5, 3, 24, 83, 1, None, 16),             # L = 3, D = 3
    (9, 4, 32, 111, 1, None, 256),           # L = 4, D = 4
    (7, 3, 40, 139, 1, None, 64),            # L = 5, D = 5
    (7, 3, 40, 167, 1, None, 64),            # L = 6, D = 6
    (6, 2, 48, 223, 1, None, 32),            # L = 7, D = 8
    (6, 3, 60, 251, 1, None, 48),            # L = 8, D = 9
    (5, 2, 24, 40, 2, None, 16),             # q = p^2 of 79 bits: L = 3, D = 3, dense reduction
]


@pytest.mark.parametrize("case", FWD, ids=lambda c: "M%d_m%d_u%d_p%d_z%d_%s" % c[:6])
def test_forward_transform_matches_oracle_fft(env, case):
    dk, torch, ctx = env
    log2_M, log2_m, u, p_bits, z, radices, alen = case
    params = _params(dk, log2_M, log2_m, u, p_bits, z, radices)
    pr = OP.Params(N=32 * alen, log2_M=log2_M, log2_m=log2_m, u=u, p_bits=p_bits, z=z)
    S = OP.setup(pr)
    a = SI.limbs(1000 + log2_M, alen)
    got = dk.to_host(ctx.forward(dk.to_device(a), alen, params))
    torch.cuda.synchronize()
    want = C.fft(C.encode(a, pr.M, pr.m, S.L, u), 2 * pr.M, pr.m, S.L, S.q, S.rho)
    assert np.array_equal(got, want)


# ---- whole products, explicit parameter tuples ----------------------------------------------

MUL = [  # (log2_M, log2_m, u, p_bits, z, radices)
    (1, 1, 32, 128, 1, None),
    (3, 2, 16, 64, 1, None),
    (4, 3, 30, 128, 1, None),
    (5, 2, 24, 32, 4, None),
    (5, 3, 40, 32, 3, None),
    (6, 2, 24, 64, 1, [1, 2, 3, 1]),
    (8, 5, 32, 128, 1, None),               # m = 32, one level of radix 64 + ...
    (9, 4, 57, 128, 1, None),               # the thesis's u = 57 ring
    (7, 3, 64, 192, 1, None),
    (6, 6, 32, 128, 1, None),               # m = 64: radix capped below 2m
    (10, 4, 60, 256, 1, None),              # L = 8
    (8, 2, 2, 64, 1, None),                 # u = 2: the decode's elements exceed an LDS tile
    (11, 1, 5, 64, 1, None),                # m = 2, u = 5
    # tight formats (L, D): (2, 2), (3, 3), (4, 4), (5, 5), (6, 6), (7, 8), (8, 9); z = 2
    (8, 3, 20, 55, 1, None),
    (9, 4, 32, 83, 1, None),
    (6, 6, 40, 111, 1, None),               # m = 64
    (7, 5, 56, 139, 1, None),
    (8, 4, 70, 167, 1, None),
    (5, 2, 90, 223, 1, None),
    (6, 3, 100, 251, 1, None),
    (6, 3, 30, 36, 2, None),                # q = p^2 of 71 bits: L = 3, D = 3
]


@pytest.mark.parametrize("case", MUL, ids=lambda c: "M%d_m%d_u%d_p%d_z%d_%s" % c)
def test_mul_parameter_tuples(env, case):
    dk = env[0]
    log2_M, log2_m, u, p_bits, z, radices = case
    cap = (1 << log2_M) * (1 << log2_m) // 2 * u // 32
    for alen, blen, seed in [(cap, cap, 1), (cap, max(1, cap // 8), 2), (max(1, cap // 3), cap, 3)]:
        print("case", case, alen, blen, flush=True)
        a, b = SI.operand_pair(seed + 10 * log2_M, alen, blen)
        got = _gpu_mul(env, a, b, _params(dk, log2_M, log2_m, u, p_bits, z, radices))
        assert np.array_equal(got, C.schoolbook(a, b))


def test_tight_format_plans(env):
    """A modulus below 2^(28 D - 1) runs on D digits, one fewer than its limbs would take; the
    tuples of the parameter tests above get the format their modulus fits."""
    dk, torch, ctx = env
    for log2_M, log2_m, u, p_bits, z, _ in MUL:
        cap = (1 << log2_M) * (1 << log2_m) // 2 * u // 32
        info = ctx.plan_info(cap, cap, _params(dk, log2_M, log2_m, u, p_bits, z))
        L = info.L
        full = (32 * L + 28) // 28
        tight = L >= 2 and info.q_bits <= 28 * (full - 1) - 1
        assert info.digits == (full - 1 if tight else full), (log2_M, log2_m, u, p_bits, z)


# ---- the thesis rule at 2^18 bits (the small configuration) and edge operands --------------

def test_mul_2e18_thesis_rule(env):
    a, b = SI.operand_pair(SI.SEED_BASE + 0, 8192, 8192)
    assert np.array_equal(_gpu_mul(env, a, b), C.schoolbook(a, b))


@pytest.mark.parametrize("kind", ["ones", "ones_favorable", "pow2", "square", "unbalanced",
                                  "one_limb", "favorable_plus_one"])
def test_mul_edge_operands(env, kind):
    if kind == "ones":
        a = b = SI.all_ones(8192)
    elif kind == "ones_favorable":
        a = b = SI.all_ones(7296)           # 3648 64-bit words: u = 57 meets the bound exactly
    elif kind == "pow2":
        a, b = SI.power_of_two(8192 * 32 - 1, 8192), SI.power_of_two(12345, 8192)
    elif kind == "square":
        a = SI.limbs(77, 8192)
        got = _gpu_mul(env, a, a, square=True)
        assert np.array_equal(got, C.schoolbook(a, a))
        return
    elif kind == "unbalanced":
        a, b = SI.operand_pair(5, 8192, 1024)
    elif kind == "one_limb":
        a, b = SI.operand_pair(6, 8192, 1)
        a[-1] = 0xFFFFFFFF
        b[0] = 0xFFFFFFFF
    else:
        a, b = SI.operand_pair(8, 7297, 7297)
    assert np.array_equal(_gpu_mul(env, a, b), C.schoolbook(a, b))


def test_mul_zero_length_and_schoolbook_path(env):
    dk, torch, ctx = env
    a = SI.limbs(3, 40)
    out = ctx.mul(dk.to_device(a), dk.to_device(np.zeros(0, np.uint32)))
    torch.cuda.synchronize()
    assert np.array_equal(dk.to_host(out), np.zeros(40, np.uint32))
    for alen, blen in [(1, 1), (5, 64), (64, 64), (700, 30), (2000, 60)]:
        a, b = SI.operand_pair(alen + blen, alen, blen)
        assert np.array_equal(_gpu_mul(env, a, b), C.schoolbook(a, b)), (alen, blen)


@pytest.mark.parametrize("alen,blen,ones", [(2048, 2048, True), (2048, 2048, False), (4095, 1, True),
                                             (2, 2, True), (31, 32, True), (1000, 3000, False),
                                             (2049, 2048, True), (4000, 3999, False), (4093, 4093, True),
                                             (6000, 5000, False), (8186, 8186, True), (8186, 8186, False),
                                             (64, 8000, False), (8100, 3, True), (3000, 7000, False)])
def test_schoolbook_base_case_up_to_its_limit(env, alen, blen, ones):
    """The base case forced (cutoff above both operands): the schoolbook up to alen + blen = 4096
    words, Karatsuba levels above it (one level up to 4094 x 4094 words, two up to 8186 x
    8186), balanced and unbalanced, with all-ones operands (every column at its largest sum,
    the largest sums a0 + a1, carries through whole rows) and random ones."""
    dk, torch, ctx = env
    if ones:
        a, b = SI.all_ones(alen), SI.all_ones(blen)
    else:
        a, b = SI.operand_pair(SI.SEED_BASE + 31 + alen, alen, blen)
    p = ctx.select_params(32 * alen, 32 * blen)
    p.cutoff_bits = 2 ** 64 - 1
    assert ctx.plan_info(alen, blen, p).schoolbook
    want = C.schoolbook(a, b)
    assert np.array_equal(_gpu_mul(env, a, b, params=p), want), (alen, blen)
    if alen == blen:
        assert np.array_equal(_gpu_mul(env, a, a, params=p, square=True), C.schoolbook(a, a))
    # the allocation-free entry point takes the same path, in its scratch
    dk_, torch_, _ = env
    da, db = dk_.to_device(a), dk_.to_device(b)
    out = torch_.empty(alen + blen, dtype=torch_.int32, device="cuda")
    ctx.mul_noalloc(da, db, out, params=p)
    torch_.cuda.synchronize()
    assert np.array_equal(dk_.to_host(out), want)


def test_karatsuba_base_case_in_batches(env):
    """A batch of base-case products of one, two and no Karatsuba levels (the TUNED-style
    schoolbook choice forced by parameters) equals the oracle's schoolbook products."""
    dk, torch, ctx = env
    lens = [(3000, 3000), (2100, 2000), (5000, 4000), (8000, 7000), (100, 100), (8184, 8184), (1, 8000)]
    lens += SI.batch_lengths(SI.SEED_BASE + 41, 40, lo_bits=16, hi_bits=18)
    pairs = [SI.operand_pair(4000 + i, al, bl) for i, (al, bl) in enumerate(lens)]
    params = []
    for al, bl in lens:
        p = ctx.select_params(32 * al, 32 * bl)
        p.cutoff_bits = 2 ** 64 - 1
        params.append(p)
    got = _batch_run(env, pairs, params=params)
    for (a, b), g in zip(pairs, got):
        assert np.array_equal(g, C.schoolbook(a, b)), (len(a), len(b))


# ---- the large configurations: 2^24 and 2^28 bits --------------------------------------------

def test_mul_2e24_vs_oracle_dkss(env):
    a, b = SI.operand_pair(SI.SEED_BASE + 1, 1 << 19, 1 << 19)
    got = _gpu_mul(env, a, b)
    assert np.array_equal(got, C.dkss_mul(a, b))
    _residue_check(a, b, got, _primes61(1, 8))


def _low_limbs_check(a, b, got, w=2048):
    """The lowest w limbs of a product are the lowest w limbs of the product of the operands'
    lowest w limbs: outputs the oracle's schoolbook computes exactly at any size."""
    assert np.array_equal(got[:w], C.schoolbook(a[:w], b[:w])[:w])


def _digest_case(name):
    """Operands of a product whose oracle-DKSS digest is stored in tests/golden/dkss_digests.txt
    (written by make_dkss_digests.py, which calls only the oracle)."""
    rows = {r[0]: r for r in golden_rows("dkss_digests.txt")}
    _, seed, alen, blen, square, want = rows[name]
    seed, alen, blen = int(seed), int(alen), int(blen)
    if int(square):
        a = SI.limbs(seed, alen)
        return a, a, True, want
    a, b = SI.operand_pair(seed, alen, blen)
    return a, b, False, want


@pytest.mark.parametrize("name", ["2p28_random", "2p28_square", "2p28_unbalanced"])
def test_mul_2e28_vs_oracle_dkss(env, name):
    """2^28-bit products (random, squaring, 8:1) equal the CPU oracle's DKSS product, through its
    stored SHA-256 (the oracle takes minutes per product), and pass residues mod 8 primes."""
    a, b, square, want = _digest_case(name)
    print("case", name, len(a), len(b), flush=True)
    got = _gpu_mul(env, a, b, square=square)
    assert sha256_limbs(got) == want
    _residue_check(a, b, got, _primes61(3, 8))


@pytest.mark.parametrize("policy", ["thesis", "learned"])
def test_mul_2e30_heldout_vs_oracle_dkss(env, policy):
    """The held-out single product at 2^30 bits (outside the selector's training grid) under the
    thesis rule and under the learned selector equals the CPU oracle's DKSS product (its stored
    SHA-256), and passes residues mod 4 primes computed by the oracle on the host."""
    dk, torch, _ = env
    a, b, _, want = _digest_case("2p30_heldout")
    ctx = dk.Context(dk.POLICY_THESIS if policy == "thesis" else dk.POLICY_LEARNED)
    print("case 2^30", policy, ctx.select_params(32 * len(a), 32 * len(b)).as_dict(), flush=True)
    c = ctx.mul(dk.to_device(a), dk.to_device(b))
    torch.cuda.synchronize()
    got = dk.to_host(c)
    assert sha256_limbs(got) == want
    qs = _primes61(30, 4)
    ra, rb, rc = host_residues([a, b, got], qs)
    assert residues_agree(ra, rb, rc, qs)


def _ones_product(n, k):
    """(2^(32n) - 1)(2^(32k) - 1) = 2^(32(n+k)) - 2^(32n) - 2^(32k) + 1 as n + k limbs (closed
    form, linear time)."""
    v = (1 << (32 * (n + k))) - (1 << (32 * n)) - (1 << (32 * k)) + 1
    return np.frombuffer(v.to_bytes(4 * (n + k), "little"), dtype=np.uint32)


@pytest.mark.parametrize("log2_bits", [24, 28])
@pytest.mark.parametrize("kind", ["ones", "ones_unbalanced", "pow2", "pow2_top"])
def test_mul_large_edge_operands(env, log2_bits, kind):
    """Edge operands at 2^24 and 2^28 bits against closed forms: all-ones factors (every encoded
    coefficient at its maximum, the largest coefficient sums), also 8:1 unbalanced, and powers of
    two (a single bit in the product), one of them at the top bit of both operands."""
    n = (1 << log2_bits) // 32
    if kind == "ones":
        a = b = SI.all_ones(n)
        want = _ones_product(n, n)
    elif kind == "ones_unbalanced":
        a, b = SI.all_ones(n), SI.all_ones(n // 8)
        want = _ones_product(n, n // 8)
    else:
        i, j = (32 * n - 1, 32 * n - 1) if kind == "pow2_top" else (12345, 32 * n - 777)
        a, b = SI.power_of_two(i, n), SI.power_of_two(j, n)
        want = np.zeros(2 * n, np.uint32)
        want[(i + j) // 32] = np.uint32(1 << ((i + j) % 32))
    print("case", kind, log2_bits, flush=True)
    got = _gpu_mul(env, a, b)
    assert np.array_equal(got, want)


def test_gpu_residues_match_oracle(env):
    dk, torch, ctx = env
    x = SI.limbs(99, 300001)
    primes = _primes61(4, 5) + [3, 2 ** 61 - 1]
    got = dk.residues(dk.to_device(x), primes)
    assert got == [C.residue(x, q) for q in primes]


def test_workspace_too_small(env):
    dk, torch, ctx = env
    a = dk.to_device(SI.limbs(1, 8192))
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(dk.DkssError) as e:
        ctx.mul(a, a, ws=ws)
    assert e.value.code == dk.ENOSPC


# ---- batched products ------------------------------------------------------------------------

def _batch_run(env, pairs, policy_ctx=None, params=None):
    dk, torch, ctx = env
    c0 = policy_ctx or ctx
    das = [dk.to_device(a) for a, _ in pairs]
    dbs = [dk.to_device(b) for _, b in pairs]
    outs = c0.mul_batch(das, dbs, params=params)
    torch.cuda.synchronize()
    return [dk.to_host(o) for o in outs]


def test_batch_mixed_small_vs_schoolbook(env):
    """Zero-length, schoolbook-range and DKSS products of many parameter tuples in one batch."""
    rng = random.Random(11)
    lens = [(0, 5), (7, 0), (1, 1), (3, 64), (64, 64), (65, 65), (100, 13)]
    lens += SI.batch_lengths(2024, 120, lo_bits=8, hi_bits=16)
    pairs = [SI.operand_pair(1000 + i, al, bl) for i, (al, bl) in enumerate(lens)]
    pairs.append((pairs[20][0], pairs[20][0]))                    # a squaring inside a batch
    got = _batch_run(env, pairs)
    for (a, b), g in zip(pairs, got):
        assert np.array_equal(g, C.schoolbook(a, b)), (len(a), len(b))


def test_batch_matches_plain_and_residues(env):
    """A batch with the C3 length distribution (2^12..2^22 bits, ratio 1..8): every product equals
    the plain single-product result and passes residue checks; a few against the oracle."""
    dk, torch, ctx = env
    lens = SI.batch_lengths(SI.SEED_BASE + 3, 256)
    pairs = [SI.operand_pair(5000 + i, al, bl) for i, (al, bl) in enumerate(lens)]
    got = _batch_run(env, pairs)
    qs = _primes61(9, 4)
    for i, ((a, b), g) in enumerate(zip(pairs, got)):
        _residue_check(a, b, g, qs)
        if i % 32 == 0:
            assert np.array_equal(g, _gpu_mul(env, a, b))
        if len(a) * len(b) < 4e6:
            assert np.array_equal(g, C.schoolbook(a, b))


@pytest.mark.parametrize("limbs", [128, 2048, 20000])
def test_every_candidate_tuple_is_bit_exact(env, limbs):
    """Parameter choices (tuner / selector search space) never change the product."""
    dk, torch, ctx = env
    a, b = SI.operand_pair(limbs, limbs, max(1, limbs // 3))
    want = C.schoolbook(a, b)
    cands = ctx.candidates(32 * limbs, 32 * limbs)
    assert cands
    for ci, p in cands:
        p.cutoff_bits = 0
        assert np.array_equal(_gpu_mul(env, a, b, p), want), ci


@pytest.mark.parametrize("log2_m,radices_fixed,radices_general", [
    (4, [5, 5, 5], [4, 4, 4, 3]),       # m = 16: radix-32 levels (compile-time shape) vs radix 16/8
    (5, [6, 6, 3], [5, 5, 5]),          # m = 32: radix-64 levels vs radix-32 levels
])
def test_compile_time_shapes_agree(env, log2_m, radices_fixed, radices_general):
    """The level kernels compiled for fixed (m, radix) shapes and those with only m fixed (any
    radix) give the same product for one tuple run with splits that take either; the product's
    lowest limbs equal the oracle's and its residues the oracle's residues.  (Every other m runs
    the fully general kernels, throughout the other tests.)"""
    dk, torch, ctx = env
    log2_M = sum(radices_fixed) - 1
    limbs = (1 << (log2_M + log2_m - 1)) * 24 // 32     # the tuple's full capacity (u = 24)
    a, b = SI.operand_pair(SI.SEED_BASE + 60 + log2_m, limbs, limbs - 5)
    got = [_gpu_mul(env, a, b, _params(dk, log2_M, log2_m, u=24, p_bits=128, radices=rad))
           for rad in (radices_fixed, radices_general)]
    assert np.array_equal(got[0], got[1])
    _low_limbs_check(a, b, got[0])
    _residue_check(a, b, got[0], _primes61(60 + log2_m, 4))


def test_tuned_policy_products(env):
    dk, torch, ctx = env
    tctx = dk.Context(dk.POLICY_TUNED)
    for limbs in [300, 5000, 1 << 15]:
        a, b = SI.operand_pair(limbs + 7, limbs, limbs)
        c = tctx.mul(dk.to_device(a), dk.to_device(b))
        torch.cuda.synchronize()
        assert np.array_equal(dk.to_host(c), C.schoolbook(a, b))


def test_tuned_policy_batch_sections(env):
    """A batch of 300 mixed products under the TUNED policy takes the table's batch 256 section
    (the schoolbook up to about 2^14.5 bits, other candidates above): it equals the thesis rule's
    batch, and its small products the oracle's."""
    dk, torch, ctx = env
    tctx = dk.Context(dk.POLICY_TUNED)
    assert tctx.select_params(2 ** 14, 2 ** 14, 300).cutoff_bits == 2 ** 64 - 1
    lens = SI.batch_lengths(SI.SEED_BASE + 41, 300, hi_bits=19)
    pairs = [SI.operand_pair(8000 + i, al, bl) for i, (al, bl) in enumerate(lens)]
    as_ = [dk.to_device(a) for a, _ in pairs]
    bs = [dk.to_device(b) for _, b in pairs]
    out_t = tctx.mul_batch(as_, bs)
    out_0 = ctx.mul_batch(as_, bs)
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(out_t, out_0))
    for (a, b), g in zip(pairs, out_t):
        if len(a) * len(b) < 2e6:
            assert np.array_equal(dk.to_host(g), C.schoolbook(a, b)), (len(a), len(b))


def test_batch_graph_replays(env):
    """A batch captured into a HIP graph: every replay equals the eager batch, with eager work
    and synchronizations between replays, outputs cleared before each replay, and new operand
    values written in place between replays (the graph reads them at the same addresses)."""
    dk, torch, ctx = env
    lens = [(0, 5), (3, 64), (64, 64), (100, 13)] + SI.batch_lengths(SI.SEED_BASE + 31, 150, hi_bits=18)
    pairs = [SI.operand_pair(7000 + i, al, bl) for i, (al, bl) in enumerate(lens)]
    as_ = [dk.to_device(a) for a, _ in pairs]
    bs = [dk.to_device(b) for _, b in pairs]
    call = dk.BatchCall(ctx, as_, bs)
    graph = call.graph()
    assert graph.products == len(pairs) and graph.kernels > 0
    eager = dk.Context()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    for rep in range(3):
        if rep == 2:                       # new operand values, same buffers
            for t in as_ + bs:
                if t.numel():
                    t.copy_(torch.randint(-2 ** 31, 2 ** 31, t.shape, dtype=torch.int32,
                                          device="cuda", generator=gen))
        for o in call.outs:
            o.zero_()
        want = eager.mul_batch(as_, bs)    # eager work between the replays
        torch.cuda.synchronize()
        graph()
        torch.cuda.synchronize()
        for i, (o, w) in enumerate(zip(call.outs, want)):
            assert torch.equal(o, w), (rep, i, lens[i])
    a0, b0 = dk.to_host(as_[5]), dk.to_host(bs[5])
    assert np.array_equal(dk.to_host(call.outs[5]), C.schoolbook(a0, b0))
    graph.close()


@pytest.mark.parametrize("opts", [{"fuse": 0}, {"overlap": 1}, {"overlap": 1, "fuse": 0},
                                  {"lds": 16384}, {"lds": 65536}, {"lds": 163840},
                                  {"lanes": 1}, {"lanes": 8}])
def test_context_options_keep_the_bits(env, opts):
    """The unfused componentwise products (separate k_pointwise, k_encode), the second stream for
    b, other LDS budgets and other numbers of batch streams give the same product, single and
    batched."""
    dk, torch, ctx0 = env
    ctx = dk.Context()
    names = {"fuse": dk.OPT_FUSE_PW, "overlap": dk.OPT_OVERLAP, "lds": dk.OPT_DFT_LDS,
             "lanes": dk.OPT_BATCH_LANES}
    for k, v in opts.items():
        ctx.set_option(names[k], v)
    for alen, blen in [(8192, 8192), (30000, 4000), (131072, 131072)]:
        a, b = SI.operand_pair(alen + 3 * blen, alen, blen)
        da, db = dk.to_device(a), dk.to_device(b)
        got = ctx.mul(da, db)
        want = ctx0.mul(da, db)
        assert torch.equal(got, want), (opts, alen, blen)
        sq = ctx.mul(da, da)
        assert torch.equal(sq, ctx0.mul(da, da)), (opts, alen)
        if alen * blen < 1e8:
            assert np.array_equal(dk.to_host(got), C.schoolbook(a, b))
    lens = SI.batch_lengths(SI.SEED_BASE + 5, 64, hi_bits=18)
    pairs = [SI.operand_pair(300 + i, al, bl) for i, (al, bl) in enumerate(lens)]
    as_ = [dk.to_device(x) for x, _ in pairs]
    bs = [dk.to_device(y) for _, y in pairs]
    for x, y in zip(ctx.mul_batch(as_, bs), ctx0.mul_batch(as_, bs)):
        assert torch.equal(x, y), opts


def test_batch_4096_full_size(env):
    """The mixed batch at its stated size (4096 products, 2^12..2^22 bits, ratio 1..8) under the
    learned selector, replayed as a graph: every product passes c = a*b modulo 8 seeded 61-bit
    primes with all residues computed by the oracle on the host, and 64 products spread over the
    batch equal the oracle's DKSS product (thesis rule) limb for limb."""
    dk, torch, _ = env
    from concurrent.futures import ThreadPoolExecutor
    pairs = SI.mixed_batch(4096)
    as_ = [dk.to_device(a) for a, _ in pairs]
    bs = [dk.to_device(b) for _, b in pairs]
    call = dk.BatchCall(dk.Context(dk.POLICY_LEARNED), as_, bs)
    graph = call.graph()
    graph()
    torch.cuda.synchronize()
    got = [dk.to_host(o) for o in call.outs]
    graph.close()
    qs = _primes61(4096, 8)
    flat = [x for (a, b), c in zip(pairs, got) for x in (a, b, c)]
    res = host_residues(flat, qs)
    bad = [i for i in range(len(pairs)) if not residues_agree(res[3 * i], res[3 * i + 1], res[3 * i + 2], qs)]
    assert not bad, bad[:10]
    sample = list(range(0, 4096, 64))
    C.lib()
    with ThreadPoolExecutor(max_workers=16) as ex:
        want = list(ex.map(lambda i: C.dkss_mul(*pairs[i]), sample))
    for i, w in zip(sample, want):
        assert np.array_equal(got[i], w), (i, len(pairs[i][0]), len(pairs[i][1]))


def test_mul_captured_on_a_fresh_context(env):
    """dkss_mul allocates nothing and does not wait: on a context that has built no table, a
    product recorded into a graph by torch's stream capture (global mode, where an allocation or
    a synchronization would fail the capture) replays correctly, several times, with eager work
    and other products of the same context between the replays."""
    dk, torch, _ = env
    a, b = SI.operand_pair(SI.SEED_BASE + 70, 30000, 20000)
    want = C.schoolbook(a, b)
    da, db = dk.to_device(a), dk.to_device(b)
    ctx = dk.Context()
    ws = torch.empty(ctx.workspace_bytes(30000, 20000), dtype=torch.uint8, device="cuda")
    out = torch.zeros(50000, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.mul(da, db, out=out, ws=ws)
    torch.cuda.synchronize()
    other = dk.to_device(SI.limbs(71, 8192))
    for rep in range(3):
        out.zero_()
        sq = ctx.mul(other, other)                   # eager work of the same context in between
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(dk.to_host(out), want), rep
        assert np.array_equal(dk.to_host(sq), C.schoolbook(dk.to_host(other), dk.to_host(other)))


def test_prepare_refused_under_capture_leaves_context_usable(env):
    """dkss_prepare on a capturing stream is refused before any work, and the context stays
    unprepared: the product captured next builds its table in the workspace, and an eager product
    afterwards (which prepares the context) is right too."""
    dk, torch, _ = env
    a, b = SI.operand_pair(SI.SEED_BASE + 72, 9000, 9000)
    want = C.schoolbook(a, b)
    da, db = dk.to_device(a), dk.to_device(b)
    ctx = dk.Context()
    ws = torch.empty(ctx.workspace_bytes(9000, 9000), dtype=torch.uint8, device="cuda")
    out = torch.zeros(18000, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        with pytest.raises(dk.DkssError) as e:
            ctx.prepare(9000, 9000)
        ctx.mul(da, db, out=out, ws=ws)
    assert e.value.code == dk.EINVAL
    torch.cuda.synchronize()
    eager = ctx.mul(da, db)
    torch.cuda.synchronize()
    assert np.array_equal(dk.to_host(eager), want)
    g.replay()
    torch.cuda.synchronize()
    assert np.array_equal(dk.to_host(out), want)


@pytest.mark.parametrize("policy", ["thesis", "learned"])
def test_products_without_prepare(env, policy):
    """Without a planning call that builds the tables, single products and a batch build them in
    their workspace on every call; the results equal the oracle's (schoolbook) and those of a
    prepared context."""
    dk, torch, _ = env
    pol = dk.POLICY_THESIS if policy == "thesis" else dk.POLICY_LEARNED
    ctx = dk.Context(pol)
    for alen, blen in [(8192, 8192), (30000, 4000), (100000, 100000)]:
        a, b = SI.operand_pair(alen + blen + 11, alen, blen)
        da, db = dk.to_device(a), dk.to_device(b)
        for _ in range(2):
            got = ctx.mul(da, db, prepare=False)
            torch.cuda.synchronize()
            if alen * blen < 1e9:
                assert np.array_equal(dk.to_host(got), C.schoolbook(a, b)), (alen, blen)
        assert torch.equal(got, dk.Context(pol).mul(da, db)), (alen, blen)
    lens = SI.batch_lengths(SI.SEED_BASE + 73, 80, hi_bits=18)
    pairs = [SI.operand_pair(400 + i, al, bl) for i, (al, bl) in enumerate(lens)]
    as_ = [dk.to_device(x) for x, _ in pairs]
    bs = [dk.to_device(y) for _, y in pairs]
    bc = dk.BatchCall(dk.Context(pol), as_, bs, prepare=False)
    for _ in range(2):
        outs = bc()
        torch.cuda.synchronize()
        for (x, y), o in zip(pairs, outs):
            assert np.array_equal(dk.to_host(o), C.schoolbook(x, y)), (len(x), len(y))


def test_mul_2e34_thesis_learned_and_square(env):
    """The largest single product: two 2^34-bit operands (2 GiB each, seeded uniform limbs from
    the host generator) under the thesis rule and under the learned selector, and the squaring
    of a.  Checked by residues mod 16 seeded 61-bit primes: the residues of a, b and the products
    modulo 2 of them are the oracle's, computed on the host; all 16 from the GPU's residue kernel
    (itself pinned to the oracle) agree with c = a*b.  Both policies give identical limbs."""
    dk, torch, _ = env
    import time
    n = (1 << 34) // 32
    ha, hb = SI.operand_pair(SI.SEED_BASE + 34, n, n)
    a, b = dk.to_device(ha), dk.to_device(hb)
    qs = _primes61(34, 16)
    host_q = qs[:2]
    hra, hrb = host_residues([ha, hb], host_q)
    ra, rb = dk.residues(a, qs), dk.residues(b, qs)
    assert ra[:2] == hra and rb[:2] == hrb
    del ha, hb
    outs = {}
    for name, policy in (("thesis", dk.POLICY_THESIS), ("learned", dk.POLICY_LEARNED)):
        ctx = dk.Context(policy)
        ws = torch.empty(ctx.workspace_bytes(n, n), dtype=torch.uint8, device="cuda")
        c = torch.empty(2 * n, dtype=torch.int32, device="cuda")
        ctx.prepare(n, n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.mul(a, b, out=c, ws=ws)
        torch.cuda.synchronize()
        print("2^34 x 2^34 %s: %.1f ms, params %s" % (name, 1e3 * (time.perf_counter() - t0),
                                                      ctx.select_params(1 << 34, 1 << 34).as_dict()), flush=True)
        rc = dk.residues(c, qs)
        assert residues_agree(ra, rb, rc, qs), name
        if name == "thesis":
            (hrc,) = host_residues([dk.to_host(c)], host_q)
            assert residues_agree(hra, hrb, hrc, host_q)
            sq = ctx.mul(a, a, ws=ws)
            rs = dk.residues(sq, qs)
            assert residues_agree(ra, ra, rs, qs)
            (hrs,) = host_residues([dk.to_host(sq)], host_q)
            assert residues_agree(hra, hra, hrs, host_q)
            del sq
        outs[name] = c
        del ws
        torch.cuda.empty_cache()
    assert torch.equal(outs["thesis"], outs["learned"])


@pytest.mark.parametrize("policy", ["thesis", "learned"])
def test_step6_by_kronecker_schoenhage(env, policy):
    """Step 6 as Sec. 3.2.6 writes it (DKSS_OPT_STEP6_KS): products in R by Kronecker-Schoenhage
    substitution, the integer products by the library itself (DKSS again above the base-case
    cutoff): the same products as the direct path and the oracle's schoolbook, single, squared
    and batched."""
    dk, torch, ctx0 = env
    ctx = dk.Context(dk.POLICY_THESIS if policy == "thesis" else dk.POLICY_LEARNED)
    ctx.set_option(dk.OPT_STEP6_KS, 1)
    for alen, blen in [(100, 70), (8192, 8192), (30000, 4000), (1 << 19, 1 << 19)]:
        a, b = SI.operand_pair(SI.SEED_BASE + 600 + alen, alen, blen)
        da, db = dk.to_device(a), dk.to_device(b)
        print("ks case", policy, alen, blen, ctx.select_params(32 * alen, 32 * blen).as_dict(), flush=True)
        got = ctx.mul(da, db)
        want = ctx0.mul(da, db)
        assert torch.equal(got, want), (alen, blen)
        if alen * blen < 1e9:
            assert np.array_equal(dk.to_host(got), C.schoolbook(a, b))
        assert torch.equal(ctx.mul(da, da), ctx0.mul(da, da)), alen
    lens = SI.batch_lengths(SI.SEED_BASE + 601, 48, hi_bits=18)
    pairs = [SI.operand_pair(900 + i, al, bl) for i, (al, bl) in enumerate(lens)]
    as_ = [dk.to_device(x) for x, _ in pairs]
    bs = [dk.to_device(y) for _, y in pairs]
    for (x, y), got in zip(pairs, ctx.mul_batch(as_, bs)):
        assert np.array_equal(dk.to_host(got), C.schoolbook(x, y))
