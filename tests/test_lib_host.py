"""CPU-side checks of libdkss: exported symbols, host planning against the oracle's rule and
prime, argument errors that are decided before any device work."""
import ctypes
import os
import re

import pytest

from oracle import params as OP

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dk():
    import paper_1503_04955_amd as dk
    try:
        dk.lib()
    except RuntimeError:
        from paper_1503_04955_amd import build
        build.build()
    return dk


def test_header_symbols_exported(dk):
    hdr = open(os.path.join(ROOT, "include", "dkss.h")).read()
    names = set(re.findall(r"\b(dkss_[a-z_]+)\s*\(", hdr))
    assert names == set(dk.EXPORTED)
    L = dk.lib()
    for n in names:
        assert hasattr(L, n), n


@pytest.mark.parametrize("N", [2 ** 12, 5000 * 32, 2 ** 18, 233472, 2 ** 24, 2 ** 28, 2 ** 30,
                               2 ** 34, 64 * 1703936, 64 * 85983232])
def test_planner_matches_oracle_rule(dk, N):
    ctx = dk.Context()
    p = ctx.select_params(N, N)
    o = OP.thesis_rule(N)
    assert (p.log2_M, p.log2_m, p.u, p.p_bits, p.z) == (o.log2_M, o.log2_m, o.u, o.p_bits, 1)
    assert sum(p.radix_log2[i] for i in range(p.n_levels)) == o.log2_M + 1


@pytest.mark.parametrize("N", [2 ** 12, 2 ** 18, 2 ** 24, 2 ** 28])
def test_planner_prime_matches_oracle(dk, N):
    ctx = dk.Context()
    n = N // 32
    info = ctx.plan_info(n, n, dk.Params.make(*_rule(N), cutoff_bits=0))
    o = OP.thesis_rule(N)
    p, h, nn = OP.proth_prime(o.p_bits, o.log2_M + 1)
    assert info.modulus == p and info.q_bits == p.bit_length()
    assert info.poly_bytes == (2 * o.M) * o.m * info.L * 4


def _rule(N):
    o = OP.thesis_rule(N)
    return o.log2_M, o.log2_m, o.u, o.p_bits, o.z


def test_planner_prime_power(dk):
    """z > 1: the modulus is p^z for the 32-bit p = 3*2^30 + 1 of the oracle."""
    ctx = dk.Context()
    info = ctx.plan_info(48, 48, dk.Params.make(5, 2, 24, 32, 4, cutoff_bits=0))
    assert info.modulus == (3 * 2 ** 30 + 1) ** 4


@pytest.mark.parametrize("N", [2 ** 12, 5000 * 32, 2 ** 18, 2 ** 22, 2 ** 26, 2 ** 30, 2 ** 34])
def test_candidate_set(dk, N):
    """The candidates of dkss_candidates, restated from their definition: 18 tuples with a prime
    modulus (Mm = 2^(t_min + c // 6), m = 2^(c % 6 + 1), the fewest whole limbs of p with
    p > Mm 2^(2u), or 28 D - 1 bits where that saves a 28-bit digit), and 6 with the square of a
    prime (z = 2, Mm = 2^t_min, the fewest bits of p with p^2 > Mm 2^(2u) for every prime of that
    length); each feasible tuple plans on the host with a modulus p^z of the oracle's Proth
    prime, and its products in R on the digits its modulus needs."""
    ctx = dk.Context()
    cands = dict(ctx.candidates(N, N))
    assert cands and max(cands) < dk.NCAND == 24

    def u_of(t):
        return -(-2 * N // 2 ** t)

    t_min = next(t for t in range(2, 63) if t + 2 * u_of(t) + 1 <= 256)
    for c, p in cands.items():
        t = t_min + (c // 6 if c < 18 else 0)
        lm = c % 6 + 1 if c < 18 else c - 17
        u = u_of(t)
        assert (p.log2_M + p.log2_m, p.log2_m, p.u) == (t, lm, u), c
        nb = t + 2 * u + 1                   # bits of the smallest prime above Mm 2^(2u)
        limbs, digits = -(-nb // 32), -(-(nb + 1) // 28)
        if c < 18:
            tight = limbs >= 2 and digits < (32 * limbs + 28) // 28
            assert p.z == 1 and p.p_bits == (28 * digits - 1 if tight else 32 * limbs), c
        else:
            assert p.z == 2 and 2 * p.p_bits - 2 >= t + 2 * u > 2 * p.p_bits - 4, c
        info = ctx.plan_info(N // 32, N // 32, p)
        prime, _, _ = OP.proth_prime(p.p_bits, p.log2_M + 1)
        assert info.modulus == prime ** p.z and info.q_bits > t + 2 * u
        # the products run on the fewest 28-bit digits that hold 2q, except one-limb moduli
        full = (32 * info.L + 28) // 28
        want = -(-(info.q_bits + 1) // 28) if info.L >= 2 else full
        assert info.digits == max(want, full - 1), c
    for c in range(18, 24):
        if c - 18 in cands:
            assert c in cands, c


def test_errors_before_device_work(dk):
    ctx = dk.Context()
    # p^z below Mm 2^(2u)
    with pytest.raises(dk.DkssError) as e:
        ctx.plan_info(64, 64, dk.Params.make(5, 2, 60, 64, 1, cutoff_bits=0))
    assert e.value.code == dk.ERANGE
    # capacity M m/2 u below the operand
    with pytest.raises(dk.DkssError) as e:
        ctx.plan_info(4096, 4096, dk.Params.make(5, 2, 20, 128, 1, cutoff_bits=0))
    assert e.value.code == dk.ERANGE
    # radices not summing to log2(2M), radix above 2m
    with pytest.raises(dk.DkssError):
        ctx.plan_info(64, 64, dk.Params.make(5, 2, 0, 128, 1, radices=[3, 2], cutoff_bits=0))
    with pytest.raises(dk.DkssError):
        ctx.plan_info(64, 64, dk.Params.make(5, 2, 0, 128, 1, radices=[4, 2], cutoff_bits=0))
    # M < m
    with pytest.raises(dk.DkssError):
        ctx.plan_info(64, 64, dk.Params.make(2, 3, 0, 128, 1, cutoff_bits=0))
    L = dk.lib()
    assert L.dkss_mul(None, None, None, 0, None, 0, None, None, 0, None) == dk.EINVAL
    assert L.dkss_ctx_create(None, 0, None) == dk.EINVAL
    h = ctypes.c_void_p()
    assert L.dkss_ctx_create(ctypes.byref(h), 7, None) == dk.EINVAL
    assert L.dkss_strerror(dk.ENOSPC) == b"workspace too small"


def test_karatsuba_base_case_routing(dk):
    """The base case covers products whose leaves fit the schoolbook after at most two Karatsuba
    levels (up to 8186 x 8186 words); such products need a workspace, plain schoolbook products
    none, and beyond two levels the product goes to DKSS."""
    ctx = dk.Context()
    for alen, blen, base in [(2048, 2048, True), (4000, 4000, True), (8184, 8184, True), (64, 8000, True),
                             (8186, 8186, True), (8187, 8187, False)]:
        p = ctx.select_params(32 * alen, 32 * blen)
        p.cutoff_bits = 2 ** 64 - 1
        assert bool(ctx.plan_info(alen, blen, p).schoolbook) == base, (alen, blen)
        ws = ctx.workspace_bytes(alen, blen, p)
        assert (ws > 0) == (alen + blen > 4096), (alen, blen, ws)


def test_workspace_and_schoolbook_routing(dk):
    ctx = dk.Context()
    assert ctx.workspace_bytes(0, 100) == 0
    assert ctx.plan_info(16, 16).schoolbook == 1          # below the default cutoff
    info = ctx.plan_info(8192, 8192)
    assert info.schoolbook == 0
    assert ctx.workspace_bytes(8192, 8192) >= 2 * info.poly_bytes


def test_transform_memory_two_polynomials(dk):
    """The transform needs no temporary polynomial (thesis Sec. 5.1 outlook; Sec. 4.5 counts three
    polynomials): a 2^28-bit product's workspace under the thesis rule is the two polynomials and
    the rho table plus less than 1 % for decode and carries, 24.6N bits against 36N for three
    polynomials of the same coefficients."""
    ctx = dk.Context(dk.POLICY_THESIS)
    n = 1 << 23
    info = ctx.plan_info(n, n)
    ws = ctx.workspace_bytes(n, n)
    base = 2 * info.poly_bytes + info.table_bytes
    assert base <= ws < base + info.poly_bytes // 64
    assert ws * 8 < 25 * (32 * n)


@pytest.mark.parametrize("a,b,batch", [(1, 1, 1), (2 ** 18, 2 ** 15, 16), (2 ** 30, 2 ** 30, 4096),
                                       (100, 5000, 3), (2 ** 36, 7, 65535), (0, 40, 1)])
def test_selector_features_match_oracle(dk, a, b, batch):
    import numpy as np
    import oracle.mlp as om
    np.testing.assert_allclose(dk.mlp_features(a, b, batch), om.features(a, b, batch), rtol=1e-6,
                               atol=1e-7)


def test_selector_weights_io_and_errors(dk, tmp_path):
    import numpy as np
    w = np.random.default_rng(3).normal(0, 1, dk.MLP_NPARAM).astype(np.float32)
    path = str(tmp_path / "w.txt")
    dk.mlp_save(path, w, comment="test weights\nsecond line")
    assert np.array_equal(dk.mlp_load(path), w)          # %.9g round-trips float32 exactly
    bad = str(tmp_path / "bad.txt")
    with open(bad, "w") as f:
        f.write("3 64 7\n" + "0\n" * dk.MLP_NPARAM)       # wrong output count
    with pytest.raises(dk.DkssError):
        dk.mlp_load(bad)
    with open(bad, "w") as f:
        f.write("3 64 %d\n" % dk.MLP_OUT + "0\n" * (dk.MLP_NPARAM - 1))   # one weight short
    with pytest.raises(dk.DkssError):
        dk.mlp_load(bad)
    ctx = dk.Context(dk.POLICY_LEARNED, tuning_dir=str(tmp_path))   # no dkss_mlp.txt there
    assert ctx.mlp_choose(2 ** 20, 2 ** 20) == -1                     # thesis fallback, no device work
    p = ctx.select_params(2 ** 20, 2 ** 20)
    t = dk.Context().select_params(2 ** 20, 2 ** 20)
    assert p.as_dict() == t.as_dict()
    w[17] = np.nan
    with pytest.raises(dk.DkssError):
        ctx.set_mlp(w)
    with pytest.raises(dk.DkssError):
        ctx.mlp_choose(0, 5)
    assert dk.lib().dkss_mlp_features(1, 1, 0, (ctypes.c_float * 3)()) == dk.EINVAL
    assert dk.lib().dkss_mlp_work_floats(10) == 10 * (dk.MLP_NPARAM + 1)


def test_committed_selector_weights_load(dk):
    path = os.path.join(dk.TUNING_DIR, "dkss_mlp.txt")
    if not os.path.exists(path):
        pytest.skip("no trained selector weights in the package")
    import numpy as np
    w = dk.mlp_load(path)
    assert w.shape == (dk.MLP_NPARAM,) and np.all(np.isfinite(w))


def test_tuned_table_with_level_split(dk, tmp_path):
    """Tuned lines may carry a level split and an LDS budget; a split that does not fit the
    candidate's transform length or radix cap is ignored (default split)."""
    N = 2 ** 28
    ctx0 = dk.Context()
    cands = dict(ctx0.candidates(N, N))
    c = sorted(cands)[0]
    p = cands[c]
    total = p.log2_M + 1
    cap = max(p.radix_log2[i] for i in range(p.n_levels))
    split = [cap - 1] * (total // (cap - 1)) + ([total % (cap - 1)] if total % (cap - 1) else [])
    with open(tmp_path / "dkss_tuning.txt", "w") as f:
        f.write("# test\n")
        f.write("0 27.5 %d %s 16384\n" % (c, ".".join(map(str, split))))
        f.write("27.5 28.5 %d %s 16384\n" % (c, ".".join(map(str, [1] * (total - 1)))))   # sum short
        f.write("28.5 64 %d\n" % c)
    ctx = dk.Context(dk.POLICY_TUNED, tuning_dir=str(tmp_path))
    q = ctx.select_params(2 ** 27, 2 ** 27)
    q27 = dict(ctx0.candidates(2 ** 27, 2 ** 27))[c]
    assert (q.log2_M, q.log2_m, q.p_bits) == (q27.log2_M, q27.log2_m, q27.p_bits)
    if sum(split) == q27.log2_M + 1:
        assert [q.radix_log2[i] for i in range(q.n_levels)] == split
    q = ctx.select_params(N, N)
    assert [q.radix_log2[i] for i in range(q.n_levels)] == [p.radix_log2[i] for i in range(p.n_levels)]
    info = ctx.plan_info(N // 32, N // 32)
    assert [info.params.radix_log2[i] for i in range(info.params.n_levels)] == \
        [p.radix_log2[i] for i in range(p.n_levels)]


def test_tuned_table_batch_sections_and_schoolbook(dk, tmp_path):
    """"@batch B" sections: a product takes the entry of the largest B not above its batch size
    whose range holds its N, falling back to smaller B; a schoolbook entry selects the base case
    (cutoff UINT64_MAX, the thesis tuple) and falls back to DKSS where the base case does not
    apply."""
    ctx0 = dk.Context()
    sizes = [2 ** 11, 2 ** 13, 2 ** 16, 2 ** 22]
    common = set.intersection(*[{c for c, _ in ctx0.candidates(N, N)} for N in sizes])
    c1, c2, c3 = sorted(common)[:3]
    with open(tmp_path / "dkss_tuning.txt", "w") as f:
        f.write("0 13 %d\n13 20 %d\n20 64 %d\n" % (dk.CAND_SCHOOLBOOK, c1, dk.CAND_SCHOOLBOOK))
        f.write("@batch 16\n0 14 %d\n14 20 %d   # comment\n" % (dk.CAND_SCHOOLBOOK, c2))
        f.write("@batch 256\n10 12 %d\n" % c3)
    ctx = dk.Context(dk.POLICY_TUNED, tuning_dir=str(tmp_path))

    def tup(p):
        return (p.log2_M, p.log2_m, p.p_bits)

    def cand(c, N):
        return tup(dict(ctx0.candidates(N, N))[c])

    thesis = {N: ctx0.select_params(N, N) for N in sizes}
    school = 2 ** 64 - 1
    for N, batch, want in [(2 ** 13, 1, c1), (2 ** 16, 1, c1), (2 ** 16, 16, c2), (2 ** 16, 300, c2),
                           (2 ** 11, 300, c3), (2 ** 11, 255, None), (2 ** 13, 16, None),
                           (2 ** 22, 16, None), (2 ** 22, 1, None), (2 ** 11, 1, None)]:
        q = ctx.select_params(N, N, batch)
        if want is None:                       # a schoolbook entry
            assert tup(q) == tup(thesis[N]) and q.cutoff_bits == school, (N, batch)
        else:
            assert tup(q) == cand(want, N) and q.cutoff_bits == 2048, (N, batch)
    # plan_info plans at batch 1: the schoolbook entry below 2^13 bits applies beyond the default
    # cutoff; the one above 2^20 bits exceeds the base case and runs the thesis tuple
    assert ctx.plan_info(200, 200).schoolbook == 1 and ctx0.plan_info(200, 200).schoolbook == 0
    big = ctx.plan_info(2 ** 16, 2 ** 16)
    assert big.schoolbook == 0 and tup(big.params) == tup(ctx0.plan_info(2 ** 16, 2 ** 16).params)


def test_tuned_table_writer_sections(dk, tmp_path):
    """tune.write_tuned_table: half-open buckets around the measured sizes, the fastest output
    per size (the schoolbook included), one "@batch B" section per measured batch size ending at
    its largest size, and a table the library reads back with the same choices."""
    from paper_1503_04955_amd import tune
    S = dk.CAND_SCHOOLBOOK
    ms = {  # (x, batch) -> {output: ms}
        (12.0, 1): {S: 0.01, 3: 0.03, "thesis": 0.05}, (12.5, 1): {S: 0.05, 3: 0.03, "thesis": 0.06},
        (13.0, 1): {2: 0.02, 3: 0.04, "thesis": 0.07},
        (12.0, 16): {S: 0.001, 2: 0.004, "thesis": 0.005}, (13.0, 16): {S: 0.009, 8: 0.003, "thesis": 0.006},
    }
    rows = [{"log2_a": x, "ratio": 1, "batch": bt, "cand": c, "ms": v}
            for (x, bt), d in ms.items() for c, v in d.items()]
    rows.append({"log2_a": 12.0, "ratio": 2, "batch": 1, "cand": 9, "ms": 0.0001})   # other ratios ignored
    path = tmp_path / "dkss_tuning.txt"
    tune.write_tuned_table(rows, str(path))
    lines = [l.split("#")[0].split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert lines == [["0.000", "12.250", "S"], ["12.250", "12.750", "3"], ["12.750", "64.000", "2"],
                     ["@batch", "16"], ["0.000", "12.500", "S"], ["12.500", "13.500", "8"]]
    ctx = dk.Context(dk.POLICY_TUNED, tuning_dir=str(tmp_path))
    school = 2 ** 64 - 1
    assert ctx.select_params(2 ** 12, 2 ** 12, 1).cutoff_bits == school
    assert ctx.select_params(2 ** 12, 2 ** 12, 20).cutoff_bits == school
    p16 = ctx.select_params(2 ** 13, 2 ** 13, 16)
    c8 = dict(dk.Context().candidates(2 ** 13, 2 ** 13))[8]
    assert (p16.log2_M, p16.log2_m, p16.p_bits) == (c8.log2_M, c8.log2_m, c8.p_bits)
    p1 = ctx.select_params(2 ** 14, 2 ** 14, 16)          # beyond the batch-16 section: batch 1's entry
    c2 = dict(dk.Context().candidates(2 ** 14, 2 ** 14))[2]
    assert (p1.log2_M, p1.log2_m, p1.p_bits) == (c2.log2_M, c2.log2_m, c2.p_bits)


def test_tuned_table_names_the_rule_where_nothing_beats_it(dk, tmp_path):
    """Where no measured candidate beats the thesis rule's own timing, the writer names the rule
    ("T"); the library then plans that size with the rule, also inside a batch section (not with
    the entry of a smaller batch size)."""
    from paper_1503_04955_amd import tune
    ms = {(16.0, 1): {3: 0.03, 8: 0.06, "thesis": 0.04}, (17.0, 1): {3: 0.05, "thesis": 0.09},
          (18.0, 1): {3: 0.05, "thesis": 0.04},
          (16.0, 16): {2: 0.02, "thesis": 0.01}, (17.0, 16): {2: 0.02, "thesis": 0.03}}
    rows = [{"log2_a": x, "ratio": 1, "batch": bt, "cand": c, "ms": v}
            for (x, bt), d in ms.items() for c, v in d.items()]
    path = tmp_path / "dkss_tuning.txt"
    tune.write_tuned_table(rows, str(path))
    lines = [l.split("#")[0].split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert lines == [["0.000", "16.500", "3"], ["16.500", "17.500", "3"], ["17.500", "64.000", "T"],
                     ["@batch", "16"], ["0.000", "16.500", "T"], ["16.500", "17.500", "2"]]
    ctx = dk.Context(dk.POLICY_TUNED, tuning_dir=str(tmp_path))
    ctx0 = dk.Context()

    def tup(p):
        return (p.log2_M, p.log2_m, p.u, p.p_bits)

    rule = {N: tup(ctx0.select_params(N, N)) for N in (2 ** 16, 2 ** 18)}
    c3 = {N: tup(dict(ctx0.candidates(N, N))[3]) for N in (2 ** 16, 2 ** 17)}
    assert c3[2 ** 16] != rule[2 ** 16]          # the rule entry of batch 16 decides, not batch 1's
    assert tup(ctx.select_params(2 ** 16, 2 ** 16, 1)) == c3[2 ** 16]
    for batch in (16, 100):
        assert tup(ctx.select_params(2 ** 16, 2 ** 16, batch)) == rule[2 ** 16], batch
    assert tup(ctx.select_params(2 ** 17, 2 ** 17)) == c3[2 ** 17]
    assert tup(ctx.select_params(2 ** 18, 2 ** 18)) == rule[2 ** 18]


def test_smul_parameters_and_product_form(dk):
    """SMUL's plan (host only): the ring for 2^16..2^30-bit products satisfies the convolution
    bound of the outermost form (min(na, nb) (2^s - 1)^2 < 2^K, n | 2K), and the componentwise
    products run on the matrix cores where their kernel exists (lw <= 16), on the vector units
    beyond; an explicit form is honoured and one the ring cannot take is refused."""
    for bits in (16, 20, 24, 26, 28, 30):
        n = (1 << bits) // 32
        p = dk.smul_select(n, n)
        N = 1 << p.log2_n
        K = p.K
        assert K == 2048 * p.lw and (2 * K) % N == 0
        na = -(-32 * n // p.s)
        assert 2 * na - 1 <= N and na * ((1 << p.s) - 1) ** 2 < (1 << K), bits
        assert p.products == (2 if p.lw <= 16 else 1), (bits, p.as_dict())
    with pytest.raises(dk.DkssError) as e:
        dk.smul_workspace_bytes(1 << 20, 1 << 20, dk.SmulParams.make(0, 32, 2))
    assert e.value.code == dk.ERANGE
    assert dk.smul_workspace_bytes(1 << 18, 1 << 18, dk.SmulParams.make(0, 0, 1)) > 0
