"""GPU tests of the learned selector: the network kernels against the float64 oracle (forward,
loss, gradient, Adam), training, and the LEARNED policy's products (bit-exact) and regret."""
import os
import time

import numpy as np
import pytest

import oracle.mlp as om
import seeded_inputs as SI
from conftest import host_residues, primes61, residues_agree

pytestmark = pytest.mark.gpu

OUT = 25                      # DKSS_MLP_OUT: 24 candidates and the base case


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1503_04955_amd as dk
    assert torch.cuda.is_available()
    dk.lib()
    return dk, torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _case(seed, n, scale=0.5):
    rng = np.random.default_rng(seed)
    th = rng.normal(0, scale, om.n_params(OUT)).astype(np.float32)
    X = rng.normal(0, 1, (n, om.IN)).astype(np.float32)
    T = rng.normal(0, 1, (n, OUT)).astype(np.float32)
    Mk = (rng.random((n, OUT)) < 0.7).astype(np.float32)
    return th, X, T, Mk


@pytest.mark.parametrize("n", [1, 3, 4, 257, 1001])
def test_forward_matches_oracle(env, n):
    dk, torch = env
    th, X, _, _ = _case(10 + n, n)
    y = dk.mlp_forward(_dev(torch, th), _dev(torch, X)).cpu().numpy()
    yo, _ = om.forward(th.astype(np.float64), X.astype(np.float64), OUT)
    # float32 sums of at most 64 products per unit
    assert np.max(np.abs(y - yo)) <= 2e-5 * max(1.0, np.max(np.abs(yo)))


@pytest.mark.parametrize("n", [1, 5, 257, 1000])
def test_loss_and_gradient_match_oracle(env, n):
    dk, torch = env
    th, X, T, Mk = _case(20 + n, n)
    ms = float(Mk.sum())
    g, loss = dk.mlp_loss_grad(_dev(torch, th), _dev(torch, X), _dev(torch, T), _dev(torch, Mk), ms)
    g = g.cpu().numpy()
    lo, go = om.loss_grad(th.astype(np.float64), X.astype(np.float64), T.astype(np.float64),
                          Mk.astype(np.float64), ms, OUT)
    assert abs(float(loss.item()) - lo) <= 1e-5 * abs(lo)
    # per-parameter float32 sums over n samples: bounded against the gradient's scale
    scale = np.max(np.abs(go))
    err = np.abs(g - go)
    assert np.max(err) <= 1e-4 * scale, (np.argmax(err), np.max(err), scale)
    # entries that are large against the scale also match relatively
    big = np.abs(go) > 0.05 * scale
    assert np.all(err[big] <= 2e-4 * np.abs(go[big]) + 1e-6 * scale)


def test_weighted_loss_and_gradient_match_oracle(env):
    """Real-valued per-output weights (as the trainer's decision weights) in place of the 0/1
    mask: the same kernels, the oracle's weighted definition."""
    dk, torch = env
    from paper_1503_04955_amd import learn
    th, X, T, Mk = _case(60, 300)
    W = learn.decision_weights(T, Mk)
    ws = float(W.sum())
    g, loss = dk.mlp_loss_grad(_dev(torch, th), _dev(torch, X), _dev(torch, T), _dev(torch, W), ws)
    lo, go = om.loss_grad(th.astype(np.float64), X.astype(np.float64), T.astype(np.float64),
                          W.astype(np.float64), ws, OUT)
    assert abs(float(loss.item()) - lo) <= 1e-5 * abs(lo)
    scale = np.max(np.abs(go))
    assert np.max(np.abs(g.cpu().numpy() - go)) <= 1e-4 * scale


def test_gradient_is_deterministic(env):
    dk, torch = env
    th, X, T, Mk = _case(31, 999)
    args = [_dev(torch, a) for a in (th, X, T, Mk)] + [float(Mk.sum())]
    g1, l1 = dk.mlp_loss_grad(*args)
    g2, l2 = dk.mlp_loss_grad(*args)
    assert torch.equal(g1, g2) and torch.equal(l1, l2)


def test_adam_matches_oracle(env):
    dk, torch = env
    rng = np.random.default_rng(40)
    th = rng.normal(0, 1, om.n_params(OUT)).astype(np.float32)
    p = _dev(torch, th)
    m1 = torch.zeros_like(p)
    m2 = torch.zeros_like(p)
    tho, m1o, m2o = th.astype(np.float64), np.zeros(th.size), np.zeros(th.size)
    for step in range(1, 4):
        g = rng.normal(0, 1, th.size).astype(np.float32)
        dk.mlp_adam(p, _dev(torch, g), m1, m2, step, 0.01)
        tho, m1o, m2o = om.adam_step(tho, g.astype(np.float64), m1o, m2o, step, 0.01)
    np.testing.assert_allclose(p.cpu().numpy(), tho, rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(m1.cpu().numpy(), m1o, rtol=1e-5, atol=1e-7)


def test_training_fits_a_teacher(env):
    """Adam on the GPU kernels fits targets made by a random teacher network (oracle forward):
    the loss falls by more than 20x and the student's argmin agrees with the teacher's on most
    samples."""
    dk, torch = env
    from paper_1503_04955_amd import learn
    rng = np.random.default_rng(50)
    teacher = rng.normal(0, 0.4, om.n_params(OUT))
    X = rng.uniform(-1, 1, (400, om.IN)).astype(np.float32)
    T, _ = om.forward(teacher, X.astype(np.float64), OUT)
    Mk = np.ones_like(T, dtype=np.float32)
    w, curve = learn.train(X, T.astype(np.float32), Mk, steps=1500, lr=0.01, seed=3)
    assert curve[-1][1] < curve[0][1] / 20, curve[::5]
    ys, _ = om.forward(w.astype(np.float64), X.astype(np.float64), OUT)
    agree = np.mean(np.argmin(ys, axis=1) == np.argmin(T, axis=1))
    assert agree > 0.6, agree


def _weights(dk):
    path = os.path.join(dk.TUNING_DIR, "dkss_mlp.txt")
    if not os.path.exists(path):
        pytest.skip("no trained selector weights in the package")
    return dk.mlp_load(path)


def test_choice_is_argmin_of_forward(env):
    """dkss_mlp_choose agrees with the argmin of the forward kernel over the feasible outputs."""
    dk, torch = env
    w = _weights(dk)
    ctx = dk.Context(dk.POLICY_LEARNED)
    ctx.set_mlp(w)
    wd = _dev(torch, w)
    for bits_a, bits_b, batch in [(2 ** 12, 2 ** 12, 1), (2 ** 16, 2 ** 14, 4096), (2 ** 22, 2 ** 20, 256),
                                  (2 ** 28, 2 ** 28, 1), (2 ** 30, 2 ** 27, 1), (3000, 70000, 77)]:
        y = dk.mlp_forward(wd, _dev(torch, dk.mlp_features(bits_a, bits_b, batch)[None, :])).cpu().numpy()[0]
        feas = [c for c, _ in ctx.candidates(bits_a, bits_b)]
        na, nb = -(-bits_a // 32), -(-bits_b // 32)
        if na + nb <= 4096:
            feas.append(dk.CAND_SCHOOLBOOK)
        want = min(feas, key=lambda c: y[c])
        assert ctx.mlp_choose(bits_a, bits_b, batch) == want
        p = ctx.select_params(bits_a, bits_b, batch)
        if want == dk.CAND_SCHOOLBOOK:
            assert p.cutoff_bits == 2 ** 64 - 1
        else:
            assert p.cutoff_bits == 0
            q = dict(ctx.candidates(bits_a, bits_b))[want]
            assert (p.log2_M, p.log2_m, p.u, p.p_bits) == (q.log2_M, q.log2_m, q.u, q.p_bits)


@pytest.mark.parametrize("alen,blen", [(128, 128), (512, 64), (2048, 2048), (3000, 1000),
                                       (8192, 8192), (40000, 5000)])
def test_learned_policy_products_exact(env, alen, blen):
    """Products under the LEARNED policy (whatever it picks, schoolbook included) equal the
    oracle's schoolbook product."""
    dk, torch = env
    from oracle import coracle
    _weights(dk)
    ctx = dk.Context(dk.POLICY_LEARNED)
    a, b = SI.operand_pair(SI.SEED_BASE + 700 + alen, alen, blen)
    c = dk.to_host(ctx.mul(dk.to_device(a), dk.to_device(b)))
    assert np.array_equal(c, coracle.schoolbook(a, b))


def test_learned_policy_batch_exact(env):
    """A mixed batch under the LEARNED policy equals the same products under the thesis rule."""
    dk, torch = env
    _weights(dk)
    lens = SI.batch_lengths(SI.SEED_BASE + 77, 300, hi_bits=18)
    as_, bs = [], []
    for i, (al, bl) in enumerate(lens):
        a, b = SI.operand_pair(SI.SEED_BASE + 9000 + i, al, bl)
        as_.append(dk.to_device(a))
        bs.append(dk.to_device(b))
    out_l = dk.Context(dk.POLICY_LEARNED).mul_batch(as_, bs)
    out_t = dk.Context().mul_batch(as_, bs)
    assert all(torch.equal(x, y) for x, y in zip(out_l, out_t))


def _time(fn, torch, reps=3):
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return sorted(ts)[len(ts) // 2]


def test_learned_beats_thesis_on_heldout_sizes(env):
    """Live timing on sizes outside the training grid, the largest 2^30 bits: the products under
    the LEARNED policy take less time in total than under the thesis rule, are identical, and pass
    residue checks against the oracle's residues of a, b and c."""
    dk, torch = env
    _weights(dk)
    ctx_t = dk.Context()
    ctx_l = dk.Context(dk.POLICY_LEARNED)
    tot_t = tot_l = 0.0
    lines = []
    for x in (13.75, 18.25, 22.75, 26.25, 30.0):
        n = int(round(2 ** x / 32))
        g = torch.Generator(device="cuda")
        g.manual_seed(int(x * 100))
        a = torch.randint(-2 ** 31, 2 ** 31, (n,), dtype=torch.int32, device="cuda", generator=g)
        b = torch.randint(-2 ** 31, 2 ** 31, (n,), dtype=torch.int32, device="cuda", generator=g)
        ct = torch.empty(2 * n, dtype=torch.int32, device="cuda")
        cl = torch.empty_like(ct)
        wt = torch.empty(max(ctx_t.workspace_bytes(n, n), 1), dtype=torch.uint8, device="cuda")
        wl = torch.empty(max(ctx_l.workspace_bytes(n, n), 1), dtype=torch.uint8, device="cuda")
        mt = _time(lambda: ctx_t.mul(a, b, out=ct, ws=wt), torch)
        ml = _time(lambda: ctx_l.mul(a, b, out=cl, ws=wl), torch)
        assert torch.equal(ct, cl)
        # c = a*b modulo 4 seeded primes, every residue computed by the oracle on the host
        qs = primes61(int(x * 100), 4)
        ra, rb, rc = host_residues([dk.to_host(a), dk.to_host(b), dk.to_host(cl)], qs)
        assert residues_agree(ra, rb, rc, qs), x
        tot_t += mt
        tot_l += ml
        lines.append("2^%.2f: thesis %.3f ms, learned %.3f ms (choice %d)"
                     % (x, mt, ml, ctx_l.mlp_choose(32 * n, 32 * n)))
        del a, b, ct, cl, wt, wl
        torch.cuda.empty_cache()
    print("\n".join(lines))
    assert tot_l < tot_t, lines


def test_library_loaded_before_torch_in_a_fresh_process(env):
    """The binding loads torch's HIP runtime before the library, whatever the caller imports
    first, so a process never holds two runtimes (the second one would see no device)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_1503_04955_amd as dk\n"
            "f = dk.mlp_features(1 << 20, 1 << 18, 4)\n"
            "import torch, numpy as np\n"
            "w = torch.zeros(dk.MLP_NPARAM, device='cuda')\n"
            "y = dk.mlp_forward(w, torch.from_numpy(f[None, :]).cuda())\n"
            "assert float(y.abs().sum()) == 0.0\n"
            "print('ok')\n" % root)
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=240)
    assert res.returncode == 0 and "ok" in res.stdout, res.stderr[-2000:]
