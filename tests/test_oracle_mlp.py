"""Pins of the selector oracle (oracle/mlp.py) against facts outside its own code: finite
differences, the closed forms of the all-active and all-inactive networks, Adam's first step."""
import numpy as np
import pytest

import oracle.mlp as om

OUT = 25


def _rand(seed, n, n_out=OUT, scale=0.5):
    rng = np.random.default_rng(seed)
    th = rng.normal(0, scale, om.n_params(n_out))
    X = rng.normal(0, 1, (n, om.IN))
    T = rng.normal(0, 1, (n, n_out))
    Mk = (rng.random((n, n_out)) < 0.7).astype(np.float64)
    return th, X, T, Mk


def test_param_count():
    # 3*64 + 64 + 64*64 + 64 + 25*64 + 25
    assert om.n_params(OUT) == 6041


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_gradient_central_differences(seed):
    """Back-propagation against (L(theta + h e_i) - L(theta - h e_i)) / 2h, every parameter of a
    network with 8 hidden units and 5 outputs (the same code at a size where all coordinates are
    checked), and a random sample of coordinates of the full-size network."""
    rng = np.random.default_rng(seed)
    for n_hid, n_out, coords in ((8, 5, None), (64, OUT, 300)):
        th = rng.normal(0, 0.5, om.n_params(n_out, om.IN, n_hid))
        X = rng.normal(0, 1, (7, om.IN))
        T = rng.normal(0, 1, (7, n_out))
        Mk = (rng.random((7, n_out)) < 0.6).astype(np.float64)
        ms = Mk.sum()
        _, g = om.loss_grad(th, X, T, Mk, ms, n_out, om.IN, n_hid)
        idx = range(th.size) if coords is None else rng.choice(th.size, coords, replace=False)
        h = 1e-6
        for i in idx:
            e = np.zeros_like(th)
            e[i] = h
            fd = (om.loss(th + e, X, T, Mk, ms, n_out, om.IN, n_hid) -
                  om.loss(th - e, X, T, Mk, ms, n_out, om.IN, n_hid)) / (2 * h)
            assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (n_hid, i, fd, g[i])


def test_all_active_is_one_affine_map():
    """With every pre-activation positive ReLU is the identity, so the network equals the
    composed affine map A x + c with A = W3 W2 W1 and c = W3 (W2 b1 + b2) + b3."""
    rng = np.random.default_rng(5)
    W1 = rng.uniform(0.1, 1, (64, 3))
    b1 = rng.uniform(0.1, 1, 64)
    W2 = rng.uniform(0.1, 1, (64, 64))
    b2 = rng.uniform(0.1, 1, 64)
    W3 = rng.normal(0, 1, (OUT, 64))
    b3 = rng.normal(0, 1, OUT)
    th = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])
    X = rng.uniform(0, 1, (9, 3))
    y, _ = om.forward(th, X, OUT)
    A = W3 @ W2 @ W1
    c = W3 @ (W2 @ b1 + b2) + b3
    np.testing.assert_allclose(y, X @ A.T + c, rtol=1e-12, atol=1e-9)
    # one hand-checked entry: output 0 of sample 0 by explicit sums
    h1 = [max(0.0, sum(W1[j, k] * X[0, k] for k in range(3)) + b1[j]) for j in range(64)]
    h2 = [max(0.0, sum(W2[i, j] * h1[j] for j in range(64)) + b2[i]) for i in range(64)]
    assert abs(y[0, 0] - (sum(W3[0, i] * h2[i] for i in range(64)) + b3[0])) < 1e-9


def test_all_inactive_first_layer():
    """b1 very negative: h1 = 0, so y = W3 relu(b2) + b3 for every input, and the gradient of
    W1 and b1 is zero."""
    th, X, T, Mk = _rand(6, 11)
    W1, b1, W2, b2, W3, b3 = (a.copy() for a in om.unpack(th, OUT))
    b1[:] = -1e6
    th2 = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])
    y, _ = om.forward(th2, X, OUT)
    np.testing.assert_allclose(y, np.tile(W3 @ np.maximum(b2, 0) + b3, (11, 1)), rtol=1e-12)
    _, g = om.loss_grad(th2, X, T, Mk, Mk.sum(), OUT)
    assert np.all(g[:64 * 3 + 64] == 0)


def test_masked_targets_do_not_matter():
    th, X, T, Mk = _rand(7, 13)
    T2 = T + (1 - Mk) * 1e3
    l1, g1 = om.loss_grad(th, X, T, Mk, Mk.sum(), OUT)
    l2, g2 = om.loss_grad(th, X, T2, Mk, Mk.sum(), OUT)
    assert l1 == l2 and np.array_equal(g1, g2)


def test_adam_first_step_is_signed_lr():
    """At step 1 with zero moments the bias-corrected ratio is g / (|g| + eps): each parameter
    moves by lr * sign(g) (up to eps / |g|)."""
    rng = np.random.default_rng(8)
    th = rng.normal(0, 1, 100)
    g = rng.normal(0, 1, 100)
    new, m1, m2 = om.adam_step(th, g, np.zeros(100), np.zeros(100), 1, 0.01)
    np.testing.assert_allclose(new, th - 0.01 * np.sign(g), atol=1e-8)
    np.testing.assert_allclose(m1, 0.1 * g)
    np.testing.assert_allclose(m2, 0.001 * g * g)


def test_adam_constant_gradient():
    """A constant gradient keeps the corrected ratio at sign(g) on every step."""
    th = np.zeros(4)
    g = np.array([2.0, -3.0, 0.5, -0.25])
    m1 = np.zeros(4)
    m2 = np.zeros(4)
    for step in range(1, 6):
        th, m1, m2 = om.adam_step(th, g, m1, m2, step, 0.1)
    np.testing.assert_allclose(th, -0.5 * np.sign(g), atol=1e-7)


def test_features_closed_form():
    f = om.features(2 ** 21, 2 ** 12, 4096)
    np.testing.assert_allclose(f, [0.0, -1.0, 1.0])
    # rounding up to whole limbs; symmetric in the operands
    np.testing.assert_allclose(om.features(33, 2 ** 30, 1), om.features(2 ** 30, 64, 1))
    np.testing.assert_allclose(om.features(0, 1, 1), [(5 - 21) / 9, (5 - 21) / 9, 0])
