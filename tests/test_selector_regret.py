"""What the trained selector gains over the thesis's rule, from committed measurements.

The package's weights (tuning/dkss_mlp.txt) choose, at every held-out point of
tuning/timings_heldout.json (sizes and batch sizes never seen in training, 2^30 bits among
them), the output of least predicted time among the outputs measured there; its regret
t(choice) / t(fastest measured) - 1 is compared with the thesis rule's.  The network is
evaluated with the float64 oracle forward pass (the GPU forward kernel is compared with it in
tests/test_gpu_mlp.py), the inputs with the library's host feature function.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle.mlp as om

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNING = os.path.join(ROOT, "paper_1503_04955_amd", "tuning")


def _limbs(x, ratio):
    n = max(1, int(round(2.0 ** x / 32)))
    return n, max(1, int(round(n / ratio)))


@pytest.fixture(scope="module")
def data():
    wpath = os.path.join(TUNING, "dkss_mlp.txt")
    hpath = os.path.join(TUNING, "timings_heldout.json")
    if not (os.path.exists(wpath) and os.path.exists(hpath)):
        pytest.skip("no trained selector or held-out timings in the package")
    import paper_1503_04955_amd as dk
    w = dk.mlp_load(wpath).astype(np.float64)
    with open(hpath) as f:
        rows = json.load(f)["rows"]
    pts = {}
    for r in rows:
        pts.setdefault((r["log2_a"], r["ratio"], r["batch"]), {})[r["cand"]] = r["ms"]
    with open(os.path.join(TUNING, "timings.json")) as f:
        train_keys = {(r["log2_a"], r["ratio"], r["batch"]) for r in json.load(f)["rows"]}
    return dk, w, pts, train_keys


def _regrets(dk, w, pts):
    out = []
    for (x, ratio, batch), ms in sorted(pts.items()):
        n, nb = _limbs(x, ratio)
        f = dk.mlp_features(32 * n, 32 * nb, batch).astype(np.float64)
        y, _ = om.forward(w, f[None, :], dk.MLP_OUT)
        meas = [c for c in ms if isinstance(c, int)]
        best = min(ms[c] for c in meas)
        choice = min(meas, key=lambda c: y[0, c])
        out.append(((x, ratio, batch), ms[choice] / best - 1, ms["thesis"] / best - 1))
    return out


def test_heldout_points_are_not_training_points(data):
    dk, w, pts, train_keys = data
    assert pts and not (set(pts) & train_keys)
    assert any(k[0] == 30.0 for k in pts)


def test_selector_beats_thesis_rule_on_heldout_points(data):
    dk, w, pts, _ = data
    regs = _regrets(dk, w, pts)
    learned = np.array([r[1] for r in regs])
    thesis = np.array([r[2] for r in regs])
    # geometric-mean time ratio to the best measured output
    g_learned = math.exp(np.mean(np.log1p(learned)))
    g_thesis = math.exp(np.mean(np.log1p(thesis)))
    print("held-out regret: learned mean %.3f (geo %.3f), thesis mean %.3f (geo %.3f), %d points"
          % (learned.mean(), g_learned, thesis.mean(), g_thesis, len(regs)))
    assert g_learned < g_thesis
    assert learned.mean() < thesis.mean()


def test_selector_at_2p30_bits(data):
    """The single 2^30-bit products (held out): the selector's choice is at least as fast as the
    thesis rule's tuple."""
    dk, w, pts, _ = data
    for key, rl, rt in _regrets(dk, w, pts):
        if key[0] == 30.0 and key[2] == 1:
            assert rl <= rt, (key, rl, rt)
