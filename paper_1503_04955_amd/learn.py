"""Train the learned parameter selector on the tuner's timings, on the GPU, with the library's own
network kernels (dkss_mlp_loss_grad, dkss_mlp_adam), and evaluate its regret.

    python -m paper_1503_04955_amd.learn [--timings DIR/timings.json] [--out DIR/dkss_mlp.txt]
                                         [--steps 3000] [--lr 0.01] [--seed 1]
    python -m paper_1503_04955_amd.learn --eval DIR/timings_heldout.json [--weights FILE]

Data: one sample per measured point (operand sizes, batch) of the tuner; input the selector's
features (dkss_mlp_features), target the natural log of milliseconds per product for each
output (DKSS candidate c, or the schoolbook), masked where the output was not measured
(infeasible at that size).  Loss: weighted mean squared error, each measured output weighted
by max(exp(-(ln t - ln t_best) / 0.3), 0.1), t_best the point's fastest output, so that the fit
is closest where it decides the argmin (an output three times slower than the best still
counts a tenth); Adam with a cosine-decayed step size; weights initialised from a seeded normal
(He scaling), output biases at the mean target.

Regret of a choice at a point = t(choice) / t(fastest measured output) - 1.
"""
import argparse
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_1503_04955_amd as dk  # noqa: E402

K = dk.MLP_OUT


def _limbs(x, ratio):
    n = max(1, int(round(2.0 ** x / 32)))
    return n, max(1, int(round(n / ratio)))


def load_points(path):
    """{(log2_a, ratio, batch): {label: ms per product}} from a tuner file."""
    with open(path) as f:
        rows = json.load(f)["rows"]
    pts = {}
    for r in rows:
        pts.setdefault((r["log2_a"], r["ratio"], r["batch"]), {})[r["cand"]] = r["ms"]
    return pts


def dataset(points):
    """(X[n][IN], T[n][K], mask[n][K], keys) float32 arrays of the measured outputs."""
    keys = sorted(points)
    X = np.zeros((len(keys), dk.MLP_IN), np.float32)
    T = np.zeros((len(keys), K), np.float32)
    Mk = np.zeros((len(keys), K), np.float32)
    for i, (x, ratio, batch) in enumerate(keys):
        n, nb = _limbs(x, ratio)
        X[i] = dk.mlp_features(32 * n, 32 * nb, batch)
        for label, ms in points[(x, ratio, batch)].items():
            if isinstance(label, int):
                T[i, label] = math.log(ms)
                Mk[i, label] = 1.0
    return X, T, Mk, keys


def decision_weights(T, Mk, tau=0.3, floor=0.1):
    """Per-output loss weights: max(exp(-(ln t - ln t_best) / tau), floor) where measured, else 0."""
    best = np.where(Mk > 0, T, np.inf).min(axis=1, keepdims=True)
    best = np.where(np.isfinite(best), best, 0.0)
    return np.where(Mk > 0, np.maximum(np.exp(-(T - best) / tau), floor), 0.0).astype(np.float32)


def init_params(seed, mean_target):
    """He-scaled normal weights, zero biases, output biases at the mean target."""
    rng = np.random.default_rng(seed)
    H, I = dk.MLP_HID, dk.MLP_IN
    parts = [rng.normal(0, math.sqrt(2.0 / I), H * I), np.zeros(H),
             rng.normal(0, math.sqrt(2.0 / H), H * H), np.zeros(H),
             rng.normal(0, math.sqrt(1.0 / H), K * H), np.full(K, mean_target)]
    return np.concatenate(parts).astype(np.float32)


def train(X, T, Mk, steps=3000, lr=0.01, seed=1, log_every=100, device="cuda"):
    """Full-batch Adam on the GPU; returns (weights, [(step, loss)])."""
    import torch
    n = X.shape[0]
    msum = float(Mk.sum())
    mean_t = float((T * Mk).sum() / msum)
    theta = torch.from_numpy(init_params(seed, mean_t)).to(device)
    x, t, mk = (torch.from_numpy(np.ascontiguousarray(a)).to(device) for a in (X, T, Mk))
    grad = torch.empty(dk.MLP_NPARAM, dtype=torch.float32, device=device)
    loss = torch.empty(1, dtype=torch.float32, device=device)
    m1 = torch.zeros(dk.MLP_NPARAM, dtype=torch.float32, device=device)
    m2 = torch.zeros_like(m1)
    work = dk.mlp_work(n, device)
    curve = []
    for step in range(1, steps + 1):
        dk.mlp_loss_grad(theta, x, t, mk, msum, grad=grad, loss=loss, work=work)
        if step == 1 or step % log_every == 0 or step == steps:
            curve.append((step, float(loss.item())))
        rate = 0.5 * lr * (1.0 + math.cos(math.pi * (step - 1) / steps))
        dk.mlp_adam(theta, grad, m1, m2, step, rate)
    dk.mlp_loss_grad(theta, x, t, mk, msum, grad=grad, loss=loss, work=work)
    curve.append((steps + 1, float(loss.item())))
    return theta.cpu().numpy(), curve


def predict(weights, X, device="cuda"):
    """Network outputs for inputs X (GPU forward kernel)."""
    import torch
    w = torch.from_numpy(np.ascontiguousarray(weights, np.float32)).to(device)
    x = torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(device)
    return dk.mlp_forward(w, x).cpu().numpy()


def tuned_choices(keys, tuning_dir=None):
    """The TUNED policy's output at each point (x, ratio, batch), from the library's own table
    lookup (dkss_select_params, host only): CAND_SCHOOLBOOK where the tuple comes with the base
    case, else the index of the candidate with the same tuple, "thesis" where none has it.  The
    candidates' timings at a point use the default level split, so the batch 1 entries' tuned
    splits and LDS budgets do not enter the comparison."""
    ctx = dk.Context(dk.POLICY_TUNED, tuning_dir=tuning_dir)
    out = []
    for x, ratio, batch in keys:
        n, nb = _limbs(x, ratio)
        q = ctx.select_params(32 * n, 32 * nb, batch)
        if 32 * min(n, nb) <= q.cutoff_bits:
            out.append(dk.CAND_SCHOOLBOOK)
            continue
        tup = (q.log2_M, q.log2_m, q.p_bits, q.z)
        same = [c for c, p in ctx.candidates(32 * n, 32 * nb)
                if (p.log2_M, p.log2_m, p.p_bits, p.z) == tup]
        out.append(same[0] if same else "thesis")
    return out


def regrets(points, pred, keys, tuned=None):
    """Per point: regret of the selector's choice (argmin of pred over measured outputs), of the
    thesis rule and, if tuned (the TUNED policy's output per point) is given, of the tuned
    table; an output not measured at the point (the base case beyond its limit) is the thesis
    rule's, as in the library."""
    out = []
    for i, key in enumerate(keys):
        ms = points[key]
        meas = [c for c in ms if isinstance(c, int)]
        best = min(ms[c] for c in meas)
        choice = min(meas, key=lambda c: pred[i, c])
        r = {"point": list(key), "choice": choice, "best": min(meas, key=lambda c: ms[c]),
             "learned": ms[choice] / best - 1, "thesis": ms["thesis"] / best - 1}
        if tuned is not None:
            r["tuned_choice"] = tuned[i]
            r["tuned"] = ms.get(tuned[i], ms["thesis"]) / best - 1
        out.append(r)
    return out


def summary(regs, field):
    v = [r[field] for r in regs if r.get(field) is not None]
    return {"mean": float(np.mean(v)), "geomean_ratio": float(np.exp(np.mean(np.log1p(v)))),
            "max": float(np.max(v)), "points": len(v)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--timings", default=os.path.join(dk.TUNING_DIR, "timings.json"))
    ap.add_argument("--out", default=os.path.join(dk.TUNING_DIR, "dkss_mlp.txt"))
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=0.01)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--eval", default="", help="held-out timings file to evaluate the weights on")
    ap.add_argument("--weights", default="", help="weights to evaluate (default: --out)")
    args = ap.parse_args()
    if args.eval:
        w = dk.mlp_load(args.weights or args.out)
        pts = load_points(args.eval)
        X, _, _, keys = dataset(pts)
        regs = regrets(pts, predict(w, X), keys, tuned_choices(keys))
        res = {"learned": summary(regs, "learned"), "tuned": summary(regs, "tuned"),
               "thesis": summary(regs, "thesis"), "points": regs}
        print(json.dumps({k: res[k] for k in ("learned", "tuned", "thesis")}), flush=True)
        with open(os.path.splitext(args.eval)[0] + "_regret.json", "w") as f:
            json.dump(res, f, indent=1)
        return
    pts = load_points(args.timings)
    X, T, Mk, keys = dataset(pts)
    w, curve = train(X, T, decision_weights(T, Mk), args.steps, args.lr, args.seed)
    regs = regrets(pts, predict(w, X), keys)
    fit = summary(regs, "learned")
    dk.mlp_save(args.out, w, comment=(
        "learned parameter selector, trained on %s (%d points, %d targets)\n"
        "Adam, %d steps, lr %g cosine, seed %d; final weighted loss %.5f; training-set regret "
        "mean %.4f"
        % (os.path.basename(args.timings), X.shape[0], int(Mk.sum()), args.steps, args.lr,
           args.seed, curve[-1][1], fit["mean"])))
    with open(os.path.splitext(args.out)[0] + "_train.json", "w") as f:
        json.dump({"curve": curve, "train_regret": fit, "thesis_regret": summary(regs, "thesis")},
                  f, indent=1)
    print("loss %.5f -> %.5f; training-set regret: learned %.4f, thesis %.4f"
          % (curve[0][1], curve[-1][1], fit["mean"], summary(regs, "thesis")["mean"]), flush=True)


if __name__ == "__main__":
    main()
