"""Autotuner: measure every candidate parameter tuple on the GPU and write the tuned table.

    python -m paper_1503_04955_amd.tune [--lo 12] [--hi 30] [--step 0.5] [--ratios 1,2,4,8]
                                        [--out DIR]

For each operand size N = 2^x bits (x from lo to hi in steps) and each length ratio, every
feasible candidate tuple (dkss_candidates: Mm offset x log2 m, the smallest modulus for it) and
the thesis's rule are timed as whole products on seeded operands (the context's tables built
beforehand, median of a few repetitions).  Writes
  DIR/dkss_tuning.txt   "lo hi cand" lines: the fastest candidate per size bucket (ratio 1)
  DIR/timings.json      every measurement: the training data of the learned selector
The table is what a DKSS_POLICY_TUNED context loads.  Choices never change result bits; each
measured product is checked by residues on the GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_1503_04955_amd as dk  # noqa: E402

CHECK_PRIMES = [2305843009213693951, 4611686018427387847, 1152921504606846883]


def _time_product(ctx, a, b, c, ws, params, reps, torch):
    ctx.prepare(a.numel(), b.numel(), params)
    ctx.mul(a, b, out=c, params=params, ws=ws)          # warm
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.mul(a, b, out=c, params=params, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def _check(a, b, c):
    ra, rb, rc = dk.residues(a, CHECK_PRIMES), dk.residues(b, CHECK_PRIMES), dk.residues(c, CHECK_PRIMES)
    return all(z == x * y % q for x, y, z, q in zip(ra, rb, rc, CHECK_PRIMES))


def tune(lo, hi, step, ratios, out_dir, reps=3, verbose=True):
    import torch
    import seeded_inputs as SI

    ctx = dk.Context()
    rows = []
    best = []
    x = lo
    while x <= hi + 1e-9:
        for ratio in ratios:
            n = max(1, int(round(2.0 ** x / 32)))
            nb = max(1, int(round(n / ratio)))
            a_h, b_h = SI.operand_pair(int(x * 100) + ratio, n, nb)
            a, b = dk.to_device(a_h), dk.to_device(b_h)
            c = torch.empty(n + nb, dtype=torch.int32, device="cuda")
            cands = [(ci, p) for ci, p in ctx.candidates(32 * n, 32 * nb)]
            entries = [("thesis", ctx.select_params(32 * n, 32 * nb))] + cands
            wsb = max(ctx.workspace_bytes(n, nb, p) for _, p in entries)
            ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
            results = {}
            for ci, p in entries:
                p.cutoff_bits = 0
                ms = _time_product(ctx, a, b, c, ws, p, reps, torch)
                if not _check(a, b, c):
                    raise RuntimeError("product check failed for candidate %s at 2^%.1f" % (ci, x))
                results[ci] = ms
                rows.append({"log2_a": x, "log2_b": x - (ratio.bit_length() - 1), "ratio": ratio,
                             "batch": 1, "cand": ci, "ms": ms, "params": p.as_dict()})
            win = min((k for k in results if k != "thesis"), key=lambda k: results[k])
            if verbose:
                print("2^%.1f ratio %d: thesis %.4f ms, best cand %d %.4f ms (%s)" % (
                    x, ratio, results["thesis"], win, results[win],
                    dict(entries)[win].as_dict()), flush=True)
            if ratio == 1:
                best.append((x, win, results[win], results["thesis"]))
        x += step
        torch.cuda.empty_cache()
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, "dkss_tuning.txt"), "w") as f:
        f.write("# log2N_lo log2N_hi candidate   (fastest measured candidate; ms best / thesis)\n")
        for i, (x, win, ms, ms_th) in enumerate(best):
            lo_b = x - step / 2 if i else 0.0
            hi_b = x + step / 2 if i + 1 < len(best) else 64.0
            f.write("%.3f %.3f %d   # %.4f / %.4f\n" % (lo_b, hi_b, win, ms, ms_th))
    with open(os.path.join(out_dir, "timings.json"), "w") as f:
        json.dump({"arch": "gfx950", "reps": reps, "rows": rows}, f)
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--lo", type=float, default=12)
    ap.add_argument("--hi", type=float, default=30)
    ap.add_argument("--step", type=float, default=0.5)
    ap.add_argument("--ratios", default="1,2,4,8")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=dk.TUNING_DIR)
    args = ap.parse_args()
    t0 = time.time()
    tune(args.lo, args.hi, args.step, [int(r) for r in args.ratios.split(",")], args.out, args.reps)
    print("tuning took %.1f s" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
