"""Autotuner: measure every candidate parameter tuple on the GPU; write the tuned table and the
training data of the learned selector.

    python -m paper_1503_04955_amd.tune [--set train|heldout] [--out DIR] [--reps 3]

A point is (x, ratio, batch): `batch` independent products of 2^x-bit by 2^x/ratio-bit operands
(whole limbs).  At each point every feasible candidate tuple (dkss_candidates: Mm offset x
log2 m with a prime modulus, and log2 m at the smallest Mm with the square of a prime, z = 2),
the base case where it applies (the schoolbook for operands of at most 4096 limbs together,
Karatsuba levels over it up to 8186 x 8186 limbs) and the thesis's rule (the context's THESIS
policy) are timed:
`reps` back-to-back calls between two HIP events after one warm call, divided by reps and by
batch, so each figure is milliseconds per product.  batch 1 runs dkss_mul, larger batches one
dkss_mul_batch call.  Every timed product is checked by residues on the GPU (all of a single
product, the first and the last of a batch).

Sets of points
  train     x in 12..29.5 step 0.5 and 30.5..32, ratios 1,2,4,8, batch 1; x in 12..22 step 0.5
            for batch 16 and 256 and step 1 for batch 4096, ratios 1,2,4,8, while
            batch * 2^x <= 2^33
  heldout   points the selector never sees in training: x = 30 and quarter points between the
            training sizes, ratio 1 and 3, batch 1; and batch 64 and 1024 at quarter points
  kernels   for each training size from 2^16 bits (ratio 1, batch 1) and its fastest candidate:
            the FFT level split (library default, balanced, balanced with one more level) and
            the LDS budget of the DFT-only levels (16, 32, 64 KiB); needs DIR/timings.json

Writes (train) DIR/dkss_tuning.txt, "lo hi cand" lines: the fastest output per size bucket at
ratio 1, for batch 1 and in an "@batch B" section per batch size of the grid (what a
DKSS_POLICY_TUNED context loads), and DIR/timings.json; (heldout)
DIR/timings_heldout.json; (kernels) DIR/timings_kernels.json and DIR/dkss_tuning.txt again, its
lines extended to "lo hi cand radices dft_lds".  Choices never change result bits.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_1503_04955_amd as dk  # noqa: E402

CHECK_PRIMES = [2305843009213693951, 4611686018427387847, 1152921504606846883]
WS_LIMIT = 64 << 30          # skip a candidate whose batched workspace exceeds this
SCHOOLBOOK = dk.CAND_SCHOOLBOOK


def train_points():
    pts = []
    x = 12.0
    while x <= 29.5 + 1e-9:
        for r in (1, 2, 4, 8):
            pts.append((x, r, 1))
        x += 0.5
    # beyond the held-out 2^30: single products up to 2^32 bits, so that the selector's inputs
    # at the largest sizes (2^34 bits) lie close to measured ones
    for x in (30.5, 31.0, 31.5, 32.0):
        for r in (1, 2, 4, 8):
            pts.append((x, r, 1))
    # batches: every half-integer size for 16 and 256 products, whole sizes for 4096 (their
    # points are the costly ones)
    for B in (16, 256, 4096):
        step = 1.0 if B == 4096 else 0.5
        x = 12.0
        while x <= 22.0 + 1e-9:
            if B * 2.0 ** x <= 2.0 ** 33:
                for r in (1, 2, 4, 8):
                    pts.append((x, r, B))
            x += step
    return pts


def heldout_points():
    pts = [(30.0, 1, 1), (30.0, 3, 1)]
    for x in (12.25, 13.75, 15.25, 16.75, 18.25, 19.75, 21.25, 22.75, 24.25, 25.75, 27.25, 28.75):
        for r in (1, 3):
            pts.append((x, r, 1))
    for B in (64, 1024):
        for x in (12.25, 14.75, 17.25, 19.75, 22.25):
            if B * 2.0 ** x <= 2.0 ** 33:
                for r in (1, 3):
                    pts.append((x, r, B))
    return pts


def _lengths(x, ratio):
    n = max(1, int(round(2.0 ** x / 32)))
    return n, max(1, int(round(n / ratio)))


def _check(a, b, c):
    ra, rb, rc = dk.residues(a, CHECK_PRIMES), dk.residues(b, CHECK_PRIMES), dk.residues(c, CHECK_PRIMES)
    return all(z == x * y % q for x, y, z, q in zip(ra, rb, rc, CHECK_PRIMES))


def _events_ms(fn, reps, torch):
    fn()                                              # warm: tables, caches
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def entries(ctx, n, nb):
    """[(label, Params)]: 'thesis', candidate indices, SCHOOLBOOK where it applies."""
    th = ctx.select_params(32 * n, 32 * nb)
    out = [("thesis", th)]
    for ci, p in ctx.candidates(32 * n, 32 * nb):
        p.cutoff_bits = 0
        out.append((ci, p))
    sb = ctx.select_params(32 * n, 32 * nb)
    sb.cutoff_bits = (1 << 64) - 1
    if ctx.plan_info(n, nb, sb).schoolbook:       # the base case applies (Karatsuba levels included)
        out.append((SCHOOLBOOK, sb))
    return out


def measure_point(ctx, x, ratio, batch, reps, torch, seed):
    """{label: ms per product} at one point."""
    n, nb = _lengths(x, ratio)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    A = torch.randint(-2 ** 31, 2 ** 31, (batch * n,), dtype=torch.int32, device="cuda", generator=g)
    B = torch.randint(-2 ** 31, 2 ** 31, (batch * nb,), dtype=torch.int32, device="cuda", generator=g)
    C = torch.empty(batch * (n + nb), dtype=torch.int32, device="cuda")
    as_ = [A[i * n:(i + 1) * n] for i in range(batch)]
    bs = [B[i * nb:(i + 1) * nb] for i in range(batch)]
    cs = [C[i * (n + nb):(i + 1) * (n + nb)] for i in range(batch)]
    res = {}
    for label, p in entries(ctx, n, nb):
        if batch == 1:
            ws = torch.empty(max(ctx.workspace_bytes(n, nb, p), 1), dtype=torch.uint8, device="cuda")
            ctx.prepare(n, nb, p)

            def fn(p=p, ws=ws):
                ctx.mul(as_[0], bs[0], out=cs[0], params=p, ws=ws)
        else:
            call = dk.BatchCall(ctx, as_, bs, cs, [p] * batch, alloc_ws=False)
            if call.ws_bytes > WS_LIMIT:
                continue
            call.ws = torch.empty(max(call.ws_bytes, 1), dtype=torch.uint8, device="cuda")
            fn = call
        ms = _events_ms(fn, reps, torch)
        for i in sorted({0, batch - 1}):
            if not _check(as_[i], bs[i], cs[i]):
                raise RuntimeError("product check failed: %s at 2^%.2f ratio %d batch %d"
                                   % (label, x, ratio, batch))
        res[label] = (ms / batch, p.as_dict())
        del fn
    del A, B, C
    torch.cuda.empty_cache()
    return res


def _dump(rows, reps, out_json):
    os.makedirs(os.path.dirname(out_json) or ".", exist_ok=True)
    tmp = out_json + ".tmp"
    with open(tmp, "w") as f:
        json.dump({"arch": "gfx950", "reps": reps, "unit": "ms per product", "rows": rows}, f)
    os.replace(tmp, out_json)


def run(points, reps, out_json, verbose=True, tuned_txt=None, merge=False, resume=False):
    """Measure the points; with merge, rows of out_json at other points are kept; with resume,
    also its rows at these points, which are then not measured again.  The file is rewritten
    after every point, so that a run cut short keeps what it measured."""
    import torch
    ctx = dk.Context()
    rows = []
    done = set()
    if (merge or resume) and os.path.exists(out_json):
        keys = {(x, r, b) for x, r, b in points}
        with open(out_json) as f:
            old = json.load(f)["rows"]
        for r in old:
            key = (r["log2_a"], r["ratio"], r["batch"])
            if key not in keys:
                if merge:
                    rows.append(r)
            elif resume:
                rows.append(r)
                done.add(key)
    t0 = time.time()
    for k, (x, ratio, batch) in enumerate(points):
        if (x, ratio, batch) in done:
            continue
        res = measure_point(ctx, x, ratio, batch, reps, torch, seed=int(x * 1000) * 100 + ratio * 10 + k)
        for label, (ms, pd) in res.items():
            rows.append({"log2_a": x, "log2_b": x - math.log2(ratio), "ratio": ratio,
                         "batch": batch, "cand": label, "ms": ms, "params": pd})
        _dump(rows, reps, out_json)
        if verbose:
            win = min((c for c in res if c != "thesis"), key=lambda c: res[c][0])
            print("[%4d/%d %6.0fs] 2^%.2f ratio %d batch %d: thesis %.5f ms, best %s %.5f ms"
                  % (k + 1, len(points), time.time() - t0, x, ratio, batch, res["thesis"][0], win,
                     res[win][0]), flush=True)
    _dump(rows, reps, out_json)
    if tuned_txt:
        write_tuned_table(rows, tuned_txt)
    return rows


def best_candidates(rows, batch=1, school=False):
    """{x: (cand, ms)}: the fastest DKSS candidate (or, with school, also the schoolbook) per size
    at ratio 1 and the given batch size."""
    best = {}
    for r in rows:
        if r["ratio"] != 1 or r["batch"] != batch or not isinstance(r["cand"], int):
            continue
        if r["cand"] == SCHOOLBOOK and not school:
            continue
        x = r["log2_a"]
        if x not in best or r["ms"] < best[x][1]:
            best[x] = (r["cand"], r["ms"])
    return best


def write_tuned_table(rows, path, kernel_rows=None):
    """Fastest output (a DKSS candidate or the schoolbook) per size at ratio 1 as half-open
    log2 N buckets, first for batch 1, then in one "@batch B" section per measured batch size;
    with kernel_rows, batch 1 entries also carry the fastest level split and DFT LDS budget
    measured for their candidate.  Sections other than batch 1 end at their largest measured
    size: beyond it a product takes the entry of a smaller batch size."""
    kbest = {}
    best1 = best_candidates(rows, 1, school=True)
    for r in kernel_rows or []:
        x = r["log2_a"]
        if x in best1 and r["cand"] == best1[x][0] and (x not in kbest or r["ms"] < kbest[x]["ms"]):
            kbest[x] = r
    batches = sorted({r["batch"] for r in rows if r["ratio"] == 1})
    with open(path, "w") as f:
        f.write("# log2N_lo log2N_hi candidate [radices] [dft_lds]   (fastest measured; ms best / thesis)\n")
        f.write("# candidate S: the base case (schoolbook, Karatsuba levels over it); T: the thesis rule\n")
        for B in batches:
            best = best_candidates(rows, B, school=True)
            thesis = {r["log2_a"]: r["ms"] for r in rows
                      if r["ratio"] == 1 and r["batch"] == B and r["cand"] == "thesis"}
            xs = sorted(best)
            if B != 1:
                f.write("@batch %d\n" % B)
            for i, x in enumerate(xs):
                lo = (xs[i - 1] + x) / 2 if i else 0.0
                if i + 1 < len(xs):
                    hi = (x + xs[i + 1]) / 2
                elif B == 1:
                    hi = 64.0
                else:
                    hi = x + (x - xs[i - 1]) / 2 if i else x + 0.5
                cfg, ms = "", best[x][1]
                if B == 1 and x in kbest:
                    k = kbest[x]
                    cfg = " %s %d" % (".".join(str(v) for v in k["radices"]), k["dft_lds"])
                    ms = k["ms"]
                name = "S" if best[x][0] == SCHOOLBOOK else str(best[x][0])
                if x in thesis and ms >= thesis[x]:
                    # nothing measured beat the rule here: name the rule, so the lookup never
                    # picks a slower tuple (nor an entry of a smaller batch size)
                    name, cfg = "T", ""
                f.write("%.3f %.3f %s%s   # %.4f / %.4f\n" % (lo, hi, name, cfg, ms, thesis.get(x, 0.0)))


def radix_splits(total, cap):
    """Level splits of 2^total into radices 2^r, r <= cap: the library default (full radices
    first), the balanced split with as many levels, and the balanced split with one more."""
    d, rem = [], total
    while rem > cap:
        d.append(cap)
        rem -= cap
    if rem:
        d.append(rem)
    out = [d]
    for n in (len(d), len(d) + 1):
        if n > 8 or n > total:
            continue
        q, r = divmod(total, n)
        bal = [q + 1] * r + [q] * (n - r)
        if max(bal) <= cap and bal not in out:
            out.append(bal)
    return out


KERNEL_LDS = (16384, 32768, 65536)


def tune_kernels(train_json, reps, out_json, tuned_txt, lo=16.0, verbose=True):
    """For each size of the training grid (ratio 1, batch 1, 2^lo bits and up) and its fastest
    candidate: time every level split of radix_splits and every DFT LDS budget of KERNEL_LDS."""
    import torch
    with open(train_json) as f:
        rows = json.load(f)["rows"]
    best = best_candidates(rows)
    ctx = dk.Context()
    krows = []
    t0 = time.time()
    xs = [x for x in sorted(best) if x >= lo]
    for k, x in enumerate(xs):
        n, nb = _lengths(x, 1)
        cand = best[x][0]
        p0 = dict(ctx.candidates(32 * n, 32 * nb))[cand]
        total = p0.log2_M + 1
        cap = max(p0.radix_log2[i] for i in range(p0.n_levels))
        g = torch.Generator(device="cuda")
        g.manual_seed(int(x * 1000) + 7)
        a = torch.randint(-2 ** 31, 2 ** 31, (n,), dtype=torch.int32, device="cuda", generator=g)
        b = torch.randint(-2 ** 31, 2 ** 31, (nb,), dtype=torch.int32, device="cuda", generator=g)
        c = torch.empty(n + nb, dtype=torch.int32, device="cuda")
        res = []
        for split in radix_splits(total, cap):
            p = dk.Params.make(p0.log2_M, p0.log2_m, p0.u, p0.p_bits, p0.z, split, 0)
            ws = torch.empty(max(ctx.workspace_bytes(n, nb, p), 1), dtype=torch.uint8, device="cuda")
            ctx.prepare(n, nb, p)
            for lds in KERNEL_LDS:
                ctx.set_option(dk.OPT_DFT_LDS, lds)
                ms = _events_ms(lambda: ctx.mul(a, b, out=c, params=p, ws=ws), reps, torch)
                if not _check(a, b, c):
                    raise RuntimeError("product check failed: split %s lds %d at 2^%.2f" % (split, lds, x))
                res.append((ms, split, lds))
                krows.append({"log2_a": x, "ratio": 1, "batch": 1, "cand": cand, "radices": split,
                              "dft_lds": lds, "ms": ms})
            del ws
        ctx.set_option(dk.OPT_DFT_LDS, 32768)
        del a, b, c
        torch.cuda.empty_cache()
        if verbose:
            ms, split, lds = min(res)
            print("[%3d/%d %6.0fs] 2^%.2f cand %d: default %.4f ms, best %s lds %d %.4f ms"
                  % (k + 1, len(xs), time.time() - t0, x, cand, best[x][1], split, lds, ms), flush=True)
    with open(out_json, "w") as f:
        json.dump({"arch": "gfx950", "reps": reps, "unit": "ms per product", "rows": krows}, f)
    write_tuned_table(rows, tuned_txt, krows)
    return krows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--set", choices=["train", "heldout", "kernels"], default="train")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=dk.TUNING_DIR)
    ap.add_argument("--batches", default="", help="measure only these batch sizes, e.g. 1 or 16,256")
    ap.add_argument("--merge", action="store_true", help="keep the file's rows at other points")
    ap.add_argument("--resume", action="store_true",
                    help="keep the file's rows at these points too and measure only the missing ones")
    args = ap.parse_args()
    if args.set == "kernels":
        t0 = time.time()
        tune_kernels(os.path.join(args.out, "timings.json"), args.reps,
                     os.path.join(args.out, "timings_kernels.json"),
                     os.path.join(args.out, "dkss_tuning.txt"))
        print("kernel tuning took %.1f s" % (time.time() - t0), flush=True)
        return
    pts = train_points() if args.set == "train" else heldout_points()
    if args.batches:
        keep = {int(b) for b in args.batches.split(",")}
        pts = [p for p in pts if p[2] in keep]
    t0 = time.time()
    if args.set == "train":
        run(pts, args.reps, os.path.join(args.out, "timings.json"),
            tuned_txt=os.path.join(args.out, "dkss_tuning.txt"), merge=args.merge, resume=args.resume)
    else:
        run(pts, args.reps, os.path.join(args.out, "timings_heldout.json"), merge=args.merge,
            resume=args.resume)
    print("tuning took %.1f s" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
