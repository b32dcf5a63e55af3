"""Benchmark: DKSS multiplication on one MI355X, operand bits multiplied per second.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--bits 28] [--no-cpu] [--batch 4096]

One step is one whole product c = a*b of two 2^bits-bit operands (default 2^28 bits, 8388608
uint32 limbs each, uniform random limbs from a seeded splitmix64 stream) through every stage of
the path: encode, forward transforms of both operands, componentwise products, inverse
transform, decode and carries.  The parameter tuple is the thesis's rule; its constants and the
table of rho powers are prepared before the timed region (cached in the context).  Operands and
workspace are resident in HBM before timing.  After timing, the product is checked by residues
modulo 8 seeded random 61-bit primes (computed on the GPU for a, b and c and compared with
Python integers).  `value` is this plain product's throughput.

The roofline object describes the dominant kernel (most time over the timed region; with the
thesis's parameters the forward FFT levels with fused rho twiddles, k_level<L, 1>), timed with
HIP events on the library's stream.  Products in R are counted in 32x32-bit multiply-adds of the
schoolbook product (m^2 L^2 per product in R) and priced against the chip's full-rate 32-bit VALU
throughput (256 CUs x 64 lanes x 2.4 GHz); other kernels in algorithmic bytes against HBM
bandwidth.  `traffic` is the HBM bytes per launch that the committed counter summary
profiles/<kernel>_traffic.txt records, when it was taken on the current kernel sources, else
null.  roofline_fft reports the FFT levels without twiddles (k_level<L, 0>) against HBM.

"tuned" and "learned" time the same product under the tuned table and the learned selector;
"cold" times a fresh context's first product of the same operands on the host clock: planning
(prime, generator, rho on the host) and the rho-power table (GPU) as setup_ms, then the product;
"sizes" times single products of 2^18 and 2^24 bits (thesis rule, learned selector, and the
thesis-rule product replayed as a one-product HIP graph, which removes the host launch cost of
the launch-bound small case).
The "batch" object: 4096 independent products, operand lengths log-uniform in 2^12..2^22 bits,
length ratios uniform in [1, 8], run as 4096 sequential plain calls (thesis rule), as one
dkss_mul_batch call per policy (thesis, tuned, learned), and as the learned batch captured in a
HIP graph and replayed; every variant's bits equal the plain calls' (checked).

The cpu_baseline leg times the CPU oracle (plain C, one thread) on a bounded sample: one whole
product of two 2^25-bit operands by the oracle's DKSS with the same parameter rule.
"""
import argparse
import json
import os
import random
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "operand bits multiplied/sec (bit-exact), batched+tuned vs plain DKSS, 1 GPU"
PEAK_HBM_GBS = 8000.0
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12     # full-rate 32-bit VALU ops (v_mad_u64_u32)


def _isprime(n):
    if n < 2 or n % 2 == 0:
        return n == 2
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def primes61(seed, count):
    rng = random.Random(seed)
    out = []
    while len(out) < count:
        q = rng.getrandbits(61) | (1 << 60) | 1
        if _isprime(q):
            out.append(q)
    return out


def cpu_baseline(bits=25):
    """Oracle (C, -O2, one thread) on one 2^bits x 2^bits product: operand bits/s."""
    import seeded_inputs as SI
    from oracle import coracle
    n = (1 << bits) // 32
    a, b = SI.operand_pair(SI.SEED_BASE + 100, n, n)
    coracle.lib()
    t0 = time.perf_counter()
    coracle.dkss_mul(a, b)
    dt = time.perf_counter() - t0
    return {"value": 2 * n * 32 / dt, "unit": "operand bits/s", "cores": 1, "kind": "oracle",
            "sample": "one 2^%d x 2^%d-bit product through the oracle's DKSS (thesis rule), "
                      "single thread, %.1f s" % (bits, bits, dt)}


def _timed(fn, reps, torch):
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def batch_bench(count, reps, dk, torch, SI):
    """count uneven products: plain sequential calls vs one batched call per policy, and the
    learned batch captured into a HIP graph and replayed."""
    lens = SI.batch_lengths(SI.SEED_BASE + 2, count)
    as_, bs = [], []
    for i, (al, bl) in enumerate(lens):
        a, b = SI.operand_pair(SI.SEED_BASE + 100000 + i, al, bl)
        as_.append(dk.to_device(a))
        bs.append(dk.to_device(b))
    bits = 32.0 * sum(al + bl for al, bl in lens)
    outs_p = [torch.empty(a.numel() + b.numel(), dtype=torch.int32, device="cuda") for a, b in zip(as_, bs)]
    ctx = dk.Context()
    wss = max(ctx.workspace_bytes(a.numel(), b.numel()) for a, b in zip(as_, bs))
    ws = torch.empty(max(wss, 1), dtype=torch.uint8, device="cuda")

    def plain():
        for a, b, o in zip(as_, bs, outs_p):
            ctx.mul(a, b, out=o, ws=ws)

    res = {"workload": "%d products, operands 2^12..2^22 bits log-uniform, length ratio U[1,8]"
                       % count, "operand_bits": bits}
    ms = _timed(plain, reps, torch)
    res["plain_sequential"] = {"ms": ms, "value": bits / (ms / 1e3)}
    same = True
    for name, policy in (("thesis", dk.POLICY_THESIS), ("tuned", dk.POLICY_TUNED),
                         ("learned", dk.POLICY_LEARNED)):
        call = dk.BatchCall(dk.Context(policy), as_, bs)
        ms = _timed(call, reps, torch)
        same = same and all(torch.equal(x, y) for x, y in zip(outs_p, call.outs))
        res["batched_" + name] = {"ms": ms, "value": bits / (ms / 1e3)}
        if name == "learned":
            for o in call.outs:
                o.zero_()
            graph = call.graph()
            ms = _timed(graph, reps, torch)
            same = same and all(torch.equal(x, y) for x, y in zip(outs_p, call.outs))
            res["graph_learned"] = {"ms": ms, "value": bits / (ms / 1e3), "kernels": graph.kernels}
            graph.close()
        del call
        torch.cuda.empty_cache()
    if not same:
        raise RuntimeError("batched products differ from the plain ones")
    best = min(res[k]["ms"] for k in ("batched_tuned", "batched_learned", "graph_learned"))
    res["speedup_best_batched_vs_plain"] = res["plain_sequential"]["ms"] / best
    res["bit_identical"] = same
    return res


def sizes_bench(bits_list, reps, dk, torch, SI):
    """Single products at other sizes (the 2^18-bit case is launch-bound): thesis rule and learned
    selector as plain calls, and the thesis-rule product captured as a one-product HIP graph;
    every variant bit-identical to the first."""
    out = {}
    for bits in bits_list:
        n = (1 << bits) // 32
        a_h, b_h = SI.operand_pair(SI.SEED_BASE + 3 + bits, n, n)
        a, b = dk.to_device(a_h), dk.to_device(b_h)
        res = {"limbs": n}
        ref = None
        for name, policy in (("thesis", dk.POLICY_THESIS), ("learned", dk.POLICY_LEARNED)):
            ctx = dk.Context(policy)
            c = torch.empty(2 * n, dtype=torch.int32, device="cuda")
            ws = torch.empty(max(ctx.workspace_bytes(n, n), 1), dtype=torch.uint8, device="cuda")
            ms = _timed(lambda: ctx.mul(a, b, out=c, ws=ws), reps, torch)
            if ref is None:
                ref = c
            elif not torch.equal(ref, c):
                raise RuntimeError("2^%d product differs between policies" % bits)
            res[name] = {"ms": ms, "value": 2 * n * 32 / (ms / 1e3)}
            if name == "thesis":
                call = dk.BatchCall(ctx, [a], [b])
                graph = call.graph()
                ms = _timed(graph, reps, torch)
                if not torch.equal(ref, call.outs[0]):
                    raise RuntimeError("2^%d graph product differs" % bits)
                res["thesis_graph"] = {"ms": ms, "value": 2 * n * 32 / (ms / 1e3),
                                       "kernels": graph.kernels}
                graph.close()
        out["2^%d" % bits] = res
    return out


def traffic_record(kernel, bits, source_files):
    """HBM bytes per launch of `kernel` in the 2^bits product from the committed counter summary,
    or None when the summary is missing or was taken on other kernel sources (sha256 of
    source_files)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "%s_dkss_mul_2p%d_traffic.txt" % (kernel, bits))
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in source_files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if kv.get("source_sha256") != h.hexdigest():
        return None
    return float(kv["hbm_bytes_per_launch"])


KERNEL_SOURCES = ["paper_1503_04955_amd/csrc/dkss_lib.hip", "paper_1503_04955_amd/csrc/kernels.hpp"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--bits", type=int, default=28)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--overlap", type=int, default=0, help="transform b on a second stream")
    ap.add_argument("--dft-lds", type=int, default=32768, help="LDS bytes per FFT-level workgroup")
    ap.add_argument("--batch", type=int, default=4096, help="products in the batch leg (0: skip)")
    ap.add_argument("--sizes", default="18,24", help="other single-product sizes, log2 bits ('' to skip)")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="end with one device-to-device copy of this many bytes (a counter "
                         "calibration kernel of known traffic)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1503_04955_amd as dk
    import seeded_inputs as SI

    dev = torch.device("cuda:0")
    n = (1 << args.bits) // 32
    a_h, b_h = SI.operand_pair(SI.SEED_BASE + 2, n, n)
    a, b = dk.to_device(a_h, dev), dk.to_device(b_h, dev)
    c = torch.empty(2 * n, dtype=torch.int32, device=dev)
    ctx = dk.Context()
    ctx.set_option(dk.OPT_OVERLAP, args.overlap)
    ctx.set_option(dk.OPT_DFT_LDS, args.dft_lds)
    params = ctx.select_params(32 * n, 32 * n)
    plan = ctx.plan_info(n, n)
    ws = torch.empty(ctx.workspace_bytes(n, n), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    ctx.prepare(n, n)
    print("plan %s L=%d S=%d bytes" % (params.as_dict(), plan.L, plan.poly_bytes), file=sys.stderr,
          flush=True)
    for _ in range(args.warmup):
        ctx.mul(a, b, out=c, ws=ws)
    torch.cuda.synchronize()
    ctx.profile_reset()
    ctx.profile(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        ctx.mul(a, b, out=c, ws=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ctx.profile(False)
    ms = e0.elapsed_time(e1)
    stats = ctx.profile_read()

    # bit-exactness by residues (GPU residue kernel, compared in Python integers)
    qs = primes61(SI.SEED_BASE, 8)
    ra, rb, rc = dk.residues(a, qs), dk.residues(b, qs), dk.residues(c, qs)
    exact = all(z == x * y % q for x, y, z, q in zip(ra, rb, rc, qs))
    if not exact:
        print("product check by residues FAILED", file=sys.stderr)
        sys.exit(1)

    ms_step = ms / args.steps
    value = args.steps * 2 * n * 32 / (ms / 1e3)
    # dominant kernel: the kind with the most time; products in R are priced against the VALU,
    # everything else against HBM bandwidth
    symbols = {"k_dft": "k_level<%d, 0>", "k_twiddle": "k_level<%d, 1>",
               "k_twiddle_inv": "k_level<%d, 2>", "k_pointwise": "k_pointwise<%d>",
               "k_decode": "k_decode<%d>", "k_encode": "k_encode<%d>"}
    dom = max(stats, key=lambda k: stats[k].total_ms)
    st = stats[dom]
    avg_ms = st.total_ms / st.launches
    if st.alg_ops > 0:
        ops_launch = st.alg_ops / st.launches
        achieved = ops_launch / (avg_ms / 1e3) / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_VALU_TOPS, 2),
                    "unit": "TOP/s", "frac": round(achieved / PEAK_VALU_TOPS, 4)}
        work = {"ops_per_launch": ops_launch}
    else:
        bytes_launch = st.alg_bytes / st.launches
        achieved = bytes_launch / (avg_ms / 1e3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                    "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4)}
        work = {"alg_bytes_per_launch": bytes_launch}
    roofline["traffic"] = traffic_record(dom, args.bits, KERNEL_SOURCES)
    roofline.update({"kernel": dom, "symbol": symbols.get(dom, dom).replace("%d", str(plan.L))
                     if "%d" in symbols.get(dom, "") else dom,
                     "avg_launch_ms": round(avg_ms, 4), "launches": int(st.launches)})
    roofline.update(work)
    dft = stats.get("k_dft")
    roofline_fft = None
    if dft and dft.launches:
        avg_ms = dft.total_ms / dft.launches
        gbs = dft.alg_bytes / dft.launches / (avg_ms / 1e3) / 1e9
        roofline_fft = {"kernel": "k_dft", "symbol": "k_level<%d, 0>" % plan.L, "bound": "hbm",
                        "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": round(gbs / PEAK_HBM_GBS, 4), "avg_launch_ms": round(avg_ms, 4),
                        "traffic": traffic_record("k_dft", args.bits, KERNEL_SOURCES)}
    kernels = {k: {"launches": int(v.launches), "ms_per_step": round(v.total_ms / args.steps, 4),
                   "avg_launch_ms": round(v.total_ms / v.launches, 4)}
               for k, v in stats.items()}
    out = {
        "metric": METRIC, "value": value, "unit": "operand bits/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic (seeded uniform uint32 limbs)",
        "config": {"workload": "plain DKSS, one product of two 2^%d-bit operands (%d uint32 limbs "
                               "each), thesis-rule parameters" % (args.bits, n),
                   "params": params.as_dict(), "L": plan.L, "overlap": args.overlap,
                   "dft_lds": args.dft_lds},
        "verified": "residues mod 8 random 61-bit primes",
        "roofline": roofline, "roofline_fft": roofline_fft, "kernels": kernels,
    }
    # the same product with the tuned policy
    ctx_t = dk.Context(dk.POLICY_TUNED)
    ctx_t.set_option(dk.OPT_OVERLAP, args.overlap)
    ctx_t.set_option(dk.OPT_DFT_LDS, args.dft_lds)
    ws_t = torch.empty(ctx_t.workspace_bytes(n, n), dtype=torch.uint8, device=dev)
    c_t = torch.empty_like(c)
    ms_t = _timed(lambda: ctx_t.mul(a, b, out=c_t, ws=ws_t), args.steps, torch)
    if not torch.equal(c, c_t):
        print("tuned product differs", file=sys.stderr)
        sys.exit(1)
    out["tuned"] = {"ms_per_step": ms_t, "value": 2 * n * 32 / (ms_t / 1e3),
                    "params": ctx_t.select_params(32 * n, 32 * n).as_dict()}
    del ws_t
    # ... and with the learned selector
    ctx_l = dk.Context(dk.POLICY_LEARNED)
    ctx_l.set_option(dk.OPT_OVERLAP, args.overlap)
    ctx_l.set_option(dk.OPT_DFT_LDS, args.dft_lds)
    ws_l = torch.empty(ctx_l.workspace_bytes(n, n), dtype=torch.uint8, device=dev)
    ms_l = _timed(lambda: ctx_l.mul(a, b, out=c_t, ws=ws_l), args.steps, torch)
    if not torch.equal(c, c_t):
        print("learned-policy product differs", file=sys.stderr)
        sys.exit(1)
    out["learned"] = {"ms_per_step": ms_l, "value": 2 * n * 32 / (ms_l / 1e3),
                      "choice": ctx_l.mlp_choose(32 * n, 32 * n),
                      "params": ctx_l.select_params(32 * n, 32 * n).as_dict()}
    # cold: a fresh context's planning (host), rho table (GPU) and first product, host clock
    ws_c = torch.empty(dk.Context().workspace_bytes(n, n), dtype=torch.uint8, device=dev)
    ctx_c = dk.Context()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx_c.prepare(n, n)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx_c.mul(a, b, out=c_t, ws=ws_c)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    if not torch.equal(c, c_t):
        print("cold product differs", file=sys.stderr)
        sys.exit(1)
    out["cold"] = {"setup_ms": 1e3 * (t1 - t0), "first_product_ms": 1e3 * (t2 - t1),
                   "ms": 1e3 * (t2 - t0)}
    del ws_l, ws, ws_c, c_t, ctx_c
    torch.cuda.empty_cache()
    if args.batch:
        out["batch"] = batch_bench(args.batch, 3, dk, torch, SI)
    if args.sizes:
        out["sizes"] = sizes_bench([int(x) for x in args.sizes.split(",")], 20, dk, torch, SI)
    if args.copy_calib:
        src = torch.empty(args.copy_calib, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calib_bytes"] = args.copy_calib
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
