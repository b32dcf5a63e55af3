"""Benchmark: DKSS multiplication on one MI355X, operand bits multiplied per second.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch 4096] [--no-cpu] [--no-c5]
                [--legs batch,2p28,sizes,smul,twforms,c5] [--copy-calib BYTES]

Headline (`value`): the mixed batch, batched and learned-tuned.  One step is one pass of the whole
hot path over the batch: 4096 independent products whose longer operand has 2^U(12,22) bits
(log-uniform, rounded to uint32 limbs), length ratio U[1, 8], limbs uniform from a seeded
splitmix64 stream (seeded_inputs.mixed_batch), each product running encode, both forward
transforms, componentwise products, inverse transform, decode and carries (or the schoolbook
base case where the selector picks it).  Parameters per product come from the learned selector
(planned once, tables prepared before timing); the batch runs as one dkss_mul_batch captured
into a HIP graph and replayed with one launch per step.  W untimed replays, then K timed ones
between two synchronizations; operands, results and workspace are resident in HBM.  `value` =
the batch's operand bits (sum of 32 (alen + blen)) / seconds per step.  Every product of the
timed runs is checked: equal to the plain per-product calls, and c = a b modulo 8 seeded 61-bit
primes (GPU residue kernel, compared in Python integers).

Beside it, under "batch": the same products as 4096 plain calls (thesis rule, one dkss_mul each:
the baseline of the metric), and as one eager dkss_mul_batch per policy (thesis, tuned, learned).

`roofline` describes the headline's dominant kernel kind (most time in a separate profiled pass
of K eager learned batches: HIP events around every launch on the library's stream, so the
timed pass above carries no event overhead): products in R counted in 32x32-bit multiply-adds of
the schoolbook product (m^2 L^2 per product in R), priced against the chip's full-rate 32-bit
VALU throughput (256 CUs x 64 lanes x 2.4 GHz); HBM-bound kinds in algorithmic bytes against
8 TB/s.  `traffic` comes from the committed counter summary of that kernel and workload
(profiles/<kernel>_<workload>_traffic.txt) while it was taken on the current kernel sources,
else null.

Other legs: "single_2p28" one 2^28 x 2^28-bit product (thesis rule, tuned table, learned
selector; its own profiled pass gives `roofline` of its dominant kernel, the forward twiddle
level); "sizes" single products of 2^18 and 2^24 bits; "smul" SMUL beside DKSS at 2^24 and 2^28
bits; "twforms" the bad multiplications of one 2^28-bit transform level on the vector units and
on the matrix cores (dkss_probe_twiddle_products); "c5" one 2^34 x 2^34-bit product (2 GiB
operands, seeded uniform limbs from the device generator) under the thesis rule and the learned
selector, plus the squaring a*a, each checked by residues mod 16 primes; "cpu_baseline" the
oracle's DKSS (C, gcc -O3 -march=native built on the machine that runs it) on a bounded sample
of the same batch: one thread, then all of the host's cores available to this process (at most
16) taking products from the batch in order, each for about 10 s.
"""
import argparse
import json
import os
import sys
import tempfile
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "operand bits multiplied/sec (bit-exact), batched+tuned vs plain DKSS, 1 GPU"
PEAK_HBM_GBS = 8000.0
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12     # full-rate 32-bit VALU ops (v_mad_u64_u32)
KERNEL_SOURCES = ["paper_1503_04955_amd/csrc/dkss_lib.hip", "paper_1503_04955_amd/csrc/kernels.hpp"]


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
    import random
    rng = random.Random(seed)
    out = []
    while len(out) < count:
        q = rng.getrandbits(61) | (1 << 60) | 1
        if _isprime(q):
            out.append(q)
    return out


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline(pairs, budget_s=10.0):
    """The oracle's DKSS (thesis rule) on products of the batch in order: one thread for about
    budget_s, then every available core (threads; the oracle's C calls run without the
    interpreter lock) for about budget_s.  Operand bits per second of completed products."""
    from oracle import coracle
    lib = coracle.lib_native(tempfile.mkdtemp(prefix="dkss_oracle_"))

    def run(i):
        a, b = pairs[i]
        coracle.dkss_mul(a, b, library=lib)
        return 32.0 * (len(a) + len(b))

    t0 = time.perf_counter()
    bits1, k = 0.0, 0
    while k < len(pairs) and (k == 0 or time.perf_counter() - t0 < budget_s):
        bits1 += run(k)
        k += 1
    dt1 = time.perf_counter() - t0
    cores = host_cores()
    lock = threading.Lock()
    state = {"next": 0, "bits": 0.0, "done": 0}
    t0 = time.perf_counter()

    def worker():
        while True:
            with lock:
                i = state["next"]
                if i >= len(pairs) or time.perf_counter() - t0 >= budget_s:
                    return
                state["next"] = i + 1
            bits = run(i)
            with lock:
                state["bits"] += bits
                state["done"] += 1

    ths = [threading.Thread(target=worker) for _ in range(cores)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    dtn = time.perf_counter() - t0
    return {"value": state["bits"] / dtn, "unit": "operand bits/s", "cores": cores, "kind": "oracle",
            "sample": "the first %d products of the 4096-product batch (%.3g operand bits) through the "
                      "oracle's DKSS on %d threads in %.1f s (gcc -O3 -march=native; host reports %d CPUs)"
                      % (state["done"], state["bits"], cores, dtn, os.cpu_count() or 0),
            "single_thread": {"value": bits1 / dt1, "unit": "operand bits/s", "cores": 1,
                              "sample": "the first %d products (%.3g operand bits) in %.1f s"
                                        % (k, bits1, dt1)}}


def _timed(fn, reps, torch, warmup=1):
    for _ in range(warmup):
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


def traffic_record(kernel, workload, source_files):
    """HBM bytes per launch of `kernel` in `workload` from the committed counter summary, or None
    when it is missing or was taken on other kernel sources (sha256 of source_files)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "%s_%s_traffic.txt" % (kernel, workload))
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


def roofline_of(stats, workload, mad_rate=None):
    """Roofline object of the kind with the most time in a profiled pass (VALU-bound kinds also
    against the measured multiply-add rate, when given)."""
    dom = max(stats, key=lambda k: stats[k].total_ms)
    st = stats[dom]
    avg_ms = st.total_ms / st.launches
    if st.alg_ops > 0:
        per = st.alg_ops / st.launches
        achieved = per / (avg_ms / 1e3) / 1e12
        r = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_VALU_TOPS, 2),
             "unit": "TOP/s", "frac": round(achieved / PEAK_VALU_TOPS, 4), "ops_per_launch": per,
             "alg_bytes_per_launch": st.alg_bytes / st.launches}
        if mad_rate:
            r["frac_of_measured_mad_rate"] = round(achieved / mad_rate, 4)
    else:
        per = st.alg_bytes / st.launches
        achieved = per / (avg_ms / 1e3) / 1e9
        r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
             "frac": round(achieved / PEAK_HBM_GBS, 4), "alg_bytes_per_launch": per}
    r["traffic"] = traffic_record(dom, workload, KERNEL_SOURCES)
    r.update({"kernel": dom, "avg_launch_ms": round(avg_ms, 4), "launches": int(st.launches),
              "workload": workload})
    return r


def kernel_table(stats, steps):
    return {k: {"launches": int(v.launches), "ms_per_step": round(v.total_ms / steps, 4),
                "avg_launch_ms": round(v.total_ms / v.launches, 4)} for k, v in stats.items()}


def check_residues(dk, as_, bs, outs, qs):
    for i, (a, b, c) in enumerate(zip(as_, bs, outs)):
        ra, rb, rc = dk.residues(a, qs), dk.residues(b, qs), dk.residues(c, qs)
        if not all(z == x * y % q for x, y, z, q in zip(ra, rb, rc, qs)):
            raise RuntimeError("product %d fails the residue check" % i)


def batch_leg(args, dk, torch, SI):
    """The headline (learned batch as a replayed graph), its profiled pass, and the other forms."""
    pairs = SI.mixed_batch(args.batch)
    as_ = [dk.to_device(a) for a, _ in pairs]
    bs = [dk.to_device(b) for _, b in pairs]
    bits = 32.0 * sum(len(a) + len(b) for a, b in pairs)
    log("batch: %d products, %.4g operand bits" % (len(pairs), bits))
    ctx_l = dk.Context(dk.POLICY_LEARNED)
    ctx_l.set_option(dk.OPT_BATCH_LANES, args.lanes)
    call = dk.BatchCall(ctx_l, as_, bs)                              # plans, infers, prepares
    graph = call.graph()
    for _ in range(args.warmup):
        graph()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        graph()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    log("batch: graph learned %.3f ms per step" % ms_step)
    head = {"ms": ms_step, "value": bits / (ms_step / 1e3), "kernels": graph.kernels,
            "lanes": args.lanes}
    if args.headline_only:
        # the profiling form: the headline's kernels alone (no plain calls, no other policies)
        call.ctx.set_option(dk.OPT_BATCH_LANES, 1)
        call.ctx.profile_reset()
        call.ctx.profile(True)
        for _ in range(args.steps):
            call()
        torch.cuda.synchronize()
        call.ctx.profile(False)
        stats = call.ctx.profile_read()
        graph.close()
        # every 64th product (the full check launches 24 residue kernels per product, which
        # would crowd a trace of this form)
        check_residues(dk, as_[::64], bs[::64], call.outs[::64], primes61(SI.SEED_BASE, 8))
        return ms_step, bits, {"workload": "4096 products (headline only)", "operand_bits": bits,
                               "graph_learned": head}, stats
    # the plain calls: thesis rule, one dkss_mul per product (tables prepared)
    ctx = dk.Context()
    outs_p = [torch.empty(a.numel() + b.numel(), dtype=torch.int32, device="cuda") for a, b in zip(as_, bs)]
    ws = torch.empty(max([ctx.workspace_bytes(a.numel(), b.numel()) for a, b in zip(as_, bs)] + [1]),
                     dtype=torch.uint8, device="cuda")

    def plain():
        for a, b, o in zip(as_, bs, outs_p):
            ctx.mul(a, b, out=o, ws=ws)

    reps = max(1, min(args.steps, 5))
    ms_plain = _timed(plain, reps, torch)
    log("batch: plain sequential %.3f ms" % ms_plain)
    if not all(torch.equal(x, y) for x, y in zip(outs_p, call.outs)):
        raise RuntimeError("graph batch differs from the plain products")
    check_residues(dk, as_, bs, outs_p, primes61(SI.SEED_BASE, 8))
    res = {"workload": "4096 products, operands 2^12..2^22 bits log-uniform, length ratio U[1,8]",
           "operand_bits": bits, "graph_learned": head,
           "plain_sequential": {"ms": ms_plain, "value": bits / (ms_plain / 1e3)}}
    # the profiled pass of the headline's kernels: the eager learned batch, K steps, its groups
    # on one stream (concurrent groups would stretch each other's kernel times)
    call.ctx.set_option(dk.OPT_BATCH_LANES, 1)
    call.ctx.profile_reset()
    call.ctx.profile(True)
    for _ in range(args.steps):
        call()
    torch.cuda.synchronize()
    call.ctx.profile(False)
    stats = call.ctx.profile_read()
    call.ctx.set_option(dk.OPT_BATCH_LANES, args.lanes)
    same = all(torch.equal(x, y) for x, y in zip(outs_p, call.outs))
    graph.close()
    for name, policy in (("thesis", dk.POLICY_THESIS), ("tuned", dk.POLICY_TUNED),
                         ("learned", dk.POLICY_LEARNED)):
        bc = dk.BatchCall(dk.Context(policy), as_, bs)
        ms = _timed(bc, reps, torch)
        same = same and all(torch.equal(x, y) for x, y in zip(outs_p, bc.outs))
        res["batched_" + name] = {"ms": ms, "value": bits / (ms / 1e3)}
        log("batch: eager %s %.3f ms" % (name, ms))
        del bc
        torch.cuda.empty_cache()
    if not same:
        raise RuntimeError("batched products differ from the plain ones")
    res["speedup_vs_plain"] = ms_plain / ms_step
    res["bit_identical"] = same
    return ms_step, bits, res, stats


def single_leg(bits_log2, reps, dk, torch, SI):
    """One 2^bits product under the thesis rule (profiled pass for its roofline), tuned, learned."""
    n = (1 << bits_log2) // 32
    a_h, b_h = SI.operand_pair(SI.SEED_BASE + 2, n, n)
    a, b = dk.to_device(a_h), dk.to_device(b_h)
    del a_h, b_h
    out = {"limbs": n}
    ref = None
    stats = None
    for name, policy in (("thesis", dk.POLICY_THESIS), ("tuned", dk.POLICY_TUNED),
                         ("learned", dk.POLICY_LEARNED)):
        ctx = dk.Context(policy)
        c = torch.empty(2 * n, dtype=torch.int32, device="cuda")
        ws = torch.empty(ctx.workspace_bytes(n, n), dtype=torch.uint8, device="cuda")
        ctx.prepare(n, n)
        ms = _timed(lambda: ctx.mul(a, b, out=c, ws=ws), reps, torch, warmup=3)
        if ref is None:
            ref = c
            qs = primes61(SI.SEED_BASE, 8)
            ra, rb, rc = dk.residues(a, qs), dk.residues(b, qs), dk.residues(c, qs)
            if not all(z == x * y % q for x, y, z, q in zip(ra, rb, rc, qs)):
                raise RuntimeError("2^%d product fails the residue check" % bits_log2)
            ctx.profile_reset()
            ctx.profile(True)
            for _ in range(reps):
                ctx.mul(a, b, out=c, ws=ws)
            torch.cuda.synchronize()
            ctx.profile(False)
            stats = ctx.profile_read()
        elif not torch.equal(ref, c):
            raise RuntimeError("2^%d product differs between policies" % bits_log2)
        out[name] = {"ms": ms, "value": 2 * n * 32 / (ms / 1e3),
                     "params": ctx.select_params(32 * n, 32 * n).as_dict()}
        log("2^%d %s: %.3f ms" % (bits_log2, name, ms))
        del ws
    torch.cuda.empty_cache()
    out["kernels"] = kernel_table(stats, reps)
    out["roofline"] = roofline_of(stats, "dkss_mul_2p%d" % bits_log2, dk.probe_mad_rate() / 1e12)
    return out


def sizes_leg(bits_list, reps, dk, torch, SI):
    """Single products at other sizes: thesis rule and learned selector as plain calls, and the
    thesis-rule product replayed as a one-product HIP graph."""
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
            ctx.prepare(n, n)
            ms = _timed(lambda: ctx.mul(a, b, out=c, ws=ws), reps, torch)
            if ref is None:
                ref = c
            elif not torch.equal(ref, c):
                raise RuntimeError("2^%d product differs between policies" % bits)
            res[name] = {"ms": ms, "value": 2 * n * 32 / (ms / 1e3)}
            if name == "thesis":
                bc = dk.BatchCall(ctx, [a], [b])
                graph = bc.graph()
                ms = _timed(graph, reps, torch)
                if not torch.equal(ref, bc.outs[0]):
                    raise RuntimeError("2^%d graph product differs" % bits)
                res["thesis_graph"] = {"ms": ms, "value": 2 * n * 32 / (ms / 1e3), "kernels": graph.kernels}
                graph.close()
        out["2^%d" % bits] = res
        log("2^%d: thesis %.4f ms, learned %.4f ms" % (bits, res["thesis"]["ms"], res["learned"]["ms"]))
    return out


def smul_leg(bits_list, reps, dk, torch, SI):
    """The thesis's comparison method on the same GPU: one 2^bits x 2^bits-bit product by SMUL
    (Schoenhage-Strassen, the library's FFT length and ring) beside DKSS under the thesis rule and
    the learned selector; the DKSS/SMUL time ratio (the thesis measures 26-36 on one CPU core)."""
    out = {}
    for bits in bits_list:
        n = (1 << bits) // 32
        a_h, b_h = SI.operand_pair(SI.SEED_BASE + 2, n, n)
        a, b = dk.to_device(a_h), dk.to_device(b_h)
        del a_h, b_h
        res = {"limbs": n}
        c_s = torch.empty(2 * n, dtype=torch.int32, device="cuda")
        p = dk.smul_select(n, n)
        ws = torch.empty(dk.smul_workspace_bytes(n, n), dtype=torch.uint8, device="cuda")
        ms = _timed(lambda: dk.smul(a, b, out=c_s, ws=ws), reps, torch, warmup=2)
        res["smul"] = {"ms": ms, "value": 2 * n * 32 / (ms / 1e3), "params": p.as_dict()}
        if p.lw <= 16:
            # the same ring with the componentwise products in the other form (A/B): 28-bit digits
            # on the vector units (1) or exact 8-bit products on the matrix cores (2)
            other = 3 - p.products
            q = dk.SmulParams.make(p.log2_n, p.lw, other)
            c_v = torch.empty(2 * n, dtype=torch.int32, device="cuda")
            ms_v = _timed(lambda: dk.smul(a, b, out=c_v, params=q, ws=ws), reps, torch, warmup=2)
            if not torch.equal(c_v, c_s):
                raise RuntimeError("2^%d SMUL products differ between the two forms" % bits)
            key = "smul_matrix_products" if other == 2 else "smul_vector_products"
            res[key] = {"ms": ms_v, "value": 2 * n * 32 / (ms_v / 1e3)}
            del c_v
        del ws
        for name, policy in (("dkss_thesis", dk.POLICY_THESIS), ("dkss_learned", dk.POLICY_LEARNED)):
            ctx = dk.Context(policy)
            c = torch.empty(2 * n, dtype=torch.int32, device="cuda")
            ws = torch.empty(ctx.workspace_bytes(n, n), dtype=torch.uint8, device="cuda")
            ctx.prepare(n, n)
            ms = _timed(lambda: ctx.mul(a, b, out=c, ws=ws), reps, torch, warmup=2)
            if not torch.equal(c, c_s):
                raise RuntimeError("2^%d SMUL and DKSS products differ" % bits)
            res[name] = {"ms": ms, "value": 2 * n * 32 / (ms / 1e3)}
            del ws, c
        res["dkss_over_smul"] = {"thesis": res["dkss_thesis"]["ms"] / res["smul"]["ms"],
                                 "learned": res["dkss_learned"]["ms"] / res["smul"]["ms"]}
        res["verified"] = "SMUL product equal to both DKSS products"
        out["2^%d" % bits] = res
        log("2^%d: smul %.3f ms (%s), dkss thesis %.3f ms, learned %.3f ms" %
            (bits, res["smul"]["ms"],
             ", ".join(["%s products" % ("matrix-core" if p.products == 2 else "vector-unit")] +
                       ["%s %.3f ms" % (k[5:].replace("_", " "), res[k]["ms"])
                        for k in ("smul_matrix_products", "smul_vector_products") if k in res]),
             res["dkss_thesis"]["ms"], res["dkss_learned"]["ms"]))
        torch.cuda.empty_cache()
    return out


def c5_leg(dk, torch, SI):
    """One 2^34 x 2^34-bit product under the thesis rule and under the learned selector, and the
    squaring a*a (thesis rule): one timed call each after a warm-up call (tables prepared)."""
    n = (1 << 34) // 32
    g = torch.Generator(device="cuda")
    g.manual_seed(SI.SEED_BASE + 34)
    a = torch.randint(-2 ** 31, 2 ** 31, (n,), dtype=torch.int32, device="cuda", generator=g)
    b = torch.randint(-2 ** 31, 2 ** 31, (n,), dtype=torch.int32, device="cuda", generator=g)
    qs = primes61(SI.SEED_BASE + 34, 16)
    ra, rb = dk.residues(a, qs), dk.residues(b, qs)
    out = {"limbs": n, "verified": "residues mod 16 random 61-bit primes"}
    ref = None
    for name, policy, sq in (("thesis", dk.POLICY_THESIS, False), ("learned", dk.POLICY_LEARNED, False),
                             ("thesis_square", dk.POLICY_THESIS, True)):
        ctx = dk.Context(policy)
        ws = torch.empty(ctx.workspace_bytes(n, n), dtype=torch.uint8, device="cuda")
        c = torch.empty(2 * n, dtype=torch.int32, device="cuda")
        y = a if sq else b
        ctx.prepare(n, n)
        ms = _timed(lambda: ctx.mul(a, y, out=c, ws=ws), 1, torch)
        rc = dk.residues(c, qs)
        ry = ra if sq else rb
        if not all(z == x * w % q for x, w, z, q in zip(ra, ry, rc, qs)):
            raise RuntimeError("2^34 %s fails the residue check" % name)
        if not sq:
            if ref is None:
                ref = c
            elif not torch.equal(ref, c):
                raise RuntimeError("2^34 product differs between policies")
        out[name] = {"ms": ms, "value": (2 * n * 32) / (ms / 1e3),
                     "params": ctx.select_params(1 << 34, 1 << 34).as_dict()}
        log("2^34 %s: %.1f ms" % (name, ms))
        del ws
        if sq:
            del c
        torch.cuda.empty_cache()
    return out


def twiddle_forms_leg(reps, dk, torch):
    """The bad multiplications of one transform level of the 2^28-bit products (thesis rule and
    learned selector: their m = 16 and modulus q) in the two forms of dkss_probe_twiddle_products:
    2M elements in groups of 32 sharing one twiddle, seeded canonical residues, every output word
    of the two forms compared.  A level that used the matrix cores would first have to gather
    the elements of each table index together: that pass is priced here as one device copy of
    the level's S bytes."""
    out = {}
    n = 1 << 23
    gen = torch.Generator(device="cuda")
    for name, policy in (("thesis", dk.POLICY_THESIS), ("learned", dk.POLICY_LEARNED)):
        plan = dk.Context(policy).plan_info(n, n)
        L, log2_M = plan.L, plan.params.log2_M
        if plan.params.log2_m != 4 or not 3 <= L <= 6:
            continue
        q = sum(int(plan.q[k]) << (32 * k) for k in range(L))
        groups = (2 << log2_M) // 32
        top = q.bit_length() - 1 - 32 * (L - 1)
        gen.manual_seed(0x44B55 + 900 + L)

        def residues(count):
            w = torch.randint(-2 ** 31, 2 ** 31, (count, L), dtype=torch.int32, device="cuda", generator=gen)
            w[:, L - 1] &= (1 << top) - 1 if top < 31 else 0x7FFFFFFF
            return w.reshape(-1)

        t = residues(groups * 16)
        x = residues(groups * 32 * 16)
        r = torch.randint(0, 32, (groups * 32,), dtype=torch.int32, device="cuda", generator=gen)
        y1, y2 = torch.empty_like(x), torch.empty_like(x)
        # the two forms and the copy timed in turn, three times: the least time of each
        ms1 = ms2 = ms_copy = float("inf")
        for _ in range(3):
            ms1 = min(ms1, _timed(lambda: dk.probe_twiddle_products(1, q, L, groups, t, x, r, y1), reps, torch))
            ms2 = min(ms2, _timed(lambda: dk.probe_twiddle_products(2, q, L, groups, t, x, r, y2), reps, torch))
            ms_copy = min(ms_copy, _timed(lambda: y1.copy_(x), reps, torch))
        dk.probe_twiddle_products(1, q, L, groups, t, x, r, y1)
        torch.cuda.synchronize()
        if not torch.equal(y1, y2):
            raise RuntimeError("the two forms of the twiddle products differ (%s)" % name)
        S = x.numel() * 4
        out[name] = {"L": L, "q_bits": q.bit_length(), "elements": groups * 32, "groups": groups,
                     "poly_bytes": S, "vector_units_ms": ms1, "matrix_cores_ms": ms2,
                     "matrix_over_vector": ms2 / ms1, "gather_pass_ms": ms_copy,
                     "verified": "all %d output words of the two forms equal" % x.numel()}
        log("twiddle products %s (L = %d, %d elements): vector units %.3f ms, matrix cores %.3f ms, "
            "a gather pass %.3f ms" % (name, L, groups * 32, ms1, ms2, ms_copy))
        del t, x, r, y1, y2
        torch.cuda.empty_cache()
    return out


def copy_calibration(args, torch, out):
    """One device-to-device copy of --copy-calib bytes: a kernel of known HBM traffic that the
    counter runs scale their FETCH_SIZE and WRITE_SIZE by."""
    if args.copy_calib:
        src = torch.empty(args.copy_calib, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calib_bytes"] = args.copy_calib


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=4096, help="products in the headline batch")
    ap.add_argument("--legs", default="batch,2p28,sizes,smul,twforms,c5",
                    help="comma-separated legs to run (the headline batch is always run)")
    ap.add_argument("--no-c5", action="store_true", help="skip the 2^34 leg")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--lanes", type=int, default=4,
                    help="stream lanes of the headline batch's groups (DKSS_OPT_BATCH_LANES)")
    ap.add_argument("--headline-only", action="store_true",
                    help="profiling form: the headline batch alone (graph and profiled pass), or, "
                         "when --legs does not name batch, only the named legs among 2p28, smul "
                         "and twforms")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="end with one device-to-device copy of this many bytes (a counter "
                         "calibration kernel of known traffic)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    legs = set(x for x in args.legs.split(",") if x)

    import torch
    import paper_1503_04955_amd as dk
    import seeded_inputs as SI

    props = torch.cuda.get_device_properties(0)
    # the VALU peak is nominal (CUs x 64 lanes x clock); the measured rate of the products'
    # multiply-add instruction is reported beside it
    mad_rate = dk.probe_mad_rate() / 1e12
    log("v_mad_u64_u32: %.2f T lane-ops/s measured (nominal %.2f)" % (mad_rate, PEAK_VALU_TOPS))
    if args.headline_only and "batch" not in legs:
        # the profiling form of the other legs alone (no headline): one JSON line of them
        sub = {}
        if "2p28" in legs:
            sub["single_2p28"] = single_leg(28, args.steps, dk, torch, SI)
        if "smul" in legs:
            sub["smul"] = smul_leg([24, 28], args.steps, dk, torch, SI)
        if "twforms" in legs:
            sub["twiddle_forms"] = twiddle_forms_leg(args.steps, dk, torch)
        copy_calibration(args, torch, sub)
        print(json.dumps(sub), flush=True)
        return
    ms_step, bits, batch, stats = batch_leg(args, dk, torch, SI)
    out = {
        "metric": METRIC, "value": bits / (ms_step / 1e3), "unit": "operand bits/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic (seeded uniform uint32 limbs)",
        "config": {"workload": "batched DKSS, learned-tuned parameters, one replayed HIP graph: 4096 "
                               "products, operands 2^12..2^22 bits log-uniform, length ratio U[1,8]",
                   "products": args.batch, "operand_bits": bits},
        "verified": "every product equal to the plain calls' and c = a*b mod 8 random 61-bit primes",
        "device": {"name": props.name, "compute_units": props.multi_processor_count,
                   "hbm_bytes": props.total_memory, "mad_u64_u32_tops_measured": round(mad_rate, 2)},
        "roofline": roofline_of(stats, "batch4096", mad_rate),
        "kernels": kernel_table(stats, args.steps),
        "batch": batch,
    }
    if "plain_sequential" in batch:
        out["config"]["baseline"] = ("plain sequential calls, thesis rule: %.3f ms (%.4g operand bits/s)"
                                     % (batch["plain_sequential"]["ms"], batch["plain_sequential"]["value"]))
    else:
        out["verified"] = "c = a*b mod 8 random 61-bit primes for every 64th product"
    if "2p28" in legs:
        out["single_2p28"] = single_leg(28, args.steps, dk, torch, SI)
    if "sizes" in legs:
        out["sizes"] = sizes_leg([18, 24], 20, dk, torch, SI)
    if "smul" in legs:
        out["smul"] = smul_leg([24, 28], 10, dk, torch, SI)
    if "twforms" in legs:
        out["twiddle_forms"] = twiddle_forms_leg(10, dk, torch)
    if "c5" in legs and not args.no_c5:
        out["c5"] = c5_leg(dk, torch, SI)
    copy_calibration(args, torch, out)
    if not args.no_cpu:
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(SI.mixed_batch(args.batch))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
