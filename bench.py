"""Benchmark: verified secure linear inference over Z_{2^64} on one MI355X.

Default workload: the VGG-shaped network (batch 32, 32x32x3, 3x3 "same" convolutions
64-64-128-128-256-256 with 2x2 average pooling, FC 4096-256-10), chained as a linear
network (ReLU / max-pool are outside this path).  One timed step evaluates one batch of
synthetic input: encode and share the batch, and for every layer im2col, the truncation
pair, Pi_Inner, truncation and pooling; then one batched Pi_BIVerify of all layer
products.  Right after each step (outside the timed window, timed on its own) the
truncation gates are verified and the logits opened with Pi_Rec.

Printed metric: verified secure-matmul GOPS = sum over layers of 2 M K N / step time,
plus the truncation-gate verification rate and the roofline of the Pi_Inner product.

--workload mix runs the mixed-request serving configuration (512 requests, batch sizes
uniform in 1..64, model uniform over MLP / LeNet / VGG) and prints its own line.
"""
import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_2411_09287_amd import workloads  # noqa: E402

INT8_PEAK_TOPS = 5000.0       # MI355X dense int8 MFMA
ENVELOPE = (32768, 2304, 256)  # largest VGG-style conv product (batch 32, 3x3x256 -> 256)
TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "pi_inner_vgg_hbm_traffic.txt")
V2_TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                               "truncation_gates_vgg_hbm_traffic.txt")
# 64-bit integer multiply-accumulate on the vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# of single-issue vector instructions (39.3 T lane-instructions/s), four per u64 MAC in the
# product kernel (one 32x32->64 multiply-add, two 32-bit low multiplies, one three-way add),
# every one counted at the full issue rate: a ceiling, not a sustained rate.
U64_ALU_PEAK_TMACS = 256 * 4 * 16 * 2.4e9 / 4 / 1e12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_gpu(args):
    import torch
    from paper_2411_09287_amd import mpc3, network

    torch.cuda.set_device(0)
    name = args.workload
    batch = workloads.MODELS[name]["batch"]
    variant = {"limb": mpc3.VARIANT_LIMB_I8, "u64": mpc3.VARIANT_U64, "auto": mpc3.VARIANT_AUTO}[args.variant]
    ctx = mpc3.Context(workloads.master_seed(4))
    ctx.set_variant(variant)
    net = network.Network(ctx, name)
    shapes = net.shapes(batch)
    if args.variant == "auto":
        for M, K, N in net.exec_shapes(batch):
            ctx.autotune(M, K, N, 3)
    # the limb kernel's launch shape per layer, tuned once before any timed step
    tuning = []
    if args.variant != "u64" and not args.no_tune:
        for M, K, N in net.exec_shapes(batch):
            sh, md, mb = ctx.autotune_launch(M, K, N, 5)
            tuning.append({"shape": [M, K, N], "launch": list(sh), "ms_builtin": round(md, 4), "ms_tuned": round(mb, 4)})
        log(f"[bench] launch tuning: {json.dumps(tuning)}")
    x = torch.from_numpy(workloads.rng(4).random((batch,) + tuple(workloads.MODELS[name]["input"]))).cuda()
    ops = sum(2.0 * M * K * N for M, K, N in shapes)
    # the products run at the contraction width padded to whole k-blocks; work is counted at
    # the model's own (the library's counter takes the executed width)
    work_scale = sum(M * K * N for M, K, N in shapes) / sum(M * K * N for M, K, N in net.exec_shapes(batch))
    ntrunc = sum(M * N for M, K, N in shapes)
    log(f"[bench] workload={name} variant={args.variant} layers={len(shapes)} ring GOP per step={ops / 1e9:.3f}")

    def step():
        out = net.forward(x)
        ok = ctx.verify(-1, mpc3.VERIFY_INNER)
        return out, ok

    def finish(out):
        t0 = time.perf_counter()
        ok = ctx.verify(-1, mpc3.VERIFY_TRUNC)
        t1 = time.perf_counter()
        logits = ctx.reconstruct(out)
        return ok, t1 - t0, logits

    for i in range(args.warmup):
        out, ok = step()
        ok2, _, _ = finish(out)
        log(f"[bench] warmup {i + 1}/{args.warmup} ok={ok and ok2}")
    torch.cuda.synchronize()
    # no collector pauses inside the timed windows (collected here, re-enabled at the end)
    gc.collect()
    gc.disable()
    times, vtimes = [], []
    for i in range(args.steps):
        ctx.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out, ok = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        ctx.profile(False)
        ok2, vt, _ = finish(out)
        vtimes.append(vt)
        if not (ok and ok2):
            raise SystemExit("verification failed in an honest run")
        log(f"[bench] step {i + 1}/{args.steps} {times[-1] * 1e3:.2f} ms (truncation gates {vt * 1e3:.1f} ms)")
    ktime, launches, macs = ctx.profile_read()
    piped = None
    if not args.no_pipeline:
        # the same steps pipelined: each batch's batched Pi_BIVerify (mpc3_verify_begin) runs
        # on the worker streams while the next batch's layers run on the context's stream; the
        # window closes when the last verification has ended.  The truncation gates of these
        # batches are verified afterwards (outside the window; measured above per step).
        def pipelined(n):
            out = None
            for i in range(n):
                out = net.forward(x)
                if i > 0 and not ctx.verify_end():
                    raise SystemExit("verification failed in an honest run")
                ctx.verify_begin(-1, mpc3.VERIFY_INNER)
            return out, ctx.verify_end()

        # one untimed pass of the same length first: the allocator's pools then hold the
        # buffers of every batch whose truncation gates wait
        out, ok = pipelined(args.steps)
        ok2, _, _ = finish(out)
        if not (ok and ok2):
            raise SystemExit("verification failed in an honest run")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out, ok = pipelined(args.steps)
        torch.cuda.synchronize()
        piped = (time.perf_counter() - t0) / args.steps
        ok2, _, _ = finish(out)
        if not (ok and ok2):
            raise SystemExit("verification failed in an honest run")
        log(f"[bench] pipelined {args.steps} steps: {piped * 1e3:.2f} ms per step")
    # the serial step's two halves on their own: the forward (issue and GPU, synchronised),
    # then the batched Pi_BIVerify of its products (synchronous)
    fw_times, v1_times = [], []
    for i in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = net.forward(x)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ok = ctx.verify(-1, mpc3.VERIFY_INNER)
        t2 = time.perf_counter()
        fw_times.append(t1 - t0)
        v1_times.append(t2 - t1)
        ok2, _, _ = finish(out)
        if not (ok and ok2):
            raise SystemExit("verification failed in an honest run")
    log(f"[bench] forward {float(np.median(fw_times)) * 1e3:.2f} ms, Pi_BIVerify {float(np.median(v1_times)) * 1e3:.2f} ms")
    env = None if args.no_envelope else envelope(ctx)
    u64_times = []
    if args.variant == "limb" and not args.no_u64_step:
        # the same step with every product on the vector ALU (u64 kernels); its truncation
        # gates are verified afterwards with the matrix-core kernels (bit-identical results)
        cu = mpc3.Context(workloads.master_seed(4))
        cu.set_variant(mpc3.VARIANT_U64)
        netu = network.Network(cu, name)
        for i in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = netu.forward(x)
            ok = cu.verify(-1, mpc3.VERIFY_INNER)
            torch.cuda.synchronize()
            if i >= args.warmup:
                u64_times.append(time.perf_counter() - t0)
            cu.set_variant(mpc3.VARIANT_LIMB_I8)
            ok = cu.verify(-1, mpc3.VERIFY_TRUNC) and ok
            cu.set_variant(mpc3.VARIANT_U64)
            if not ok:
                raise SystemExit("verification failed in an honest run")
        log(f"[bench] u64 step {float(np.median(u64_times)) * 1e3:.2f} ms")
    gc.enable()
    return {"batch": batch, "shapes": shapes, "ops": ops, "ntrunc": ntrunc, "times": times, "vtimes": vtimes,
            "ktime": ktime, "launches": launches, "macs": macs * work_scale, "envelope": env, "u64_times": u64_times,
            "piped": piped, "fw_times": fw_times, "v1_times": v1_times, "tuning": tuning}


# Truncation-gate verification: the HBM bytes the method must move per truncation once its
# gates are materialised after five symbolic rounds (4 elements per truncation and plane, two
# planes of 64-word elements): the two planes written once (4096 B), and every later round
# reading both planes and writing the folded halves, 3 n 512 B for n rows per plane, n =
# 4, 2, 1, ... per truncation (sum 8): 12288 B.
V2_BYTES_PER_TRUNCATION = 4096 + 12288
HBM_PEAK_GBPS = 8000.0


def v2_measured_bytes_per_truncation():
    """HBM bytes per truncation of the truncation-gate phase measured with rocprofv3 counters
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy), valid only while the sources of its
    kernels and host steps are the ones they were taken on; None otherwise."""
    import hashlib
    try:
        lines = open(V2_TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    kv = dict(ln.split(":", 1) for ln in lines if ln.startswith(("source_sha256:", "bytes_per_truncation:")))
    h = hashlib.sha256()
    for name in ("gemm_limb.hip", "kernels.hip", "engine.cpp"):
        h.update(open(os.path.join(ROOT, "paper_2411_09287_amd", "csrc", name), "rb").read())
    if kv.get("source_sha256", "").strip() != h.hexdigest() or "bytes_per_truncation" not in kv:
        return None
    return float(kv["bytes_per_truncation"])


def v2_roofline(ntrunc, seconds, variant="limb"):
    achieved = V2_BYTES_PER_TRUNCATION * ntrunc / seconds / 1e9
    per = v2_measured_bytes_per_truncation() if variant == "limb" else None
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS, "traffic": per * ntrunc if per else None,
            "kernel": "truncation-gate verification, whole phase (algorithmic bytes of its materialised rounds: "
                      f"{V2_BYTES_PER_TRUNCATION} B per truncation)"}


def measured_traffic(variant):
    """HBM bytes per Pi_Inner product call measured with rocprofv3 counters (FETCH_SIZE and
    WRITE_SIZE, scaled by a plain copy), valid only while the product kernel's source is
    the one they were taken on; None otherwise."""
    import hashlib
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    kv = dict(ln.split(":", 1) for ln in lines if ln.startswith(("source_sha256:", "bytes_per_call_")))
    src = os.path.join(ROOT, "paper_2411_09287_amd", "csrc", "gemm_limb.hip" if variant != "u64" else "gemm_u64.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if kv.get("source_sha256", "").strip() != digest:
        return None
    v = kv.get(f"bytes_per_call_{variant}")
    return float(v) if v else None


def envelope(ctx, reps=5):
    """Both kernel families on the envelope product (three-party form)."""
    M, K, N = ENVELOPE
    _, ms_u64, ms_limb = ctx.autotune(M, K, N, reps)
    ops = 72.0 * 5 * M * K * N
    return {"shape": list(ENVELOPE), "u64_ms": ms_u64, "limb_ms": ms_limb, "limb_over_u64": ms_u64 / ms_limb,
            "limb_int8_tops": ops / (ms_limb * 1e-3) / 1e12, "limb_int8_frac": ops / (ms_limb * 1e-3) / 1e12 / INT8_PEAK_TOPS}


def _oracle_rows(job):
    """One worker of the CPU baseline: the oracle on `rows_of(M)` rows of every layer."""
    from oracle.protocol import Ctx
    from oracle.ring import encode

    shapes, frac, part, parts = job
    o = Ctx(workloads.master_seed(4))
    g = workloads.rng(9 + part)
    ops = 0.0
    for M, K, N in shapes:
        rows = max(1, M // frac // parts)
        X = o.share(encode(g.random((rows, K)), 13))
        W = o.share(encode(g.standard_normal((K, N)) * 0.05, 13))
        pair = o.trunc_pair(rows * N, 13)
        o.trunc(pair, o.inner(X, W, pair))
        ops += 2.0 * rows * K * N
    if not o.verify(kinds=1):
        raise SystemExit("oracle verification failed in an honest run")
    return ops


def cpu_baseline(args, shapes):
    """The oracle on a row sample of every layer of the step: share, truncation pair,
    Pi_Inner and truncation per layer, then one batched verification of the sampled
    products (no truncation gates), as in the timed GPU step.  Once on one core (1/frac of
    the rows) and once on `cores` worker processes, each taking 1/cores of a 4x larger
    sample (its own context and verification: the same work split by row blocks)."""
    import multiprocessing

    frac = args.cpu_sample
    t0 = time.perf_counter()
    ops1 = _oracle_rows((shapes, frac, 0, 1))
    dt1 = time.perf_counter() - t0
    cores = args.cpu_cores
    out = {"value": ops1 / dt1 / 1e9, "unit": "GOPS", "cores": 1, "kind": "oracle",
           "sample": f"1/{frac} of the rows of every layer product (same K, N): share, truncation pair, "
                     f"Pi_Inner, truncation per layer, one batched verification; {dt1:.1f} s on one core"}
    if cores > 1:
        frac_m = max(1, frac // 4)
        t0 = time.perf_counter()
        with multiprocessing.get_context("fork").Pool(cores) as pool:
            opsm = sum(pool.map(_oracle_rows, [(shapes, frac_m, i, cores) for i in range(cores)]))
        dtm = time.perf_counter() - t0
        out["multi_core"] = {"value": opsm / dtm / 1e9, "unit": "GOPS", "cores": cores,
                             "sample": f"1/{frac_m} of the rows in {cores} row blocks, one process each; "
                                       f"{dtm:.1f} s wall"}
    return out


def comparisons(name, batch):
    """Comparisons (ReLU evaluations) of one batch: every output of every layer but the last,
    and for each 2x2 max pool of N outputs 2 N / 4 + N / 4 more."""
    from paper_2411_09287_amd import network
    plan = network.plan(name)
    n = 0
    for i, d in enumerate(plan):
        M, K, N = workloads.layer_gemm_shape(d["layer"], batch)
        if i + 1 < len(plan):
            n += M * N
            if d["pool_after"]:
                n += M * N // 4 * 3
    return n


def _oracle_network(job):
    """The oracle through network.Network's call sequence with ReLU and max pooling on
    `batch` images, every product verified; returns the images done."""
    from oracle.layers import im2col_share
    from oracle.protocol import Share, Ctx
    from oracle.ring import encode
    from paper_2411_09287_amd import network

    name, batch, seed = job
    o = Ctx(workloads.master_seed(2))
    plan = network.plan(name)
    weights = []
    for d, w in zip(plan, network.float_weights(name, nonlinear=True)):
        if d.get("kpad", w.shape[0]) > w.shape[0]:
            w = np.concatenate([w, np.zeros((d["kpad"] - w.shape[0], w.shape[1]))])
        weights.append(o.share(encode(w, 13)))
    x = workloads.rng(seed).random((batch,) + tuple(workloads.MODELS[name]["input"]))
    h = o.share(encode(x, 13).reshape(batch, -1))
    for i, (d, W) in enumerate(zip(plan, weights)):
        layer = d["layer"]
        if layer[0] == "conv":
            _, kh, kw, cin, cout, pad, (hh, ww) = layer[:7]
            X = im2col_share(h.map(lambda a: a.reshape(batch, hh, ww, cin)), kh, kw, pad, workloads.conv_stride(layer))
            extra = d["kpad"] - X.m.shape[1]
            if extra:
                X = X.map(lambda a: np.concatenate([a, np.zeros((a.shape[0], extra), dtype=np.uint64)], axis=1))
        else:
            X = h.map(lambda a: a.reshape(batch, -1))
        pair = o.trunc_pair(X.m.shape[0] * W.m.shape[1], 13)
        Y = o.trunc(pair, o.inner(X, W, pair))
        if i + 1 < len(plan):
            Y = o.relu(Y)
        if d["pool_after"]:
            oh, ow = d["out_hw"]
            Y = o.maxpool2(Y.map(lambda a: a.reshape(batch, -1)), batch, oh, ow, layer[4])
        h = Share(*[a.reshape(batch, -1) for a in Y.comps()])
    if not o.verify():
        raise SystemExit("oracle verification failed in an honest run")
    o.reconstruct(h)
    return batch


def cpu_baseline_nonlinear(args, comparisons_per_image):
    """The oracle's secure inference with ReLU and max pooling, every product verified, on
    one core, in images/s: the whole network on one image for the MLP; for the larger
    networks (one image takes the oracle hours) the ReLU of 64 values with its verification
    (the comparisons dominate the oracle's time), scaled by the comparisons of one image."""
    from oracle.protocol import Ctx
    from oracle.ring import encode

    t0 = time.perf_counter()
    if args.workload == "mlp":
        n = _oracle_network((args.workload, 1, 3))
        dt = time.perf_counter() - t0
        return {"value": n / dt, "unit": "inferences/s", "cores": 1, "kind": "oracle",
                "sample": f"one image of the mlp network with ReLU, every product verified; {dt:.1f} s on one core"}
    o = Ctx(workloads.master_seed(2))
    o.relu(o.share(encode(workloads.rng(3).standard_normal(64), 13)))
    if not o.verify():
        raise SystemExit("oracle verification failed in an honest run")
    dt = time.perf_counter() - t0
    return {"value": 64.0 / dt / comparisons_per_image, "unit": "inferences/s", "cores": 1, "kind": "oracle",
            "sample": f"ReLU of 64 values with every product verified, {dt:.1f} s on one core, scaled to the "
                      f"{comparisons_per_image} comparisons of one image (linear layers not counted)"}


def run_nonlinear(args, cpu):
    """Secure inference with ReLU and max pooling: one step evaluates a batch and verifies
    every product it made (the layer products, the truncation gates, the Pi_Mult triples
    and the Boolean triples of the non-linear layers), then opens the logits."""
    import torch
    from paper_2411_09287_amd import mpc3, network

    torch.cuda.set_device(0)
    name = args.workload
    batch = workloads.MODELS[name]["batch"]
    variant = {"limb": mpc3.VARIANT_LIMB_I8, "u64": mpc3.VARIANT_U64, "auto": mpc3.VARIANT_LIMB_I8}[args.variant]
    ctx = mpc3.Context(workloads.master_seed(2))
    ctx.set_variant(variant)
    net = network.Network(ctx, name, nonlinear=True)
    x = torch.from_numpy(workloads.rng(2).random((batch,) + tuple(workloads.MODELS[name]["input"]))).cuda()
    phases = {}

    def step():
        out = net.forward(x)
        ok = True
        for label, kind in (("inner", mpc3.VERIFY_INNER), ("mult", mpc3.VERIFY_MULT),
                            ("nonlinear", mpc3.VERIFY_NONLINEAR), ("trunc", mpc3.VERIFY_TRUNC)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ok = ctx.verify(-1, kind) and ok
            phases.setdefault(label, []).append(time.perf_counter() - t0)
        ctx.reconstruct(out)
        return ok

    for i in range(args.warmup):
        if not step():
            raise SystemExit("verification failed in an honest run")
        log(f"[bench] warmup {i + 1}/{args.warmup}")
    phases.clear()
    times = []
    c0 = ctx.comm_stats()
    for i in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if not step():
            raise SystemExit("verification failed in an honest run")
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log(f"[bench] step {i + 1}/{args.steps} {times[-1] * 1e3:.1f} ms")
    cb, cr = ctx.comm_stats()
    t = float(np.median(times))
    nrelu = comparisons(name, batch)
    return {"metric": "verified secure inferences/s", "value": batch / t, "unit": "inferences/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": t * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": {"u64": "u64"}.get(args.variant, "int8-limb"),
            "data": "synthetic",
            "config": {"workload": f"{name} with ReLU and 2x2 max pooling, batch {batch}",
                       "comparisons_per_batch": nrelu,
                       "verify_ms": {k: float(np.median(v)) * 1e3 for k, v in phases.items()},
                       "comm_bytes_per_batch": int((np.asarray(cb, dtype=np.int64) - np.asarray(c0[0], dtype=np.int64)).sum()) // max(args.steps, 1),
                       "comm_rounds_per_batch": [(a - b) // max(args.steps, 1) for a, b in zip(cr, c0[1])]},
            "roofline": None, "cpu_baseline": cpu}


def run_depth(args):
    """Multiplication circuits of depth 32 and 128 (Sec. 5.1, Fig. "dep"): a batch of
    `width` values multiplied layer by layer, x_(k+1) = Pi_Mult(x_k, y_k), then one
    verification of every layer's triples (R chosen by the cost model on the MAN setting).
    Reports the GPU time of the evaluation and of the verification, the counted
    communication and rounds, and the modelled MAN time of the whole run."""
    import torch
    from paper_2411_09287_amd import mpc3, netmodel

    torch.cuda.set_device(0)
    width = args.depth_width
    g = workloads.rng(7)
    out = {}
    for depth in (32, 128):
        ctx = mpc3.Context(workloads.master_seed(7))
        ctx.set_variant(mpc3.VARIANT_LIMB_I8)
        rtt, bw = netmodel.NETWORKS["MAN"]
        ctx.set_network(rtt * 1e3, bw / 1e6, 0.1)
        x0 = g.integers(0, 1 << 64, (width, 1), dtype=np.uint64, endpoint=False)
        ys = [g.integers(0, 1 << 64, (width, 1), dtype=np.uint64, endpoint=False) for _ in range(depth)]
        X = ctx.share(mpc3.to_words(x0))
        Ys = [ctx.share(mpc3.to_words(y)) for y in ys]
        torch.cuda.synchronize()
        c0 = ctx.comm_stats()
        t0 = time.perf_counter()
        for k in range(depth):
            X = ctx.mult(X, Ys[k])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ok = ctx.verify(mpc3.R_NETWORK, mpc3.VERIFY_MULT)
        t2 = time.perf_counter()
        if not ok:
            raise SystemExit("verification failed in an honest run")
        cb, cr = netmodel.diff(ctx.comm_stats(), c0)
        got = mpc3.from_words(ctx.reconstruct(X)).reshape(-1)
        want = x0.reshape(-1).copy()
        for y in ys:
            want = want * y.reshape(-1)
        if not np.array_equal(got, want):
            raise SystemExit("opened product differs from the plaintext product")
        phases = (netmodel.OFFLINE, netmodel.ONLINE, netmodel.VERIFY_OFFLINE, netmodel.VERIFY_ONLINE)
        man = netmodel.seconds(cb, cr, phases, "MAN")
        out[f"depth_{depth}"] = {"eval_gpu_ms": (t1 - t0) * 1e3, "verify_gpu_ms": (t2 - t1) * 1e3,
                                 "comm_bytes": int(np.asarray(cb).sum()), "rounds": cr,
                                 "man_model_s": man, "mults_per_s_gpu": width * depth / (t2 - t0)}
        log(f"[depth] {depth}: {json.dumps(out[f'depth_{depth}'])}")
    return out


def run_mix(args):
    """Mixed-request serving: packed with direct calls (every request at time 0), packed
    per (model, batch bucket) from HIP graphs where the replay was measured faster than
    direct calls (every request at time 0, and open-loop Poisson arrivals at 70% of that
    server's measured capacity), and the u64 per-request baseline."""
    import torch
    from paper_2411_09287_amd import mpc3, serve

    torch.cuda.set_device(0)
    reqs = serve.request_mix(args.requests, seed=5)
    out = {}
    runs = [("limb_packed", mpc3.VARIANT_AUTO, True, False), ("limb_packed_graphs", mpc3.VARIANT_AUTO, True, "auto")]
    if not args.no_baseline:
        runs.append(("u64_per_request", mpc3.VARIANT_U64, False, False))
    for label, variant, pack, graphs in runs:
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            ctx = mpc3.Context(workloads.master_seed(5))
            ctx.set_variant(variant)
            srv = serve.Server(ctx, graphs=graphs)
            if variant == mpc3.VARIANT_AUTO:
                n = srv.tune(reqs, log=lambda m: log(f"[mix] {m}"))
                log(f"[mix] tuned {n} layer shapes")
            if graphs == "auto":
                picks = srv.tune_graphs()
                out["graph_buckets"] = sorted(f"{m}_b{b}" for (m, b), v in picks.items() if v)
                log(f"[mix] graphs chosen for {out['graph_buckets']}")
            res = srv.run(reqs, pack=pack, log=lambda m: log(f"[mix] {label} {m}"))
            out[label] = serve.summary(res)
            log(f"[mix] {label}: {json.dumps(out[label])}")
            if graphs:
                # requests per second at 70% of the capacity just measured
                rate = 0.7 * len(reqs) / res["makespan"]
                res = srv.run(reqs, pack=pack, arrivals=serve.poisson_arrivals(reqs, rate),
                              log=lambda m: log(f"[mix] open-loop {m}"))
                out["limb_graphs_open_loop"] = {**serve.summary(res), "arrival_rate_per_s": rate}
                log(f"[mix] open loop: {json.dumps(out['limb_graphs_open_loop'])}")
            ctx.close()
    out["forward_ms"] = forward_graph_vs_direct()
    return reqs, out


def forward_graph_vs_direct(reps=20):
    """Wall time (host issue + GPU, synchronised) of one linear forward per model and batch
    bucket: direct calls against the replay of the recorded graph (median of reps; each
    replay is verified, untimed, before the next)."""
    import time

    import torch
    from paper_2411_09287_amd import mpc3, network, serve

    res = {}
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        ctx = mpc3.Context(workloads.master_seed(9))
        ctx.set_variant(mpc3.VARIANT_LIMB_I8)
        for name in serve.MODEL_NAMES:
            net = network.Network(ctx, name)
            for b in (1, 8, 64):
                x = serve.request_input(name, b, 0, ctx.device)
                rf = network.RecordedForward(net, b)
                tt = {"direct": [], "graph": []}
                for _ in range(reps):
                    for kind in ("direct", "graph"):
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        h = net.forward(x) if kind == "direct" else rf(x)
                        torch.cuda.synchronize()
                        tt[kind].append(time.perf_counter() - t0)
                        assert ctx.verify()
                        del h
                res[f"{name}_b{b}"] = {k: float(np.median(v) * 1e3) for k, v in tt.items()}
                res[f"{name}_b{b}"]["kernel_nodes"] = rf.nodes()[0]
                log(f"[mix] forward {name} batch {b}: {json.dumps(res[f'{name}_b{b}'])}")
                rf.close()
        ctx.close()
    return res


def run_rtrade(args):
    """Verification time against the repetition parameter R: Pi_MultVerify of n Pi_Mult
    triples (n = 2^18, 2^20) for R = 0..10, GPU time measured, network time of the counted
    verification messages from the LAN/MAN/WAN model; the R that minimises the sum."""
    import torch
    from paper_2411_09287_amd import mpc3, netmodel

    torch.cuda.set_device(0)
    ctx = mpc3.Context(workloads.master_seed(6))
    ctx.set_variant(mpc3.VARIANT_LIMB_I8)
    g = workloads.rng(6)
    out = {}
    for logn in (18, 20):
        n = 1 << logn
        a = ctx.share(mpc3.to_words(g.integers(0, 1 << 63, n, dtype=np.uint64)))
        b = ctx.share(mpc3.to_words(g.integers(0, 1 << 63, n, dtype=np.uint64)))
        table = {}
        for R in range(0, 11):
            best = None
            for rep in range(3):
                ctx.mult(a, b)
                torch.cuda.synchronize()
                c0 = ctx.comm_stats()
                t0 = time.perf_counter()
                ok = ctx.verify(R, mpc3.VERIFY_MULT)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                if not ok:
                    raise SystemExit("verification failed in an honest run")
                cb, cr = netmodel.diff(ctx.comm_stats(), c0)
                if best is None or dt < best[0]:
                    best = (dt, cb, cr)
            table[R] = best
            log(f"[rtrade] |G|=2^{logn} R={R} gpu {best[0] * 1e3:.2f} ms")
        out[f"2^{logn}"] = {
            "gpu_ms": {R: v[0] * 1e3 for R, v in table.items()},
            "verify_rounds": {R: v[2][2] + v[2][3] for R, v in table.items()},
            "verify_bytes": {R: int(v[1][2].sum() + v[1][3].sum()) for R, v in table.items()},
            "best": {net: {"R": R, "ms": tot * 1e3} for net in netmodel.NETWORKS
                     for R, tot in [netmodel.best_r(table, net)]},
        }
    return out


def hbm_copy(gib):
    """A plain device-to-device copy of `gib` GiB: its time gives the achievable HBM rate and,
    under rocprofv3 --pmc, the counter reading of a known byte count."""
    import torch
    torch.cuda.set_device(0)
    n = int(gib * (1 << 30)) // 8
    a = torch.empty(n, dtype=torch.int64, device="cuda").fill_(1)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    print(json.dumps({"copy_bytes": 8 * n, "ms": ms, "read_plus_write_GBps": 2 * 8 * n / (ms * 1e-3) / 1e9}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--variant", choices=["u64", "limb", "auto"], default="limb")
    ap.add_argument("--workload", default="vgg", choices=["vgg", "lenet", "mlp", "matmul", "snn", "lenet5", "vgg16",
                                                          "depth", "mix", "rtrade"])
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--depth-width", type=int, default=1 << 16, help="values per layer of the depth workload")
    ap.add_argument("--no-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=16)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-cores", type=int, default=8, help="worker processes of the multi-core CPU baseline")
    ap.add_argument("--nonlinear", action="store_true",
                    help="networks with ReLU and max pooling (edaBits); the step verifies every product")
    ap.add_argument("--no-envelope", action="store_true")
    ap.add_argument("--no-u64-step", action="store_true", help="skip the u64-kernel run of the step")
    ap.add_argument("--no-tune", action="store_true", help="built-in launch shapes (no launch-shape autotuning)")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="report the synchronised one-step-at-a-time time only")
    ap.add_argument("--hbm-copy", type=float, default=0.0, help="only time a device copy of this many GiB")
    ap.add_argument("--envelope-only", action="store_true", help="only time the envelope product")
    args = ap.parse_args()
    if args.hbm_copy > 0:
        hbm_copy(args.hbm_copy)
        return
    if args.envelope_only:
        import torch
        from paper_2411_09287_amd import mpc3
        torch.cuda.set_device(0)
        print(json.dumps(envelope(mpc3.Context(workloads.master_seed(4)))))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU benchmark: --gpus above 1 is not supported (the multi-GPU layout is a design note only)"}))
        raise SystemExit(2)

    if args.workload == "rtrade":
        res = run_rtrade(args)
        best = res["2^20"]["best"]["MAN"]
        line = {"metric": "verification time at the best R (Pi_MultVerify, 2^20 triples, MAN model)",
                "value": best["ms"], "unit": "ms", "n_gpus": 1, "steps": 1, "warmup": 0,
                "ms_per_step": best["ms"], "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
                "dtype": "int8-limb", "data": "synthetic",
                "config": {"workload": "Pi_MultVerify of 2^18 and 2^20 triples, R = 0..10", **res}}
        print(json.dumps(line))
        return

    if args.workload == "depth":
        res = run_depth(args)
        d = res["depth_128"]
        line = {"metric": "verified secure multiplications/s (depth-128 circuit, GPU time)",
                "value": d["mults_per_s_gpu"], "unit": "mults/s", "n_gpus": 1, "steps": 1, "warmup": 0,
                "ms_per_step": d["eval_gpu_ms"] + d["verify_gpu_ms"], "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "int8-limb", "data": "synthetic",
                "config": {"workload": f"multiplication circuits of depth 32 and 128, width {args.depth_width}",
                           **res}}
        print(json.dumps(line))
        return

    if args.workload == "mix":
        reqs, res = run_mix(args)
        main_res = res["limb_packed_graphs"]
        line = {"metric": "verified secure inferences/s (linear path)", "value": main_res["inferences_per_s"],
                "unit": "inferences/s", "n_gpus": 1, "steps": 1, "warmup": 0,
                "ms_per_step": main_res["makespan_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "int8-limb", "data": "synthetic",
                "config": {"workload": f"mixed requests: {len(reqs)} requests, batch 1..64, mlp/lenet/vgg",
                           **{k: v for k, v in res.items()}}}
        print(json.dumps(line))
        return

    # the CPU baseline runs first, before this process initialises the GPU (its worker
    # processes are forked)
    if args.nonlinear:
        cpu = None if args.no_cpu else cpu_baseline_nonlinear(args, comparisons(args.workload, 1))
        print(json.dumps(run_nonlinear(args, cpu)))
        return
    cpu = None if args.no_cpu else cpu_baseline(args, workloads.model_shapes(args.workload))
    r = run_gpu(args)
    ts = float(np.median(r["times"]))              # one step at a time, synchronised
    t = r["piped"] if r["piped"] is not None else ts
    vt = float(np.median(r["vtimes"]))
    avg_launch_ms = r["ktime"] / max(r["launches"], 1)
    macs_per_launch = r["macs"] / max(r["launches"], 1)
    if args.variant == "u64":
        achieved = macs_per_launch / (avg_launch_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": U64_ALU_PEAK_TMACS, "unit": "T u64-MAC/s",
                "frac": achieved / U64_ALU_PEAK_TMACS, "traffic": None}
    else:
        achieved = macs_per_launch * 72 / (avg_launch_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": INT8_PEAK_TOPS, "unit": "TOPS",
                "frac": achieved / INT8_PEAK_TOPS, "traffic": None}
    traffic = measured_traffic(args.variant)
    roof["traffic"] = traffic
    roof["kernel"] = "Pi_Inner three-party product (one call: B-digit conversion + product), all layers"
    roof["avg_launch_ms"] = avg_launch_ms
    roof["launches"] = r["launches"]
    line = {
        "metric": "verified Z_2^64 secure-matmul GOPS",
        "value": r["ops"] / t / 1e9, "unit": "GOPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"u64": "u64", "limb": "int8-limb", "auto": "autotuned"}[args.variant], "data": "synthetic",
        "config": {"workload": f"{args.workload} linear network (no activations; 2x2 sum pooling, its 1/4 folded into "
                               f"the next weights, in place of max pooling), batch {r['batch']}", "variant": args.variant,
                   "layers": [list(s) for s in r["shapes"]],
                   "window": "encode+share, im2col, truncation pairs, Pi_Inner, truncation, pooling, "
                             "one batched Pi_BIVerify of every layer product"
                             + ("; steps pipelined (a batch's Pi_BIVerify overlaps the next batch's layers)"
                                if r["piped"] is not None else ""),
                   "serial_ms_per_step": ts * 1e3,
                   "forward_ms": float(np.median(r["fw_times"])) * 1e3,
                   "pi_biverify_ms": float(np.median(r["v1_times"])) * 1e3,
                   "linear_images_per_s": r["batch"] / t,
                   "truncation_gate_verify_ms": vt * 1e3,
                   "truncations_per_s": r["ntrunc"] / vt,
                   "images_per_s_incl_truncation_gates": r["batch"] / (t + vt),
                   "envelope_product": r["envelope"],
                   "launch_tuning": r["tuning"]},
        "roofline": roof,
        "v2_roofline": v2_roofline(r["ntrunc"], vt, args.variant),
        "cpu_baseline": cpu,
    }
    if r["u64_times"]:
        tu = float(np.median(r["u64_times"]))
        line["config"]["u64_step"] = {"serial_ms_per_step": tu * 1e3, "GOPS": r["ops"] / tu / 1e9,
                                      "limb_over_u64_serial": tu / ts}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
