"""Benchmark: verified secure linear layers over Z_{2^64} on one MI355X.

One step = one pass of the linear path of the VGG-style network (batch 32, 32x32x3,
3x3 same convolutions 64-64-128-128-256-256 and FC 4096-256-10) over one batch of
synthetic input: for every layer, encode and share its input activation (im2col for
convolutions) and evaluate Pi_Inner; then verify every product of the step (one
compressed Pi_BIVerify per layer) and open the logits with Pi_Rec.  With --trunc the
step also generates each layer's truncation pair, truncates, and verifies the
truncation gates.  Weights are shared once, outside the timed region.

Printed metric: verified secure-matmul GOPS = sum over layers of 2 M K N / step time.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_2411_09287_amd import workloads  # noqa: E402

INT8_PEAK_TOPS = 5000.0       # MI355X dense int8 MFMA
HBM_PEAK_GBS = 8000.0
# 64-bit integer multiply-accumulate on the vector ALU: 256 CUs x 64 lanes x 2.4 GHz of
# 32-bit multiplies at quarter rate, three multiplies per u64 MAC.
U64_ALU_PEAK_TMACS = 256 * 64 * 2.4e9 / 4 / 3 / 1e12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def layer_plan(name):
    spec = workloads.MODELS[name]
    plan = []
    for i, layer in enumerate(spec["layers"]):
        M, K, N = workloads.layer_gemm_shape(layer, spec["batch"])
        plan.append({"i": i, "layer": layer, "M": M, "K": K, "N": N})
    return spec["batch"], plan


def gpu_step(ctx, mpc3, batch, plan, inputs, weights, trunc):
    last = None
    for L in plan:
        layer = L["layer"]
        xs = ctx.share(ctx.encode(inputs[L["i"]]).reshape(batch, -1))
        if layer[0] == "conv":
            _, kh, kw, cin, cout, pad, (h, w) = layer
            xs = ctx.im2col(xs, batch, h, w, cin, kh, kw, pad)
        if trunc:
            pair = ctx.trunc_pair(L["M"] * L["N"], workloads.FRAC_BITS)
            last = ctx.trunc(pair, ctx.inner(xs, weights[L["i"]], pair))
        else:
            last = ctx.inner(xs, weights[L["i"]])
    ok = ctx.verify(-1, mpc3.VERIFY_ALL)
    out = ctx.reconstruct(last)
    return ok, out


def run_gpu(args):
    import torch
    from paper_2411_09287_amd import mpc3

    torch.cuda.set_device(0)
    batch, plan = layer_plan(args.workload)
    seed = workloads.master_seed(4)
    variant = mpc3.VARIANT_LIMB_I8 if args.variant == "limb" else mpc3.VARIANT_U64
    ctx = mpc3.Context(seed)
    ctx.set_variant(variant)
    inputs, weights = [], []
    for L in plan:
        layer = L["layer"]
        x = workloads.layer_input(layer, batch, 100 + L["i"])
        inputs.append(torch.from_numpy(x).cuda())
        w = workloads.layer_weight(layer, 200 + L["i"]).reshape(L["K"], L["N"])
        weights.append(ctx.share(ctx.encode(torch.from_numpy(w).cuda())))
    ops = sum(2.0 * L["M"] * L["K"] * L["N"] for L in plan)
    log(f"[bench] workload={args.workload} variant={args.variant} layers={len(plan)} "
        f"ring GOP per step={ops / 1e9:.2f}")
    for i in range(args.warmup):
        ok, _ = gpu_step(ctx, mpc3, batch, plan, inputs, weights, args.trunc)
        log(f"[bench] warmup {i + 1}/{args.warmup} ok={ok}")
    torch.cuda.synchronize()
    ctx.profile(True)
    times = []
    for i in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ok, out = gpu_step(ctx, mpc3, batch, plan, inputs, weights, args.trunc)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        if not ok:
            raise SystemExit("verification failed in an honest run")
        log(f"[bench] step {i + 1}/{args.steps} {times[-1] * 1e3:.2f} ms")
    ctx.profile(False)
    ktime, launches, macs = ctx.profile_read()
    return plan, batch, ops, times, (ktime, launches, macs)


def cpu_baseline(args, plan, batch):
    """The oracle on a row sample of every layer: share, truncation pair, Pi_Inner, truncation
    and the compressed per-layer verification, as in one GPU step (no V2)."""
    from oracle.layers import im2col_share
    from oracle.protocol import Ctx
    from oracle.ring import encode

    frac = args.cpu_sample
    o = Ctx(workloads.master_seed(4), chunk=1 << 14)
    t0 = time.perf_counter()
    ops = 0.0
    for L in plan:
        layer = L["layer"]
        rows = max(1, L["M"] // frac)
        if layer[0] == "conv":
            _, kh, kw, cin, cout, pad, (h, w) = layer
            imgs = max(1, batch // frac)
            x = workloads.layer_input(layer, imgs, 100 + L["i"])
            xs = o.share(encode(x, 13).reshape(imgs, -1))
            X = im2col_share(xs.map(lambda a: a.reshape(imgs, h, w, cin)), kh, kw, pad)
            rows = X.m.shape[0]
        else:
            x = workloads.layer_input(layer, batch, 100 + L["i"])[:rows]
            X = o.share(encode(x, 13))
        Wt = workloads.layer_weight(layer, 200 + L["i"]).reshape(L["K"], L["N"])
        W = o.share(encode(Wt, 13))
        o.inner(X, W)
        o.verify(kinds=1)
        ops += 2.0 * rows * L["K"] * L["N"]
    dt = time.perf_counter() - t0
    return {"value": ops / dt / 1e9, "unit": "GOPS", "cores": 1, "kind": "oracle",
            "sample": f"1/{frac} of the rows (images) of every layer: share, Pi_Inner and the per-layer "
                      f"compressed verification; {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--variant", choices=["u64", "limb"], default="limb")
    ap.add_argument("--workload", default="vgg", choices=["vgg", "lenet", "mlp", "matmul"])
    ap.add_argument("--trunc", action="store_true",
                    help="truncation pairs, truncation and their gate verification inside the step")
    ap.add_argument("--cpu-sample", type=int, default=64)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus above 1 is not supported"}))
        raise SystemExit(2)

    plan, batch, ops, times, (ktime, launches, macs) = run_gpu(args)
    t = float(np.median(times))
    value = ops / t / 1e9
    avg_launch_ms = ktime / max(launches, 1)
    macs_per_launch = macs / max(launches, 1)
    if args.variant == "limb":
        achieved = macs_per_launch * 72 / (avg_launch_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": INT8_PEAK_TOPS, "unit": "TOPS",
                "frac": achieved / INT8_PEAK_TOPS, "traffic": None}
    else:
        achieved = macs_per_launch / (avg_launch_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": U64_ALU_PEAK_TMACS, "unit": "T u64-MAC/s",
                "frac": achieved / U64_ALU_PEAK_TMACS, "traffic": None}
    roof["kernel"] = "Pi_Inner party product (all layers)"
    roof["avg_launch_ms"] = avg_launch_ms
    cpu = None if args.no_cpu else cpu_baseline(args, plan, batch)
    line = {
        "metric": "verified Z_2^64 secure-matmul GOPS",
        "value": value, "unit": "GOPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int8-limb" if args.variant == "limb" else "u64", "data": "synthetic",
        "config": {"workload": f"{args.workload} linear path, batch {batch}", "variant": args.variant,
                   "layers": [[L["M"], L["K"], L["N"]] for L in plan], "trunc_in_step": bool(args.trunc),
                   "linear_images_per_s": batch / t},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
