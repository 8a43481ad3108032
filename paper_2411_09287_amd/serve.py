"""Batched serving of mixed secure-inference requests on one GPU.

Requests (model, batch size) arrive together; requests of the same model are packed, in
arrival order, into row-blocks of at most `cap[model]` images.  A pack runs as one
secure evaluation: every layer is one Pi_Inner over the packed rows (rows are images x
output positions, so requests simply stack), one truncation pair, and one verification
per layer for the whole pack; the opened logits are split back per request.  Packing
amortises the verification (whose cost does not grow with the number of rows beyond
the compression products) and the per-launch costs over many requests.

The packer also orders packs so that a model's first pack runs as soon as possible
(first-come order of each pack's first request).
"""
import time

import numpy as np
import torch

from . import mpc3, workloads
from .network import Network

MODEL_NAMES = ("mlp", "lenet", "vgg")


def m_bucket(M):
    """Rows rounded up to a power of two: the autotuner keeps one choice per bucket."""
    b = 1
    while b < M:
        b *= 2
    return b
DEFAULT_CAP = {"mlp": 512, "lenet": 256, "vgg": 64}


def request_mix(n=512, seed=5):
    """Seeded mix: batch sizes uniform in 1..64, model uniform over the three networks."""
    g = workloads.rng(seed)
    bs = g.integers(1, 65, size=n)
    ms = g.integers(0, 3, size=n)
    return [(i, MODEL_NAMES[m], int(b)) for i, (m, b) in enumerate(zip(ms, bs))]


def request_input(name, b, rid, device="cuda"):
    """Uniform [0, 1) images of the model's input shape, seeded per request."""
    shape = (b,) + tuple(workloads.MODELS[name]["input"])
    gen = torch.Generator(device=device)
    gen.manual_seed(1000 + rid)
    return torch.rand(shape, generator=gen, dtype=torch.float64, device=device)


def packs_of(reqs, cap, pack=True):
    """Group requests of one model into packs of at most cap images, in arrival order."""
    out = []
    for name in MODEL_NAMES:
        cur, n = [], 0
        for r in (r for r in reqs if r[1] == name):
            if cur and (not pack or n + r[2] > cap[name]):
                out.append(cur)
                cur, n = [], 0
            cur.append(r)
            n += r[2]
        if cur:
            out.append(cur)
    out.sort(key=lambda p: p[0][0])
    return out


class Server:
    def __init__(self, ctx, models=MODEL_NAMES, cap=None):
        self.ctx = ctx
        self.nets = {m: Network(ctx, m) for m in models}
        self.cap = dict(DEFAULT_CAP if cap is None else cap)

    def tune(self, reqs, reps=3, log=None):
        """Autotune the kernel family for every layer shape the packs will produce.  The
        library keeps one choice per (M rounded up to a power of two, K, N), so each such
        bucket is timed once, at its largest M."""
        shapes = set()
        for p in packs_of(reqs, self.cap):
            b = sum(r[2] for r in p)
            shapes.update((m_bucket(M), K, N) for M, K, N in self.nets[p[0][1]].exec_shapes(b))
        for i, (M, K, N) in enumerate(sorted(shapes)):
            self.ctx.autotune(M, K, N, reps)
            if log and (i + 1) % 16 == 0:
                log(f"tuned {i + 1}/{len(shapes)} shapes")
        return len(shapes)

    def run(self, reqs, pack=True, log=None):
        """Serve all requests; returns per-request latency (s), makespan (s) and images."""
        ctx = self.ctx
        inputs = {r[0]: request_input(r[1], r[2], r[0], ctx.device) for r in reqs}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat = {}
        ok_all = True
        packs = packs_of(reqs, self.cap, pack)
        for n_done, p in enumerate(packs):
            if log and n_done % 64 == 0:
                log(f"pack {n_done}/{len(packs)}")
            net = self.nets[p[0][1]]
            x = torch.cat([inputs[r[0]] for r in p]) if len(p) > 1 else inputs[p[0][0]]
            out = net.forward(x)
            ok_all &= ctx.verify()
            logits = ctx.reconstruct(out)          # synchronises: the pack's results are final
            t = time.perf_counter() - t0
            row = 0
            for r in p:
                lat[r[0]] = t
                row += r[2]
            del logits
        makespan = time.perf_counter() - t0
        images = sum(r[2] for r in reqs)
        return {"ok": ok_all, "latency": lat, "makespan": makespan, "images": images,
                "packs": len(packs)}


def summary(res):
    lat = np.array(sorted(res["latency"].values()))
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "inferences_per_s": res["images"] / res["makespan"], "makespan_s": res["makespan"],
            "images": res["images"], "packs": res["packs"], "verified": bool(res["ok"])}
