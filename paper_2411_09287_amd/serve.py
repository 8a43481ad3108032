"""Batched serving of mixed secure-inference requests on one GPU.

Requests (model, batch size) are packed per model, in arrival order, into row-blocks of at
most `cap[model]` images.  A pack runs as one secure evaluation: every layer is one
Pi_Inner over the packed rows (rows are images x output positions, so requests simply
stack) with one truncation pair, and one verification covers the whole pack; the opened
logits are split back per request.  Packing amortises the verification (whose cost does
not grow with the number of rows beyond the compression products) and the per-launch
costs over many requests.  With graphs, a pack is padded to its batch bucket (a power of
two) and its layers replay a HIP graph recorded once per (model, bucket), which removes
the per-call host work of the linear forward.

Requests either all arrive at time 0 (packs in the order of their first request) or
arrive open-loop at given times (the oldest waiting request's model is served next).
"""
import time

import numpy as np
import torch

from . import mpc3, workloads
from .network import Network, RecordedForward

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


def bucket_of(b, cap):
    """The batch bucket of a pack of b images: b rounded up to a power of two, at most cap."""
    return min(m_bucket(b), max(cap, b))


def poisson_arrivals(reqs, rate, seed=7):
    """Open-loop arrivals: exponential gaps of mean 1/rate seconds, in request order."""
    g = workloads.rng(seed)
    t = np.cumsum(g.exponential(1.0 / rate, size=len(reqs)))
    return {r[0]: float(ti) for r, ti in zip(reqs, t)}


class Server:
    """graphs=True: every pack runs at its batch bucket (power of two, zero images padding
    it) from a HIP graph recorded on first use per (model, bucket) (network.RecordedForward;
    buckets whose layers exceed the library's fixed workspace run by direct calls).
    graphs="auto": the same for the (model, bucket) pairs where tune_graphs measured the
    replay faster than direct calls (the direct calls can use kernels a recording cannot,
    such as the implicit lowering of convolutions); the other packs run unpadded by direct
    calls.  buckets=True without graphs pads every pack the same way but makes the calls
    directly, buckets="picked" pads only the packs whose bucket has a graph picked: both draw
    the masks of the graph servers.  The context of a graph server needs a stream of its own."""

    def __init__(self, ctx, models=MODEL_NAMES, cap=None, graphs=False, buckets=None):
        self.ctx = ctx
        self.nets = {m: Network(ctx, m) for m in models}
        self.cap = dict(DEFAULT_CAP if cap is None else cap)
        self.graphs = graphs
        if buckets is None:
            buckets = "picked" if graphs == "auto" else bool(graphs)
        self.buckets = buckets
        self.recorded = {}
        self.graph_pick = {}

    def tune(self, reqs, reps=3, log=None):
        """Autotune the kernel family for every layer shape the packs will produce, and the
        limb kernel's launch shape where that family wins on a product large enough for it.
        The library keeps one choice per (M rounded up to a power of two, K, N), so each such
        bucket is timed once, at its largest M."""
        shapes = set()
        for p in packs_of(reqs, self.cap):
            b = sum(r[2] for r in p)
            # the pack's own size, and its bucket where packs may be padded
            for bb in {b, bucket_of(b, self.cap[p[0][1]]) if self.buckets else b}:
                shapes.update((m_bucket(M), K, N) for M, K, N in self.nets[p[0][1]].exec_shapes(bb))
        for i, (M, K, N) in enumerate(sorted(shapes)):
            choice, _, _ = self.ctx.autotune(M, K, N, reps)
            if choice == mpc3.VARIANT_LIMB_I8 and M * K * N >= (1 << 22):
                self.ctx.autotune_launch(M, K, N, reps)
            if log and (i + 1) % 16 == 0:
                log(f"tuned {i + 1}/{len(shapes)} shapes")
        return len(shapes)

    def tune_graphs(self, reps=3, log=None):
        """graphs="auto": for every model and batch bucket up to its cap, time a direct
        forward against the replay of the recorded graph (median of reps, each verified
        before the next, synchronised wall time) and keep the faster.  Returns the picks."""
        ctx = self.ctx
        for name, net in self.nets.items():
            bk = 1
            while bk <= self.cap[name]:
                rf = self._graph(name, bk)
                if rf is None:
                    self.graph_pick[(name, bk)] = False
                else:
                    x = request_input(name, bk, 0, ctx.device)
                    tt = {"direct": [], "graph": []}
                    for _ in range(reps):
                        for kind in tt:
                            torch.cuda.synchronize()
                            t0 = time.perf_counter()
                            h = net.forward(x) if kind == "direct" else rf(x)
                            torch.cuda.synchronize()
                            tt[kind].append(time.perf_counter() - t0)
                            if not ctx.verify():
                                raise RuntimeError("verification failed in an honest run")
                            del h
                    self.graph_pick[(name, bk)] = float(np.median(tt["graph"])) < float(np.median(tt["direct"]))
                if log:
                    log(f"graph pick {name} bucket {bk}: {self.graph_pick[(name, bk)]}")
                bk *= 2
        return dict(self.graph_pick)

    def _graph(self, name, bk):
        key = (name, bk)
        if key not in self.recorded:
            try:
                self.recorded[key] = RecordedForward(self.nets[name], bk)
            except mpc3.Mpc3Error as e:
                if e.code != mpc3.E_LIMIT:
                    raise
                self.recorded[key] = None
        return self.recorded[key]

    def forward(self, name, x):
        """Shared logits of the images x (rows beyond x.shape[0] belong to padding) and
        whether a recorded graph produced them."""
        net = self.nets[name]
        b = x.shape[0]
        bk = bucket_of(b, self.cap[name])
        pick = self.graph_pick.get((name, bk), False)
        if not (self.buckets is True or (self.buckets == "picked" and pick)):
            return net.forward(x), False
        use = self.graphs is True or (self.graphs == "auto" and pick)
        rf = self._graph(name, bk) if use else None
        if rf is not None:
            return rf(x), True
        if bk > b:
            x = torch.cat([x, torch.zeros((bk - b,) + tuple(x.shape[1:]), dtype=x.dtype, device=x.device)])
        return net.forward(x), False

    def _run_pack(self, p, inputs, keep_logits, out):
        ctx = self.ctx
        x = torch.cat([inputs[r[0]] for r in p]) if len(p) > 1 else inputs[p[0][0]]
        h, from_graph = self.forward(p[0][1], x)
        out["graph_packs"] += int(from_graph)
        out["ok"] &= ctx.verify()
        logits = ctx.reconstruct(h)            # synchronises: the pack's results are final
        if keep_logits:
            row = 0
            for r in p:
                out["logits"][r[0]] = ctx.decode(logits[row:row + r[2]].contiguous())
                row += r[2]

    def run(self, reqs, pack=True, log=None, arrivals=None, keep_logits=False):
        """Serve all requests; returns per-request latency (s), makespan (s) and images.

        arrivals=None: every request is there at time 0 and the packs run in the order of
        their first request (packs_of).  arrivals={request id: seconds}: an open-loop run
        on a virtual clock advanced by the measured service time of each pack: when the
        GPU is free, the model of the oldest waiting request is served with its waiting
        requests of that model (arrival order, at most cap images); latency is completion
        minus arrival."""
        ctx = self.ctx
        inputs = {r[0]: request_input(r[1], r[2], r[0], ctx.device) for r in reqs}
        torch.cuda.synchronize()
        out = {"ok": True, "graph_packs": 0, "logits": {}}
        lat = {}
        if arrivals is None:
            t0 = time.perf_counter()
            packs = packs_of(reqs, self.cap, pack)
            for n_done, p in enumerate(packs):
                if log and n_done % 64 == 0:
                    log(f"pack {n_done}/{len(packs)}")
                self._run_pack(p, inputs, keep_logits, out)
                t = time.perf_counter() - t0
                for r in p:
                    lat[r[0]] = t
            makespan = time.perf_counter() - t0
            npacks = len(packs)
        else:
            waiting = sorted(reqs, key=lambda r: (arrivals[r[0]], r[0]))
            clock, npacks, i = 0.0, 0, 0
            queue = []
            while i < len(waiting) or queue:
                while i < len(waiting) and arrivals[waiting[i][0]] <= clock:
                    queue.append(waiting[i])
                    i += 1
                if not queue:
                    clock = arrivals[waiting[i][0]]
                    continue
                name = queue[0][1]
                p, n = [], 0
                for r in queue:
                    if r[1] != name:
                        continue
                    if p and (not pack or n + r[2] > self.cap[name]):
                        break
                    p.append(r)
                    n += r[2]
                queue = [r for r in queue if r not in p]
                t0 = time.perf_counter()
                self._run_pack(p, inputs, keep_logits, out)
                clock += time.perf_counter() - t0
                for r in p:
                    lat[r[0]] = clock - arrivals[r[0]]
                npacks += 1
                if log and npacks % 64 == 0:
                    log(f"pack {npacks}, {i}/{len(waiting)} arrived")
            makespan = clock - min(arrivals.values())
        images = sum(r[2] for r in reqs)
        res = {"ok": out["ok"], "latency": lat, "makespan": makespan, "images": images, "packs": npacks,
               "graph_packs": out["graph_packs"]}
        if keep_logits:
            res["logits"] = out["logits"]
        return res


def summary(res):
    lat = np.array(sorted(res["latency"].values()))
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "inferences_per_s": res["images"] / res["makespan"], "makespan_s": res["makespan"],
            "images": res["images"], "packs": res["packs"], "graph_packs": res.get("graph_packs", 0),
            "verified": bool(res["ok"])}
