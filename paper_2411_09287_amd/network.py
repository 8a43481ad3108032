"""Secure evaluation of a chained network through the C ABI.

The layers of the MLP, LeNet-shaped and VGG-shaped networks are chained: convolution
(im2col) or dense product with Pi_Inner, Pi_Trunc by the fixed-point precision, then

  * nonlinear=True: ReLU after every layer but the last and 2x2 max pooling between
    stages (Sec. 4.3: edaBits, bit extraction, B2A, Pi_Mult);
  * nonlinear=False (the linear path alone): no activation, and 2x2 average pooling as a
    sum pool of the shares (a local linear map) with the factor 1/4 folded into the next
    layer's plaintext weights before encoding.

Weights are encoded and shared once; every call of `forward` shares a new input batch,
evaluates the layers and leaves the products pending for `verify`.
"""
import numpy as np
import torch

from . import mpc3, workloads


def plan(name):
    """Layers of a model with the pooling that links them: list of dicts."""
    spec = workloads.MODELS[name]
    layers = spec["layers"]
    out = []
    for i, layer in enumerate(layers):
        d = {"layer": layer, "pool_after": False}
        if layer[0] == "conv":
            _, kh, kw, cin, cout, pad, (h, w) = layer[:7]
            oh, ow = workloads.conv_out_hw(layer)
            d["out_hw"] = (oh, ow)
            # contraction width of the product: kh kw cin zero-padded to whole 32-deep
            # k-blocks of the matrix-core kernel (zero columns of the lowered input against
            # zero rows of the weights leave every output unchanged)
            d["kpad"] = -(-kh * kw * cin // 32) * 32
            if i + 1 < len(layers):
                nxt = layers[i + 1]
                if nxt[0] == "conv":
                    d["pool_after"] = tuple(nxt[6]) == (oh // 2, ow // 2) and (oh, ow) != tuple(nxt[6])
                else:
                    d["pool_after"] = nxt[1] == (oh // 2) * (ow // 2) * cout
        out.append(d)
    return out


def float_weights(name, seed=200, nonlinear=False):
    """Plaintext weights (K x N); on the linear path 1/4 is folded in after every average pool."""
    ws = []
    pooled = False
    for i, d in enumerate(plan(name)):
        layer = d["layer"]
        M, K, N = workloads.layer_gemm_shape(layer, 1)
        w = workloads.layer_weight(layer, seed + i).reshape(K, N)
        if pooled and not nonlinear:
            w = w / 4.0
        ws.append(w)
        pooled = d["pool_after"]
    return ws


class Network:
    """Shared weights of one model on one context."""

    def __init__(self, ctx, name, seed=200, nonlinear=False):
        self.ctx = ctx
        self.name = name
        self.nonlinear = nonlinear
        self.plan = plan(name)
        self.frac = ctx.frac_bits
        self.w_float = float_weights(name, seed, nonlinear)
        self.weights = []
        with torch.cuda.stream(ctx.stream):
            for d, w in zip(self.plan, self.w_float):
                if d.get("kpad", w.shape[0]) > w.shape[0]:
                    w = np.concatenate([w, np.zeros((d["kpad"] - w.shape[0], w.shape[1]))])
                self.weights.append(ctx.share(ctx.encode(torch.from_numpy(w).to(ctx.device))))

    def shapes(self, batch):
        """The layers' products M x K x N as the model defines them."""
        return [workloads.layer_gemm_shape(d["layer"], batch) for d in self.plan]

    def exec_shapes(self, batch):
        """The products as evaluated (convolutions with the padded contraction width)."""
        return [(M, self.plan[i].get("kpad", K), N) for i, (M, K, N) in enumerate(self.shapes(batch))]

    def forward(self, x, trunc=True):
        """x: float64 tensor (batch, ...) of the model's input shape on the device, ready on
        the current stream.  Returns the shared logits (batch x classes); products stay
        pending."""
        st = self.ctx.stream
        cur = torch.cuda.current_stream(x.device)
        if cur == st:
            return self._forward(x, trunc)
        st.wait_stream(cur)
        x.record_stream(st)
        with torch.cuda.stream(st):
            return self._forward(x, trunc)

    def _forward(self, x, trunc):
        ctx = self.ctx
        batch = x.shape[0]
        h = ctx.share(ctx.encode(x).reshape(batch, -1))
        for i, d in enumerate(self.plan):
            layer = d["layer"]
            Wt = self.weights[i]
            if layer[0] == "conv":
                # the lowering and the product in one call, verified from the layer's input
                _, kh, kw, cin, cout, pad, (hh, ww) = layer[:7]
                oh, ow = workloads.conv_out_hw(layer)
                M = batch * oh * ow

                def product(pair, layer=layer, kh=kh, kw=kw, cin=cin, pad=pad, hh=hh, ww=ww, h=h, d=d, Wt=Wt):
                    return ctx.inner_conv(h, batch, hh, ww, cin, kh, kw, pad, Wt, pair, ld=d["kpad"],
                                          stride=workloads.conv_stride(layer))
            else:
                X = h if h.cols == layer[1] else mpc3.DShare(*[t.reshape(batch, -1) for t in (h.m, h.r1, h.r2)])
                M = X.rows

                def product(pair, X=X, Wt=Wt):
                    return ctx.inner(X, Wt, pair)
            if trunc:
                pair = ctx.trunc_pair(M * Wt.cols, self.frac)
                Y = ctx.trunc(pair, product(pair))
            else:
                Y = product(None)
            if self.nonlinear and i + 1 < len(self.plan):
                Y = ctx.relu(Y)
            if d["pool_after"]:
                oh, ow = d["out_hw"]
                pool = ctx.maxpool2 if self.nonlinear else ctx.sumpool2
                Y = pool(mpc3.DShare(*[t.reshape(batch, -1) for t in (Y.m, Y.r1, Y.r2)]), batch, oh, ow, layer[4])
            h = Y if layer[0] == "fc" else mpc3.DShare(*[t.reshape(batch, -1) for t in (Y.m, Y.r1, Y.r2)])
        return h


class RecordedForward:
    """The linear forward of `net` (nonlinear=False) at one batch size, recorded once into a
    HIP graph and replayed per call.

    The calls are those of `Network.forward` in the same order (encode, share, then per
    layer im2col, truncation pair, Pi_Inner with the library's fixed workspace, Pi_Trunc and
    the sum pool), on buffers allocated here before recording; a replay therefore draws the
    same masks and registers the same products as those calls made directly at that point
    of the context's history, and each replay's masks are fresh.  The context must run on a
    stream of its own (not the null stream).  `__call__` copies the images into the recorded
    input buffer on the context's stream and launches the graph; the returned logits share
    is the recorded output buffer, overwritten by the next replay, which the library refuses
    until the products of this one are verified."""

    def __init__(self, net, batch):
        if net.nonlinear:
            raise ValueError("only the linear layers can be recorded (the non-linear ones allocate)")
        ctx = net.ctx
        self.net, self.batch, self.ctx = net, batch, ctx
        dev = ctx.device
        shape = (batch,) + tuple(workloads.MODELS[net.name]["input"])
        with torch.cuda.stream(ctx.stream):
            self._alloc(shape, dev)
        torch.cuda.synchronize(dev)
        ctx.capture_begin()
        try:
            with torch.cuda.stream(ctx.stream):
                self.out = self._calls()
        except Exception:
            try:
                ctx.capture_end()
            except mpc3.Mpc3Error:
                pass
            raise
        self.graph = ctx.capture_end()

    def _alloc(self, shape, dev):
        net, batch = self.net, self.batch
        self.x = torch.zeros(shape, dtype=torch.float64, device=dev)
        self.enc = torch.empty(shape, dtype=torch.int64, device=dev)
        self.h0 = mpc3.DShare.empty(batch, int(np.prod(shape[1:])), dev)
        self.layers = []
        for i, d in enumerate(net.plan):
            layer = d["layer"]
            M, K, N = net.exec_shapes(batch)[i]
            b = {"pair": mpc3.DPair(M * N, dev), "Z": mpc3.DShare.empty(M, N, dev),
                 "Y": mpc3.DShare.empty(M, N, dev)}
            if layer[0] == "conv":
                b["cols"] = mpc3.DShare.empty(M, K, dev)
            if d["pool_after"]:
                oh, ow = d["out_hw"]
                b["pool"] = mpc3.DShare.empty(batch, (oh // 2) * (ow // 2) * layer[4], dev)
            self.layers.append(b)

    def _calls(self):
        ctx, net, batch = self.ctx, self.net, self.batch
        h = ctx.share(ctx.encode(self.x, out=self.enc).reshape(batch, -1), out=self.h0)
        for i, (d, b) in enumerate(zip(net.plan, self.layers)):
            layer = d["layer"]
            if layer[0] == "conv":
                _, kh, kw, cin, cout, pad, (hh, ww) = layer[:7]
                X = ctx.im2col(h, batch, hh, ww, cin, kh, kw, pad, d["kpad"], stride=workloads.conv_stride(layer),
                               out=b["cols"])
            else:
                X = h if h.cols == layer[1] else mpc3.DShare(*[t.reshape(batch, -1) for t in (h.m, h.r1, h.r2)])
            M, N = X.rows, net.weights[i].cols
            pair = ctx.trunc_pair(M * N, net.frac, out=b["pair"])
            Z = ctx.inner_static(X, net.weights[i], pair, out=b["Z"])
            Y = ctx.trunc(pair, Z, out=b["Y"])
            if d["pool_after"]:
                oh, ow = d["out_hw"]
                Y = ctx.sumpool2(mpc3.DShare(*[t.reshape(batch, -1) for t in (Y.m, Y.r1, Y.r2)]), batch, oh, ow,
                                 layer[4], out=b["pool"])
            h = Y if layer[0] == "fc" else mpc3.DShare(*[t.reshape(batch, -1) for t in (Y.m, Y.r1, Y.r2)])
        return h

    def nodes(self):
        """(kernel nodes, other nodes) of the recorded graph."""
        return self.ctx.graph_nodes(self.graph)

    def __call__(self, x):
        """x: float64 images (at most `batch`, the rest of the recorded batch is zero)."""
        ctx = self.ctx
        n = x.shape[0]
        if n > self.batch:
            raise ValueError(f"{n} images for a graph recorded at batch {self.batch}")
        st = ctx.stream
        st.wait_stream(torch.cuda.current_stream(x.device))
        with torch.cuda.stream(st):
            self.x[:n].copy_(x)
            if n < self.batch:
                self.x[n:].zero_()
        x.record_stream(st)
        ctx.graph_launch(self.graph)
        return self.out

    def close(self):
        if self.graph:
            self.ctx.graph_destroy(self.graph)
            self.graph = 0
