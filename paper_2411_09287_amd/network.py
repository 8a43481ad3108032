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
        """x: float64 tensor (batch, ...) of the model's input shape on the device.
        Returns the shared logits (batch x classes); products stay pending."""
        ctx = self.ctx
        batch = x.shape[0]
        h = ctx.share(ctx.encode(x).reshape(batch, -1))
        for i, d in enumerate(self.plan):
            layer = d["layer"]
            if layer[0] == "conv":
                _, kh, kw, cin, cout, pad, (hh, ww) = layer[:7]
                X = ctx.im2col(h, batch, hh, ww, cin, kh, kw, pad, d["kpad"], stride=workloads.conv_stride(layer))
            else:
                X = h if h.cols == layer[1] else mpc3.DShare(*[t.reshape(batch, -1) for t in (h.m, h.r1, h.r2)])
            M, N = X.rows, self.weights[i].cols
            if trunc:
                pair = ctx.trunc_pair(M * N, self.frac)
                Z = ctx.inner(X, self.weights[i], pair)
                Y = ctx.trunc(pair, Z)
            else:
                Y = ctx.inner(X, self.weights[i])
            if self.nonlinear and i + 1 < len(self.plan):
                Y = ctx.relu(Y)
            if d["pool_after"]:
                oh, ow = d["out_hw"]
                pool = ctx.maxpool2 if self.nonlinear else ctx.sumpool2
                Y = pool(mpc3.DShare(*[t.reshape(batch, -1) for t in (Y.m, Y.r1, Y.r2)]), batch, oh, ow, layer[4])
            h = Y if layer[0] == "fc" else mpc3.DShare(*[t.reshape(batch, -1) for t in (Y.m, Y.r1, Y.r2)])
        return h
