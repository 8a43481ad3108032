"""Seeded synthetic workloads: layer shapes and float64 inputs.

This module holds no arithmetic of the protocol (no encoding, sharing or ring
operations).  It only draws the plaintext floats that both the HIP path and
the CPU oracle start from, so that the two can be compared on identical data.

Data come from numpy's PCG64 with data seed 1 + cfg; the MPC master seed of a
configuration is SHA-256("mpc3-cfg" || cfg).  Image workloads are MNIST- and
CIFAR-shaped stand-ins (uniform [0, 1) pixels); weights are N(0, 0.05^2) at
random initialisation.  No dataset is read.
"""
import hashlib

import numpy as np

FRAC_BITS = 13


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def master_seed(cfg):
    return hashlib.sha256(b"mpc3-cfg" + str(cfg).encode()).digest()


# Conv layers are (kh, kw, cin, cout, pad); "valid" = 0, "same" 3x3 = 1, stride 1.
# Pooling (2x2, stride 2) between stages is a non-linear layer and not part of the
# linear path; each linear layer gets its own synthetic input of its input shape.
MODELS = {
    "matmul": {"batch": 64, "input": (128,), "layers": [("fc", 128, 64)]},
    "mlp": {"batch": 128, "input": (784,),
            "layers": [("fc", 784, 128), ("fc", 128, 128), ("fc", 128, 10)]},
    "lenet": {"batch": 64, "input": (28, 28, 1),
              "layers": [("conv", 5, 5, 1, 20, 0, (28, 28)), ("conv", 5, 5, 20, 50, 0, (12, 12)),
                         ("fc", 800, 500), ("fc", 500, 10)]},
    "vgg": {"batch": 32, "input": (32, 32, 3),
            "layers": [("conv", 3, 3, 3, 64, 1, (32, 32)), ("conv", 3, 3, 64, 64, 1, (32, 32)),
                       ("conv", 3, 3, 64, 128, 1, (16, 16)), ("conv", 3, 3, 128, 128, 1, (16, 16)),
                       ("conv", 3, 3, 128, 256, 1, (8, 8)), ("conv", 3, 3, 256, 256, 1, (8, 8)),
                       ("fc", 4096, 256), ("fc", 256, 10)]},
    "snn": {"batch": 30, "input": (28, 28, 1),
            "layers": [("conv", 5, 5, 1, 5, 1, (28, 28), 2), ("fc", 845, 10)]},
    "lenet5": {"batch": 30, "input": (32, 32, 1),
               "layers": [("conv", 5, 5, 1, 6, 0, (32, 32)), ("conv", 5, 5, 6, 16, 0, (14, 14)),
                          ("fc", 400, 120), ("fc", 120, 84), ("fc", 84, 10)]},
    "vgg16": {"batch": 30, "input": (64, 64, 3),
              "layers": [("conv", 3, 3, 3, 64, 1, (64, 64)), ("conv", 3, 3, 64, 64, 1, (64, 64)),
                         ("conv", 3, 3, 64, 128, 1, (32, 32)), ("conv", 3, 3, 128, 128, 1, (32, 32)),
                         ("conv", 3, 3, 128, 256, 1, (16, 16)), ("conv", 3, 3, 256, 256, 1, (16, 16)),
                         ("conv", 3, 3, 256, 256, 1, (16, 16)),
                         ("conv", 3, 3, 256, 512, 1, (8, 8)), ("conv", 3, 3, 512, 512, 1, (8, 8)),
                         ("conv", 3, 3, 512, 512, 1, (8, 8)),
                         ("conv", 3, 3, 512, 512, 1, (4, 4)), ("conv", 3, 3, 512, 512, 1, (4, 4)),
                         ("conv", 3, 3, 512, 512, 1, (4, 4)),
                         ("fc", 2048, 512), ("fc", 512, 512), ("fc", 512, 200)]},
}

CONFIG_MODEL = {1: "matmul", 2: "mlp", 3: "lenet", 4: "vgg"}


def layer_gemm_shape(layer, batch):
    """(M, K, N) of the layer's matrix product (conv via im2col: rows b,oh,ow; cols kh,kw,cin)."""
    if layer[0] == "fc":
        return batch, layer[1], layer[2]
    oh, ow = conv_out_hw(layer)
    _, kh, kw, cin, cout = layer[:5]
    return batch * oh * ow, kh * kw * cin, cout


def conv_stride(layer):
    return layer[7] if len(layer) > 7 else 1


def conv_out_hw(layer):
    """Output image size of a convolution layer."""
    _, kh, kw, cin, cout, pad, (h, w) = layer[:7]
    s = conv_stride(layer)
    return (h + 2 * pad - kh) // s + 1, (w + 2 * pad - kw) // s + 1


def model_shapes(name, batch=None):
    spec = MODELS[name]
    b = spec["batch"] if batch is None else batch
    return [layer_gemm_shape(l, b) for l in spec["layers"]]


def layer_input(layer, batch, seed, dist="uniform"):
    """Synthetic activation for one layer: (batch, K) for fc, (batch, h, w, cin) for conv."""
    g = rng(seed)
    shape = (batch, layer[1]) if layer[0] == "fc" else (batch,) + tuple(layer[6]) + (layer[3],)
    if dist == "normal":
        return g.standard_normal(shape)
    return g.random(shape)


def layer_weight(layer, seed, std=0.05):
    g = rng(seed)
    shape = (layer[1], layer[2]) if layer[0] == "fc" else (layer[1], layer[2], layer[3], layer[4])
    return g.standard_normal(shape) * std


def matmul_inputs(seed, M=64, K=128, N=64):
    """The plain secure-matmul workload: X, W ~ N(0, 1)."""
    g = rng(seed)
    return g.standard_normal((M, K)), g.standard_normal((K, N))


def uniform_u64(seed, n):
    """Uniform 64-bit words for ring-level tests (returned as uint64)."""
    return rng(seed).integers(0, 1 << 64, size=n, dtype=np.uint64, endpoint=False)
