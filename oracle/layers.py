"""Convolution lowering (oracle; test infrastructure only).

Sec. 4.1 evaluates a convolution as one inner product per output.  A convolution of an
NHWC tensor with KH x KW x C kernels, zero padding p and stride s is the matrix product of
the rows (b, oh, ow) of the patch matrix, whose columns are (kh, kw, c), with the weights
reshaped to (KH*KW*C) x Cout; output (oh, ow) reads input (s oh + kh - p, s ow + kw - p).
Each share plane is rearranged alone, which is local and linear.
"""
import numpy as np


def im2col(x, kh, kw, pad, stride=1):
    """x: (B, H, W, C) uint64 plane -> (B*OH*OW, KH*KW*C), OH = (H + 2 pad - KH) // stride + 1."""
    B, H, W, C = x.shape
    xp = np.zeros((B, H + 2 * pad, W + 2 * pad, C), dtype=np.uint64)
    xp[:, pad:pad + H, pad:pad + W, :] = x
    OH, OW = (H + 2 * pad - kh) // stride + 1, (W + 2 * pad - kw) // stride + 1
    out = np.zeros((B, OH, OW, kh, kw, C), dtype=np.uint64)
    for i in range(kh):
        for j in range(kw):
            out[:, :, :, i, j, :] = xp[:, i:i + stride * (OH - 1) + 1:stride, j:j + stride * (OW - 1) + 1:stride, :]
    return out.reshape(B * OH * OW, kh * kw * C)


def im2col_share(s, kh, kw, pad, stride=1):
    from .protocol import Share
    return Share(*[im2col(p, kh, kw, pad, stride) for p in s.comps()])


def sumpool2(x):
    """2x2 sum pooling with stride 2 of a (B, H, W, C) uint64 plane (wraps mod 2^64)."""
    B, H, W, C = x.shape
    v = x.reshape(B, H // 2, 2, W // 2, 2, C)
    return v[:, :, 0, :, 0] + v[:, :, 0, :, 1] + v[:, :, 1, :, 0] + v[:, :, 1, :, 1]


def sumpool2_share(s, B, H, W, C):
    from .protocol import Share
    return Share(*[sumpool2(p.reshape(B, H, W, C)).reshape(B, -1) for p in s.comps()])
