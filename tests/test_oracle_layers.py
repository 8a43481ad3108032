"""Pins of the oracle's convolution lowering and sum pooling against their definitions,
written out with Python integers (Sec. 4.1 evaluates a convolution as one inner product
per output; pooling sums are local linear maps of the shares).

A convolution of an NHWC input with KH x KW x C x Cout weights, stride 1 and zero
padding p is, by definition,
    out[b, oh, ow, co] = sum_{kh, kw, c} x[b, oh + kh - p, ow + kw - p, c] W[kh, kw, c, co]
with x read as 0 outside the image.  The lowering must give the same numbers as the
product of its patch matrix with the weights reshaped to (KH KW C) x Cout, so an error in
the (kh, kw, c) column order, the padding offset or the output-row order fails here."""
import numpy as np
import pytest

from oracle.layers import im2col, sumpool2

MASK = (1 << 64) - 1


def direct_conv(x, w, pad, stride=1):
    B, H, W, C = x.shape
    KH, KW, _, CO = w.shape
    OH, OW = (H + 2 * pad - KH) // stride + 1, (W + 2 * pad - KW) // stride + 1
    out = np.zeros((B, OH, OW, CO), dtype=np.uint64)
    for b in range(B):
        for oh in range(OH):
            for ow in range(OW):
                for co in range(CO):
                    acc = 0
                    for kh in range(KH):
                        for kw in range(KW):
                            ih, iw = stride * oh + kh - pad, stride * ow + kw - pad
                            if not (0 <= ih < H and 0 <= iw < W):
                                continue
                            for c in range(C):
                                acc += int(x[b, ih, iw, c]) * int(w[kh, kw, c, co])
                    out[b, oh, ow, co] = acc & MASK
    return out


@pytest.mark.parametrize("B,H,W,C,KH,KW,CO,pad", [
    (1, 5, 5, 1, 3, 3, 2, 0),
    (2, 5, 7, 3, 3, 3, 2, 1),      # odd, non-square image, C > 1, "same" padding
    (1, 6, 5, 2, 2, 3, 3, 0),      # KH != KW: a swapped (kh, kw) order fails
    (1, 4, 4, 2, 3, 2, 1, 1),
    (2, 7, 6, 3, 5, 5, 2, 2),
])
def test_im2col_product_is_the_direct_convolution(B, H, W, C, KH, KW, CO, pad):
    g = np.random.default_rng(B * 1000 + H * 100 + W * 10 + C + KH + pad)
    x = g.integers(0, 1 << 64, size=(B, H, W, C), dtype=np.uint64, endpoint=False)
    w = g.integers(0, 1 << 64, size=(KH, KW, C, CO), dtype=np.uint64, endpoint=False)
    cols = im2col(x, KH, KW, pad)
    OH, OW = H + 2 * pad - KH + 1, W + 2 * pad - KW + 1
    assert cols.shape == (B * OH * OW, KH * KW * C)
    got = (cols @ w.reshape(KH * KW * C, CO)).reshape(B, OH, OW, CO)
    assert np.array_equal(got, direct_conv(x, w, pad))


@pytest.mark.parametrize("B,H,W,C,KH,KW,CO,pad,stride", [
    (1, 28, 28, 1, 5, 5, 2, 1, 2),     # the S-NN layer's geometry: 13 x 13 outputs
    (2, 7, 6, 3, 3, 3, 2, 1, 2),
    (1, 9, 8, 2, 3, 2, 1, 0, 3),
])
def test_strided_im2col_product_is_the_direct_convolution(B, H, W, C, KH, KW, CO, pad, stride):
    g = np.random.default_rng(H * 10 + stride)
    x = g.integers(0, 1 << 64, size=(B, H, W, C), dtype=np.uint64, endpoint=False)
    w = g.integers(0, 1 << 64, size=(KH, KW, C, CO), dtype=np.uint64, endpoint=False)
    cols = im2col(x, KH, KW, pad, stride)
    OH, OW = (H + 2 * pad - KH) // stride + 1, (W + 2 * pad - KW) // stride + 1
    assert cols.shape == (B * OH * OW, KH * KW * C)
    got = (cols @ w.reshape(KH * KW * C, CO)).reshape(B, OH, OW, CO)
    assert np.array_equal(got, direct_conv(x, w, pad, stride))


def test_im2col_entries_by_index():
    # entry (row (b, oh, ow), column (kh, kw, c)) is x[b, oh + kh - p, ow + kw - p, c] or 0
    B, H, W, C, KH, KW, pad = 2, 4, 3, 2, 3, 2, 1
    x = np.arange(1, B * H * W * C + 1, dtype=np.uint64).reshape(B, H, W, C)
    cols = im2col(x, KH, KW, pad)
    OH, OW = H + 2 * pad - KH + 1, W + 2 * pad - KW + 1
    for b in range(B):
        for oh in range(OH):
            for ow in range(OW):
                row = (b * OH + oh) * OW + ow
                for kh in range(KH):
                    for kw in range(KW):
                        for c in range(C):
                            ih, iw = oh + kh - pad, ow + kw - pad
                            want = x[b, ih, iw, c] if 0 <= ih < H and 0 <= iw < W else 0
                            assert cols[row, (kh * KW + kw) * C + c] == want


@pytest.mark.parametrize("B,H,W,C", [(1, 2, 2, 1), (2, 4, 6, 3), (1, 8, 4, 5)])
def test_sumpool2_is_the_direct_window_sum(B, H, W, C):
    g = np.random.default_rng(H * W * C)
    x = g.integers(0, 1 << 64, size=(B, H, W, C), dtype=np.uint64, endpoint=False)
    got = sumpool2(x)
    assert got.shape == (B, H // 2, W // 2, C)
    for b in range(B):
        for i in range(H // 2):
            for j in range(W // 2):
                for c in range(C):
                    s = sum(int(x[b, 2 * i + di, 2 * j + dj, c]) for di in (0, 1) for dj in (0, 1))
                    assert int(got[b, i, j, c]) == s & MASK
