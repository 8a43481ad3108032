"""GF(2^d) = Z_2[x] / f(x) (oracle; test infrastructure only).

Sec. 4.3 verifies the Boolean (Z_2) multiplications of the non-linear layers with the same
Pi_MultVerify as over Z_{2^l}, taken with l = 1: the Galois ring GR(2, d) is the field
GF(2^d).  f is the modulus of the Z_{2^64} verification ring reduced mod 2 (the paper does
not name it; it is irreducible over GF(2)); d = 64 in the protocol, smaller d only in
soundness tests.

An element is one uint64 word, bit k the coefficient of x^k (bits d and above are 0).
Addition is XOR.  A product is the carry-less product (schoolbook over the bits of one
factor) reduced modulo f from the top coefficient down.
"""
import numpy as np

from .gr import MODULI

U64 = np.uint64


def clmul(a, b):
    """Carry-less product of uint64 arrays: (lo, hi) words of the 127-bit result."""
    a = np.asarray(a, U64)
    b = np.asarray(b, U64)
    shape = np.broadcast_shapes(a.shape, b.shape)
    lo = np.zeros(shape, U64)
    hi = np.zeros(shape, U64)
    for k in range(64):
        sel = np.zeros(shape, U64) - ((b >> U64(k)) & U64(1))      # all ones where bit k of b is set
        lo ^= (a << U64(k)) & sel
        if k:
            hi ^= (a >> U64(64 - k)) & sel
    return lo, hi


class GF:
    def __init__(self, d=64):
        if d not in MODULI or d < 2:
            raise ValueError(f"unsupported degree {d}")
        self.d = d
        self.taps = MODULI[d]
        self.mask = U64((1 << d) - 1) if d < 64 else U64(0xFFFFFFFFFFFFFFFF)
        self.X = U64(2)
        self.ONE = U64(1)

    def reduce(self, lo, hi):
        """lo + 2^64 hi modulo f: for each coefficient k from 2d - 2 down to d, clear it and
        add x^(k - d) (f - x^d), i.e. x^(k - d + t) for every low term x^t of f."""
        lo = np.asarray(lo, U64).copy()
        hi = np.asarray(hi, U64).copy()
        d = self.d

        def bit(k):
            return ((hi >> U64(k - 64)) if k >= 64 else (lo >> U64(k))) & U64(1)

        def flip(k, sel):
            if k >= 64:
                hi[...] ^= sel << U64(k - 64)
            else:
                lo[...] ^= sel << U64(k)

        for k in range(2 * d - 2, d - 1, -1):
            sel = bit(k)
            flip(k, sel)
            for t in self.taps:
                flip(k - d + t, sel)
        return lo

    def mul(self, a, b):
        return self.reduce(*clmul(a, b))

    def dot(self, a, b, axis=0):
        """XOR-sum of elementwise products along an axis."""
        return np.bitwise_xor.reduce(self.mul(a, b), axis=axis)

    def pow(self, a, e):
        out = np.ones_like(np.asarray(a, U64))
        base = np.asarray(a, U64)
        while e:
            if e & 1:
                out = self.mul(out, base)
            base = self.mul(base, base)
            e >>= 1
        return out

    def powers(self, a, n):
        """[a^0, ..., a^(n-1)] of one element: with the first L powers known, the next L are
        their products with a^L (L = 1, 2, 4, ...)."""
        out = np.ones(1, U64)
        step = np.asarray(a, U64)             # a^L
        while out.size < n:
            out = np.concatenate([out, self.mul(out, step)])
            step = self.mul(step, step)
        return out[:n]

    def inv(self, a):
        """a^(2^d - 2), the inverse in the multiplicative group of order 2^d - 1."""
        if not np.all(np.asarray(a, U64)):
            raise ZeroDivisionError("0 has no inverse")
        return self.pow(a, (1 << self.d) - 2)
