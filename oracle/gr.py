"""Galois ring GR(2^64, d) = Z_{2^64}[x] / f(x) (oracle; test infrastructure only).

Sec. 3 ("Ring-Specific Challenges") moves verification into Z_{2^l}[x]/f(x)
with f of degree d irreducible over Z_2; the constants 0, 1, 2 used by
Pi_Reduce are the ring elements whose free coefficient is 0, 1, 2.  The paper
does not give f.  Reading: f(x) = x^d + sum_{i in taps} x^i with the
trinomials/pentanomials below (irreducible over GF(2)), taken monic over
Z_{2^64}.  d = 64 is the paper's setting (Sec. 5, "Benchmark setting").

An element is a uint64 vector of d coefficients, coefficient of x^0 first.
Products are the schoolbook polynomial product followed by reduction with
x^d = -sum_{i in taps} x^i.
"""
import numpy as np

U64 = np.uint64

# Low-order terms of the monic modulus f(x) = x^d + sum x^i.
MODULI = {
    1: (0,),            # x + 1      (d = 1 is plain Z_{2^64}: only constants)
    2: (1, 0),          # x^2 + x + 1
    4: (1, 0),          # x^4 + x + 1
    8: (4, 3, 1, 0),    # x^8 + x^4 + x^3 + x + 1
    16: (5, 3, 1, 0),   # x^16 + x^5 + x^3 + x + 1
    32: (7, 3, 2, 0),   # x^32 + x^7 + x^3 + x^2 + 1
    64: (4, 3, 1, 0),   # x^64 + x^4 + x^3 + x + 1
}


class GR:
    def __init__(self, d=64):
        if d not in MODULI:
            raise ValueError(f"unsupported extension degree {d}")
        self.d = d
        self.taps = MODULI[d]

    # -- constructors ---------------------------------------------------
    def zeros(self, *shape):
        return np.zeros(shape + (self.d,), dtype=U64)

    def const(self, c, *shape):
        """Constant-term embedding of a Z_{2^64} value (or array of values)."""
        c = np.asarray(c, dtype=U64)
        out = np.zeros(c.shape + (self.d,), dtype=U64)
        out[..., 0] = c
        return out

    def lift(self, v):
        """Pi_Tran: a Z_{2^64} share becomes the free coefficient; the other coefficients are 0."""
        return self.const(v)

    # -- arithmetic -----------------------------------------------------
    def add(self, a, b):
        return np.asarray(a, U64) + np.asarray(b, U64)

    def sub(self, a, b):
        return np.asarray(a, U64) - np.asarray(b, U64)

    def neg(self, a):
        return np.zeros_like(a) - a

    def scale(self, s, a):
        """Z_{2^64} scalar (array broadcast over the leading axes) times a ring element."""
        return np.asarray(s, U64)[..., None] * np.asarray(a, U64)

    def reduce(self, full):
        """Reduce a product of length 2d-1 modulo f, top coefficient first."""
        d = self.d
        full = full.copy()
        for k in range(2 * d - 2, d - 1, -1):
            c = full[..., k]
            for t in self.taps:
                full[..., k - d + t] -= c
        return full[..., :d]

    def mul(self, a, b):
        """Elementwise ring product over broadcast leading axes."""
        a = np.asarray(a, U64)
        b = np.asarray(b, U64)
        d = self.d
        shape = np.broadcast_shapes(a.shape[:-1], b.shape[:-1])
        full = np.zeros(shape + (2 * d - 1,), dtype=U64)
        for j in range(d):
            full[..., j:j + d] += a[..., j:j + 1] * b
        return self.reduce(full)

    def dot(self, a, b):
        """sum_i a_i * b_i over axis -2 (a ring inner product)."""
        return self.mul(a, b).sum(axis=-2, dtype=U64)

    def pow(self, a, e):
        out = self.const(1)
        base = np.asarray(a, U64)
        while e:
            if e & 1:
                out = self.mul(out, base)
            base = self.mul(base, base)
            e >>= 1
        return out

    def powers(self, a, n):
        """[a^0, a^1, ..., a^(n-1)] by repeated multiplication."""
        out = np.zeros((n, self.d), dtype=U64)
        cur = self.const(1)
        for i in range(n):
            out[i] = cur
            cur = self.mul(cur, a)
        return out

    def mulmat(self, t):
        """d x d matrix T with T @ v == t * v (column j holds t * x^j)."""
        d = self.d
        eye = np.eye(d, dtype=U64)
        return self.mul(np.broadcast_to(np.asarray(t, U64), (d, d)), eye).T.copy()

    def var(self):
        """The ring element x (coefficient vector e_1)."""
        out = self.zeros()
        out[1] = 1
        return out

    def inv(self, a):
        """Inverse of a unit: a^(2^d - 2) is an inverse modulo 2 (GF(2^d)* has order
        2^d - 1); Newton's step y <- y (2 - a y) then doubles the 2-adic precision."""
        a = np.asarray(a, U64)
        if not np.any(a & U64(1)):
            raise ZeroDivisionError("not a unit (zero modulo 2)")
        y = self.pow(a, (1 << self.d) - 2)
        two = self.const(2)
        for _ in range(7):
            y = self.mul(y, self.sub(two, self.mul(a, y)))
        return y

    def is_zero(self, a):
        return not np.any(np.asarray(a, U64))
