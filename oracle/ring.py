"""Z_{2^64} helpers and fixed-point encoding (oracle; test infrastructure only).

Fixed point follows the Preliminaries ("Notation"): a real x with k fractional
bits is encoded as floor(x * 2^k) when x >= 0 and as 2^l + floor(x * 2^k) when
x < 0, i.e. the two's complement of the floor.
"""
import numpy as np

U64 = np.uint64
MASK64 = (1 << 64) - 1


def u64(a):
    """Python ints / int arrays -> uint64 array, reducing modulo 2^64."""
    if isinstance(a, np.ndarray) and a.dtype == np.uint64:
        return a
    arr = np.asarray(a, dtype=object)
    return np.vectorize(lambda v: int(v) & MASK64, otypes=[np.uint64])(arr) if arr.ndim else U64(int(a) & MASK64)


def encode(x, frac_bits):
    """Preliminaries, "Notation": floor(x * 2^k) modulo 2^64 (two's complement of the floor)."""
    x = np.asarray(x, dtype=np.float64)
    scaled = np.floor(x * float(1 << frac_bits))
    return scaled.astype(np.int64).view(np.uint64)


def decode(v, frac_bits):
    """Inverse of encode: signed value / 2^k."""
    return np.asarray(v, dtype=np.uint64).view(np.int64).astype(np.float64) / float(1 << frac_bits)


def ash(v, t):
    """Arithmetic right shift of a two's-complement 64-bit word by t bits (floor(v / 2^t))."""
    return (np.asarray(v, dtype=np.uint64).view(np.int64) >> np.int64(t)).view(np.uint64)


def signed(v):
    return np.asarray(v, dtype=np.uint64).view(np.int64)
