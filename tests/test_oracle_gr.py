"""Pins of the oracle's Galois-ring arithmetic against sympy and closed forms."""
import numpy as np
import pytest
import sympy as sp

from oracle.gr import GR, MODULI

MASK = (1 << 64) - 1
xs = sp.symbols("x")


def _rand(g, gr, *shape):
    return g.integers(0, 1 << 64, size=shape + (gr.d,), dtype=np.uint64, endpoint=False)


def _fpoly(d):
    return sp.Poly(xs ** d + sum(xs ** t for t in MODULI[d]), xs)


@pytest.mark.parametrize("d", [2, 4, 8, 16, 32, 64])
def test_modulus_irreducible_over_gf2(d):
    assert sp.Poly(_fpoly(d).as_expr(), xs, modulus=2).is_irreducible


@pytest.mark.parametrize("d", [4, 8, 64])
def test_product_mod2_is_gf2d_product(d):
    gr = GR(d)
    g = np.random.default_rng(d)
    f2 = sp.Poly(_fpoly(d).as_expr(), xs, modulus=2)
    for _ in range(3):
        a, b = _rand(g, gr), _rand(g, gr)
        c = gr.mul(a, b)
        pa = sp.Poly([int(v) & 1 for v in a[::-1]], xs, modulus=2)
        pb = sp.Poly([int(v) & 1 for v in b[::-1]], xs, modulus=2)
        pc = (pa * pb).rem(f2)
        want = [0] * d
        for (k,), v in pc.terms():
            want[k] = int(v) % 2
        assert [int(v) & 1 for v in c] == want


@pytest.mark.parametrize("d", [8, 64])
def test_product_is_integer_remainder_mod_2_64(d):
    """The full product over Z, remainder by the monic f over Z, then mod 2^64 (catches sign errors)."""
    gr = GR(d)
    g = np.random.default_rng(7 + d)
    f = _fpoly(d).set_domain(sp.ZZ)
    for _ in range(2):
        a, b = _rand(g, gr), _rand(g, gr)
        pa = sp.Poly([int(v) for v in a[::-1]], xs, domain=sp.ZZ)
        pb = sp.Poly([int(v) for v in b[::-1]], xs, domain=sp.ZZ)
        rem = (pa * pb).rem(f)
        want = [0] * d
        for (k,), v in rem.terms():
            want[k] = int(v) & MASK
        assert [int(v) for v in gr.mul(a, b)] == want


@pytest.mark.parametrize("d", [4, 64])
def test_x_to_the_d_closed_form(d):
    gr = GR(d)
    xd = gr.pow(gr.var(), d)
    want = np.zeros(d, dtype=np.uint64)
    for t in MODULI[d]:
        want[t] = np.uint64(MASK)          # x^d = -(sum of the low terms)
    assert np.array_equal(xd, want)


def test_ring_axioms():
    gr = GR(64)
    g = np.random.default_rng(3)
    a, b, c = _rand(g, gr), _rand(g, gr), _rand(g, gr)
    assert np.array_equal(gr.mul(a, b), gr.mul(b, a))
    assert np.array_equal(gr.mul(gr.mul(a, b), c), gr.mul(a, gr.mul(b, c)))
    assert np.array_equal(gr.mul(a, b + c), gr.mul(a, b) + gr.mul(a, c))
    assert np.array_equal(gr.mul(a, gr.const(1)), a)


def test_mulmat_and_powers():
    gr = GR(64)
    g = np.random.default_rng(4)
    t, v = _rand(g, gr), _rand(g, gr, 5)
    T = gr.mulmat(t)
    assert np.array_equal(v @ T.T, gr.mul(t, v))
    p = gr.powers(t, 9)
    for k in range(9):
        assert np.array_equal(p[k], gr.pow(t, k))


@pytest.mark.parametrize("d", [4, 64])
def test_inverse(d):
    gr = GR(d)
    g = np.random.default_rng(5)
    X = gr.var()
    one = gr.const(1)
    for u in [X, gr.sub(one, X), gr.mul(X, gr.sub(X, one)), _rand(g, gr) | np.uint64(1)]:
        assert np.array_equal(gr.mul(u, gr.inv(u)), one)
    if d == 64:
        # x * (x^63 + x^3 + x^2 + 1) = x^64 + x^4 + x^3 + x = -1, so x^-1 = -(x^63 + x^3 + x^2 + 1)
        want = np.zeros(64, dtype=np.uint64)
        for k in (63, 3, 2, 0):
            want[k] = np.uint64(MASK)
        assert np.array_equal(gr.inv(X), want)
