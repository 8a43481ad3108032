"""Pins of the oracle's non-linear layers (Sec. 4.3, Fig. "The maliciously edaBits
generation") and of its GF(2^64) verification: sympy's GF(2) polynomial arithmetic, closed
forms (AND, the top bit, max(x, 0), 2x2 maxima of plaintext), the consistency of the two
sharings of an edaBit or daBit, honest verification passing and injected errors failing,
and the false-accept rate of the field verification at a small degree against its bound."""
import numpy as np
import pytest
import sympy as sp

from oracle.gf2 import GF
from oracle.gr import MODULI
from oracle.nonlinear import SITE_AND_GAMMA2, SITE_EDA_W_M1, BShare
from oracle.protocol import Aborted, Ctx, SITE_MULT_GAMMA2, OFFLINE, ONLINE
from oracle.ring import encode

SEED = bytes(range(40, 72))
U64 = np.uint64


def _u64(g, *shape):
    return g.integers(0, 1 << 64, size=shape, dtype=np.uint64, endpoint=False)


def _poly(v, x):
    return sp.Poly(sum(((int(v) >> k) & 1) * x ** k for k in range(64)), x, modulus=2)


@pytest.mark.parametrize("d", [8, 64])
def test_gf_product_is_sympy_product_mod_f(d):
    x = sp.symbols("x")
    f = sp.Poly(x ** d + sum(x ** t for t in MODULI[d]), x, modulus=2)
    F = GF(d)
    g = np.random.default_rng(d)
    a = _u64(g, 12) & F.mask
    b = _u64(g, 12) & F.mask
    got = F.mul(a, b)
    for ai, bi, ci in zip(a, b, got):
        want = (_poly(ai, x) * _poly(bi, x)).rem(f)
        w = sum(int(c) % 2 << k for (k,), c in want.terms())
        assert int(ci) == w


def test_gf_field_laws_and_inverse():
    F = GF(64)
    g = np.random.default_rng(3)
    a, b, c = _u64(g, 8), _u64(g, 8), _u64(g, 8)
    assert np.array_equal(F.mul(a, b ^ c), F.mul(a, b) ^ F.mul(a, c))
    assert np.array_equal(F.mul(F.mul(a, b), c), F.mul(a, F.mul(b, c)))
    assert np.array_equal(F.mul(a, F.inv(a)), np.ones(8, U64))
    # squaring is additive (Frobenius) and x^64 = x^4 + x^3 + x + 1
    assert np.array_equal(F.mul(a ^ b, a ^ b), F.mul(a, a) ^ F.mul(b, b))
    assert int(F.pow(U64(2), 64)) == 0b11011
    p = F.powers(U64(0x1234567), 37)
    assert all(int(p[i]) == int(F.pow(U64(0x1234567), i)) for i in range(37))


def test_boolean_and_is_bitwise_and_with_table1_traffic():
    ctx = Ctx(SEED)
    g = np.random.default_rng(4)
    a = BShare(_u64(g, 9), _u64(g, 9), _u64(g, 9))
    b = BShare(_u64(g, 9), _u64(g, 9), _u64(g, 9))
    item = {"triples": []}
    c = ctx.and_words(a, b, item)
    assert np.array_equal(c.value(), a.value() & b.value())
    # one word (64 gates): 8 bytes offline (P0 -> P2) and 8 bytes each way online
    assert ctx.comm[OFFLINE][0][2] == 8 * 9
    assert ctx.comm[ONLINE][1][2] == 8 * 9 and ctx.comm[ONLINE][2][1] == 8 * 9
    assert len(item["triples"]) == 1


def test_edabits_two_sharings_agree():
    ctx = Ctx(SEED)
    r, R = ctx.edabits(50)
    assert np.array_equal(r.value(), R.value())
    bits = np.unpackbits(R.value().view(np.uint8))
    assert 0.35 < bits.mean() < 0.65                  # random bits, not a constant
    assert ctx.verify()


def test_dabits_are_bits_in_both_sharings():
    ctx = Ctx(SEED)
    s, sb = ctx.dabits(64)
    v = s.value()
    assert set(np.unique(v)) <= {0, 1}
    assert np.array_equal(v, sb.value())
    assert 0 < v.sum() < 64
    assert ctx.verify()


def test_msb_is_top_bit():
    ctx = Ctx(SEED)
    g = np.random.default_rng(5)
    x0 = np.concatenate([_u64(g, 20), np.array([0, 1, (1 << 63) - 1, 1 << 63, (1 << 64) - 1,
                                                (1 << 62), 3 << 62], dtype=U64)])
    X = ctx.share(x0)
    eda = ctx.edabits(x0.size)
    item = {"triples": []}
    ctx.pending.append(("and", item))
    m = ctx.msb(X, eda, item)
    assert np.array_equal(m.value(), x0 >> U64(63))
    assert len(item["triples"]) == 6                  # one Boolean Pi_Mult round per prefix level


def test_relu_is_max_with_zero():
    ctx = Ctx(SEED)
    g = np.random.default_rng(6)
    x = encode(g.standard_normal(12) * 5, 13)
    x[:3] = np.array([0, 1, (1 << 64) - 1], dtype=U64)
    y = ctx.relu(ctx.share(x))
    assert ctx.verify()
    got = ctx.reconstruct(y)
    assert np.array_equal(got, np.where(x.view(np.int64) > 0, x, U64(0)))


def test_maxpool2_is_window_maximum():
    ctx = Ctx(SEED)
    g = np.random.default_rng(7)
    B, H, W, C = 1, 4, 2, 2
    x = encode(g.standard_normal(B * H * W * C) * 3, 13).reshape(B, H * W * C)
    y = ctx.maxpool2(ctx.share(x), B, H, W, C)
    assert ctx.verify()
    got = ctx.reconstruct(y).view(np.int64).reshape(B, H // 2, W // 2, C)
    v = x.view(np.int64).reshape(B, H, W, C)
    want = np.maximum(np.maximum(v[:, 0::2, 0::2], v[:, 0::2, 1::2]), np.maximum(v[:, 1::2, 0::2], v[:, 1::2, 1::2]))
    assert np.array_equal(got, want)


@pytest.mark.parametrize("site,index,e", [(SITE_AND_GAMMA2, 2, 1 << 17), (SITE_AND_GAMMA2, 0, 1),
                                          (SITE_EDA_W_M1, 1, 1 << 63), (SITE_MULT_GAMMA2, 5, 1)])
def test_injected_errors_in_nonlinear_layer_abort(site, index, e):
    ctx = Ctx(SEED)
    x = encode(np.random.default_rng(8).standard_normal(4), 13)
    X = ctx.share(x)
    ctx.inject(site, index, e)
    ctx.relu(X)
    assert not ctx.verify()
    with pytest.raises(Aborted):
        ctx.relu(X)


def test_gf_verification_false_accept_rate_small_degree():
    """A wrong Boolean triple (64 gates, one of them off by one) is accepted by the GF(2^8)
    Pi_MultVerify with probability at most about (|G| + 2 R + 1) / 2^8 (Schwartz-Zippel on
    the power-weighted sum, two per reduction round, one for the final check)."""
    trials, acc = 120, 0
    G, R = 64, 3
    for t in range(trials):
        ctx = Ctx(bytes([t % 256, t // 256]) + bytes(30), d=8)
        g = np.random.default_rng(100 + t)
        a = BShare(_u64(g, 1), _u64(g, 1), _u64(g, 1))
        b = BShare(_u64(g, 1), _u64(g, 1), _u64(g, 1))
        c = ctx.and_words(a, b, {"triples": []})
        bad = BShare(c.m ^ U64(1 << int(g.integers(0, 64))), c.r1, c.r2)
        acc += ctx.verify_and_item({"triples": [(a, b, bad)]}, ctx.next_op(), 0, R, {})
    bound = (G + 2 * R + 1) / 256
    assert acc / trials <= bound + 0.08
