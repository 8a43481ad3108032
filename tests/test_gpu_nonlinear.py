"""Parity of the non-linear layers on the GPU (edaBits, daBits, ReLU, 2x2 max pooling, and
their verification: the edaBit inner products over GR(2^64, 64), the Boolean triples over
GF(2^64)) with the CPU oracle, bit for bit, on the same seeds and call sequence; plus
properties at sizes the oracle does not reach."""
import numpy as np
import pytest

from oracle.protocol import Ctx
from oracle.ring import encode

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2411_09287_amd import mpc3  # noqa: E402

SEED = bytes(range(3, 35))


def pair_of(variant=0):
    o = Ctx(SEED)
    c = mpc3.Context(SEED)
    c.set_variant(variant)
    return o, c


def same(gs, os_):
    gm, g1, g2 = gs.numpy()
    return all(np.array_equal(a.reshape(-1), b.reshape(-1)) for a, b in zip((gm, g1, g2), os_.comps()))


def word0(a):
    """A transcript slot of the oracle as the GPU logs it: 64 words, or one word (GF(2^64))
    in word 0 of a zero slot."""
    a = np.atleast_1d(np.asarray(a, dtype=np.uint64)).reshape(-1)
    if a.size == 64:
        return a
    out = np.zeros(64, np.uint64)
    out[:a.size] = a
    return out


def compare_transcripts(o, c):
    for s, log in enumerate(o.vlog):
        r, R, dim = c.verify_log(s, mpc3.LOG_R)
        assert np.array_equal(r, word0(log["r"])), (s, log["kind"])
        assert R == log["R"] and dim == log["npad"], (s, log["kind"])
        assert np.array_equal(c.verify_log(s, mpc3.LOG_Z)[0], word0(log["z"].m)), s
        for k, rl in enumerate(log["rounds"]):
            assert np.array_equal(c.verify_log(s, mpc3.LOG_ZETA, k)[0], word0(rl["zeta"])), (s, k)
            for slot, key in [(mpc3.LOG_H0_M1, "m1"), (mpc3.LOG_H0_M2, "m2"), (mpc3.LOG_H0_G2, "gamma2")]:
                assert np.array_equal(c.verify_log(s, slot, k)[0], word0(rl["h0"][key])), (s, k, key)
            for slot, key in [(mpc3.LOG_H2_M1, "m1"), (mpc3.LOG_H2_M2, "m2"), (mpc3.LOG_H2_G2, "gamma2")]:
                assert np.array_equal(c.verify_log(s, slot, k)[0], word0(rl["h2"][key])), (s, k, key)
        assert np.array_equal(c.verify_log(s, mpc3.LOG_DELTA)[0], word0(log["delta"])), s
        for slot, key in [(mpc3.LOG_DELTA_M1, "m1"), (mpc3.LOG_DELTA_M2, "m2"), (mpc3.LOG_DELTA_G2, "gamma2")]:
            assert np.array_equal(c.verify_log(s, slot)[0], word0(log["delta_tr"][key])), (s, key)


def comm_equal(o, c):
    bg, rg = c.comm_stats()
    return np.array_equal(bg, np.array(o.comm, dtype=np.uint64)) and rg == o.rounds


@pytest.mark.parametrize("n", [1, 37, 130])
def test_edabits_and_dabits_parity(n):
    o, c = pair_of()
    ra, rb = o.edabits(n)
    ga, gb = c.edabits(n)
    assert same(ga, ra) and same(gb, rb)
    sa, sb = o.dabits(n)
    ha, hb = c.dabits(n)
    assert same(ha, sa) and same(hb, sb)
    assert comm_equal(o, c)
    assert o.verify() and c.verify()
    compare_transcripts(o, c)
    assert comm_equal(o, c)


def _values(g, n):
    x = encode(g.standard_normal(n) * 6, 13)
    x[:4] = np.array([0, 1, (1 << 64) - 1, 1 << 63], dtype=np.uint64)[:min(4, n)]
    return x


_ORACLE = {}


def _oracle_relu(n, inj=None):
    """The oracle's run of share -> ReLU -> verify on n seeded values (computed once per case;
    it does not depend on the kernel family compared with it)."""
    key = (n, inj)
    if key not in _ORACLE:
        g = np.random.default_rng(n if inj is None else inj[0] * 7 + inj[1])
        x = _values(g, n)
        o = Ctx(SEED)
        if inj:
            o.inject(*inj)
        Yo = o.relu(o.share(x))
        before = ([[list(r) for r in ph] for ph in o.comm], list(o.rounds))
        ok = o.verify()
        _ORACLE[key] = (x, o, Yo, before, ok)
    return _ORACLE[key]


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("n", [5, 64, 97])
def test_relu_parity_and_transcript(variant, n):
    x, o, Yo, before, ok_o = _oracle_relu(n)
    c = mpc3.Context(SEED)
    c.set_variant(variant)
    Yg = c.relu(c.share(mpc3.to_words(x)))
    assert same(Yg, Yo)
    bg, rg = c.comm_stats()
    assert np.array_equal(bg, np.array(before[0], dtype=np.uint64)) and rg == before[1]
    assert ok_o and c.verify()
    compare_transcripts(o, c)
    assert comm_equal(o, c)
    got = mpc3.from_words(c.reconstruct(Yg)).reshape(-1)
    assert np.array_equal(got, np.where(x.view(np.int64) > 0, x, np.uint64(0)))


@pytest.mark.parametrize("B,H,W,C", [(1, 4, 4, 3), (2, 2, 6, 1)])
def test_maxpool2_parity(B, H, W, C):
    g = np.random.default_rng(H * W + C)
    x = encode(g.standard_normal(B * H * W * C) * 3, 13).reshape(B, H * W * C)
    o, c = pair_of(1)
    Xo, Xg = o.share(x), c.share(mpc3.to_words(x))
    Yo, Yg = o.maxpool2(Xo, B, H, W, C), c.maxpool2(Xg, B, H, W, C)
    assert same(Yg, Yo)
    assert o.verify() and c.verify()
    compare_transcripts(o, c)
    assert comm_equal(o, c)
    v = x.view(np.int64).reshape(B, H, W, C)
    want = np.maximum(np.maximum(v[:, 0::2, 0::2], v[:, 0::2, 1::2]), np.maximum(v[:, 1::2, 0::2], v[:, 1::2, 1::2]))
    assert np.array_equal(mpc3.from_words(c.reconstruct(Yg)).view(np.int64).reshape(want.shape), want)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("site,index,e", [(mpc3.SITE_AND_GAMMA2, 3, 1 << 17), (mpc3.SITE_AND_GAMMA2, 0, 1 << 63),
                                          (mpc3.SITE_EDA_W_M1, 2, 1 << 63), (mpc3.SITE_EDA_W_M1, 0, 5),
                                          (mpc3.SITE_MULT_GAMMA2, 100, 1)])
def test_injected_error_in_relu_detected(variant, site, index, e):
    x, o, Yo, _, ok_o = _oracle_relu(6, (site, index, e))
    c = mpc3.Context(SEED)
    c.set_variant(variant)
    c.inject(site, index, e)
    Yg = c.relu(c.share(mpc3.to_words(x)))
    assert same(Yg, Yo)
    assert not ok_o and not c.verify()
    compare_transcripts(o, c)
    with pytest.raises(mpc3.Mpc3Error) as ei:
        c.reconstruct(Yg)
    assert ei.value.code == mpc3.E_ABORTED


@pytest.mark.parametrize("variant", [0, 1])
def test_relu_large_verifies_and_rejects(variant):
    """40000 values: three edaBit Pi_BIVerify instances (16384 per instance), a 28 M-gate
    GF(2^64) instance; the opened values are max(x, 0), an injected error in the last
    Boolean word is caught.  (The oracle's verification is too slow at this size.)"""
    g = np.random.default_rng(9)
    n = 40000
    x = _values(g, n)
    for inj in (None, (mpc3.SITE_AND_GAMMA2, n - 1, 1 << 5)):
        c = mpc3.Context(SEED)
        c.set_variant(variant)
        if inj:
            c.inject(*inj)
        Xg = c.share(mpc3.to_words(x))
        Yg = c.relu(Xg)
        ok = c.verify()
        assert ok == (inj is None)
        if ok:
            got = mpc3.from_words(c.reconstruct(Yg)).reshape(-1)
            assert np.array_equal(got, np.where(x.view(np.int64) > 0, x, np.uint64(0)))


def test_nonlinear_kind_selection():
    """Verifying the Z_2^64 products first and the non-linear kind afterwards gives the same
    outcome as the oracle, and reconstruct waits for both."""
    g = np.random.default_rng(12)
    x = _values(g, 9)
    o, c = pair_of(1)
    Yo, Yg = o.relu(o.share(x)), c.relu(c.share(mpc3.to_words(x)))
    assert o.verify(kinds=4) and c.verify(kinds=mpc3.VERIFY_MULT)
    with pytest.raises(mpc3.Mpc3Error) as ei:
        c.reconstruct(Yg)
    assert ei.value.code == mpc3.E_UNVERIFIED
    assert o.verify(kinds=8) and c.verify(kinds=mpc3.VERIFY_NONLINEAR)
    compare_transcripts(o, c)
    assert np.array_equal(mpc3.from_words(c.reconstruct(Yg)).reshape(-1), o.reconstruct(Yo).reshape(-1))


@pytest.mark.parametrize("variant", [0, 1])
def test_mult_verify_in_chunks_parity(variant):
    """1100 Pi_Mult triples verified in instances of 500: three challenges, transcripts as
    the oracle's with the same chunking."""
    g = np.random.default_rng(44)
    o = Ctx(SEED, chunk_mult=500)
    c = mpc3.Context(SEED)
    c.set_variant(variant)
    c.set_verify_chunks(500, 0)
    a0 = g.integers(0, 1 << 64, size=(1100, 1), dtype=np.uint64, endpoint=False)
    b0 = g.integers(0, 1 << 64, size=(1100, 1), dtype=np.uint64, endpoint=False)
    co = o.mult(o.share(a0), o.share(b0))
    cg = c.mult(c.share(mpc3.to_words(a0)), c.share(mpc3.to_words(b0)))
    assert same(cg, co)
    assert o.verify() and c.verify()
    assert len(o.vlog) == 3
    compare_transcripts(o, c)
    assert comm_equal(o, c)


def test_edabit_rows_in_chunks_parity():
    """40 edaBits with instances of 16 inner products: three Pi_BIVerify instances of the
    edaBit gates, as the oracle's with the same chunking."""
    o = Ctx(SEED, chunk_rows=16)
    c = mpc3.Context(SEED)
    c.set_verify_chunks(0, 16)
    ra, rb = o.edabits(40)
    ga, gb = c.edabits(40)
    assert same(ga, ra) and same(gb, rb)
    assert o.verify() and c.verify()
    assert [lg["kind"] for lg in o.vlog] == ["mult", "rows", "rows", "rows"]
    compare_transcripts(o, c)
    assert comm_equal(o, c)
