"""Pins of the oracle's protocol steps against plaintext arithmetic, closed forms,
brute force on tiny inputs, the paper's communication figures and soundness bounds."""
import itertools

import numpy as np
import pytest

from oracle import prg
from oracle.gr import GR
from oracle.protocol import (Aborted, Ctx, Share, Unverified, SITE_INNER_GAMMA2, SITE_INNER_M1,
                             SITE_MULT_GAMMA2, SITE_REC_R1, SITE_TRUNC_GAMMA2, SITE_TRUNC_M1,
                             SITE_VER_DELTA_M1, SITE_VER_H0_M1, SITE_VER_H2_GAMMA2, OFFLINE, ONLINE)
from oracle.ring import decode, encode
from paper_2411_09287_amd import workloads

MASK = (1 << 64) - 1
SEED = bytes(range(32))


def _u64(g, *shape):
    return g.integers(0, 1 << 64, size=shape, dtype=np.uint64, endpoint=False)


def _total(comm, phase):
    return sum(sum(row) for row in comm[phase])


def test_encode_decode_floor():
    g = np.random.default_rng(0)
    x = g.standard_normal(1000) * 100
    err = decode(encode(x, 13), 13) - x
    assert np.all(err <= 0) and np.all(err > -2.0 ** -13)
    # the encoding of a negative value is 2^64 + floor(x 2^k)
    assert int(encode(np.array([-1.5]), 13)[0]) == (1 << 64) - 3 * (1 << 12)


@pytest.mark.parametrize("owner", [0, 1, 2])
def test_share_reconstructs_to_input(owner):
    ctx = Ctx(SEED)
    x = _u64(np.random.default_rng(1), 37)
    s = ctx.share(x, owner=owner)
    assert np.array_equal(s.m - s.r1 - s.r2, x)
    assert np.array_equal(ctx.reconstruct(s), x)


def test_inner_is_plain_matmul_mod_2_64():
    g = np.random.default_rng(2)
    ctx = Ctx(SEED)
    M, K, N = 9, 33, 7
    X0, W0 = _u64(g, M, K), _u64(g, K, N)
    Z = ctx.inner(ctx.share(X0), ctx.share(W0))
    assert np.array_equal(Z.value(), X0 @ W0)           # numpy uint64 matmul wraps mod 2^64


def test_inner_brute_force_tiny():
    for M, K, N in [(1, 1, 1), (2, 3, 4), (4, 4, 4), (3, 1, 2)]:
        g = np.random.default_rng(M * 100 + K * 10 + N)
        ctx = Ctx(SEED)
        X0, W0 = _u64(g, M, K), _u64(g, K, N)
        Z = ctx.inner(ctx.share(X0), ctx.share(W0))
        for m, n in itertools.product(range(M), range(N)):
            want = sum(int(X0[m, k]) * int(W0[k, n]) for k in range(K)) & MASK
            assert int(Z.value()[m, n]) == want


def test_inner_communication_matches_table1():
    """Table 1 ("Ours"): inner product of any dimension costs 1 l offline, 2 l online."""
    g = np.random.default_rng(3)
    ctx = Ctx(SEED)
    X, W = ctx.share(_u64(g, 5, 40)), ctx.share(_u64(g, 40, 6))
    before = [_total(ctx.comm, p) for p in range(4)]
    ctx.inner(X, W)
    assert _total(ctx.comm, OFFLINE) - before[OFFLINE] == 8 * 30
    assert _total(ctx.comm, ONLINE) - before[ONLINE] == 16 * 30


def test_inner_with_truncation_communication_matches_table1():
    """Table 1: inner product with truncation costs 7 l offline and 2 l online;
    the truncation pair alone is 6 l offline (Sec. 4.2)."""
    g = np.random.default_rng(4)
    ctx = Ctx(SEED)
    X, W = ctx.share(_u64(g, 4, 10)), ctx.share(_u64(g, 10, 3))
    b0 = _total(ctx.comm, OFFLINE)
    pair = ctx.trunc_pair(12, 13)
    assert _total(ctx.comm, OFFLINE) - b0 == 48 * 12
    b1 = [_total(ctx.comm, p) for p in range(2)]
    Z = ctx.inner(X, W, pair)
    ctx.trunc(pair, Z)
    assert _total(ctx.comm, OFFLINE) - b0 == 56 * 12
    assert _total(ctx.comm, ONLINE) - b1[ONLINE] == 16 * 12


def test_trunc_pair_reconstructs_xor_and_shift():
    """<r_x> opens to B1 xor B2 (bitwise, from the two pairwise bit lists) and <r_z> to
    floor(r_x / 2^t) of the signed word, computed here with Python integers."""
    ctx = Ctx(SEED)
    n, t = 50, 13
    pair = ctx.trunc_pair(n, t)
    op = pair["op"]
    B1 = prg.words(ctx.seeds[(0, 1)], prg.tag(op, prg.TRUNC_B, 1), n)
    B2 = prg.words(ctx.seeds[(0, 2)], prg.tag(op, prg.TRUNC_B, 2), n)
    rx, rz = pair["rx"].value(), pair["rz"].value()
    for p in range(n):
        v = int(B1[p]) ^ int(B2[p])
        assert int(rx[p]) == v
        sv = v - (1 << 64) if v >> 63 else v
        assert int(rz[p]) == (sv >> t) & MASK


def test_truncation_error_is_one_lsb():
    g = np.random.default_rng(5)
    ctx = Ctx(SEED)
    x, w = g.standard_normal((16, 20)), g.standard_normal((20, 8))
    X0, W0 = encode(x, 13), encode(w, 13)
    pair = ctx.trunc_pair(16 * 8, 13)
    Zt = ctx.trunc(pair, ctx.inner(ctx.share(X0), ctx.share(W0), pair))
    assert ctx.verify()
    out = ctx.reconstruct(Zt).view(np.int64)
    exact = (X0 @ W0).view(np.int64)
    diff = out - (exact >> 13)
    assert set(np.unique(diff)) <= {0, 1}


def test_truncation_large_error_probability():
    """Sec. 4.2: the probabilistic truncation makes a large error when m = x + r_x wraps the
    signed range, which for a uniform r_x happens with probability |x| / 2^64 per value; for
    values of l_x bits that is at most 2^(l_x - l + 1).  Values with |x| < 2^60 (l_x = 61)."""
    ctx = Ctx(SEED)
    n = 4096
    g = np.random.default_rng(6)
    v = (g.integers(-(1 << 60), 1 << 60, size=n)).astype(np.int64)
    # a 1-dimensional product x * 1 feeds the truncation
    X = ctx.share(v.view(np.uint64).reshape(n, 1))
    W = ctx.share(np.ones((1, 1), dtype=np.uint64))
    pair = ctx.trunc_pair(n, 13)
    Zt = ctx.trunc(pair, ctx.inner(X, W, pair))
    ctx.pending = []      # honest run; verification is pinned by the tests below
    out = ctx.reconstruct(Zt).view(np.int64).reshape(-1)
    big = np.abs(out - (v >> 13)) > 1
    p = np.abs(v).astype(np.float64) / 2.0 ** 64
    mean, sd = p.sum(), np.sqrt((p * (1 - p)).sum())
    assert abs(big.sum() - mean) < 4 * sd
    assert big.mean() <= 2.0 ** (61 - 64 + 1)


def test_verify_honest_all_kinds():
    g = np.random.default_rng(7)
    ctx = Ctx(SEED, chunk=8)
    X, W = ctx.share(_u64(g, 4, 6)), ctx.share(_u64(g, 6, 5))
    pair = ctx.trunc_pair(20, 13)
    Z = ctx.inner(X, W, pair)
    ctx.trunc(pair, Z)
    ctx.mult(ctx.share(_u64(g, 7)), ctx.share(_u64(g, 7)))
    ctx.inner(ctx.share(_u64(g, 3, 2)), ctx.share(_u64(g, 2, 4)))
    assert ctx.verify()
    kinds = [l["kind"] for l in ctx.vlog]
    assert kinds == ["inner", "trunc", "trunc", "trunc", "mult"]   # all Pi_Inner products in one
    assert all(not np.any(l["delta"]) for l in ctx.vlog)


SITES = [SITE_INNER_GAMMA2, SITE_INNER_M1, SITE_TRUNC_GAMMA2, SITE_TRUNC_M1, SITE_MULT_GAMMA2,
         SITE_VER_H0_M1, SITE_VER_H2_GAMMA2, SITE_VER_DELTA_M1]


VERIFY_SITES = {SITE_VER_H0_M1, SITE_VER_H2_GAMMA2, SITE_VER_DELTA_M1}


@pytest.mark.parametrize("site", SITES)
@pytest.mark.parametrize("e", [1, 1 << 63, 0xDEADBEEF << 20])
def test_verify_detects_injected_error(site, e):
    g = np.random.default_rng(8)
    ctx = Ctx(SEED, chunk=4)
    # verification sites index (instance << 16 | round << 8 | coefficient): instance 1 is
    # the first truncation chunk (the batched Pi_Inner instance, 0, has no rounds here)
    ctx.inject(site, (1 << 16) | 3 if site in VERIFY_SITES else 3, e)
    X, W = ctx.share(_u64(g, 2, 5)), ctx.share(_u64(g, 5, 3))
    pair = ctx.trunc_pair(6, 13)
    Z = ctx.inner(X, W, pair)
    Zt = ctx.trunc(pair, Z)
    ctx.mult(ctx.share(_u64(g, 5)), ctx.share(_u64(g, 5)))
    assert (site in ctx.injections) == (site in VERIFY_SITES)
    assert not ctx.verify()
    assert site not in ctx.injections          # the error was applied
    with pytest.raises(Aborted):
        ctx.reconstruct(Zt)


def test_reconstruct_requires_verification():
    g = np.random.default_rng(9)
    ctx = Ctx(SEED)
    Z = ctx.inner(ctx.share(_u64(g, 2, 2)), ctx.share(_u64(g, 2, 2)))
    with pytest.raises(Unverified):
        ctx.reconstruct(Z)
    assert ctx.verify()
    ctx.reconstruct(Z)


def test_reconstruct_detects_inconsistent_share():
    ctx = Ctx(SEED)
    s = ctx.share(_u64(np.random.default_rng(10), 6))
    ctx.inject(SITE_REC_R1, 2, 5)
    with pytest.raises(Aborted):
        ctx.reconstruct(s)
    assert ctx.aborted


def test_compressed_claim_equals_literal_claim():
    """One instance for a batch of products: sum_k x_k y_k and z of the compressed form
    equal the literal consolidated sum over all gates i = o_l + n M_l + m, each weighted
    by r^i (brute force on two tiny products of different shapes)."""
    g = np.random.default_rng(11)
    ctx = Ctx(SEED)
    gr = ctx.gr
    items = []
    for M, K, N in [(3, 4, 2), (2, 3, 3)]:
        X, W = ctx.share(_u64(g, M, K)), ctx.share(_u64(g, K, N))
        items.append((X, W, ctx.inner(X, W)))
    r = g.integers(0, 1 << 64, size=64, dtype=np.uint64, endpoint=False)
    U, V, zc = ctx.instance_inner_compressed(items, r)
    x, y, zl = ctx.instance_inner_literal(items, r)
    assert U.m.shape == (4 + 3, 64)
    for c in range(3):
        assert np.array_equal(zc.comps()[c], zl.comps()[c])
    for c1, c2 in itertools.product(range(3), repeat=2):
        assert np.array_equal(gr.dot(U.comps()[c1], V.comps()[c2]), gr.dot(x.comps()[c1], y.comps()[c2]))
    assert np.array_equal(gr.dot(U.value(), V.value()), zc.value())
    # z is the weighted sum of the products' gates, written out with Python integers
    want = np.zeros(64, dtype=np.uint64)
    i = 0
    for X, W, Z in items:
        Zv = Z.value()
        for n in range(Zv.shape[1]):
            for m in range(Zv.shape[0]):
                want = want + gr.scale(Zv[m, n], gr.pow(r, i))
                i += 1
    assert np.array_equal(zc.value(), want)
    ctx.pending = []


def test_literal_form_verifies_and_rejects():
    g = np.random.default_rng(12)
    for inj in (None, (SITE_INNER_M1, 1, 1 << 63)):
        ctx = Ctx(SEED)
        if inj:
            ctx.inject(*inj)
        ctx.inner(ctx.share(_u64(g, 2, 3)), ctx.share(_u64(g, 3, 2)))
        assert ctx.verify(R=2, literal=True) == (inj is None)


def _random_share(g, gr, n):
    return Share(*[g.integers(0, 1 << 64, size=(n, gr.d), dtype=np.uint64, endpoint=False) for _ in range(3)])


def test_reduce_round_preserves_honest_relation_and_error():
    g = np.random.default_rng(13)
    ctx = Ctx(SEED)
    gr = ctx.gr
    n = 8
    x, y = _random_share(g, gr, n), _random_share(g, gr, n)
    zval = gr.dot(x.value(), y.value())
    r1, r2 = _u64(g, 64), _u64(g, 64)
    z = Share(zval + r1 + r2, r1, r2)
    log = {"rounds": []}
    for k in range(3):
        x, y, z = ctx.reduce_round(x, y, z, 99, 0, k, log)
        assert x.m.shape[0] == n >> (k + 1)
        assert np.array_equal(gr.dot(x.value(), y.value()), z.value())
    # a wrong claim stays wrong
    x, y = _random_share(g, gr, n), _random_share(g, gr, n)
    z = Share(gr.dot(x.value(), y.value()) + gr.const(1 << 63) + r1 + r2, r1, r2)
    x, y, z = ctx.reduce_round(x, y, z, 99, 1, 0, log)
    assert not np.array_equal(gr.dot(x.value(), y.value()), z.value())


def test_lagrange_weights_over_nodes_0_1_x():
    g = np.random.default_rng(14)
    ctx = Ctx(SEED)
    gr = ctx.gr
    one, X = gr.const(1), gr.var()
    zeta = _u64(g, 64)
    c0, c1, c2 = _u64(g, 64), _u64(g, 64), _u64(g, 64)

    def p(t):
        return c0 + gr.mul(c1, t) + gr.mul(c2, gr.mul(t, t))

    L0 = gr.mul(gr.mul(zeta - one, zeta - X), ctx.inv_x)
    L1 = gr.mul(gr.mul(zeta, zeta - X), ctx.inv_1mx)
    L2 = gr.mul(gr.mul(zeta, zeta - one), ctx.inv_xxm1)
    assert np.array_equal(L0 + L1 + L2, one)
    lhs = gr.mul(L0, p(gr.const(0))) + gr.mul(L1, p(one)) + gr.mul(L2, p(X))
    assert np.array_equal(lhs, p(zeta))


def test_ring_attack_without_extension():
    """Sec. 3: in plain Z_{2^l} (d = 1) an error e = 2^(l-1) at a gate i >= 1 vanishes from
    sum r^i e_i whenever r is even, i.e. with probability 1/2; in GR(2^64, 64) the same
    error survives for random r (it vanishes only when r^2 is 0 modulo 2, i.e. r = 0 mod 2)."""
    g = np.random.default_rng(15)
    gr1, gr64 = GR(1), GR(64)
    e = np.zeros(4, dtype=np.uint64)
    e[2] = np.uint64(1 << 63)
    passes1 = 0
    trials = 4000
    for _ in range(trials):
        r = _u64(g, 1)
        s = gr1.scale(e, gr1.powers(r, 4)).sum(axis=0, dtype=np.uint64)
        passes1 += not np.any(s)
    assert abs(passes1 / trials - 0.5) < 0.05
    for _ in range(50):
        r = _u64(g, 64)
        s = gr64.scale(e, gr64.powers(r, 4)).sum(axis=0, dtype=np.uint64)
        assert np.any(s)


def test_inner_verify_soundness_small_d():
    """Lemma polyvv: a wrong claim passes Pi_InnerVerify with probability <= 1/2^d.
    With d = 4 the bound is 1/16; the empirical rate over seeded trials must not exceed
    it by more than 3 sigma."""
    trials = 1500
    d = 4
    passes = 0
    for s in range(trials):
        ctx = Ctx(s.to_bytes(32, "little"), d=d)
        gr = ctx.gr
        g = np.random.default_rng(1000 + s)
        x, y = _random_share(g, gr, 2), _random_share(g, gr, 2)
        e = g.integers(1, 1 << 64, size=d, dtype=np.uint64)
        r1, r2 = _u64(g, d), _u64(g, d)
        z = Share(gr.dot(x.value(), y.value()) + e + r1 + r2, r1, r2)
        passes += ctx.inner_verify(x, y, z, 5, 0, {})
    bound = 1 / 2 ** d
    assert passes / trials <= bound + 3 * np.sqrt(bound * (1 - bound) / trials)


def test_mult_verify_soundness_small_d():
    """Theorem multvv: false accepts of Pi_MultVerify^R stay under (|G|+1) / 2^(d-R-2)."""
    trials = 600
    d, n, R = 8, 4, 1
    passes = 0
    for s in range(trials):
        ctx = Ctx((s + 7).to_bytes(32, "little"), d=d)
        g = np.random.default_rng(5000 + s)
        ctx.inject(SITE_MULT_GAMMA2, int(g.integers(0, n)), int(g.integers(1, 1 << 63)) << 1)
        ctx.mult(ctx.share(_u64(g, n)), ctx.share(_u64(g, n)))
        passes += ctx.verify(R=R)
    bound = (n + 1) / 2 ** (d - R - 2)
    assert passes / trials <= bound + 3 * np.sqrt(bound * (1 - bound) / trials)


def test_workload_inputs_are_seeded():
    a = workloads.matmul_inputs(1)
    b = workloads.matmul_inputs(1)
    assert all(np.array_equal(u, v) for u, v in zip(a, b))
    assert workloads.model_shapes("vgg")[1] == (32768, 576, 64)
    assert workloads.model_shapes("lenet")[:2] == [(36864, 25, 20), (4096, 500, 50)]
