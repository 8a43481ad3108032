"""Verification-phase communication of the oracle against a closed form written from the
message list of the protocols (Sec. 3), with the paper's own cost statements beside it.

Messages of one verification instance with R Pi_Reduce rounds and final dimension
n_R = npad / 2^R (d-word Galois-ring elements, 8d bytes each):
  * Pi_Rec^{l[x]} of a d-word value (the challenge r, each zeta, Delta): P0 -> P2 [r]_1,
    P0 -> P1 [r]_2, P1 -> P0 m (8d bytes each) and three 32-byte hashes P1 -> P2,
    P2 -> P0, P2 -> P1; one round.  R + 2 of them per instance.
  * Pi_PolyEvl (h(0) and h(x) of every round, Delta): P0 -> P2 [Gamma]_2 (8d, offline),
    P1 <-> P2 their m halves (8d each way, online).  2R + 1 of them, R + 1 rounds.
  * Pi_Mult over GR of alpha and the n_R final x elements: 8d n_R offline (P0 -> P2),
    8d n_R each way online, one round.
Hence per instance
    offline bytes  P0->P2 = 8d (2R + n_R + 1)
    online  bytes  P0->P1 = P0->P2 = P1->P0 = 8d (R + 2),  P2->P0 = 32 (R + 2),
                   P1->P2 = P2->P1 = 8d (2R + n_R + 1) + 32 (R + 2)
    online rounds  2R + 4.

The paper states (after Fig. "The Batch Multiplication Verification Protocol") that
Pi_MultVerify costs (R + |G|/2^R) l d bits offline and (5R + 3 + |G|/2^R) l d bits online
in R + 2 rounds.  With l d bits = 8d bytes its offline figure has one Gamma share per
round where this message set has two (h(0) and h(x) are separate Pi_PolyEvl calls) plus
the one of Delta: 8d (R + 1) bytes more.  Its online figure counts one direction of each
exchange and three words per reveal: 5 per round (h(0), h(x), the reveal of zeta), 3 for
Delta's reveal and n_R for the final products; the message set here also counts the
return direction of every exchange, the challenge r's reveal, Delta's exchange and the
hashes.  The per-round Pi_Reduce cost it states (5 l d online, l d offline, after Fig.
"The Inner Product Dimension Reduction Protocol") is the same accounting."""
import math

import numpy as np
import pytest

from oracle import protocol as P
from paper_2411_09287_amd import netmodel, workloads


def rounds_and_pad(n0, R):
    need = math.ceil(math.log2(n0)) if n0 > 1 else 0
    R = max(0, need - 3) if R < 0 else min(R, need)
    npad = -(-n0 // (1 << R)) * (1 << R)
    return R, npad


def closed_form(d, instances):
    """bytes[phase][src][dst] and rounds[phase] of the verification phases for instances
    given as (R, n_R): the cost model's per-instance message list (netmodel, the formula
    the library's choice of R prices) summed."""
    b = np.zeros((4, 3, 3), dtype=np.int64)
    rounds = [0, 0, 0, 0]
    for R, nR in instances:
        bi, ri = netmodel.instance_messages(8 * d, R, nR)
        b += np.array(bi, dtype=np.int64)
        rounds = [x + y for x, y in zip(rounds, ri)]
    return b, rounds


def paper_mult_verify(d, R, G):
    """The paper's Pi_MultVerify cost in bytes (offline, online one direction) and rounds."""
    w = 8 * d
    nR = G // (1 << R)
    return w * (R + nR), w * (5 * R + 3 + nR), R + 2


def measured(ctx, fn):
    b0, r0 = np.array(ctx.comm, dtype=np.int64), list(ctx.rounds)
    ok = fn()
    b1, r1 = np.array(ctx.comm, dtype=np.int64), list(ctx.rounds)
    return ok, b1 - b0, [x - y for x, y in zip(r1, r0)]


@pytest.mark.parametrize("R", [-1, 0, 1, 3, 6])
@pytest.mark.parametrize("n", [64, 100])
def test_mult_verify_messages_closed_form(R, n):
    d = 8
    c = P.Ctx(workloads.master_seed(5), d=d)
    g = np.random.default_rng(n + R)
    a = c.share(g.integers(0, 1 << 64, n, dtype=np.uint64, endpoint=False))
    b = c.share(g.integers(0, 1 << 64, n, dtype=np.uint64, endpoint=False))
    c.mult(a, b)
    ok, db, dr = measured(c, lambda: c.verify(R=R, kinds=4))
    assert ok
    Rr, npad = rounds_and_pad(n, R)
    want_b, want_r = closed_form(d, [(Rr, npad >> Rr)])
    assert np.array_equal(db[2:], want_b[2:]) and not db[:2].any()
    assert dr == want_r
    # beside the paper's statement (G = npad, a power-of-two multiple of 2^R here)
    off_p, on_p, rounds_p = paper_mult_verify(d, Rr, npad)
    assert db[P.VER_OFF].sum() - off_p == 8 * d * (Rr + 1)
    assert dr[P.VER_ON] == 2 * rounds_p     # an exchange round and a reveal round per step
    # the paper's one-way online count: one direction of every exchange plus three words
    # per reveal of zeta and of Delta; it is one word below this message set's, which also
    # counts Delta's own Pi_PolyEvl exchange (the challenge r's reveal is left out of both)
    one_way = (db[P.VER_ON][1][2] - 32 * (Rr + 2)) + 3 * 8 * d * (Rr + 1)
    assert one_way - on_p == 8 * d


@pytest.mark.parametrize("R", [-1, 0, 2, 4])
def test_inner_and_trunc_verify_messages_closed_form(R):
    """A batch of two Pi_Inner products (one instance over sum K pairs) and a truncation
    pair of 6 outputs in chunks of 4 (instances of 128 T elements)."""
    d = 8
    c = P.Ctx(workloads.master_seed(6), d=d, chunk=4)
    g = np.random.default_rng(40 + R)

    def sh(*shape):
        return c.share(g.integers(0, 1 << 64, shape, dtype=np.uint64, endpoint=False))

    X1, W1 = sh(3, 5), sh(5, 2)
    X2, W2 = sh(2, 9), sh(9, 3)
    pair = c.trunc_pair(6, 13)
    c.inner(X1, W1, pair)
    c.inner(X2, W2)
    ok, db, dr = measured(c, lambda: c.verify(R=R))
    assert ok
    inst = []
    Rr, npad = rounds_and_pad(5 + 9, R)
    inst.append((Rr, npad >> Rr))
    for T in (4, 2):
        Rr, npad = rounds_and_pad(128 * T, R)
        inst.append((Rr, npad >> Rr))
    want_b, want_r = closed_form(d, inst)
    assert np.array_equal(db[2:], want_b[2:]) and not db[:2].any()
    assert dr == want_r
    assert [(lg["R"], lg["npad"] >> lg["R"]) for lg in c.vlog] == inst


def test_reduce_round_cost_against_the_paper():
    """One more Pi_Reduce round adds, per instance, two Pi_PolyEvl and one reveal: 2 x 8d
    offline (the paper: l d) and 7 x 8d + 96 online over both directions (the paper: 5 l d
    one way), while halving the final products."""
    d = 8
    n = 256
    res = {}
    for R in (2, 3):
        c = P.Ctx(workloads.master_seed(8), d=d)
        g = np.random.default_rng(9)
        a = c.share(g.integers(0, 1 << 64, n, dtype=np.uint64, endpoint=False))
        b = c.share(g.integers(0, 1 << 64, n, dtype=np.uint64, endpoint=False))
        c.mult(a, b)
        res[R] = measured(c, lambda: c.verify(R=R, kinds=4))
    w = 8 * d
    d_off = res[3][1][P.VER_OFF].sum() - res[2][1][P.VER_OFF].sum()
    assert d_off == 2 * w - w * ((n >> 2) - (n >> 3))
    d_on = res[3][1][P.VER_ON].sum() - res[2][1][P.VER_ON].sum()
    assert d_on == 7 * w + 96 - 2 * w * ((n >> 2) - (n >> 3))
    assert res[3][2][P.VER_ON] - res[2][2][P.VER_ON] == 2


@pytest.mark.parametrize("to_party", [-1, 0, 1, 2])
def test_reconstruct_messages_per_receiver(to_party):
    """Pi_Rec^{l,k}: party k receives its missing plane (8 bytes per element) and one hash;
    opening to all is the union of the three."""
    n = 10
    c = P.Ctx(workloads.master_seed(9))
    x = np.arange(n, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)
    s = c.share(x)
    b0 = np.array(c.comm, dtype=np.int64)
    assert np.array_equal(c.reconstruct(s, to_party), x)
    db = np.array(c.comm, dtype=np.int64) - b0
    plane_from = {0: 1, 1: 0, 2: 0}          # who sends party k its missing plane
    hash_from = {0: 2, 1: 2, 2: 1}
    want = np.zeros((4, 3, 3), dtype=np.int64)
    for k in ((0, 1, 2) if to_party < 0 else (to_party,)):
        want[P.ONLINE][plane_from[k]][k] += 8 * n
        want[P.ONLINE][hash_from[k]][k] += 32
    assert np.array_equal(db, want)


def test_reconstruct_to_one_party_ignores_messages_it_does_not_receive():
    # an error on P0 -> P2's [r]_1 aborts an opening that P2 takes part in, and is never
    # sent when only P1 receives
    c = P.Ctx(workloads.master_seed(9))
    s = c.share(np.arange(4, dtype=np.uint64))
    c.inject(P.SITE_REC_R1, 1, 5)
    assert np.array_equal(c.reconstruct(s, 1), np.arange(4))
    with pytest.raises(P.Aborted):
        c.reconstruct(s, 2)
