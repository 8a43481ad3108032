"""Network cost model of the counted communication (host side) and the two sides of the R
trade-off in the oracle's message counts (the paper's experiments, Sec. 5: more Pi_Reduce
repetitions cost rounds and save final-check bytes)."""
import numpy as np
import pytest

from oracle import protocol as P
from paper_2411_09287_amd import netmodel, workloads


def test_phase_seconds_rounds_plus_busiest_link():
    b = np.zeros((3, 3), dtype=np.uint64)
    b[1][2] = 1_000_000          # 8 Mbit on the busiest link
    b[2][1] = 500_000
    b[0][2] = 10
    # LAN: 3 rounds x 0.2 ms + 8e6 bit / 1e9 bit/s
    assert netmodel.phase_seconds(b, 3, "LAN") == pytest.approx(3 * 0.2e-3 + 8e-3)
    # WAN: 3 x 80 ms + 8e6 / 40e6
    assert netmodel.phase_seconds(b, 3, "WAN") == pytest.approx(3 * 80e-3 + 0.2)


def test_best_r_balances_round_trips_against_bytes():
    # a synthetic table: each R adds a round and halves the final-check bytes.  With
    # B bytes at R = 0, the total (R + 2) rtt + 8 B 2^-R / bw is least where one more
    # round (rtt) outweighs the bytes it saves (8 B 2^-(R+1) / bw).
    B = 1 << 24
    table = {}
    for R in range(0, 11):
        b = np.zeros((4, 3, 3), dtype=np.uint64)
        b[netmodel.VERIFY_ONLINE][1][2] = B >> R
        table[R] = (0.0, b, [0, 0, 0, R + 2])
    for net, (rtt, bw) in netmodel.NETWORKS.items():
        R, t = netmodel.best_r(table, net)
        assert rtt >= 8 * (B >> (R + 1)) / bw or R == 10
        assert R == 0 or rtt < 8 * (B >> R) / bw
        assert t == pytest.approx((R + 2) * rtt + 8 * (B >> R) / bw)
    # cheap round trips favour more repetitions
    assert netmodel.best_r(table, "LAN")[0] > netmodel.best_r(table, "WAN")[0]
    # with no bytes at stake the fewest rounds win
    flat = {R: (0.0, np.zeros((4, 3, 3), dtype=np.uint64), [0, 0, 0, R + 2]) for R in range(4)}
    assert netmodel.best_r(flat, "WAN")[0] == 0


def test_oracle_counts_trade_rounds_for_bytes():
    # Pi_MultVerify of 256 triples (d = 8 for speed): rounds grow with R, bytes shrink
    res = {}
    for R in (0, 2, 4, 6):
        c = P.Ctx(workloads.master_seed(7), d=8)
        g = np.random.default_rng(3)
        a = c.share(g.integers(0, 1 << 63, 256, dtype=np.uint64))
        b = c.share(g.integers(0, 1 << 63, 256, dtype=np.uint64))
        c.mult(a, b)
        b0, r0 = np.array(c.comm, dtype=np.int64), list(c.rounds)
        assert c.verify(R=R, kinds=4)
        db = np.array(c.comm, dtype=np.int64) - b0
        dr = [x - y for x, y in zip(c.rounds, r0)]
        res[R] = (int(db[P.VER_OFF].sum() + db[P.VER_ON].sum()), dr[P.VER_OFF] + dr[P.VER_ON])
    Rs = sorted(res)
    assert all(res[x][1] < res[y][1] for x, y in zip(Rs, Rs[1:]))       # more rounds
    assert all(res[x][0] > res[y][0] for x, y in zip(Rs, Rs[1:]))       # fewer bytes
