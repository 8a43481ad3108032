"""Network cost model over the communication the library counts (host side, no GPU work).

The paper's experiments simulate three settings (experimental setup, Sec. 6): LAN with a
0.2 ms round-trip time and 1 Gbps, MAN with 12 ms and 100 Mbps, WAN with 80 ms and 40 Mbps.
Its trade-off of the repetition parameter R (Sec. 6, verification time against R) weighs
the extra rounds of more Pi_Reduce repetitions against the smaller final check.

Model: a phase costs its message rounds times the round-trip time, plus the bytes of its
busiest directed party-to-party link over the bandwidth (the six links of three parties
run in parallel, full duplex).  Bytes and rounds are the counters of `Context.comm_stats()`
(bytes[phase][src][dst], rounds[phase]).
"""

NETWORKS = {
    "LAN": (0.2e-3, 1e9),      # round-trip time (s), bandwidth (bit/s)
    "MAN": (12e-3, 100e6),
    "WAN": (80e-3, 40e6),
}

OFFLINE, ONLINE, VERIFY_OFFLINE, VERIFY_ONLINE = 0, 1, 2, 3


def phase_seconds(link_bytes, rounds, net):
    """Seconds for one phase: link_bytes is a 3 x 3 matrix (src, dst) of bytes."""
    rtt, bw = NETWORKS[net] if isinstance(net, str) else net
    busiest = max(int(link_bytes[s][d]) for s in range(3) for d in range(3) if s != d)
    return rounds * rtt + busiest * 8.0 / bw


def seconds(comm_bytes, rounds, phases, net):
    """Sum of phase_seconds over the given phases (comm_bytes: 4 x 3 x 3, rounds: 4)."""
    return sum(phase_seconds(comm_bytes[p], rounds[p], net) for p in phases)


def diff(after, before):
    """Counter difference of two comm_stats() results (bytes array, rounds list)."""
    (b1, r1), (b0, r0) = after, before
    return b1 - b0, [x - y for x, y in zip(r1, r0)]


def best_r(table, net):
    """table: {R: (gpu_seconds, comm_bytes, rounds)} -> (R, total seconds) minimising the
    GPU time plus the verification phases' network time on `net`."""
    tot = {R: g + seconds(b, r, (VERIFY_OFFLINE, VERIFY_ONLINE), net) for R, (g, b, r) in table.items()}
    R = min(tot, key=tot.get)
    return R, tot[R]
