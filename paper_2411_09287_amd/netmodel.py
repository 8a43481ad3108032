"""Network cost model over the communication the library counts (host side, no GPU work).

The paper's experiments simulate three settings (experimental setup, Sec. 5): LAN with a
0.2 ms round-trip time and 1 Gbps, MAN with 12 ms and 100 Mbps, WAN with 80 ms and 40 Mbps.
Its trade-off of the repetition parameter R (Sec. 5.1, verification time against R) weighs
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


def instance_messages(w, R, nR):
    """bytes[phase][src][dst] and rounds[phase] of the verification phases of one instance
    with R Pi_Reduce rounds and nR final pairs of w-byte ring elements (512 in GR(2^64, 64),
    8 in GF(2^64)), from the message list of Sec. 3: R + 2 openings of one element (the
    challenge, every zeta, Delta: P0 -> P2, P0 -> P1, P1 -> P0 w bytes and three 32-byte
    hashes), 2R + 1 Pi_PolyEvl (P0 -> P2 w offline, P1 <-> P2 w each way online), and the
    Pi_Mult of alpha with the nR final elements (w nR offline, w nR each way online)."""
    b = [[[0] * 3 for _ in range(3)] for _ in range(4)]
    rounds = [0, 0, 0, 0]
    b[VERIFY_OFFLINE][0][2] += w * (2 * R + nR + 1)
    for s_, t in ((0, 1), (0, 2), (1, 0)):
        b[VERIFY_ONLINE][s_][t] += w * (R + 2)
    b[VERIFY_ONLINE][2][0] += 32 * (R + 2)
    for s_, t in ((1, 2), (2, 1)):
        b[VERIFY_ONLINE][s_][t] += w * (2 * R + nR + 1) + 32 * (R + 2)
    rounds[VERIFY_ONLINE] += 2 * R + 4
    return b, rounds


def padded_final(n0, R):
    """Final pairs of an instance of n0 pairs after R halvings (zero-padded to 2^R)."""
    return -(-n0 // (1 << R))


def model_r(n0, w, net, gpu_round_s=0.0):
    """The R in 0 .. ceil(log2 n0) of least modelled time for an instance of n0 pairs: the
    verification phases of instance_messages priced by `seconds`, plus R rounds of GPU
    latency (ties to the smaller R).  Returns (R, seconds)."""
    need = (n0 - 1).bit_length() if n0 > 1 else 0
    best = None
    for R in range(0, need + 1):
        b, r = instance_messages(w, R, padded_final(n0, R))
        t = seconds(b, r, (VERIFY_OFFLINE, VERIFY_ONLINE), net) + R * gpu_round_s
        if best is None or t < best[1]:
            best = (R, t)
    return best


def best_r(table, net):
    """table: {R: (gpu_seconds, comm_bytes, rounds)} -> (R, total seconds) minimising the
    GPU time plus the verification phases' network time on `net`."""
    tot = {R: g + seconds(b, r, (VERIFY_OFFLINE, VERIFY_ONLINE), net) for R, (g, b, r) in table.items()}
    R = min(tot, key=tot.get)
    return R, tot[R]
