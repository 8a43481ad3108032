"""The three parties' steps, run one by one in one process (oracle; test infrastructure only).

Shares (Preliminaries, "<.>-sharing"): <v> = (m, [r]_1, [r]_2) with
m = v + [r]_1 + [r]_2; P1 holds (m, [r]_1), P2 holds (m, [r]_2), P0 holds
([r]_1, [r]_2).  A Share below keeps the three planes; each protocol step is
written as the computation of the party that performs it, and every "sent"
message is counted in bytes per (phase, sender, receiver).

Readings of the paper taken here:
  * m = v + r (the Notation section), not the m = v - r of the introduction.
  * Gamma = sum r_x r_y + r_z, shared by P0 with Pi_[.](Gamma): [Gamma]_1 from eta_01,
    [Gamma]_2 = Gamma - [Gamma]_1 sent to P2.
  * Bit shares of Pi_Trunc are <b_1j> = (0, -b, 0) and <b_2j> = (0, 0, -b) so they
    reconstruct to +b under m = v + r; r_z is the arithmetic shift of r_x by t.
  * Both truncation inner products run over all 64 bit positions (weights 0 below
    bit t in the second), so each truncation gives two 64-element gates.
  * Pi_PolyEvl is one-round semi-honest evaluation of a sum of products (Pi_Inner over
    the Galois ring).  Pi_InnerVerify evaluates Delta = sum x'_i y_i + (-alpha) z as one
    Pi_PolyEvl of n + 1 products.
  * Pi_Reduce interpolates h over the nodes {0, 1, x} (x the ring element with
    coefficient vector e_1) instead of {0, 1, 2}: 2 - 0 is not a unit of the Galois
    ring, so h(0), h(1), h(2) do not determine h and the Lagrange weights would need
    a division by 2.  0, 1 and x differ pairwise by units, so the printed Lagrange
    formula applies unchanged; zeta is revealed and used as the point.
  * Pi_BIVerify on an M x K by K x N product uses gate g = m*N + n and the separable
    challenge r^g = (r^N)^m r^n, which compresses the M*N*K-dimensional consolidated
    inner product to a K-dimensional one with an identical claimed value.
  * Dimensions are zero-padded at the tail to a multiple of 2^R.
"""
import hashlib
import math

import numpy as np

from . import prg
from .gr import GR
from .nonlinear import NonlinearMixin
from .ring import ash

U64 = np.uint64
MASK64 = (1 << 64) - 1

OFFLINE, ONLINE, VER_OFF, VER_ON = 0, 1, 2, 3

# Injection sites: an additive error e at one word of one message (tests only).
SITE_INNER_GAMMA2 = 1
SITE_INNER_M1 = 2
SITE_TRUNC_GAMMA2 = 3
SITE_TRUNC_M1 = 4
SITE_MULT_GAMMA2 = 5
SITE_VER_H0_M1 = 6
SITE_VER_H2_GAMMA2 = 7
SITE_VER_DELTA_M1 = 8
SITE_REC_R1 = 9

DEFAULT_CHUNK = 1 << 19     # truncations per Pi_BIVerify instance of the truncation gates
DEFAULT_CHUNK_ROWS = 1 << 14  # edaBit inner products (64-element gates) per Pi_BIVerify instance
DEFAULT_CHUNK_MULT = 1 << 20  # Pi_Mult triples per Pi_MultVerify instance


class Aborted(Exception):
    pass


class Unverified(Exception):
    pass


def neg(a):
    a = np.asarray(a, U64)
    return np.zeros_like(a) - a


class Share:
    """<v> as three planes; any trailing shape (scalars or Galois-ring coefficient vectors)."""

    __slots__ = ("m", "r1", "r2")

    def __init__(self, m, r1, r2):
        self.m = np.asarray(m, U64)
        self.r1 = np.asarray(r1, U64)
        self.r2 = np.asarray(r2, U64)

    def value(self):
        return self.m - self.r1 - self.r2

    def comps(self):
        return (self.m, self.r1, self.r2)

    def map(self, fn):
        return Share(fn(self.m), fn(self.r1), fn(self.r2))

    def __add__(self, o):
        return Share(self.m + o.m, self.r1 + o.r1, self.r2 + o.r2)

    def __sub__(self, o):
        return Share(self.m - o.m, self.r1 - o.r1, self.r2 - o.r2)

    def __getitem__(self, k):
        return Share(self.m[k], self.r1[k], self.r2[k])


def _wt(v):
    """Python int -> uint64 (mod 2^64)."""
    return U64(v & MASK64)


class Ctx(NonlinearMixin):
    def __init__(self, master_seed, d=64, frac_bits=13, chunk=DEFAULT_CHUNK, chunk_rows=DEFAULT_CHUNK_ROWS,
                 chunk_mult=DEFAULT_CHUNK_MULT):
        self.seeds = prg.pair_seeds(master_seed)
        if d < 2:
            raise ValueError("the verification needs d >= 2 (three interpolation nodes)")
        self.gr = GR(d)
        self.d = d
        X = self.gr.var()
        self.inv_x = self.gr.inv(X)
        self.inv_1mx = self.gr.inv(self.gr.sub(self.gr.const(1), X))
        self.inv_xxm1 = self.gr.inv(self.gr.mul(X, self.gr.sub(X, self.gr.const(1))))
        self.frac_bits = frac_bits
        self.chunk = chunk
        self.chunk_rows = chunk_rows
        self.chunk_mult = chunk_mult
        self.op = 0
        self.comm = [[[0] * 3 for _ in range(3)] for _ in range(4)]
        self.rounds = [0, 0, 0, 0]
        self.pending = []
        self.aborted = False
        self.injections = {}
        self.msgs = {}          # last message of each kind (for parity of messages)
        self.vlog = []          # public transcript of each verification instance

    # -- bookkeeping ----------------------------------------------------
    def next_op(self):
        op = self.op
        self.op += 1
        return op

    def G(self, who, tg, n, start=0):
        return prg.words(self.seeds[who], tg, n, start)

    def send(self, phase, src, dst, nbytes):
        self.comm[phase][src][dst] += int(nbytes)

    def inject(self, site, index, e):
        self.injections[site] = (int(index), int(e) & MASK64)

    def _apply(self, site, msg, index_fn=None):
        """Add the pending error for `site` to a message, if its index falls in it."""
        if site not in self.injections:
            return msg
        index, e = self.injections[site]
        flat_index = index if index_fn is None else index_fn(index)
        if flat_index is None or not (0 <= flat_index < msg.size):
            return msg
        del self.injections[site]
        msg = msg.copy()
        flat = msg.reshape(-1)
        flat[flat_index:flat_index + 1] += np.array([e], dtype=U64)
        return msg

    def check(self):
        if self.aborted:
            raise Aborted()

    # ======================================================================
    # Sharing (Preliminaries, "Secret sharing")
    # ======================================================================
    def share(self, x, owner=0):
        """Pi_<.>^{l,k}(x): [r_x] from the pairwise PRGs, the owner sends m = x + r1 + r2."""
        self.check()
        op = self.next_op()
        x = np.asarray(x, U64)
        n = x.size
        s1 = (0, 1) if owner in (0, 1) else (0, 1, 2)
        s2 = (0, 2) if owner in (0, 2) else (0, 1, 2)
        r1 = self.G(s1, prg.tag(op, prg.SHARE_R, 1), n).reshape(x.shape)
        r2 = self.G(s2, prg.tag(op, prg.SHARE_R, 2), n).reshape(x.shape)
        m = x + r1 + r2                                  # computed by the owner
        for dst in (1, 2):
            if dst != owner:
                self.send(ONLINE, owner, dst, 8 * n)
        self.rounds[ONLINE] += 1
        return Share(m, r1, r2)

    def random_gr(self, purpose, op, sub):
        """Pi_<.>^{l[x]} of a random ring element: m from eta_12, [r]_j from eta_0j."""
        d = self.d
        return Share(self.G((1, 2), prg.tag(op, purpose, 0, sub), d),
                     self.G((0, 1), prg.tag(op, purpose, 1, sub), d),
                     self.G((0, 2), prg.tag(op, purpose, 2, sub), d))

    def reveal_gr(self, s, phase=VER_ON):
        """Pi_Rec^{l[x]}: P0 sends [r]_1 to P2 and [r]_2 to P1, P1 sends m to P0,
        hashes cross-check the copies, then v = m - [r]_1 - [r]_2."""
        d = self.d
        self.send(phase, 0, 2, 8 * d)
        self.send(phase, 0, 1, 8 * d)
        self.send(phase, 1, 0, 8 * d)
        self.send(phase, 1, 2, 32)
        self.send(phase, 2, 0, 32)
        self.send(phase, 2, 1, 32)
        self.rounds[phase] += 1
        return s.value()

    # ======================================================================
    # Pi_Inner / Pi_Mult over Z_{2^64} (Fig. "The Inner Product Protocol",
    # Fig. "The Multiplication Protocol", ASTRA-style online formula)
    # ======================================================================
    def inner(self, X, W, pair=None):
        """M x K by K x N product as M*N calls of Pi_Inner (Sec. 4.1, matrix products)."""
        self.check()
        op = self.next_op()
        M, K = X.m.shape
        K2, N = W.m.shape
        assert K == K2
        n = M * N
        # Preprocessing: the output-wire mask [r_Z], and P0's Gamma shared with Pi_[.].
        if pair is None:
            rz1 = self.G((0, 1), prg.tag(op, prg.INNER_RZ, 1), n).reshape(M, N)
            rz2 = self.G((0, 2), prg.tag(op, prg.INNER_RZ, 2), n).reshape(M, N)
        else:
            assert pair["n"] == n
            rx = pair["rx"]
            # Pi_Trunc: P1 sets [r_x]_1 = m_{r_x} - [r_{r_x}]_1, P2 sets [r_x]_2 = -[r_{r_x}]_2.
            rz1 = (rx.m - rx.r1).reshape(M, N)
            rz2 = neg(rx.r2).reshape(M, N)
        # P0
        RX = X.r1 + X.r2
        RW = W.r1 + W.r2
        gamma = RX @ RW + rz1 + rz2
        g1 = self.G((0, 1), prg.tag(op, prg.INNER_GAMMA, 1), n).reshape(M, N)
        g2 = self._apply(SITE_INNER_GAMMA2, gamma - g1)            # P0 -> P2
        self.send(OFFLINE, 0, 2, 8 * n)
        self.rounds[OFFLINE] += 1
        # Online: P1 and P2 evaluate their part and exchange it.
        m1 = neg(X.m @ W.r1) - X.r1 @ W.m + g1                     # P1
        m2 = X.m @ W.m - X.m @ W.r2 - X.r2 @ W.m + g2              # P2
        m1 = self._apply(SITE_INNER_M1, m1)                        # P1 -> P2
        self.send(ONLINE, 1, 2, 8 * n)
        self.send(ONLINE, 2, 1, 8 * n)
        self.rounds[ONLINE] += 1
        Z = Share(m1 + m2, rz1, rz2)
        self.msgs["inner"] = {"gamma2": g2, "m1": m1, "m2": m2}
        self.pending.append(("inner", X, W, Z))
        return Z

    def mult(self, a, b, phase_on=ONLINE):
        """Pi_Mult on equal-shaped arrays of shares (elementwise).  phase_on: the counter
        phase of the P1 <-> P2 exchange (OFFLINE for input-independent preprocessing)."""
        self.check()
        op = self.next_op()
        n = a.m.size
        shp = a.m.shape
        rz1 = self.G((0, 1), prg.tag(op, prg.MULT_RZ, 1), n).reshape(shp)
        rz2 = self.G((0, 2), prg.tag(op, prg.MULT_RZ, 2), n).reshape(shp)
        gamma = (a.r1 + a.r2) * (b.r1 + b.r2) + rz1 + rz2           # P0
        g1 = self.G((0, 1), prg.tag(op, prg.MULT_GAMMA, 1), n).reshape(shp)
        g2 = self._apply(SITE_MULT_GAMMA2, gamma - g1)
        self.send(OFFLINE, 0, 2, 8 * n)
        self.rounds[OFFLINE] += 1
        m1 = neg(a.m * b.r1) - b.m * a.r1 + g1                      # P1
        m2 = a.m * b.m - a.m * b.r2 - b.m * a.r2 + g2               # P2
        self.send(phase_on, 1, 2, 8 * n)
        self.send(phase_on, 2, 1, 8 * n)
        self.rounds[phase_on] += 1
        c = Share(m1 + m2, rz1, rz2)
        self.msgs["mult"] = {"gamma2": g2, "m1": m1, "m2": m2}
        self.pending.append(("mult", a, b, c))
        return c

    def _inner_rows(self, xs, ys, op, p_r, p_g, site_g2=None, site_m1=None, phase_off=OFFLINE,
                    phase_on=OFFLINE):
        """Batched Pi_Inner: row p of xs and ys is one inner product; fresh output masks."""
        n = xs.m.shape[0]
        r1 = self.G((0, 1), prg.tag(op, p_r, 1), n)
        r2 = self.G((0, 2), prg.tag(op, p_r, 2), n)
        gamma = ((xs.r1 + xs.r2) * (ys.r1 + ys.r2)).sum(axis=1, dtype=U64) + r1 + r2   # P0
        g1 = self.G((0, 1), prg.tag(op, p_g, 1), n)
        g2 = gamma - g1
        if site_g2 is not None:
            g2 = self._apply(site_g2, g2)
        self.send(phase_off, 0, 2, 8 * n)
        m1 = (neg(xs.m * ys.r1) - ys.m * xs.r1).sum(axis=1, dtype=U64) + g1            # P1
        m2 = (xs.m * ys.m - xs.m * ys.r2 - ys.m * xs.r2).sum(axis=1, dtype=U64) + g2   # P2
        if site_m1 is not None:
            m1 = self._apply(site_m1, m1)
        self.send(phase_on, 1, 2, 8 * n)
        self.send(phase_on, 2, 1, 8 * n)
        return Share(m1 + m2, r1, r2)

    # ======================================================================
    # Pi_Trunc (Fig. "The maliciously secure truncation protocol")
    # ======================================================================
    @staticmethod
    def trunc_weights(t):
        """Weights of the two inner products: x-gate 2^{j+1}, z-gate 2 c_j (both negated onto <b_1j>)."""
        wx = [(-(1 << (j + 1))) & MASK64 for j in range(64)]
        c = [0] * 64
        for j in range(t, 63):
            c[j] = 1 << (j - t)
        c[63] = (-(1 << (63 - t))) & MASK64
        wz = [(-2 * c[j]) & MASK64 for j in range(64)]
        return np.array(wx, dtype=U64), np.array(wz, dtype=U64), np.array([v & MASK64 for v in c], dtype=U64)

    def trunc_gates(self, op, n, t):
        """Per truncation output p: the bit shares and the two 64-element gates (x, y) pairs."""
        B1 = self.G((0, 1), prg.tag(op, prg.TRUNC_B, 1), n)       # P0 and P1
        B2 = self.G((0, 2), prg.tag(op, prg.TRUNC_B, 2), n)       # P0 and P2
        j = np.arange(64, dtype=U64)
        b1 = (B1[:, None] >> j) & U64(1)
        b2 = (B2[:, None] >> j) & U64(1)
        zero = np.zeros((n, 64), dtype=U64)
        sb1 = Share(zero, neg(b1), zero)       # <b_1j> = (0, -b, 0)
        sb2 = Share(zero, zero, neg(b2))       # <b_2j> = (0, 0, -b)
        wx, wz, c = self.trunc_weights(t)
        ones = (np.ones(64, dtype=U64) << j)   # 2^j
        xg = sb1.map(lambda a: a * wx)         # x_j = -2^{j+1} <b_1j>
        zg = sb1.map(lambda a: a * wz)         # x_j = -2 c_j <b_1j>
        return B1, B2, sb1, sb2, xg, zg, ones, c

    def trunc_pair(self, n, t):
        """Preprocessing of Pi_Trunc^t for n outputs: <r_x> and <r_z> = <ash(r_x, t)>."""
        self.check()
        op = self.next_op()
        B1, B2, sb1, sb2, xg, zg, ones, c = self.trunc_gates(op, n, t)
        wx_ = self._inner_rows(xg, sb2, op, prg.TRUNC_WX_R, prg.TRUNC_WX_GAMMA,
                               site_g2=SITE_TRUNC_GAMMA2)
        wz_ = self._inner_rows(zg, sb2, op, prg.TRUNC_WZ_R, prg.TRUNC_WZ_GAMMA,
                               site_m1=SITE_TRUNC_M1)
        self.rounds[OFFLINE] += 1
        lin_x = (sb1 + sb2).map(lambda a: (a * ones).sum(axis=1, dtype=U64))   # sum 2^j (<b1>+<b2>)
        lin_z = (sb1 + sb2).map(lambda a: (a * c).sum(axis=1, dtype=U64))      # sum c_j (<b1>+<b2>)
        rx = lin_x + wx_
        rz = lin_z + wz_
        pair = {"op": op, "n": n, "t": t, "rx": rx, "rz": rz, "wx": wx_, "wz": wz_,
                "r_x_p0": B1 ^ B2, "r_z_p0": ash(B1 ^ B2, t)}
        self.pending.append(("trunc", pair))
        return pair

    def trunc(self, pair, Z):
        """Online Pi_Trunc: m' = ash(m, t) locally; the output mask is <r_z>'s [.] form."""
        self.check()
        t = pair["t"]
        rz = pair["rz"]
        shp = Z.m.shape
        return Share(ash(Z.m, t), (rz.m - rz.r1).reshape(shp), neg(rz.r2).reshape(shp))

    # ======================================================================
    # Verification over the Galois ring (Sec. 3)
    # ======================================================================
    def poly_evl(self, a, b, op, p_r, p_g, sub, site_m1=None, site_g2=None, tr=None):
        """Pi_PolyEvl reading: semi-honest one-round sum_i a_i * b_i over GR with a fresh mask."""
        gr, d = self.gr, self.d
        rc1 = self.G((0, 1), prg.tag(op, p_r, 1, sub), d)
        rc2 = self.G((0, 2), prg.tag(op, p_r, 2, sub), d)
        gamma = gr.dot(a.r1 + a.r2, b.r1 + b.r2) + rc1 + rc2                   # P0
        g1 = self.G((0, 1), prg.tag(op, p_g, 1, sub), d)
        g2 = gamma - g1
        if site_g2 is not None:
            g2 = self._apply(site_g2[0], g2, site_g2[1])
        self.send(VER_OFF, 0, 2, 8 * d)
        m1 = neg(gr.dot(a.m, b.r1)) - gr.dot(b.m, a.r1) + g1                   # P1
        m2 = gr.dot(a.m, b.m) - gr.dot(a.m, b.r2) - gr.dot(b.m, a.r2) + g2     # P2
        if site_m1 is not None:
            m1 = self._apply(site_m1[0], m1, site_m1[1])
        self.send(VER_ON, 1, 2, 8 * d)
        self.send(VER_ON, 2, 1, 8 * d)
        if tr is not None:
            tr.update({"gamma2": g2, "m1": m1, "m2": m2})
        return Share(m1 + m2, rc1, rc2)

    def reduce_round(self, x, y, z, op, s, k, log):
        """Pi_Reduce (Fig. "The Inner Product Dimension Reduction Protocol"), n -> n/2."""
        gr = self.gr
        sub = (s << 8) | k
        f0, f1 = x[0::2], x[1::2]
        g0, g1 = y[0::2], y[1::2]
        X, Xm1 = gr.var(), gr.sub(gr.var(), gr.const(1))

        def at_x(v0, v1):         # the line through (0, v0), (1, v1) at the node x
            return gr.mul(X, v1) - gr.mul(Xm1, v0)

        f2 = Share(*[at_x(a, b) for a, b in zip(f0.comps(), f1.comps())])
        g2 = Share(*[at_x(a, b) for a, b in zip(g0.comps(), g1.comps())])

        def site(idx):
            return idx & 0xFF if (idx >> 16) == s and ((idx >> 8) & 0xFF) == k else None

        t0, t2 = {}, {}
        h0 = self.poly_evl(f0, g0, op, prg.VER_H0_R, prg.VER_H0_GAMMA, sub,
                           site_m1=(SITE_VER_H0_M1, site), tr=t0)
        h2 = self.poly_evl(f2, g2, op, prg.VER_H2_R, prg.VER_H2_GAMMA, sub,
                           site_g2=(SITE_VER_H2_GAMMA2, site), tr=t2)
        self.rounds[VER_ON] += 1
        h1 = z - h0
        zeta = self.reveal_gr(self.random_gr(prg.VER_ZETA, op, sub))
        # Lagrange weights over the nodes {0, 1, x}; every denominator is a unit.
        one, X = gr.const(1), gr.var()
        zm1, zmx = gr.sub(zeta, one), gr.sub(zeta, X)
        L0 = gr.mul(gr.mul(zm1, zmx), self.inv_x)                 # (z-1)(z-x) / ((0-1)(0-x))
        L1 = gr.mul(gr.mul(zeta, zmx), self.inv_1mx)              # z(z-x) / ((1-0)(1-x))
        L2 = gr.mul(gr.mul(zeta, zm1), self.inv_xxm1)             # z(z-1) / ((x-0)(x-1))

        def at_tau(v0, v1):       # f(zeta) = zeta * f(1) - (zeta - 1) * f(0)
            return gr.mul(zeta, v1) - gr.mul(zm1, v0)

        xn = Share(*[at_tau(a, b) for a, b in zip(f0.comps(), f1.comps())])
        yn = Share(*[at_tau(a, b) for a, b in zip(g0.comps(), g1.comps())])
        zn = Share(*[gr.mul(L0, a) + gr.mul(L1, b) + gr.mul(L2, c)
                     for a, b, c in zip(h0.comps(), h1.comps(), h2.comps())])
        log["rounds"].append({"zeta": zeta, "h0": t0, "h2": t2,
                              "h0_share": h0, "h2_share": h2})
        return xn, yn, zn

    def inner_verify(self, x, y, z, op, s, log):
        """Pi_InnerVerify (Fig. "The Inner Product Verification Protocol")."""
        gr, d = self.gr, self.d
        n = x.m.shape[0]
        alpha = self.random_gr(prg.VER_ALPHA, op, s)
        # <x'_i> = Pi_Mult over GR of <x_i> and <alpha>, fresh masks per element.
        r1 = self.G((0, 1), prg.tag(op, prg.VER_XP_R, 1, s), n * d).reshape(n, d)
        r2 = self.G((0, 2), prg.tag(op, prg.VER_XP_R, 2, s), n * d).reshape(n, d)
        gamma = gr.mul(x.r1 + x.r2, alpha.r1 + alpha.r2) + r1 + r2            # P0
        g1 = self.G((0, 1), prg.tag(op, prg.VER_XP_GAMMA, 1, s), n * d).reshape(n, d)
        g2 = gamma - g1
        self.send(VER_OFF, 0, 2, 8 * n * d)
        m1 = neg(gr.mul(x.m, alpha.r1)) - gr.mul(alpha.m, x.r1) + g1          # P1
        m2 = gr.mul(x.m, alpha.m) - gr.mul(x.m, alpha.r2) - gr.mul(alpha.m, x.r2) + g2   # P2
        self.send(VER_ON, 1, 2, 8 * n * d)
        self.send(VER_ON, 2, 1, 8 * n * d)
        self.rounds[VER_ON] += 1
        xp = Share(m1 + m2, r1, r2)
        # <Delta> = sum <x'_i><y_i> + <-alpha><z>, one Pi_PolyEvl of n + 1 products.
        A = Share(*[np.concatenate([a, neg(b)[None]]) for a, b in zip(xp.comps(), alpha.comps())])
        B = Share(*[np.concatenate([a, b[None]]) for a, b in zip(y.comps(), z.comps())])

        def site(idx):
            return idx & 0xFF if (idx >> 16) == s else None

        td = {}
        delta = self.poly_evl(A, B, op, prg.VER_DELTA_R, prg.VER_DELTA_GAMMA, s,
                              site_m1=(SITE_VER_DELTA_M1, site), tr=td)
        self.rounds[VER_ON] += 1
        dv = self.reveal_gr(delta)
        log["delta"] = dv
        log["delta_tr"] = td
        log["xp"] = xp
        return not np.any(dv)

    @staticmethod
    def auto_rounds(n0, R):
        need = max(0, math.ceil(math.log2(n0))) if n0 > 1 else 0
        if R is None or R < 0:
            R = max(0, need - 3)
        return min(R, need)

    def fold_and_check(self, x, y, z, op, s, R, log):
        """Zero-pad to a multiple of 2^R, R x Pi_Reduce, then Pi_InnerVerify."""
        n0 = x.m.shape[0]
        R = self.auto_rounds(n0, R)
        npad = -(-n0 // (1 << R)) * (1 << R)
        if npad != n0:
            pad = np.zeros((npad - n0, self.d), dtype=U64)
            x = x.map(lambda a: np.concatenate([a, pad]))
            y = y.map(lambda a: np.concatenate([a, pad]))
        log.update({"R": R, "n0": n0, "npad": npad, "rounds": []})
        for k in range(R):
            x, y, z = self.reduce_round(x, y, z, op, s, k, log)
        return self.inner_verify(x, y, z, op, s, log)

    def challenge(self, op, s, log):
        r = self.reveal_gr(self.random_gr(prg.VER_R, op, s))
        log["r"] = r
        return r

    # -- building the Galois-ring instance for each kind of pending triple ----
    @staticmethod
    def _inner_offsets(items):
        """Gate offsets o_l of a batch of Pi_Inner products: gate (m, n) of product l is
        i = o_l + n M_l + m (column-major inside a product, products in call order)."""
        offs, o = [], 0
        for X, W, Z in items:
            offs.append(o)
            o += X.m.shape[0] * W.m.shape[1]
        return offs

    def instance_inner_compressed(self, items, r):
        """One Pi_BIVerify instance for a batch of Pi_Inner products, gate i weighted by r^i
        on the x side.  With i = o_l + n M_l + m the weight factors as
        r^{o_l} * r^m * (r^{M_l})^n, so product l contributes the K_l pairs
            x_k = r^{o_l} sum_m r^m X[m,k],   y_k = sum_n (r^{M_l})^n W[k,n]
        and z = sum_l r^{o_l} sum_{m,n} r^m (r^{M_l})^n Z[m,n]."""
        gr = self.gr
        offs = self._inner_offsets(items)
        xs, ys = [[], [], []], [[], [], []]
        zs = [np.zeros(self.d, dtype=U64) for _ in range(3)]
        for (X, W, Z), o in zip(items, offs):
            M, K = X.m.shape
            N = W.m.shape[1]
            rho = gr.powers(r, M)                       # r^m
            sigma = gr.powers(gr.pow(r, M), N)          # (r^M)^n
            c = gr.pow(r, o)                            # r^{o_l}
            for q, (Xc, Wc, Zc) in enumerate(zip(X.comps(), W.comps(), Z.comps())):
                xs[q].append(gr.mul(c[None, :], Xc.T @ rho))
                ys[q].append(Wc @ sigma)
                zs[q] = zs[q] + gr.mul(c, gr.dot(sigma, Zc.T @ rho))
        return (Share(*[np.concatenate(v) for v in xs]), Share(*[np.concatenate(v) for v in ys]), Share(*zs))

    def instance_inner_literal(self, items, r):
        """The same batch as printed: every gate i = o_l + n M_l + m lifted and weighted by
        r^i, consolidated to M_l N_l K_l pairs per product."""
        gr = self.gr
        offs = self._inner_offsets(items)
        total = offs[-1] + items[-1][0].m.shape[0] * items[-1][1].m.shape[1]
        pw = gr.powers(r, total)
        xs, ys, zs = [[], [], []], [[], [], []], [np.zeros(self.d, dtype=U64) for _ in range(3)]
        for (X, W, Z), o in zip(items, offs):
            M, K = X.m.shape
            N = W.m.shape[1]
            for c in range(3):
                Xc, Wc, Zc = X.comps()[c], W.comps()[c], Z.comps()[c]
                xe = np.zeros((M * N * K, self.d), dtype=U64)
                ye = np.zeros((M * N * K, self.d), dtype=U64)
                for n in range(N):
                    for m in range(M):
                        i = o + n * M + m
                        for k in range(K):
                            xe[((n * M) + m) * K + k] = gr.scale(Xc[m, k], pw[i])
                            ye[((n * M) + m) * K + k] = gr.const(Wc[k, n])
                        zs[c] = zs[c] + gr.scale(Zc[m, n], pw[i])
                xs[c].append(xe)
                ys[c].append(ye)
        return (Share(*[np.concatenate(v) for v in xs]), Share(*[np.concatenate(v) for v in ys]), Share(*zs))

    def instance_trunc(self, pair, lo, hi, r):
        """Pi_BIVerify of the truncation gates of outputs [lo, hi): 128 elements per output."""
        gr = self.gr
        op, t = pair["op"], pair["t"]
        n = pair["n"]
        _, _, sb1, sb2, xg, zg, _, _ = self.trunc_gates(op, n, t)
        T = hi - lo
        pw = gr.powers(r, 2 * T)
        xs, ys, zs = [], [], []
        for comp in range(3):
            xa = np.concatenate([xg.comps()[comp][lo:hi, None, :], zg.comps()[comp][lo:hi, None, :]], axis=1)
            ya = np.concatenate([sb2.comps()[comp][lo:hi, None, :]] * 2, axis=1)
            # element (p, s, j): gate g = 2 (p - lo) + s, weight r^g on the x side
            xe = gr.scale(xa.reshape(2 * T, 64), pw[:, None, :]).reshape(T * 128, self.d)
            ye = gr.const(ya.reshape(T * 128))
            w = np.stack([pair["wx"].comps()[comp][lo:hi], pair["wz"].comps()[comp][lo:hi]], axis=1)
            ze = gr.scale(w.reshape(2 * T), pw).sum(axis=0, dtype=U64)
            xs.append(xe)
            ys.append(ye)
            zs.append(ze)
        return Share(*xs), Share(*ys), Share(*zs)

    def instance_mult(self, a, b, c, r, lo=0, hi=None):
        """Pi_Tran (Fig. "Compression of Multiplication Triples") of triples [lo, hi)."""
        gr = self.gr
        hi = a.m.size if hi is None else hi
        pw = gr.powers(r, hi - lo)
        x = Share(*[gr.scale(v.reshape(-1)[lo:hi], pw) for v in a.comps()])
        y = Share(*[gr.const(v.reshape(-1)[lo:hi]) for v in b.comps()])
        z = Share(*[gr.scale(v.reshape(-1)[lo:hi], pw).sum(axis=0, dtype=U64) for v in c.comps()])
        return x, y, z

    KIND = {"inner": 1, "trunc": 2, "mult": 4, "rows": 8, "and": 8}

    def verify(self, R=-1, literal=False, kinds=15):
        """Post-processing: one Pi_BIVerify for all pending Pi_Inner products (first), then
        in call order the truncation gates in chunks, one Pi_MultVerify per Pi_Mult call,
        (in chunks of triples), the edaBit inner products in chunks, and one Pi_MultVerify over GF(2^d) per layer
        call's Boolean triples; abort unless every Delta is 0.  `kinds` selects which
        pending products are verified now (1 inner, 2 trunc, 4 mult, 8 the non-linear
        layers' edaBit inner products and Boolean triples)."""
        self.check()
        op = self.next_op()
        ok = True
        s = 0
        self.vlog = []
        selected = [it for it in self.pending if self.KIND[it[0]] & kinds]
        rest = [it for it in self.pending if not self.KIND[it[0]] & kinds]
        inner = [it[1:] for it in selected if it[0] == "inner"]
        if inner:
            log = {"kind": "inner", "s": s}
            r = self.challenge(op, s, log)
            inst = self.instance_inner_literal if literal else self.instance_inner_compressed
            x, y, z = inst(inner, r)
            log["z"] = z
            ok &= self.fold_and_check(x, y, z, op, s, R, log)
            self.vlog.append(log)
            s += 1
        for item in selected:
            if item[0] == "inner":
                continue
            if item[0] == "trunc":
                pair = item[1]
                for lo in range(0, pair["n"], self.chunk):
                    hi = min(pair["n"], lo + self.chunk)
                    log = {"kind": "trunc", "s": s, "lo": lo, "hi": hi}
                    r = self.challenge(op, s, log)
                    x, y, z = self.instance_trunc(pair, lo, hi, r)
                    log["z"] = z
                    ok &= self.fold_and_check(x, y, z, op, s, R, log)
                    self.vlog.append(log)
                    s += 1
            elif item[0] == "rows":
                _, xs, ys, zs = item
                for lo in range(0, xs.m.shape[0], self.chunk_rows):
                    hi = min(xs.m.shape[0], lo + self.chunk_rows)
                    log = {"kind": "rows", "s": s, "lo": lo, "hi": hi}
                    r = self.challenge(op, s, log)
                    x, y, z = self.instance_rows(xs, ys, zs, lo, hi, r)
                    log["z"] = z
                    ok &= self.fold_and_check(x, y, z, op, s, R, log)
                    self.vlog.append(log)
                    s += 1
            elif item[0] == "and":
                log = {"kind": "and", "s": s}
                ok &= self.verify_and_item(item[1], op, s, R, log)
                self.vlog.append(log)
                s += 1
            else:
                _, a, b, c = item
                n = a.m.size
                for lo in range(0, max(n, 1), self.chunk_mult):
                    hi = min(n, lo + self.chunk_mult)
                    log = {"kind": "mult", "s": s, "lo": lo, "hi": hi}
                    r = self.challenge(op, s, log)
                    x, y, z = self.instance_mult(a, b, c, r, lo, hi)
                    log["z"] = z
                    ok &= self.fold_and_check(x, y, z, op, s, R, log)
                    self.vlog.append(log)
                    s += 1
        self.pending = rest
        if not ok:
            self.aborted = True
        return bool(ok)

    # ======================================================================
    # Pi_Rec (Preliminaries, "Verifiability of share reconstruction")
    # ======================================================================
    def reconstruct(self, X, to_party=-1):
        """Pi_Rec^{l} to every party (to_party < 0) or Pi_Rec^{l,k} to party k alone.
        Each party lacks one plane: P0 gets m from P1 (P2 sends H(m)), P1 gets [r]_2 from
        P0 (P2 sends H([r]_2)), P2 gets [r]_1 from P0 (P1 sends H([r]_1)); a receiver
        whose copy disagrees with the hash aborts before anything is opened."""
        self.check()
        if self.pending:
            raise Unverified()
        n = X.m.size
        receivers = (0, 1, 2) if to_party < 0 else (to_party,)

        def H(a):
            return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).digest()

        ok = True
        if 2 in receivers:
            to_p2 = self._apply(SITE_REC_R1, X.r1.copy())        # P0 -> P2: [r]_1
            ok &= H(to_p2) == H(X.r1)                            # against P1's hash of it
            self.send(ONLINE, 0, 2, 8 * n)
            self.send(ONLINE, 1, 2, 32)
        if 1 in receivers:
            to_p1 = X.r2.copy()                                  # P0 -> P1: [r]_2
            ok &= H(to_p1) == H(X.r2)                            # against P2's hash of it
            self.send(ONLINE, 0, 1, 8 * n)
            self.send(ONLINE, 2, 1, 32)
        if 0 in receivers:
            to_p0 = X.m.copy()                                   # P1 -> P0: m
            ok &= H(to_p0) == H(X.m)                             # against P2's hash of it
            self.send(ONLINE, 1, 0, 8 * n)
            self.send(ONLINE, 2, 0, 32)
        self.rounds[ONLINE] += 1
        if not ok:
            self.aborted = True
            raise Aborted()
        return X.m - X.r1 - X.r2
