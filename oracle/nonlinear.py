"""Non-linear layers: edaBits, daBits, bit extraction, B2A, ReLU and 2x2 max pooling, with
the Boolean multiplications verified over GF(2^d) (oracle; test infrastructure only).

Sec. 4.3 ("Secure Non-linear Function Evaluation") and Fig. "The maliciously edaBits
generation".  Boolean shares <v>^1 = (m, [r]_1, [r]_2) with m = v XOR r1 XOR r2 (the
Notation's m = v + r over Z_2) are stored bit-sliced: one uint64 word per plane holds 64
Boolean values, and for a 64-bit ring value its bits x[0..63] sit in one word, bit i = x[i].

Readings of the paper taken here (each a place where it is silent or ambiguous):
  * The arithmetic bit shares of the figure, <b_i,1> = (0, b, 0) and <b_i,2> = (0, 0, b),
    open to -b under m = v + r; they are taken as (0, -b, 0) and (0, 0, -b) so that they
    open to +b (the same reading as for the truncation bits).  <m_i> = (m_i, 0, 0) opens to
    +m_i as printed.
  * The second multiplication of the edaBits figure is "combined with a single inner
    product": <r> = sum_i 2^i (<m_i> + <r'_i>) - Pi_Inner(x_i = 2^(i+1) <m_i>, y_i = <r'_i>)
    over the 64 bit positions, one 64-element gate per edaBit, verified as a Pi_BIVerify
    instance of such gates.
  * Bit extraction adds the opened Delta = x - r to r's Boolean bits with a parallel-prefix
    (Kogge-Stone) carry: generate g = Delta AND r and propagate p = Delta XOR r are local
    (Delta is public), and each of the six levels k = 1, 2, 4, ..., 32 takes
    G <- G XOR (P AND (G << k)), P <- P AND (P << k) (the last level only G): one Boolean
    Pi_Mult round per level on whole words.  Only the top bit is needed by the comparisons:
    msb(x) = Delta_63 XOR r_63 XOR carry_63, the carry being bit 62 of the final G.
  * B2A of a bit d with a daBit (<s>^l, <s>^1): e = d XOR s is opened (Pi_Rec over Z_2) and
    <d>^l = e + (1 - 2e) <s>^l, the paper's Delta + r - 2 Delta r with Delta public.
  * ReLU(x) = x * (1 - msb(x)) (a Pi_Mult of x with the converted bit); the maximum of two
    values is q + ReLU(p - q); 2x2 max pooling takes the maximum of the two row pairs, then
    of the two results.
  * Pi_Mult over Z_2 is the Pi_Mult figure with XOR for + and -, AND for the product.
  * The Z_2 triples are verified by Pi_MultVerify over GR(2, d) = GF(2^d) (Sec. 4.3, last
    paragraph): the Sec. 3 machinery with XOR for + and -, the carry-less product modulo f
    for the product, the interpolation nodes {0, 1, x} (units apart in the field), gate
    g = 64 * word + bit weighted by r^g.
"""
import numpy as np

from . import prg
from .gf2 import GF

U64 = np.uint64
MASK64 = (1 << 64) - 1

# keystream purposes (beside those of the linear path)
EDA_BITS = 32
DA_BITS = 33
AND_RZ = 34
AND_GAMMA = 35
EDA_W_R = 36
EDA_W_GAMMA = 37

SITE_AND_GAMMA2 = 10      # P0 -> P2 [Gamma]_2 of a Boolean Pi_Mult; index = word, error XORed
SITE_EDA_W_M1 = 11        # P1 -> P2 [m]_1 of the edaBits inner products; index = edaBit

LEVELS = (1, 2, 4, 8, 16, 32)


class BShare:
    """<v>^1, bit-sliced: m = v ^ r1 ^ r2 per word (64 Boolean values per word)."""

    __slots__ = ("m", "r1", "r2")

    def __init__(self, m, r1, r2):
        self.m = np.asarray(m, U64)
        self.r1 = np.asarray(r1, U64)
        self.r2 = np.asarray(r2, U64)

    def value(self):
        return self.m ^ self.r1 ^ self.r2

    def comps(self):
        return (self.m, self.r1, self.r2)

    def map(self, fn):
        return BShare(fn(self.m), fn(self.r1), fn(self.r2))

    def __xor__(self, o):
        return BShare(self.m ^ o.m, self.r1 ^ o.r1, self.r2 ^ o.r2)

    def xor_pub(self, c):
        """XOR of a public word: it enters m only."""
        return BShare(self.m ^ np.asarray(c, U64), self.r1, self.r2)

    def and_pub(self, c):
        """AND with a public word: every plane."""
        c = np.asarray(c, U64)
        return BShare(self.m & c, self.r1 & c, self.r2 & c)

    def __getitem__(self, k):
        return BShare(self.m[k], self.r1[k], self.r2[k])


def bcat(parts):
    return BShare(*[np.concatenate([p.comps()[c] for p in parts]) for c in range(3)])


def _bits(words):
    """uint64 words -> (n, 64) array of their bits, bit i in column i."""
    j = np.arange(64, dtype=U64)
    return (np.asarray(words, U64)[:, None] >> j) & U64(1)


class NonlinearMixin:
    """Methods of the oracle context for the non-linear layers.  They use the context's
    PRG (self.G), counters (self.send, self.rounds), Pi_Mult (self.mult) and its batched
    row inner products (self._inner_rows)."""

    # ------------------------------------------------------------------
    # Pi_Mult over Z_2 on words (64 AND gates per word)
    # ------------------------------------------------------------------
    def and_words(self, a, b, item):
        """<a AND b>^1 with a fresh output mask; the triple is appended to `item` (the
        pending record of the calling layer)."""
        from .protocol import OFFLINE, ONLINE
        op = self.next_op()
        n = a.m.size
        rz1 = self.G((0, 1), prg.tag(op, AND_RZ, 1), n)
        rz2 = self.G((0, 2), prg.tag(op, AND_RZ, 2), n)
        gamma = ((a.r1 ^ a.r2) & (b.r1 ^ b.r2)) ^ rz1 ^ rz2                 # P0
        g1 = self.G((0, 1), prg.tag(op, AND_GAMMA, 1), n)
        g2 = self._apply_xor(SITE_AND_GAMMA2, gamma ^ g1)                   # P0 -> P2
        self.send(OFFLINE, 0, 2, 8 * n)
        self.rounds[OFFLINE] += 1
        m1 = (a.m & b.r1) ^ (b.m & a.r1) ^ g1                               # P1
        m2 = (a.m & b.m) ^ (a.m & b.r2) ^ (b.m & a.r2) ^ g2                 # P2
        self.send(ONLINE, 1, 2, 8 * n)
        self.send(ONLINE, 2, 1, 8 * n)
        self.rounds[ONLINE] += 1
        c = BShare(m1 ^ m2, rz1, rz2)
        item["triples"].append((a, b, c))
        self.msgs["and"] = {"gamma2": g2, "m1": m1, "m2": m2}
        return c

    def _apply_xor(self, site, msg):
        if site not in self.injections:
            return msg
        index, e = self.injections[site]
        if not 0 <= index < msg.size:
            return msg
        del self.injections[site]
        msg = msg.copy()
        msg.reshape(-1)[index] ^= U64(e)
        return msg

    # ------------------------------------------------------------------
    # Preprocessing: edaBits and daBits (Fig. "The maliciously edaBits generation")
    # ------------------------------------------------------------------
    def edabits(self, n):
        """n edaBits: (<r>^l, <r[0..63]>^1 as one word per edaBit)."""
        from .protocol import OFFLINE, Share, neg
        self.check()
        op = self.next_op()
        B1 = self.G((0, 1), prg.tag(op, EDA_BITS, 1), n)        # P0 and P1
        B2 = self.G((0, 2), prg.tag(op, EDA_BITS, 2), n)        # P0 and P2
        Mb = self.G((1, 2), prg.tag(op, EDA_BITS, 0), n)        # P1 and P2
        b1, b2, mb = _bits(B1), _bits(B2), _bits(Mb)
        zero = np.zeros((n, 64), U64)
        sb1 = Share(zero, neg(b1), zero)                        # opens to +b_i,1
        sb2 = Share(zero, zero, neg(b2))                        # opens to +b_i,2
        smb = Share(mb, zero, zero)                             # opens to +m_i
        prod = self.mult(sb1, sb2, phase_on=OFFLINE)            # <b_i,1 b_i,2>
        rp = (sb1 + sb2) - prod.map(lambda a: a * U64(2))       # <r'_i> = <b1 XOR b2>
        j = np.arange(64, dtype=U64)
        w2 = (np.ones(64, U64) << (j + U64(1)))                 # 2^(i+1) (0 at i = 63)
        xs = smb.map(lambda a: a * w2)
        w = self._inner_rows(xs, rp, op, EDA_W_R, EDA_W_GAMMA, site_m1=SITE_EDA_W_M1)
        self.rounds[OFFLINE] += 1
        self.pending.append(("rows", xs, rp, w))
        pow2 = np.ones(64, U64) << j
        lin = (smb + rp).map(lambda a: (a * pow2).sum(axis=1, dtype=U64))
        r = lin - w
        return r, BShare(Mb, B1, B2)

    def dabits(self, n):
        """n daBits: (<s>^l, <s>^1 in bit 0 of one word each), s a random bit."""
        from .protocol import OFFLINE, Share, neg
        self.check()
        op = self.next_op()
        b1 = self.G((0, 1), prg.tag(op, DA_BITS, 1), n) & U64(1)
        b2 = self.G((0, 2), prg.tag(op, DA_BITS, 2), n) & U64(1)
        mb = self.G((1, 2), prg.tag(op, DA_BITS, 0), n) & U64(1)
        zero = np.zeros(n, U64)
        sb1, sb2, smb = Share(zero, neg(b1), zero), Share(zero, zero, neg(b2)), Share(mb, zero, zero)
        p1 = self.mult(sb1, sb2, phase_on=OFFLINE)
        rp = (sb1 + sb2) - p1.map(lambda a: a * U64(2))         # b1 XOR b2
        p2 = self.mult(smb, rp, phase_on=OFFLINE)
        s = (smb + rp) - p2.map(lambda a: a * U64(2))           # m XOR b1 XOR b2
        return s, BShare(mb, b1, b2)

    # ------------------------------------------------------------------
    # Bit extraction and conversions (Sec. 4.3)
    # ------------------------------------------------------------------
    def reveal_words(self, s, phase=None, nbytes=None):
        """Pi_Rec of n words (arithmetic or Boolean planes; `nbytes` per message)."""
        from .protocol import ONLINE
        phase = ONLINE if phase is None else phase
        nb = 8 * s.m.size if nbytes is None else nbytes
        self.send(phase, 0, 2, nb)
        self.send(phase, 0, 1, nb)
        self.send(phase, 1, 0, nb)
        self.send(phase, 1, 2, 32)
        self.send(phase, 2, 0, 32)
        self.send(phase, 2, 1, 32)
        self.rounds[phase] += 1

    def msb(self, x, eda, item):
        """<msb(x)>^1 (bit 0 of one word per value) from <x>^l and an edaBit per value."""
        r, R = eda
        D = (x - r)                                             # local
        self.reveal_words(D)
        delta = D.value()                                       # public Delta = x - r
        P0 = R.xor_pub(delta)                                   # p = Delta XOR r
        G = R.and_pub(delta)                                    # g = Delta AND r
        P = P0
        for k in LEVELS:
            sk = U64(k)
            if k < LEVELS[-1]:
                t = self.and_words(bcat([P, P]), bcat([G.map(lambda a: a << sk), P.map(lambda a: a << sk)]), item)
                n = P.m.size
                G = G ^ t[:n]
                P = t[n:]
            else:
                G = G ^ self.and_words(P, G.map(lambda a: a << sk), item)
        top = P0 ^ G.map(lambda a: a << U64(1))                 # bit 63: Delta_63 ^ r_63 ^ carry
        return top.map(lambda a: a >> U64(63))

    def b2a_mult(self, x, d, da):
        """<x * d>^l for a Boolean bit d (bit 0 of one word per value) and a daBit per value:
        open e = d XOR s, convert <d>^l = e + (1 - 2e) <s>^l locally, then Pi_Mult."""
        from .protocol import Share
        s, sb = da
        n = d.m.size
        self.reveal_words(d ^ sb, nbytes=(n + 7) // 8)          # single bits, packed
        e = (d ^ sb).value() & U64(1)
        f = U64(1) - U64(2) * e                                 # 1 - 2e mod 2^64
        dl = Share(e + f * s.m, f * s.r1, f * s.r2)
        return self.mult(x, dl)

    def relu(self, x):
        """ReLU of every value of <x>^l (any shape): x * (1 - msb(x))."""
        self.check()
        shape = x.m.shape
        flat = x.map(lambda a: a.reshape(-1))
        n = flat.m.size
        eda = self.edabits(n)
        da = self.dabits(n)
        item = {"triples": []}
        self.pending.append(("and", item))
        d = self.msb(flat, eda, item).xor_pub(U64(1))           # 1 - msb
        out = self.b2a_mult(flat, d, da)
        return out.map(lambda a: a.reshape(shape))

    def maxpool2(self, x, B, H, W, C):
        """2x2 max pooling, stride 2, of an NHWC <x>^l (B*H*W*C values per plane)."""
        from .protocol import Share
        v = x.map(lambda a: a.reshape(B, H, W, C))
        a, b = v[:, 0::2, 0::2], v[:, 0::2, 1::2]
        c, d = v[:, 1::2, 0::2], v[:, 1::2, 1::2]
        N = B * (H // 2) * (W // 2) * C

        def cat(p, q):
            return Share(*[np.concatenate([u.reshape(-1), w.reshape(-1)]) for u, w in zip(p.comps(), q.comps())])

        p, q = cat(a, c), cat(b, d)
        u = q + self.relu(p - q)                                # max(a, b), max(c, d)
        u1, u2 = u[:N], u[N:]
        out = u2 + self.relu(u1 - u2)
        return out.map(lambda t: t.reshape(B, -1))

    # ------------------------------------------------------------------
    # Pi_MultVerify over GF(2^d) of Boolean triples (Sec. 3 with l = 1)
    # ------------------------------------------------------------------
    def gf(self):
        if getattr(self, "_gf", None) is None or self._gf.d != self.d:
            self._gf = GF(self.d)
            F = self._gf
            X, one = F.X, F.ONE
            self._gf_inv = (F.inv(X), F.inv(one ^ X), F.inv(F.mul(X, X ^ one)))
        return self._gf

    def gf_random(self, purpose, op, sub):
        F = self.gf()
        return BShare(self.G((1, 2), prg.tag(op, purpose, 0, sub), 1) & F.mask,
                      self.G((0, 1), prg.tag(op, purpose, 1, sub), 1) & F.mask,
                      self.G((0, 2), prg.tag(op, purpose, 2, sub), 1) & F.mask)

    def gf_reveal(self, s):
        from .protocol import VER_ON
        self.reveal_words(s, phase=VER_ON, nbytes=8)
        return s.value()

    def gf_poly_evl(self, a, b, op, p_r, p_g, sub, tr=None):
        """Pi_PolyEvl over GF(2^d): one-round sum_i a_i b_i with a fresh mask."""
        from .protocol import VER_OFF, VER_ON
        F = self.gf()
        rc1 = self.G((0, 1), prg.tag(op, p_r, 1, sub), 1) & F.mask
        rc2 = self.G((0, 2), prg.tag(op, p_r, 2, sub), 1) & F.mask
        gamma = F.dot(a.r1 ^ a.r2, b.r1 ^ b.r2) ^ rc1[0] ^ rc2[0]              # P0
        g1 = self.G((0, 1), prg.tag(op, p_g, 1, sub), 1)[0] & F.mask
        g2 = gamma ^ g1
        self.send(VER_OFF, 0, 2, 8)
        m1 = F.dot(a.m, b.r1) ^ F.dot(b.m, a.r1) ^ g1                          # P1
        m2 = F.dot(a.m, b.m) ^ F.dot(a.m, b.r2) ^ F.dot(b.m, a.r2) ^ g2        # P2
        self.send(VER_ON, 1, 2, 8)
        self.send(VER_ON, 2, 1, 8)
        if tr is not None:
            tr.update({"gamma2": U64(g2), "m1": U64(m1), "m2": U64(m2)})
        return BShare(np.array([m1 ^ m2], U64), rc1, rc2)

    def gf_reduce_round(self, x, y, z, op, s, k, log):
        """Pi_Reduce over GF(2^d), n -> n/2 (nodes 0, 1, x)."""
        from .protocol import VER_ON
        F = self.gf()
        sub = (s << 8) | k
        X, one = F.X, F.ONE
        f0, f1 = x[0::2], x[1::2]
        g0, g1 = y[0::2], y[1::2]

        def at_x(v0, v1):       # x f(1) - (x - 1) f(0) = x f(1) + (x + 1) f(0)
            return F.mul(X, v1) ^ F.mul(X ^ one, v0)

        f2 = BShare(*[at_x(a, b) for a, b in zip(f0.comps(), f1.comps())])
        g2 = BShare(*[at_x(a, b) for a, b in zip(g0.comps(), g1.comps())])
        t0, t2 = {}, {}
        h0 = self.gf_poly_evl(f0, g0, op, prg.VER_H0_R, prg.VER_H0_GAMMA, sub, tr=t0)
        h2 = self.gf_poly_evl(f2, g2, op, prg.VER_H2_R, prg.VER_H2_GAMMA, sub, tr=t2)
        self.rounds[VER_ON] += 1
        h1 = z ^ h0
        zeta = self.gf_reveal(self.gf_random(prg.VER_ZETA, op, sub))[0]
        ix, i1x, ixx = self._gf_inv
        L0 = F.mul(F.mul(zeta ^ one, zeta ^ X), ix)
        L1 = F.mul(F.mul(zeta, zeta ^ X), i1x)
        L2 = F.mul(F.mul(zeta, zeta ^ one), ixx)

        def at_zeta(v0, v1):
            return F.mul(zeta, v1) ^ F.mul(zeta ^ one, v0)

        xn = BShare(*[at_zeta(a, b) for a, b in zip(f0.comps(), f1.comps())])
        yn = BShare(*[at_zeta(a, b) for a, b in zip(g0.comps(), g1.comps())])
        zn = BShare(*[F.mul(L0, a) ^ F.mul(L1, b) ^ F.mul(L2, c)
                      for a, b, c in zip(h0.comps(), h1.comps(), h2.comps())])
        log["rounds"].append({"zeta": U64(zeta), "h0": t0, "h2": t2})
        return xn, yn, zn

    def gf_inner_verify(self, x, y, z, op, s, log):
        """Pi_InnerVerify over GF(2^d)."""
        from .protocol import VER_OFF, VER_ON
        F = self.gf()
        n = x.m.size
        alpha = self.gf_random(prg.VER_ALPHA, op, s)
        r1 = self.G((0, 1), prg.tag(op, prg.VER_XP_R, 1, s), n) & F.mask
        r2 = self.G((0, 2), prg.tag(op, prg.VER_XP_R, 2, s), n) & F.mask
        gamma = F.mul(x.r1 ^ x.r2, alpha.r1 ^ alpha.r2) ^ r1 ^ r2              # P0
        g1 = self.G((0, 1), prg.tag(op, prg.VER_XP_GAMMA, 1, s), n) & F.mask
        g2 = gamma ^ g1
        self.send(VER_OFF, 0, 2, 8 * n)
        m1 = F.mul(x.m, alpha.r1) ^ F.mul(alpha.m, x.r1) ^ g1                  # P1
        m2 = F.mul(x.m, alpha.m) ^ F.mul(x.m, alpha.r2) ^ F.mul(alpha.m, x.r2) ^ g2   # P2
        self.send(VER_ON, 1, 2, 8 * n)
        self.send(VER_ON, 2, 1, 8 * n)
        self.rounds[VER_ON] += 1
        xp = BShare(m1 ^ m2, r1, r2)
        A = bcat([xp, alpha])                 # -alpha = alpha in characteristic 2
        B = bcat([y, z])
        td = {}
        delta = self.gf_poly_evl(A, B, op, prg.VER_DELTA_R, prg.VER_DELTA_GAMMA, s, tr=td)
        self.rounds[VER_ON] += 1
        dv = self.gf_reveal(delta)
        log["delta"] = dv
        log["delta_tr"] = td
        return not np.any(dv)

    def gf_instance_and(self, triples, r):
        """Pi_Tran over GF(2^d) of Boolean triples: gate g = 64 * word + bit (words of the
        triples concatenated in call order) weighted by r^g on the x side."""
        F = self.gf()
        a = bcat([t[0] for t in triples])
        b = bcat([t[1] for t in triples])
        c = bcat([t[2] for t in triples])
        G = 64 * a.m.size
        pw = F.powers(r, G)
        sel = [(_bits(v).reshape(-1)) for v in a.comps()]
        xs = BShare(*[pw * s_ for s_ in sel])                   # r^g where the bit is 1
        ys = BShare(*[_bits(v).reshape(-1) for v in b.comps()])
        zs = BShare(*[np.array([np.bitwise_xor.reduce(pw * _bits(v).reshape(-1))], U64) for v in c.comps()])
        return xs, ys, zs

    def gf_fold_and_check(self, x, y, z, op, s, R, log):
        n0 = x.m.size
        R = self.auto_rounds(n0, R)
        npad = -(-n0 // (1 << R)) * (1 << R)
        if npad != n0:
            pad = np.zeros(npad - n0, U64)
            x = x.map(lambda a: np.concatenate([a, pad]))
            y = y.map(lambda a: np.concatenate([a, pad]))
        log.update({"R": R, "n0": n0, "npad": npad, "rounds": []})
        for k in range(R):
            x, y, z = self.gf_reduce_round(x, y, z, op, s, k, log)
        return self.gf_inner_verify(x, y, z, op, s, log)

    def verify_and_item(self, item, op, s, R, log):
        """One GF(2^d) Pi_MultVerify instance over every Boolean triple of one layer call."""
        r = self.gf_reveal(self.gf_random(prg.VER_R, op, s))[0]
        log["r"] = U64(r)
        x, y, z = self.gf_instance_and(item["triples"], r)
        log["z"] = z
        return self.gf_fold_and_check(x, y, z, op, s, R, log)

    def instance_rows(self, xs, ys, zs, lo, hi, r):
        """Pi_BIVerify of row gates [lo, hi) (row p: a 64-element inner product with output
        z_p): x'_{p,j} = r^(p - lo) x_{p,j}, y lifted, z = sum_p r^(p - lo) z_p."""
        gr = self.gr
        T = hi - lo
        pw = gr.powers(r, T)
        from .protocol import Share
        x = Share(*[gr.scale(v[lo:hi], pw[:, None, :]).reshape(T * v.shape[1], self.d) for v in xs.comps()])
        y = Share(*[gr.const(v[lo:hi].reshape(-1)) for v in ys.comps()])
        z = Share(*[gr.scale(v[lo:hi], pw).sum(axis=0, dtype=U64) for v in zs.comps()])
        return x, y, z
