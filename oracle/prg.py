"""Pairwise-seed PRG (oracle; test infrastructure only).

Preliminaries ("Secret sharing"): when P_j and P_k "pick random values
together" they run a PRG on their common seed eta_{j,k}.  The paper names no
PRG.  Reading: ChaCha20 in counter mode, RFC 8439 Sec. 2.3 block function,
written here from the RFC.

  G(eta, tag, i) = 64-bit word i of the keystream with key = eta (32 bytes),
                   96-bit nonce = tag, 32-bit block counter = floor(i / 8);
                   the word is little-endian bytes 8*(i mod 8) .. +7 of the block.
  eta_{jk}       = SHA-256(master_seed || "eta" || bytes(j, k))
  tag            = (op:u32, purpose:u16 | component:u16 << 16, sub:u32)
"""
import hashlib

import numpy as np

U32 = np.uint32
SIGMA = np.array([0x61707865, 0x3320646E, 0x79622D32, 0x6B206574], dtype=U32)

# Purposes of keystream draws.  Component: 0 = the m word (eta_12),
# 1 = [.]_1 word (eta_01), 2 = [.]_2 word (eta_02).
SHARE_R = 1
INNER_RZ = 2
INNER_GAMMA = 3
TRUNC_B = 4
TRUNC_WX_R = 5
TRUNC_WX_GAMMA = 6
TRUNC_WZ_R = 7
TRUNC_WZ_GAMMA = 8
MULT_RZ = 9
MULT_GAMMA = 10
VER_R = 16
VER_H0_R = 17
VER_H0_GAMMA = 18
VER_H2_R = 19
VER_H2_GAMMA = 20
VER_ZETA = 21
VER_ALPHA = 22
VER_XP_R = 23
VER_XP_GAMMA = 24
VER_DELTA_R = 25
VER_DELTA_GAMMA = 26


def _rotl(v, c):
    return (v << U32(c)) | (v >> U32(32 - c))


def chacha20_blocks(key, nonce_words, counters):
    """RFC 8439 Sec. 2.3: 16 output words for each 32-bit block counter; shape (n, 16)."""
    k = np.frombuffer(bytes(key), dtype="<u4")
    counters = np.asarray(counters, dtype=U32)
    n = counters.shape[0]
    init = np.empty((16, n), dtype=U32)
    init[0:4] = SIGMA[:, None]
    init[4:12] = k[:, None]
    init[12] = counters
    init[13:16] = np.asarray(nonce_words, dtype=U32)[:, None]
    x = init.copy()

    def qr(a, b, c, d):
        x[a] += x[b]; x[d] ^= x[a]; x[d] = _rotl(x[d], 16)
        x[c] += x[d]; x[b] ^= x[c]; x[b] = _rotl(x[b], 12)
        x[a] += x[b]; x[d] ^= x[a]; x[d] = _rotl(x[d], 8)
        x[c] += x[d]; x[b] ^= x[c]; x[b] = _rotl(x[b], 7)

    for _ in range(10):          # 20 rounds = 10 column + 10 diagonal rounds
        qr(0, 4, 8, 12); qr(1, 5, 9, 13); qr(2, 6, 10, 14); qr(3, 7, 11, 15)
        qr(0, 5, 10, 15); qr(1, 6, 11, 12); qr(2, 7, 8, 13); qr(3, 4, 9, 14)
    return (x + init).T.copy()


def tag(op, purpose, comp=0, sub=0):
    return (op & 0xFFFFFFFF, (purpose & 0xFFFF) | ((comp & 0xFFFF) << 16), sub & 0xFFFFFFFF)


def words(seed, tg, count, start=0):
    """G(seed, tag, i) for i in [start, start + count) as uint64."""
    if count == 0:
        return np.zeros(0, dtype=np.uint64)
    b0 = start // 8
    b1 = (start + count - 1) // 8 + 1
    ks = chacha20_blocks(seed, tg, np.arange(b0, b1, dtype=np.uint64).astype(U32))
    w = np.ascontiguousarray(ks).view("<u8").reshape(-1)
    off = start - 8 * b0
    return w[off:off + count].astype(np.uint64)


def keystream_bytes(seed, tg, nbytes, counter=0):
    """Raw keystream bytes starting at a block counter (for comparison with other ChaCha20 code)."""
    nb = (nbytes + 63) // 64
    ks = chacha20_blocks(seed, tg, np.arange(counter, counter + nb, dtype=np.uint64).astype(U32))
    return np.ascontiguousarray(ks).astype("<u4").tobytes()[:nbytes]


def pair_seeds(master_seed):
    """eta_01, eta_02, eta_12 and the all-party seed used when P1 or P2 owns an input."""
    master_seed = bytes(master_seed)
    assert len(master_seed) == 32

    def h(*ids):
        return hashlib.sha256(master_seed + b"eta" + bytes(ids)).digest()

    return {(0, 1): h(0, 1), (0, 2): h(0, 2), (1, 2): h(1, 2), (0, 1, 2): h(0, 1, 2)}
