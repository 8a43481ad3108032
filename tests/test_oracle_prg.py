"""Pins of the oracle's ChaCha20 PRG against the RFC 8439 test vector and OpenSSL."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import prg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rfc8439_2_3_2_block.txt")


def _golden():
    vals = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        k, v = line.split()
        vals[k] = v
    return vals


def test_rfc8439_block_function_vector():
    g = _golden()
    key = bytes.fromhex(g["key"])
    nonce = np.frombuffer(bytes.fromhex(g["nonce"]), dtype="<u4")
    out = prg.chacha20_blocks(key, nonce, [int(g["counter"])])
    assert out.astype("<u4").tobytes() == bytes.fromhex(g["block"])


@pytest.mark.skipif(shutil.which("openssl") is None, reason="openssl CLI absent")
@pytest.mark.parametrize("case", range(4))
def test_keystream_matches_openssl(case):
    g = np.random.default_rng(100 + case)
    key = g.integers(0, 256, 32, dtype=np.uint8).tobytes()
    nonce = g.integers(0, 256, 12, dtype=np.uint8).tobytes()
    counter = int(g.integers(0, 1 << 20))
    n = 64 * 5 + 24
    iv = counter.to_bytes(4, "little") + nonce          # OpenSSL: 32-bit counter || 96-bit nonce
    res = subprocess.run(["openssl", "enc", "-chacha20", "-K", key.hex(), "-iv", iv.hex()],
                         input=bytes(n), capture_output=True, check=True)
    ours = prg.keystream_bytes(key, np.frombuffer(nonce, dtype="<u4"), n, counter=counter)
    assert ours == res.stdout


def test_word_offsets_consistent():
    seed = bytes(range(32))
    tg = prg.tag(7, prg.INNER_GAMMA, 1, 3)
    full = prg.words(seed, tg, 100)
    for start, cnt in [(0, 1), (3, 9), (8, 8), (13, 50), (99, 1)]:
        assert np.array_equal(prg.words(seed, tg, cnt, start), full[start:start + cnt])
    # word i is little-endian bytes 8*(i mod 8).. of block floor(i/8)
    raw = prg.keystream_bytes(seed, tg, 800)
    assert np.array_equal(np.frombuffer(raw, dtype="<u8")[:100], full)


def test_tags_separate_streams():
    seed = bytes(32)
    a = prg.words(seed, prg.tag(0, prg.INNER_RZ, 1), 16)
    b = prg.words(seed, prg.tag(0, prg.INNER_RZ, 2), 16)
    c = prg.words(seed, prg.tag(1, prg.INNER_RZ, 1), 16)
    assert not np.array_equal(a, b) and not np.array_equal(a, c)
