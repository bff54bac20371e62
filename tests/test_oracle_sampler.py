"""Pins for the oracle's ChaCha20 stream (RFC 8439 block function) and samplers."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "chacha20_openssl.txt")


def _block(lib, key_hex, ctr_hex, nonce_hex):
    key = np.frombuffer(bytes.fromhex(key_hex), dtype="<u4").copy()
    nonce = np.frombuffer(bytes.fromhex(nonce_hex), dtype="<u4").copy()
    ctr = int.from_bytes(bytes.fromhex(ctr_hex), "little")
    out = np.zeros(16, dtype=np.uint32)
    vp = ctypes.c_void_p
    lib.oracle_chacha20_block(key.ctypes.data_as(vp), ctr, nonce.ctypes.data_as(vp), out.ctypes.data_as(vp))
    return out.astype("<u4").tobytes()


def test_chacha20_block_matches_openssl_golden(oracle_lib):
    # golden keystream written by tests/golden/make_chacha_golden.sh (openssl enc -chacha20)
    with open(GOLD) as f:
        for line in f:
            key, ctr, nonce, ks = line.split()
            ks = bytes.fromhex(ks)
            c = int.from_bytes(bytes.fromhex(ctr), "little")
            got = _block(oracle_lib, key, ctr, nonce) + _block(oracle_lib, key, (c + 1).to_bytes(4, "little").hex(), nonce)
            assert got == ks


@pytest.mark.skipif(shutil.which("openssl") is None, reason="openssl CLI not present")
def test_chacha20_stream_words_match_openssl_live(oracle_lib):
    seed, purpose, obj, lane = 0x0123456789ABCDEF, 5, (77 << 8) | 3, 9
    key = (seed.to_bytes(8, "little") + purpose.to_bytes(8, "little") + obj.to_bytes(8, "little")
           + bytes.fromhex("4845514701000000"))
    iv = (0).to_bytes(4, "little") + lane.to_bytes(4, "little") + bytes(8)
    ks = subprocess.run(["openssl", "enc", "-chacha20", "-K", key.hex(), "-iv", iv.hex()],
                        input=bytes(64 * 40), capture_output=True, check=True).stdout
    words = np.zeros(300, dtype=np.uint64)
    vp = ctypes.c_void_p
    oracle_lib.oracle_stream_words(seed, purpose, obj, lane, 5, 300, words.ctypes.data_as(vp))
    ref = np.frombuffer(ks, dtype="<u8")[5:305]
    assert np.array_equal(words, ref)


def _stream(lib, seed, purpose, obj, lane, n, first=0):
    w = np.zeros(n, dtype=np.uint64)
    lib.oracle_stream_words(seed, purpose, obj, lane, first, n, w.ctypes.data_as(ctypes.c_void_p))
    return w


def test_ternary_and_cbd_follow_stream(oracle_lib):
    n = 4096
    vp = ctypes.c_void_p
    t = np.zeros(n, dtype=np.int64)
    c = np.zeros(n, dtype=np.int64)
    oracle_lib.oracle_sample_ternary(42, 6, 7, n, t.ctypes.data_as(vp))
    oracle_lib.oracle_sample_cbd(42, 7, 7, n, c.ctypes.data_as(vp))
    wt = _stream(oracle_lib, 42, 6, 7, 0, n)
    wc = _stream(oracle_lib, 42, 7, 7, 0, n)
    assert list(t) == [[0, 1, -1][int(w) % 3] for w in wt]
    assert list(c) == [bin(int(w) & 0x1FFFFF).count("1") - bin((int(w) >> 21) & 0x1FFFFF).count("1") for w in wc]
    # distribution: ternary ~ 1/3 each, CBD(21) variance 21/2
    for v in (-1, 0, 1):
        assert abs((t == v).mean() - 1 / 3) < 0.04
    assert abs(c.var() - 10.5) < 1.2 and abs(c.mean()) < 0.3 and np.abs(c).max() <= 21


def test_uniform_follows_stream(oracle_lib):
    q = 1099511480321
    n = 2048
    out = np.zeros(n, dtype=np.uint64)
    oracle_lib.oracle_sample_uniform(9, 2, 0, 4, q, n, out.ctypes.data_as(ctypes.c_void_p))
    w = _stream(oracle_lib, 9, 2, 0, 4, 2 * n)
    assert [int(v) for v in out] == [((int(w[2 * k + 1]) << 64) | int(w[2 * k])) % q for k in range(n)]
    assert abs(out.astype(np.float64).mean() / q - 0.5) < 0.03
