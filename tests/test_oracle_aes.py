"""Pins for the oracle's AES-128, PRG and randomness source (CPU only).

AES is pinned to FIPS-197's printed known answers (tests/golden) and, when
the host has the OpenSSL command-line tool, to OpenSSL on random blocks.  The
PRG and randomness conventions (byte order, tweak position, key layout) are
pinned to OpenSSL's AES as an independent implementation.
"""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fips197_aes128.txt")


def _golden():
    rows = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tag, *kv = line.split()
        rows.append((tag, dict(x.split("=") for x in kv)))
    return rows


def test_fips197_known_answers():
    n = 0
    for tag, kv in _golden():
        if "out" in kv:
            got = O.aes128(bytes.fromhex(kv["key"]), bytes.fromhex(kv["in"]))
            assert got.hex() == kv["out"], tag
            n += 1
    assert n == 2


def test_fips197_key_schedule_last_round_key():
    for tag, kv in _golden():
        if tag == "A.1":
            ks = (C.c_uint8 * 176)()
            key = (C.c_uint8 * 16).from_buffer_copy(bytes.fromhex(kv["key"]))
            O.lib().orc_aes128_expand(key, ks)
            assert bytes(ks)[160:176].hex() == kv["w40_43"]


def test_sbox_entries_and_bijection():
    sb = O.sbox()
    for tag, kv in _golden():
        if tag == "SBOX":
            for a, b in kv.items():
                assert sb[int(a, 16)] == int(b, 16)
    assert sorted(sb) == list(range(256))
    # no fixed points and no "opposite fixed points" (design property of the S-box)
    assert all(sb[a] != a and sb[a] != (a ^ 0xFF) for a in range(256))


def _openssl_ecb(key: bytes, data: bytes) -> bytes:
    return subprocess.run(["openssl", "enc", "-aes-128-ecb", "-nopad", "-K", key.hex()],
                          input=data, stdout=subprocess.PIPE, check=True).stdout


need_openssl = pytest.mark.skipif(shutil.which("openssl") is None, reason="no openssl CLI")


@need_openssl
def test_aes_random_blocks_vs_openssl():
    g = np.random.Generator(np.random.PCG64(7))
    for trial in range(4):
        key = g.bytes(16)
        data = g.bytes(16 * 2500)
        ref = _openssl_ecb(key, data)
        got = b"".join(O.aes128(key, data[i:i + 16]) for i in range(0, len(data), 16))
        assert got == ref


def _blk_bytes(lo, hi):
    return lo.to_bytes(8, "little") + hi.to_bytes(8, "little")


@need_openssl
def test_prg_convention_vs_openssl():
    """H(s, j) = AES_K(s ^ J_j) ^ (s ^ J_j), K = 00..0f, J_j = byte 15 set to j."""
    g = np.random.Generator(np.random.PCG64(11))
    key = bytes(range(16))
    cases = [(int(g.integers(0, 2**63)) * 2 + 1, int(g.integers(0, 2**63)), j) for j in range(8)]
    ins = b""
    for lo, hi, j in cases:
        x = bytearray(_blk_bytes(lo, hi))
        x[15] ^= j
        ins += bytes(x)
    ref = _openssl_ecb(key, ins)
    for i, (lo, hi, j) in enumerate(cases):
        x = ins[16 * i:16 * i + 16]
        want = bytes(a ^ b for a, b in zip(ref[16 * i:16 * i + 16], x))
        glo, ghi = O.prg(lo, hi, j)
        assert _blk_bytes(glo, ghi) == want


@need_openssl
def test_randomness_convention_vs_openssl():
    """R(e, pi, c) = AES_{seed LE || 0^8}(e LE || pi u16 LE || c u16 LE || 0^4)."""
    seed = 0x0123456789ABCDEF
    key = seed.to_bytes(8, "little") + bytes(8)
    cases = [(5, 0, 0), (2**40 + 3, 66, 0), (393215, 67, 1), (0, 64, 9)]
    ins = b"".join(e.to_bytes(8, "little") + p.to_bytes(2, "little") + c.to_bytes(2, "little")
                   + bytes(4) for e, p, c in cases)
    ref = _openssl_ecb(key, ins)
    for i, (e, p, c) in enumerate(cases):
        lo, hi = O.rand(seed, e, p, c)
        assert _blk_bytes(lo, hi) == ref[16 * i:16 * i + 16]
