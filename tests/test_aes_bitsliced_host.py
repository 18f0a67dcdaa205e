"""Host pins of the library's bitsliced AES-128 (csrc/fss_aes_bs.hpp, the VGPR
alternative to the local-memory T-tables), compiled with g++ for the CPU:
the bitsliced SubBytes equals the FIPS-197 S-box on all 256 inputs (taken
from the oracle's own byte-oriented AES), the pair layout round-trips, and
encryption under the PRG key (the FIPS-197 Appendix C.1 key) matches the
Appendix C.1 known answer and the oracle's AES on random blocks."""
import os
import random
import shutil
import subprocess

import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host", "aes_bs_check.cpp")
KEY = bytes(range(16))


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    out = str(tmp_path_factory.mktemp("aesbs") / "aesbs")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-Wall", "-Wno-unknown-pragmas", "-o", out, SRC])
    return out


def _golden_c1():
    """(key, plaintext, ciphertext) of FIPS-197 Appendix C.1 from the golden file."""
    for line in open(os.path.join(HERE, "golden", "fips197_aes128.txt")):
        if line.startswith("C.1 "):
            kv = dict(f.split("=", 1) for f in line.split()[1:])
            return bytes.fromhex(kv["key"]), bytes.fromhex(kv["in"]), bytes.fromhex(kv["out"])
    raise AssertionError("no C.1 line in the golden file")


def test_pair_layout_round_trips(exe):
    assert subprocess.run([exe, "roundtrip"], stdout=subprocess.PIPE, text=True).stdout.strip() == "ok"


def test_bitsliced_sbox_all_inputs(exe):
    out = subprocess.run([exe, "sbox"], stdout=subprocess.PIPE, text=True, check=True).stdout.split()
    assert bytes(int(v, 16) for v in out) == O.sbox()


def _encrypt_pairs(exe, blocks):
    lines = []
    for i in range(0, len(blocks), 2):
        p, q = blocks[i], blocks[i + 1]
        lines.append(" ".join(f"{b:02x}" for b in KEY) + " | " + " ".join(f"{b:02x}" for b in p) + " | "
                     + " ".join(f"{b:02x}" for b in q))
    out = subprocess.run([exe], input="\n".join(lines) + "\n", stdout=subprocess.PIPE, text=True,
                         check=True).stdout.split()
    return [bytes.fromhex(h) for h in out]


def test_fips197_c1_known_answer(exe):
    key, pt, ct = _golden_c1()
    assert key == KEY
    got = _encrypt_pairs(exe, [pt, bytes(16)])
    assert got[0] == ct
    assert got[1] == O.aes128(KEY, bytes(16))


def test_random_blocks_match_oracle(exe):
    rnd = random.Random(11)
    blocks = [bytes(rnd.getrandbits(8) for _ in range(16)) for _ in range(400)]
    got = _encrypt_pairs(exe, blocks)
    assert got == [O.aes128(KEY, b) for b in blocks]
