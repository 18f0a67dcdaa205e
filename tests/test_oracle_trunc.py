"""Pins for the oracle's rescaling gate (CPU only): arithmetic right shift of a
masked 64-bit value.  For a signed y with |y| < 2^62 (the bound every compiled
piece satisfies) opened as yhat = y + r_in, the two parties' outputs must
reconstruct to floor(y / 2^s) + r_out, checked against Python's integer floor
division for random and edge values of y and r_in, and by brute force over
small y and masks whose low bits and top bit take every value."""
import random

import numpy as np
import pytest

import oracle as O

M64 = 2**64 - 1


def _check(shift, ys, r_ins, r=3, seed=0x7E):
    ys = [int(y) for y in ys]
    r_ins = [int(v) & M64 for v in r_ins]
    yhat = np.array([(y + v) & M64 for y, v in zip(ys, r_ins)], dtype=np.uint64)
    elems = np.arange(len(ys), dtype=np.int64)
    z0, z1, r_out = O.trunc(shift, seed, elems, np.array(r_ins, dtype=np.uint64), yhat, lookup_r=r)
    got = [(int(a) + int(b) - int(c)) & M64 for a, b, c in zip(z0, z1, r_out)]
    want = [(y >> shift) & M64 for y in ys]   # Python's >> floors: ARS with sign extension
    bad = [i for i in range(len(ys)) if got[i] != want[i]]
    assert not bad, (shift, r, [(ys[i], r_ins[i]) for i in bad[:4]])
    return r_out


@pytest.mark.parametrize("r", [2, 3, 4])
@pytest.mark.parametrize("shift", [1, 2, 3, 7, 12, 24, 31, 32])
def test_trunc_random_and_edges(shift, r):
    rnd = random.Random(1000 * shift + r)
    lim = 2**62
    ys = [rnd.randrange(-lim + 1, lim) for _ in range(150)]
    ys += [rnd.randrange(-2**20, 2**20) for _ in range(50)]
    ys += [0, -1, 1, lim - 1, -lim + 1, 2**shift, -(2**shift), 2**shift - 1, -(2**shift) + 1,
           2**shift + 1, -(2**shift) - 1, lim - 2**shift, -lim + 2**shift]
    r_ins = [rnd.getrandbits(64) for _ in ys]
    r_ins[:8] = [0, M64, 2**63, 2**63 - 1, 1, 2**shift - 1, 2**63 + 2**shift - 1, 2**shift]
    _check(shift, ys, r_ins, r)


def test_trunc_bruteforce_small():
    """s = 3: every y in [-256, 256) against masks whose low 3 bits run over
    all values and whose top bit is set or clear, plus random high bits."""
    rnd = random.Random(9)
    masks = []
    for low in range(8):
        for top in (0, 1):
            masks.append((top << 63) | (rnd.getrandbits(60) << 3) | low)
    ys, rs = [], []
    for m in masks:
        for y in range(-256, 256):
            ys.append(y)
            rs.append(m)
    _check(3, ys, rs, r=2)


def test_trunc_output_mask_is_drawn_from_the_seed():
    """r_out = R(e, 0).lo of the gate's own seed, whatever the input."""
    r_out = _check(5, [12345, -777], [99, 2**63 + 5], seed=0xABC)
    assert [int(v) for v in r_out] == [O.rand(0xABC, e, 0)[0] for e in range(2)]


def test_trunc_rejects_bad_shift():
    for s in (0, 33):
        with pytest.raises(ValueError):
            O.trunc(s, 1, np.arange(1), np.zeros(1, np.uint64), np.zeros(1, np.uint64))
