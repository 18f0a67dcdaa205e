"""Pins for the oracle's post-processing subprotocols and the literal interval
lookup (CPU only).

Sec. "Standard Preprocessing Subprotocols": Beaver multiplication over the
ring and the Boolean AND correlation; Sec. "Mixed-Domain Conversions": B2A.
Each is checked by reconstruction against the operation it implements,
computed here with Python integers (products mod 2^64, bitwise AND, the bit
itself).  The literal lookup (Definition "Interval lookup with vector
payload", one vector DCF per inner boundary of the compilation protocol's
translated partition) is checked for every input of small domains: the
coefficient shares add to the active piece's coefficients, found here by
scanning the spec's boundaries, and the Horner pipeline's output adds to
P(x) + r_out, evaluated here with Python integers, and to the single-key
pipeline's output for the same seed.
"""
import random

import numpy as np
import pytest

import oracle as O
from paper_2606_09551_amd import workloads as W

M64 = 2**64 - 1


def test_beaver_multiplication_reconstructs_products():
    rnd = random.Random(31)
    for i in range(3000):
        seed = rnd.getrandbits(128)
        e, step = rnd.getrandbits(40), rnd.randint(0, 3)
        a, b, c = O.triple(seed, e, step)
        A, B = (int(a[0]) + int(a[1])) & M64, (int(b[0]) + int(b[1])) & M64
        assert (int(c[0]) + int(c[1])) & M64 == (A * B) & M64
        u, v = rnd.getrandbits(64), rnd.getrandbits(64)
        if i % 7 == 0:
            u, v = rnd.choice([(0, v), (u, 0), (M64, M64), (1, M64)])
        u0, v0 = rnd.getrandbits(64), rnd.getrandbits(64)
        u1, v1 = (u - u0) & M64, (v - v0) & M64
        d = ((u0 - int(a[0])) + (u1 - int(a[1]))) & M64   # the openings
        f = ((v0 - int(b[0])) + (v1 - int(b[1]))) & M64
        z = (O.beaver_mul(0, d, f, int(a[0]), int(b[0]), int(c[0]))
             + O.beaver_mul(1, d, f, int(a[1]), int(b[1]), int(c[1]))) & M64
        assert z == (u * v) & M64


def test_and_gate_every_bit_combination():
    rnd = random.Random(32)
    for _ in range(500):
        seed = rnd.getrandbits(128)
        a, b, c = O.and_triple(seed, rnd.getrandbits(32), rnd.randint(0, 7))
        assert int(c[0]) ^ int(c[1]) == (int(a[0]) ^ int(a[1])) & (int(b[0]) ^ int(b[1]))
        # 64 bit positions, with words that hold every (x, y) pair
        x = (rnd.getrandbits(64) & ~0b1111) | 0b1010
        y = (rnd.getrandbits(64) & ~0b1111) | 0b1100
        x0, y0 = rnd.getrandbits(64), rnd.getrandbits(64)
        x1, y1 = x ^ x0, y ^ y0
        d = x0 ^ int(a[0]) ^ x1 ^ int(a[1])
        f = y0 ^ int(b[0]) ^ y1 ^ int(b[1])
        z = O.and_gate(0, d, f, int(a[0]), int(b[0]), int(c[0])) ^ O.and_gate(1, d, f, int(a[1]), int(b[1]), int(c[1]))
        assert z == x & y


def test_b2a_both_bits():
    rnd = random.Random(33)
    seen = set()
    for _ in range(400):
        seed = rnd.getrandbits(128)
        e, step = rnd.getrandbits(30), rnd.randint(0, 3)
        t, T = O.b2a_rand(seed, e, step)
        tb = int(t[0]) ^ int(t[1])
        assert tb in (0, 1) and (int(T[0]) + int(T[1])) & M64 == tb
        for z in (0, 1):
            z0 = rnd.getrandbits(1)
            z1 = z ^ z0
            c = z0 ^ int(t[0]) ^ z1 ^ int(t[1])   # the opening of z ^ t
            s = (O.b2a(0, c, int(T[0])) + O.b2a(1, c, int(T[1]))) & M64
            assert s == z
            seen.add((tb, z))
    assert seen == {(0, 0), (0, 1), (1, 0), (1, 1)}


def _piece(t: dict, x: int, n: int, is_int: bool) -> int:
    """Index of the interval holding x, by scanning the spec's boundaries."""
    if is_int:
        rep = x % (1 << n)
        return max(i for i in range(t["m"]) if t["aprime"][i] <= rep)
    return max(i for i in range(t["m"]) if t["alpha"][i] <= x)


def _poly(coef, x: int) -> int:
    return sum(c * pow(x, k, 2**64) for k, c in enumerate(coef)) & M64


def _check_lit(S, n: int, is_int: bool, seed: int, xs):
    t = O.spec_tables(S)
    got = O.lit(S, seed, np.arange(len(xs)), xs)
    for i, x in enumerate(xs):
        x = int(x)
        k = _piece(t, x, n, is_int)
        coef = [(int(a) + int(b)) & M64 for a, b in zip(got["c0"][i], got["c1"][i])]
        want = [c & M64 for c in t["coef"][k]]
        want[0] = (want[0] + int(got["r_out"][i])) & M64  # the output mask rides in the constant term
        assert coef == want, (x, k)
        y = (int(got["y0"][i]) + int(got["y1"][i]) - int(got["r_out"][i])) & M64
        assert y == _poly(t["coef"][k], x), x
    return got


@pytest.mark.parametrize("r", [2, 3, 4])
def test_literal_lookup_every_input_real_specs(r):
    """Clip-ReLU (n = 8) and a degree-2 GELU fit (n = 9), every input, 3 seeds."""
    for desc, n, f in ((W.clip_relu_spec(), 8, 4), (W.gelu_spec(f=4), 9, 4)):
        S = O.compile_spec(desc, n, f, lookup_r=r)
        xs = np.arange(-(1 << (n - 1)), 1 << (n - 1), dtype=np.int64)
        for seed in (1, 2**90 + 17, 0xF00D):
            _check_lit(S, n, False, seed, xs)


@pytest.mark.parametrize("r", [2, 3, 4])
def test_literal_lookup_every_input_integer_specs(r):
    """Random integer partitions at n = 5..7, including m = 2^n at n = 5, 6
    (every value its own interval: no padding) and m = 1, every input."""
    rnd = random.Random(600 + r)
    for n in (5, 6, 7):
        N = 1 << n
        mmax = min(N, 64)  # the spec's interval limit
        for m in (1, 2, rnd.randint(3, mmax - 1), mmax):
            alpha = [0] + sorted(rnd.sample(range(1, N), m - 1)) + [N]
            d = rnd.randint(0, 3)
            coef = [[rnd.getrandbits(64) for _ in range(d + 1)] for _ in range(m)]
            S = O.compile_spec_int(n, alpha, coef, lookup_r=r)
            xs = np.arange(-(N // 2), N // 2, dtype=np.int64)
            _check_lit(S, n, True, rnd.getrandbits(128), xs)


def test_literal_and_single_key_pipelines_agree():
    """Same seed, same masks: the literal lookup with Beaver Horner and the
    single-key lookup combined at the public x-hat open to the same
    y + r_out (GELU, n = 24, f = 12, random inputs)."""
    desc = W.gelu_spec()
    S = O.compile_spec(desc, 24, 12)
    g = np.random.Generator(np.random.PCG64(12))
    x = W.quantize(g.normal(0.0, 1.5, size=300), 24, 12)
    elems = np.arange(300) * 1301
    lit = O.lit(S, 77, elems, x)
    y0, y1, _, _, r_in, r_out, _ = O.full(S, 77, elems, x, masks=True)
    assert np.array_equal(lit["r_in"], r_in) and np.array_equal(lit["r_out"], r_out)
    assert np.array_equal(lit["y0"] + lit["y1"], y0 + y1)
