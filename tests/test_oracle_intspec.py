"""Pins for the oracle's integer operator specifications (CPU only).

Definition "Operator specification" states a spec with integer boundaries
0 = alpha_0 < ... < alpha_m = 2^n over canonical representatives and
polynomials evaluated in the ring; the worked example of the appendix
"Example: A Complete (F, Phi) Pair" is the signed ReLU with alpha_1 = N/2.
Reconstruction is checked for every input of small domains against values
computed here from the definitions (interval found by scanning, polynomial
and predicates evaluated with Python integers), independently of the
oracle's plaintext evaluator.  Also pins the 128-bit dealer seed.
"""
import random
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O
from paper_2606_09551_amd import workloads as W
from maxspec import max_int_spec

M64 = 2**64 - 1
P = W.PredDesc


def _pred_value(q, x: int, n: int) -> int:
    """One primitive predicate of the Definition at the n-bit signed input x."""
    N = 1 << n
    rep = x % N
    if q.kind == W.LT_SIGNED:
        bit = int(x < int(q.thr))
    elif q.kind == W.LT_UNSIGNED:
        bit = int(rep < int(q.thr))
    elif q.kind == W.LOWBITS_LT:
        bit = int((x % (1 << q.f_bits)) < q.gamma)
    else:  # MSB(x + c)
        bit = ((x + q.c) % N) >> (n - 1)
    return bit ^ int(q.negate)


def _direct(alpha, coef, preds, x: int, n: int):
    """(P_{i*}(x) mod 2^64, predicate bits) straight from the definition."""
    N = 1 << n
    rep = x % N
    i = next(i for i in range(len(alpha) - 1) if alpha[i] <= rep < alpha[i + 1])
    y = sum(c * pow(x, l, 2**64) for l, c in enumerate(coef[i])) & M64
    z = 0
    for q in preds:
        z ^= _pred_value(q, x, n) << q.out
    return y, z


@pytest.mark.parametrize("r", [2, 3, 4])
@pytest.mark.parametrize("n", [4, 7, 10])
def test_worked_example_relu_integer_spec(n, r):
    """alpha = (0, N/2, N), P_0 = x, P_1 = 0, z = MSB(x): y_0 + y_1 = max(x, 0) + r_out
    and z_0 ^ z_1 = MSB(x) for every x; the lookup partition has M = 3 intervals.
    The packed comparison's two queries are 1[v < (r + N/2) mod N] and the mask
    query 1[v < r] on the canonical view, which is the lookup's own view: the
    threshold query has an atom of width n, the mask query is answered by the
    lookup DCF at v (so T = 1)."""
    N = 2**n
    alpha = [0, N // 2, N]
    S = O.compile_spec_int(n, alpha, [[0, 1], [0, 0]], [P(W.MSB_SHIFT, 0, c=0)], lookup_r=r)
    t = O.spec_tables(S)
    assert (t["m"], t["p"], t["T"]) == (2, 2, 1)
    assert S.n_prim == 1 and S.n_views == 1 and S.lookup_view == 0
    assert t["atoms"] == [(n, 0, 0)]
    for rr in (0, 1, N // 2, N - 1, 12345 % N):
        B, ordv = O.protocol3(n, alpha, rr)
        assert len(B) == 4 and len(ordv) == 3
    xs = np.arange(-N // 2, N // 2, dtype=np.int64)
    for seed in (5, 2**64 + 17, 2**127 + 3):
        y0, y1, z0, z1, r_in, r_out, _ = O.full(S, seed, np.arange(N, dtype=np.int64) + 9, xs, masks=True)
        assert np.array_equal(y0 + y1 - r_out, np.maximum(xs, 0).astype(np.uint64))
        assert np.array_equal(z0 ^ z1, (xs < 0).astype(np.uint64))


def _random_int_spec(rnd: random.Random, n: int):
    N = 1 << n
    s = N // 2
    m = rnd.randint(1, min(12, N))
    alpha = [0] + sorted(rnd.sample(range(1, N), m - 1)) + [N]
    d = rnd.randint(0, 3)
    coef = [[rnd.getrandbits(64) for _ in range(d + 1)] for _ in range(m)]
    preds = [P(W.LT_SIGNED, 0, thr=float(rnd.randint(-s, s))),
             P(W.LT_UNSIGNED, 1, thr=float(rnd.randint(0, N)), negate=True),
             P(W.LOWBITS_LT, 1, f_bits=rnd.randint(1, n), gamma=0),
             P(W.MSB_SHIFT, 2, c=rnd.randint(0, N - 1)),
             P(W.LT_UNSIGNED, 3, thr=float(N))]           # sentinel C_N: constant 1
    fb = preds[2].f_bits
    preds[2] = P(W.LOWBITS_LT, 1, f_bits=fb, gamma=rnd.randint(0, 1 << fb))
    return alpha, coef, preds


@pytest.mark.parametrize("r", [2, 3, 4])
def test_random_integer_specs_reconstruct(r):
    """Random partitions (including m = 1), ring coefficients of degree 0..3 and
    every predicate kind: exhaustive reconstruction at n = 5..8."""
    rnd = random.Random(300 + r)
    for trial in range(10):
        n = rnd.randint(5, 8)
        N = 1 << n
        alpha, coef, preds = _random_int_spec(rnd, n)
        S = O.compile_spec_int(n, alpha, coef, preds, lookup_r=r)
        xs = np.arange(-N // 2, N // 2, dtype=np.int64)
        want = [_direct(alpha, coef, preds, int(x), n) for x in xs]
        yw = np.array([w[0] for w in want], dtype=np.uint64)
        zw = np.array([w[1] for w in want], dtype=np.uint64)
        seed = rnd.getrandbits(128)
        y0, y1, z0, z1, r_in, r_out, _ = O.full(S, seed, np.arange(N, dtype=np.int64), xs, masks=True)
        assert np.array_equal(y0 + y1 - r_out, yw), (trial, n)
        assert np.array_equal(z0 ^ z1, zw), (trial, n)
        yp, zp = O.plain_many(S, xs)
        assert np.array_equal(yp, yw) and np.array_equal(zp, zw)


@pytest.mark.parametrize("r", [2, 3, 4])
def test_narrowest_domains_reconstruct(r):
    """n = 2, 3, 4 (one lookup level at r >= n, leading zero bits, atoms that
    are a leaf only): exhaustive reconstruction of random integer specs."""
    rnd = random.Random(500 + r)
    for n in (2, 3, 4):
        N = 1 << n
        for trial in range(4):
            alpha, coef, preds = _random_int_spec(rnd, n)
            S = O.compile_spec_int(n, alpha, coef, preds, lookup_r=r)
            xs = np.arange(-N // 2, N // 2, dtype=np.int64)
            want = [_direct(alpha, coef, preds, int(x), n) for x in xs]
            seed = rnd.getrandbits(128)
            y0, y1, z0, z1, r_in, r_out, _ = O.full(S, seed, np.arange(N, dtype=np.int64), xs, masks=True)
            assert np.array_equal(y0 + y1 - r_out, np.array([w[0] for w in want], dtype=np.uint64)), (n, trial)
            assert np.array_equal(z0 ^ z1, np.array([w[1] for w in want], dtype=np.uint64)), (n, trial)


@pytest.mark.parametrize("r", [2, 3, 4])
def test_maximum_sizes_reconstruct(r):
    """At the interface's limits (m = 64, p = 4, 16 predicates, T = 16,
    ell = 64): exhaustive reconstruction at n = 8 against the definition."""
    rnd = random.Random(700 + r)
    n, N = 8, 256
    alpha, coef, preds = max_int_spec(rnd, n)
    S = O.compile_spec_int(n, alpha, coef, preds, lookup_r=r)
    t = O.spec_tables(S)
    assert (t["m"], t["p"], t["T"], S.ell) == (64, 4, 16, 64)
    xs = np.arange(-N // 2, N // 2, dtype=np.int64)
    want = [_direct(alpha, coef, preds, int(x), n) for x in xs]
    yw = np.array([w[0] for w in want], dtype=np.uint64)
    zw = np.array([w[1] for w in want], dtype=np.uint64)
    for seed in (rnd.getrandbits(128), 2**127 + 1):
        y0, y1, z0, z1, r_in, r_out, _ = O.full(S, seed, np.arange(N, dtype=np.int64), xs, masks=True)
        assert np.array_equal(y0 + y1 - r_out, yw)
        assert np.array_equal(z0 ^ z1, zw)
    yp, zp = O.plain_many(S, xs)
    assert np.array_equal(yp, yw) and np.array_equal(zp, zw)
    # one predicate more, or one more atom, is past the limit
    with pytest.raises(O.SpecError):
        O.compile_spec_int(n, alpha, coef, preds + [P(W.LT_UNSIGNED, 1, thr=3.0)], lookup_r=r)
    with pytest.raises(O.SpecError):
        O.compile_spec_int(n, alpha, coef, preds[:-1] + [P(W.LOWBITS_LT, 2, f_bits=2, gamma=1)], lookup_r=r)


def test_integer_spec_rejections():
    n, N = 6, 64
    good = ([0, 32, N], [[1], [2]])
    O.compile_spec_int(n, *good)
    for alpha in ([1, 32, N], [0, 32, N - 1], [0, 32, 32, N], [0, 40, 32, N]):
        coef = [[0]] * (len(alpha) - 1)
        with pytest.raises(O.SpecError):
            O.compile_spec_int(n, alpha, coef)
    with pytest.raises(O.SpecError):
        O.compile_spec_int(n, *good, preds=[P(W.LT_SIGNED, 0, thr=2.5)])


def test_lookup_view_shift():
    """Real specs look intervals up in the offset-binary view (shift 2^(n-1)),
    integer specs in the canonical view (shift 0)."""
    S = O.compile_spec(W.clip_relu_spec(), 10, 4)
    assert S.lookup_c == 2**9 and S.is_int == 0
    Si = O.compile_spec_int(10, [0, 512, 1024], [[0, 1], [0, 0]])
    assert Si.lookup_c == 0 and Si.is_int == 1


def test_seed_is_128_bits():
    """Seeds that differ only above bit 64 give different masks; a seed below
    2^64 keys AES with its 8 bytes followed by zeros."""
    a = O.rand(7, 3, 0)
    b = O.rand(7 + 2**100, 3, 0)
    assert a != b
    S = O.compile_spec(W.clip_relu_spec(), 10, 4)
    xs = np.zeros(4, np.int64)
    r1 = O.full(S, 11, np.arange(4), xs, masks=True)[4]
    r2 = O.full(S, 11 + 2**64, np.arange(4), xs, masks=True)[4]
    assert not np.array_equal(r1, r2)


@pytest.mark.skipif(shutil.which("openssl") is None, reason="no openssl CLI")
def test_randomness_128_bit_key_vs_openssl():
    """R(e, pi, c) = AES_{seed as 16 LE bytes}(e | pi | c | 0) for a seed above 2^64."""
    seed = (0xFEDCBA9876543210 << 64) | 0x0123456789ABCDEF
    key = seed.to_bytes(16, "little")
    cases = [(5, 0, 0), (2**40 + 3, 66, 0), (393215, 70, 7)]
    ins = b"".join(e.to_bytes(8, "little") + p.to_bytes(2, "little") + c.to_bytes(2, "little")
                   + bytes(4) for e, p, c in cases)
    ref = subprocess.run(["openssl", "enc", "-aes-128-ecb", "-nopad", "-K", key.hex()],
                         input=ins, stdout=subprocess.PIPE, check=True).stdout
    for i, (e, p, c) in enumerate(cases):
        lo, hi = O.rand(seed, e, p, c)
        assert lo.to_bytes(8, "little") + hi.to_bytes(8, "little") == ref[16 * i:16 * i + 16]
