"""The paper's rewrite lemmas and Protocol 3, checked exhaustively (CPU only).

These pin the identities the oracle's keygen and evaluation rely on, and the
oracle's implementation of the Protocol "Compile a scalar gate instance"
(lookup part), by brute force over tiny domains.
"""
import itertools
import random

import pytest

import oracle as O

M64 = 2**64 - 1


@pytest.mark.parametrize("n", [1, 3, 5])
def test_masked_rewrite_unsigned(n):
    """Lemma (masked rewrite): 1[x<b] = 1[xh<theta] ^ 1[xh<r] ^ w."""
    N = 2**n
    for x, r, b in itertools.product(range(N), range(N), range(N + 1)):
        xh = (x + r) % N
        theta, w = (r + b) % N, int(r + b >= N)
        assert int(x < b) == int(xh < theta) ^ int(xh < r) ^ w


@pytest.mark.parametrize("n,f", [(5, 1), (5, 3), (6, 6)])
def test_masked_rewrite_lowbits(n, f):
    """Low-bit lemma: 1[(x mod 2^f)<g] = 1[xh_f<theta] ^ 1[xh_f<r_f] ^ w."""
    N, Nf = 2**n, 2**f
    for x, r, g in itertools.product(range(N), range(N), range(Nf + 1)):
        xh = (x + r) % N
        rf, xf = r % Nf, xh % Nf
        theta, w = (rf + g) % Nf, int(rf + g >= Nf)
        assert int((x % Nf) < g) == int(xf < theta) ^ int(xf < rf) ^ w


@pytest.mark.parametrize("n", [2, 4])
def test_signed_and_msb_shift_rewrites(n):
    N, s = 2**n, 2**(n - 1)

    def signed(u):
        return u - N if u >= s else u

    for x, r in itertools.product(range(N), range(N)):
        xh = (x + r) % N
        for beta in range(-s, s):
            bp = (beta + s) % N
            theta, w = (r + bp) % N, int(r + bp >= N)
            v = (xh + s) % N
            assert int(signed(x) < beta) == int(v < theta) ^ int(v < r) ^ w
        for c in range(N):
            xc = (xh + c) % N
            th, w = (r + s) % N, int(r + s >= N)
            msb = int((x + c) % N >= s)
            assert msb == 1 ^ (int(xc < th) ^ int(xc < r) ^ w)


def test_interval_indicator_partition():
    """Lemmas: 1[x in I_i] = 1[x<a_{i+1}] ^ 1[x<a_i]; exactly one is set."""
    n, N = 5, 32
    rnd = random.Random(3)
    for _ in range(40):
        m = rnd.randint(1, 10)
        alpha = [0] + sorted(rnd.sample(range(1, N), m - 1)) + [N]
        for x in range(N):
            J = [int(x < alpha[i + 1]) ^ int(x < alpha[i]) for i in range(m)]
            assert sum(J) == 1 and alpha[J.index(1)] <= x < alpha[J.index(1) + 1]


def test_masked_interval_indicator_corollary():
    n, N = 4, 16
    alpha = [0, 3, 7, 12, 16]
    for x, r in itertools.product(range(N), range(N)):
        xh = (x + r) % N
        w = [int(r + a >= N) for a in alpha]
        assert w[0] == 0 and w[-1] == 1
        for i in range(len(alpha) - 1):
            ind = int((xh < (alpha[i + 1] + r) % N) ^ (xh < (alpha[i] + r) % N) ^ w[i + 1] ^ w[i])
            assert ind == int(alpha[i] <= x < alpha[i + 1])


def test_interval_translation_at_most_one_split():
    n, N = 5, 32
    rnd = random.Random(4)
    for _ in range(60):
        m = rnd.randint(1, 12)
        alpha = [0] + sorted(rnd.sample(range(1, N), m - 1)) + [N]
        for r in range(N):
            splits = sum(1 for i in range(m) if alpha[i] + r < N < alpha[i + 1] + r)
            assert splits <= 1
            if r == 0 or (N - r) in alpha:
                assert splits == 0


@pytest.mark.parametrize("n", [2, 3, 5, 6])
def test_protocol3_lookup_table(n):
    """Protocol 3: |B| = M+1, |ord| = M, M = min(m+1, N); the table maps every
    masked value to the x-space interval of its preimage."""
    N = 2**n
    rnd = random.Random(50 + n)
    parts = [[0, N]]
    for _ in range(25):
        m = rnd.randint(1, N)
        parts.append([0] + sorted(rnd.sample(range(1, N), m - 1)) + [N])
    parts.append(list(range(N + 1)))  # m = N: no padding possible
    for alpha in parts:
        m = len(alpha) - 1
        for r in range(N):
            B, ordv = O.protocol3(n, alpha, r)
            M = min(m + 1, N)
            assert len(B) == M + 1 and len(ordv) == M
            assert B[0] == 0 and B[-1] == N and all(B[j] < B[j + 1] for j in range(M))
            for j in range(M):
                for v in range(B[j], B[j + 1]):
                    x = (v - r) % N
                    assert alpha[ordv[j]] <= x < alpha[ordv[j] + 1]


def test_protocol3_literal_lookup_with_dcfs():
    """Literal interval lookup (one vector DCF per Protocol-3 boundary):
    LUT(v) = v_{M-1} + sum_{j>=1} (v_{j-1} - v_j) 1[v < B_j] reconstructs the
    active interval's payload for every v."""
    n, N = 5, 32
    rnd = random.Random(77)
    alpha = [0, 5, 11, 12, 20, 32]
    payload = [[rnd.getrandbits(64) for _ in range(3)] for _ in range(len(alpha) - 1)]
    for r in rnd.sample(range(N), 8) + [0]:
        B, ordv = O.protocol3(n, alpha, r)
        M = len(ordv)
        vals = [payload[o] for o in ordv]
        keys = []
        for j in range(1, M):
            beta = [(a - b) & M64 for a, b in zip(vals[j - 1], vals[j])]
            keys.append(O.dcf_gen(n, 3, B[j], beta, (rnd.getrandbits(64), 0),
                                  (rnd.getrandbits(64), 1)))
        s0 = [rnd.getrandbits(64) for _ in range(3)]
        s1 = [(a - b) & M64 for a, b in zip(vals[M - 1], s0)]
        for v in range(N):
            tot = [(a + b) & M64 for a, b in zip(s0, s1)]
            for k0, k1 in keys:
                for q, (a, b) in enumerate(zip(O.dcf_eval(0, k0, v), O.dcf_eval(1, k1, v))):
                    tot[q] = (tot[q] + a + b) & M64
            x = (v - r) % N
            istar = next(i for i in range(len(alpha) - 1) if alpha[i] <= x < alpha[i + 1])
            assert tot == payload[istar]
