"""Pins for the oracle's DCF (CPU only).

A DCF key pair for (alpha, beta) must satisfy Eval_0(x) + Eval_1(x) =
beta * 1[x < alpha] for every x (the comparison function of Boyle et al.,
EUROCRYPT 2021, used by the paper's backend).  Checked by brute force over
every alpha and x on small domains, for the Z_2 group and Z_{2^64}^p.
"""
import random

import pytest

import oracle as O

M64 = 2**64 - 1


def _roots(rnd):
    return ((rnd.getrandbits(64), rnd.getrandbits(64)), (rnd.getrandbits(64), rnd.getrandbits(64)))


@pytest.mark.parametrize("n", [1, 2, 3, 6])
def test_dcf_z2_bruteforce(n):
    rnd = random.Random(100 + n)
    for alpha in range(2**n):
        for beta in (0, 1):
            k0, k1 = O.dcf_gen(n, 0, alpha, beta, *_roots(rnd))
            for x in range(2**n):
                got = O.dcf_eval(0, k0, x) ^ O.dcf_eval(1, k1, x)
                assert got == (beta if x < alpha else 0), (n, alpha, beta, x)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("n", [1, 4, 6])
def test_dcf_vector_bruteforce(n, p):
    rnd = random.Random(1000 * n + p)
    for alpha in range(2**n):
        beta = [rnd.getrandbits(64) for _ in range(p)]
        k0, k1 = O.dcf_gen(n, p, alpha, beta, *_roots(rnd))
        for x in range(2**n):
            a, b = O.dcf_eval(0, k0, x), O.dcf_eval(1, k1, x)
            got = [(u + v) & M64 for u, v in zip(a, b)]
            assert got == (beta if x < alpha else [0] * p), (n, p, alpha, x)


def test_dcf_wide_domain_sampled():
    """n = 24 and 32: sampled points around alpha and across the domain."""
    rnd = random.Random(5)
    for n in (24, 32):
        for _ in range(6):
            alpha = rnd.getrandbits(n)
            beta = [rnd.getrandbits(64) for _ in range(3)]
            k0, k1 = O.dcf_gen(n, 3, alpha, beta, *_roots(rnd))
            z0, z1 = O.dcf_gen(n, 0, alpha, 1, *_roots(rnd))
            pts = {0, 2**n - 1, alpha, (alpha - 1) % 2**n, (alpha + 1) % 2**n}
            pts |= {rnd.getrandbits(n) for _ in range(20)}
            for x in pts:
                got = [(u + v) & M64 for u, v in zip(O.dcf_eval(0, k0, x), O.dcf_eval(1, k1, x))]
                assert got == (beta if x < alpha else [0, 0, 0])
                assert O.dcf_eval(0, z0, x) ^ O.dcf_eval(1, z1, x) == int(x < alpha)


def test_dcf_keys_share_corrections_and_differ_in_roots():
    rnd = random.Random(9)
    k0, k1 = O.dcf_gen(8, 3, 77, [1, 2, 3], *_roots(rnd))
    assert (k0.root.lo, k0.root.hi) != (k1.root.lo, k1.root.hi)
    assert k0.root.lo & 3 == 0 and k1.root.lo & 3 == 0
    for i in range(8):
        assert (k0.scw[i].lo, k0.scw[i].hi) == (k1.scw[i].lo, k1.scw[i].hi)
        assert k0.scw[i].lo & 3 == 0
        assert list(k0.vcw[i][:3]) == list(k1.vcw[i][:3])
    assert list(k0.fin[:3]) == list(k1.fin[:3])


# ---- 2^r children per level (call 2's vector DCF) ---------------------------

def _keep_rand(rnd, n, p, r):
    levels, per = -(-n // r), 1 + (p + 1) // 2
    return [(rnd.getrandbits(64), rnd.getrandbits(64)) for _ in range(levels * per)]


@pytest.mark.parametrize("r", [2, 3, 4])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 6])
def test_dcfr_z2_bruteforce(n, r):
    rnd = random.Random(300 + 10 * n + r)
    for alpha in range(2**n):
        for beta in (0, 1):
            k0, k1 = O.dcfr_gen(n, r, 0, alpha, beta, *_roots(rnd), _keep_rand(rnd, n, 0, r))
            for x in range(2**n):
                got = O.dcfr_eval(0, k0, x) ^ O.dcfr_eval(1, k1, x)
                assert got == (beta if x < alpha else 0), (n, r, alpha, beta, x)


@pytest.mark.parametrize("r", [2, 3, 4])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("n", [1, 3, 4, 6, 7])
def test_dcfr_vector_bruteforce(n, p, r):
    rnd = random.Random(3000 * n + 10 * p + r)
    for alpha in range(2**n):
        beta = [rnd.getrandbits(64) for _ in range(p)]
        k0, k1 = O.dcfr_gen(n, r, p, alpha, beta, *_roots(rnd), _keep_rand(rnd, n, p, r))
        for x in range(2**n):
            a, b = O.dcfr_eval(0, k0, x), O.dcfr_eval(1, k1, x)
            got = [(u + v) & M64 for u, v in zip(a, b)]
            assert got == (beta if x < alpha else [0] * p), (n, p, r, alpha, x)


@pytest.mark.parametrize("r", [2, 3, 4])
def test_dcfr_wide_domain_sampled(r):
    """n = 23, 24 and 32: sampled points around alpha and across the domain."""
    rnd = random.Random(15 + r)
    for n in (23, 24, 32):
        for _ in range(6):
            alpha = rnd.getrandbits(n)
            beta = [rnd.getrandbits(64) for _ in range(3)]
            k0, k1 = O.dcfr_gen(n, r, 3, alpha, beta, *_roots(rnd), _keep_rand(rnd, n, 3, r))
            pts = {0, 2**n - 1, alpha, (alpha - 1) % 2**n, (alpha + 1) % 2**n}
            pts |= {alpha ^ (1 << j) for j in range(n)}
            pts |= {rnd.getrandbits(n) for _ in range(20)}
            for x in pts:
                got = [(u + v) & M64 for u, v in zip(O.dcfr_eval(0, k0, x), O.dcfr_eval(1, k1, x))]
                assert got == (beta if x < alpha else [0, 0, 0]), (n, r, alpha, x)


@pytest.mark.parametrize("r", [2, 3, 4])
def test_dcfr_corrections(r):
    """Both keys carry the same corrections; alpha's child gets the supplied
    randomness at every level but the last, every other child corrects the
    parties' children to equal seeds and values (checked on the first level,
    where both parties expand their roots: child c is H(root, c), its value
    H(root, 2^r + j), child c taking words c p .. c p + p - 1).  At the last level alpha's child's value is corrected
    like the others (the brute-force tests check that this zeroes x = alpha)
    and all seed and control-bit corrections are zero (never used)."""
    rnd = random.Random(21 + r)
    n, p = 12, 3
    alpha = rnd.getrandbits(n)
    beta = [5, 6, 7]
    kr = _keep_rand(rnd, n, p, r)
    r0, r1 = _roots(rnd)
    k0, k1 = O.dcfr_gen(n, r, p, alpha, beta, r0, r1, kr)
    assert k0.root.lo & 3 == 0 and k1.root.lo & 3 == 0
    levels, per, C = n // r, 1 + (p + 1) // 2, 1 << r
    for i in range(levels):
        a = (alpha >> (r * (levels - 1 - i))) & (C - 1)
        for c in range(C):
            assert (k0.scw[i][c].lo, k0.scw[i][c].hi) == (k1.scw[i][c].lo, k1.scw[i][c].hi)
            assert k0.tcw[i][c] == k1.tcw[i][c] and k0.scw[i][c].lo & 3 == 0
            assert list(k0.vcw[i][c][:p]) == list(k1.vcw[i][c][:p])
        lo, hi = kr[i * per]
        on_path = ((k0.scw[i][a].lo, k0.scw[i][a].hi) == (lo & ~3, hi) and
                   list(k0.vcw[i][a][:p]) == [kr[i * per + 1][0], kr[i * per + 1][1], kr[i * per + 2][0]])
        assert on_path == (i < levels - 1), (r, i)
    for c in range(C):
        assert (k0.scw[levels - 1][c].lo, k0.scw[levels - 1][c].hi, k0.tcw[levels - 1][c]) == (0, 0, 0)
    # level 0: the parties' roots carry t = 0 and t = 1, V_alpha = 0
    a0 = alpha >> (n - r)
    for c in range(C):
        if c == a0:
            continue
        c0, c1 = O.prg(k0.root.lo, k0.root.hi, c), O.prg(k1.root.lo, k1.root.hi, c)
        assert k0.scw[0][c].lo == (c0[0] ^ c1[0]) & ~3 and k0.scw[0][c].hi == c0[1] ^ c1[1]
        assert k0.tcw[0][c] == (c0[0] ^ c1[0]) & 1
        # child c's values: words c p .. c p + p - 1 of H(s, C), H(s, C + 1), ...
        stream0 = [w for j in range(((c + 1) * p + 1) // 2) for w in O.prg(k0.root.lo, k0.root.hi, C + j)]
        stream1 = [w for j in range(((c + 1) * p + 1) // 2) for w in O.prg(k1.root.lo, k1.root.hi, C + j)]
        v0, v1 = stream0[c * p:(c + 1) * p], stream1[c * p:(c + 1) * p]
        for q in range(p):
            w = (v1[q] - v0[q] + (beta[q] if c < a0 else 0)) & M64
            assert k0.vcw[0][c][q] == (-w) & M64, (r, c, q)   # (-1)^{t_1}, t_1 = 1 at the root


@pytest.mark.parametrize("r", [2, 3, 4])
def test_dcfr_corrections_do_not_single_out_alpha_child(r):
    """The per-child corrections must not show which child lies on alpha's
    path: over 600 keys, the control-bit correction of alpha's child and of
    the other children are each 1 about half the time (a constant on alpha's
    child would single it out; its seed correction is the supplied randomness,
    checked in test_dcfr_corrections)."""
    rnd = random.Random(77 + r)
    n, p = 12, 3
    C, levels = 1 << r, 12 // r
    on = [0, 0]
    off = [0, 0]
    for _ in range(600):
        alpha = rnd.getrandbits(n)
        k0, _ = O.dcfr_gen(n, r, p, alpha, [1, 2, 3], *_roots(rnd), _keep_rand(rnd, n, p, r))
        for i in range(levels - 1):  # the last level's control-bit corrections are zero
            a = (alpha >> (r * (levels - 1 - i))) & (C - 1)
            for c in range(C):
                bucket = on if c == a else off
                bucket[0] += k0.tcw[i][c]
                bucket[1] += 1
    frac_on, frac_off = on[0] / on[1], off[0] / off[1]
    # at least 1200 and 3600 Bernoulli(1/2) samples: 5 sigma is about 0.072 and 0.042
    assert abs(frac_on - 0.5) < 0.072, frac_on
    assert abs(frac_off - 0.5) < 0.042, frac_off


# ---- the Z_2 DCF with early termination (a 2^nu-bit leaf, nu = min(7, n)) ----

@pytest.mark.parametrize("n", [1, 3, 6, 7, 8, 9, 10])
def test_dcfz_bruteforce(n):
    """Every alpha and x: Eval_0(x) ^ Eval_1(x) = 1[x < alpha].  n <= 7 is a
    single leaf (no tree level), n = 8..10 one to three levels above the leaves."""
    rnd = random.Random(700 + n)
    assert O.dcfz_nu(n) == min(7, n)
    alphas = range(2**n) if n <= 8 else sorted({0, 1, 127, 128, 129, 2**n - 1} | {rnd.getrandbits(n) for _ in range(40)})
    for alpha in alphas:
        k0, k1 = O.dcfz_gen(n, alpha, *_roots(rnd))
        for x in range(2**n):
            assert O.dcfz_eval(0, k0, x) ^ O.dcfz_eval(1, k1, x) == int(x < alpha), (n, alpha, x)


def test_dcfz_wide_domain_sampled():
    rnd = random.Random(77)
    for n in (16, 24, 31, 32):
        for _ in range(8):
            alpha = rnd.getrandbits(n)
            k0, k1 = O.dcfz_gen(n, alpha, *_roots(rnd))
            pts = {0, 2**n - 1, alpha, (alpha - 1) % 2**n, (alpha + 1) % 2**n, alpha ^ 64, alpha ^ 128}
            pts |= {rnd.getrandbits(n) for _ in range(30)}
            for x in pts:
                assert O.dcfz_eval(0, k0, x) ^ O.dcfz_eval(1, k1, x) == int(x < alpha), (n, alpha, x)


@pytest.mark.parametrize("n", [8, 12, 24])
def test_dcfz_tree_is_the_textbook_dcf_on_the_high_bits(n):
    """The levels above the leaves are the textbook construction over the high
    n - nu bits: same roots give the same seed, control-bit and value
    corrections as orc_dcf_gen(n - nu, Z_2, alpha >> nu, beta = 1)."""
    rnd = random.Random(n)
    nu = O.dcfz_nu(n)
    for _ in range(5):
        alpha = rnd.getrandbits(n)
        roots = _roots(rnd)
        z0, z1 = O.dcfz_gen(n, alpha, *roots)
        t0, t1 = O.dcf_gen(n - nu, 0, alpha >> nu, 1, *roots)
        assert (z0.root.lo, z0.root.hi) == (t0.root.lo, t0.root.hi)
        for i in range(n - nu):
            assert (z0.scw[i].lo, z0.scw[i].hi) == (t0.scw[i].lo, t0.scw[i].hi)
            assert (z0.tl[i], z0.tr[i], z0.vcw[i]) == (t0.tl[i], t0.tr[i], t0.vcw[i][0])
            assert (z1.scw[i].lo, z1.scw[i].hi) == (z0.scw[i].lo, z0.scw[i].hi)
        assert (z0.leaf.lo, z0.leaf.hi) == (z1.leaf.lo, z1.leaf.hi)


def test_dcfz_leaf_outputs_agree_off_alpha_leaf():
    """At every leaf other than alpha's the parties' 128-bit leaf vectors are
    equal (their seeds and control bits agree), so only the path decides."""
    rnd = random.Random(3)
    n, alpha = 10, 0b1011001101
    k0, k1 = O.dcfz_gen(n, alpha, *_roots(rnd))
    for hi in range(2**(n - 7)):
        if hi == alpha >> 7:
            continue
        f = [O.dcfz_eval(0, k0, (hi << 7) | j) ^ O.dcfz_eval(1, k1, (hi << 7) | j) for j in range(128)]
        assert f == [int(hi < alpha >> 7)] * 128
