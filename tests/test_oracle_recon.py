"""Reconstruction pins for the oracle's keygen + evaluation (CPU only).

For every x of small domains and several dealer seeds:
  y_0 + y_1 = P_{i*}(x) + r_out (mod 2^64) and z_0 ^ z_1 = predicate bits,
compared with the plaintext evaluator; the plaintext evaluator is itself
pinned by closed forms (clip-ReLU is exact in fixed point) and by the
rounding bound against the real-valued pieces.  Also pins the paper's
worked example (appendix "A complete (F, Phi) pair").
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2606_09551_amd import workloads as W

M64 = 2**64 - 1
P = W.PredDesc


def _mixed_pred_spec():
    """Every predicate kind, XOR-combined outputs, degree 3 pieces (p = 4)."""
    preds = [P(W.LT_SIGNED, 0, thr=-1.0), P(W.LT_SIGNED, 0, thr=2.5),       # x in [-1, 2.5)
             P(W.LT_UNSIGNED, 1, thr=5.0),
             P(W.LOWBITS_LT, 2, f_bits=3, gamma=5, negate=True),
             P(W.MSB_SHIFT, 3, c=37),
             P(W.MSB_SHIFT, 4, c=0), P(W.LT_SIGNED, 4, thr=0.75)]
    iv = [(-math.inf, -3.0), (-3.0, -0.5), (-0.5, 0.25), (0.25, 4.0), (4.0, math.inf)]
    pcs = [[1.5], [0.25, -1.0, 0.5], [0.0, 2.0, 0.0, -0.125], [-1.0, 0.5, 0.25, 0.0625], [3.0, -0.5]]
    return W.SpecDesc("mixed", iv, pcs, preds)


def _degree0_spec():
    iv = [(-math.inf, -1.0), (-1.0, 1.0), (1.0, math.inf)]
    return W.SpecDesc("steps", iv, [[-2.0], [0.5], [3.0]], [P(W.LT_SIGNED, 0, thr=1.0)])


CASES = [
    (W.clip_relu_spec(), 10, 4),
    (W.clip_relu_spec(), 8, 2),
    (W.gelu_spec(f=5), 10, 5),
    (W.exp_spec(f=4), 10, 4),
    (W.recip_spec(3, f=5), 10, 5),
    (W.relu_worked_example_spec(), 8, 0),
    (_mixed_pred_spec(), 9, 3),
    (_degree0_spec(), 6, 2),
]


@pytest.mark.parametrize("r", [2, 3, 4])
@pytest.mark.parametrize("desc,n,f", CASES, ids=lambda v: getattr(v, "name", str(v)))
def test_reconstruction_exhaustive(desc, n, f, r):
    S = O.compile_spec(desc, n, f, lookup_r=r)
    s = 2**(n - 1)
    xs = np.arange(-s, s, dtype=np.int64)
    yp, zp = O.plain_many(S, xs)
    for seed in (1, 0xC2, 2**64 - 5):
        elems = np.arange(len(xs), dtype=np.int64) + seed % 1000
        y0, y1, z0, z1, _ = O.full(S, seed, elems, xs)
        _, _, _, r_out = O.keygen(S, seed, elems[:64])
        assert np.array_equal(y0[:64] + y1[:64] - r_out, yp[:64])
        # r_out of every element, without storing all keys
        rout = np.array([O.rand(seed, int(e), 0)[1] for e in elems], dtype=np.uint64)
        assert np.array_equal(y0 + y1 - rout, yp), desc.name
        assert np.array_equal(z0 ^ z1, zp), desc.name


def test_clip_relu_closed_form_exact():
    """clip(x, 0, 6) is exact at F_out = 2f: y = clip(x, 0, 6 * 2^f) * 2^f."""
    n, f = 16, 8
    S = O.compile_spec(W.clip_relu_spec(), n, f)
    for x in list(range(-2**15, -2**15 + 50)) + list(range(-300, 2000)) + [2**15 - 1]:
        y, z = O.plain(S, x)
        want = min(max(x, 0), 6 * 2**f) * 2**f
        assert y == want % 2**64
        assert z == int(x < 0) | (int(x < 6 * 2**f) << 1)


@pytest.mark.parametrize("desc,n,f", [(W.gelu_spec(), 24, 12), (W.exp_spec(), 24, 12),
                                      (W.recip_spec(7), 24, 12), (W.rsqrt_spec(), 24, 12),
                                      (_mixed_pred_spec(), 14, 5)],
                         ids=lambda v: getattr(v, "name", str(v)))
def test_plaintext_within_rounding_bound(desc, n, f):
    """|y / 2^F_out - P_real(x)| <= sum_l 0.5 |x|^l / 2^F_out (coefficient rounding)."""
    S = O.compile_spec(desc, n, f)
    t = O.spec_tables(S)
    g = np.random.Generator(np.random.PCG64(3))
    s = 2**(n - 1)
    xs = list(g.integers(-s, s, size=400)) + [a for a in t["alpha"][1:-1]] + \
        [a - 1 for a in t["alpha"][1:-1]] + [-s, s - 1]
    for x in xs:
        x = int(x)
        y, _ = O.plain(S, x)
        y = y - 2**64 if y >= 2**63 else y
        i = next(i for i, (lo, hi) in enumerate(desc.intervals) if lo <= x / 2**f < hi)
        real = sum(c * (x / 2**f) ** l for l, c in enumerate(desc.pieces[i]))
        bound = sum(0.5 * abs(x) ** l for l in range(t["p"])) / 2**t["F_out"]
        assert abs(y / 2**t["F_out"] - real) <= bound + 1e-12 * (1 + abs(real))


@pytest.mark.parametrize("n", [4, 8, 10])
def test_worked_example_relu(n):
    """Paper appendix: m = 2 intervals, M = 3, p = 2 (a, b); packed comparison
    holds exactly the two atoms 1[xh < (r + N/2) mod N] and 1[xh < r]."""
    N = 2**n
    S = O.compile_spec(W.relu_worked_example_spec(), n, 0)
    t = O.spec_tables(S)
    assert (t["m"], t["p"], t["T"]) == (2, 2, 2)
    B, ordv = O.protocol3(n, t["aprime"], 12345 % N)
    assert len(ordv) == min(t["m"] + 1, N) == 3
    seed = 99
    elems = np.arange(6, dtype=np.int64)
    K0, K1, r_in, r_out = O.keygen(S, seed, elems)
    for i in range(len(elems)):
        r = int(r_in[i]) % N
        thr = []
        for a in range(2):
            f = [O.dcfz_eval(0, K0[i].atom[a], u) ^ O.dcfz_eval(1, K1[i].atom[a], u) for u in range(N)]
            # reconstructs a threshold function 1[u < theta]
            theta = sum(f)
            assert f == [1] * theta + [0] * (N - theta)
            thr.append(theta)
        assert thr == [(r + N // 2) % N, r]
    xs = np.arange(-N // 2, N // 2, dtype=np.int64)
    y0, y1, z0, z1, _ = O.full(S, seed, np.arange(N, dtype=np.int64), xs)
    rout = np.array([O.rand(seed, e, 0)[1] for e in range(N)], dtype=np.uint64)
    assert np.array_equal(y0 + y1 - rout, np.maximum(xs, 0).astype(np.uint64))
    assert np.array_equal(z0 ^ z1, (xs < 0).astype(np.uint64))


def test_key_shape_is_mask_independent():
    """Shape (T, atom widths, payload p, n) is identical across dealer seeds."""
    S = O.compile_spec(_mixed_pred_spec(), 12, 4)
    shapes = set()
    for seed in range(0, 1000, 7):
        K0, K1, _, _ = O.keygen(S, seed, np.arange(2, dtype=np.int64))
        for K in (K0[0], K1[1]):
            shapes.add((tuple(K.atom[t].n for t in range(S.T)),
                        tuple(K.atom[t].nu for t in range(S.T)), K.coeff.n, K.coeff.p))
    assert len(shapes) == 1


def test_wide_domain_sampled_reconstruction():
    """Config-sized specs (n = 24): sampled elements, including boundary inputs."""
    for desc in (W.gelu_spec(), W.exp_spec(), W.recip_spec(8), W.rsqrt_spec()):
        S = O.compile_spec(desc, 24, 12)
        t = O.spec_tables(S)
        g = np.random.Generator(np.random.PCG64(21))
        xs = np.concatenate([g.integers(-2**23, 2**23, size=24),
                             np.array(t["alpha"][1:-1]), np.array(t["alpha"][1:-1]) - 1,
                             np.array([-2**23, 2**23 - 1])]).astype(np.int64)
        elems = np.arange(len(xs), dtype=np.int64) * 7919
        y0, y1, z0, z1, _ = O.full(S, 0xABC, elems, xs)
        rout = np.array([O.rand(0xABC, int(e), 0)[1] for e in elems], dtype=np.uint64)
        yp, zp = O.plain_many(S, xs)
        assert np.array_equal(y0 + y1 - rout, yp)
        assert np.array_equal(z0 ^ z1, zp)
