"""Host-side checks of the C-ABI library (CPU only: no kernel is launched).

The shared library must load, export every function include/fusefss.h
declares, quantise specs to exactly the oracle's integer tables (two
independent implementations of the same rules), reject invalid specs with
the documented codes, and size keys independently of masks.
"""
import ctypes as C
import math
import os
import re

import pytest

import oracle as O
from paper_2606_09551_amd import fss as F
from paper_2606_09551_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            src = open(os.path.join(inc, fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"^\s*(?:const\s+)?[\w]+\s*\*?\s*(fss_\w+)\s*\(", src, flags=re.M))
    return names


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 20
    for n in sorted(names):
        assert hasattr(F.lib, n), n
    assert "gfx950" in F.version()


# The calls of the boundary: the spec in both forms, keygen, the plain and
# the fused evaluators, the autotuner.
BOUNDARY = ["fss_compile_spec", "fss_compile_spec_int", "fss_key_bytes", "fss_keygen", "fss_eval",
            "fss_eval_batch", "fss_autotune", "fss_spec_free"]


def test_boundary_calls_declared_and_exported():
    names = declared_functions()
    for n in BOUNDARY:
        assert n in names, n
        assert hasattr(F.lib, n), n


def test_integer_spec_tables_match_oracle():
    """The worked ReLU (alpha = 0, N/2, N) and random integer specs: the
    library's quantised tables equal the oracle's, with the unshifted lookup view."""
    import random
    P = W.PredDesc
    rnd = random.Random(41)
    cases = [(10, [0, 512, 1024], [[0, 1], [0, 0]], [P(W.MSB_SHIFT, 0, c=0)])]
    for _ in range(6):
        n = rnd.randint(4, 24)
        N = 1 << n
        m = rnd.randint(1, 12)
        alpha = [0] + sorted(rnd.sample(range(1, N), m - 1)) + [N]
        d = rnd.randint(0, 3)
        coef = [[rnd.getrandbits(64) for _ in range(d + 1)] for _ in range(m)]
        preds = [P(W.LT_SIGNED, 0, thr=float(rnd.randint(-N // 2, N // 2))),
                 P(W.LT_UNSIGNED, 1, thr=float(rnd.randint(1, N - 1))),
                 P(W.LOWBITS_LT, 1, f_bits=min(n, 3), gamma=2), P(W.MSB_SHIFT, 2, c=rnd.randint(0, N - 1))]
        cases.append((n, alpha, coef, preds))
    # the interface's largest spec (64 intervals, degree 3, 16 predicates,
    # 16 atoms, 64 output bits) at n = 8 and 32
    from maxspec import max_int_spec
    cases += [(n, *max_int_spec(rnd, n)) for n in (8, 32)]
    for n, alpha, coef, preds in cases:
        lib_t = F.Spec.integer(n, alpha, coef, preds).query(n, 0)
        orc = O.spec_tables(O.compile_spec_int(n, alpha, coef, preds))
        for k in ("m", "d", "p", "F_out", "T", "ell", "aprime", "coef"):
            assert lib_t[k] == orc[k], (n, k)
        atoms = [(k, c % 2**64, msk) for k, c, msk in zip(lib_t["atom_k"], lib_t["atom_c"], lib_t["atom_is_mask"])]
        assert atoms == [(a[0], a[1], a[2]) for a in orc["atoms"]]


def test_integer_spec_rejections():
    P = W.PredDesc
    N = 64
    F.Spec.integer(6, [0, 32, N], [[1], [2]])
    for alpha in ([1, 32, N], [0, 32, N - 1], [0, 32, 32, N], [0, 40, 32, N]):
        with pytest.raises(F.FssError) as e:
            F.Spec.integer(6, alpha, [[0]] * (len(alpha) - 1))
        assert e.value.code == -1
    with pytest.raises(F.FssError) as e:
        F.Spec.integer(6, [0, 32, N], [[1], [2]], [P(W.LT_SIGNED, 0, thr=2.5)])
    assert e.value.code == -1
    with pytest.raises(F.FssError) as e:
        F.Spec.integer(40, [0, 2**40], [[1]])
    assert e.value.code == -2
    s = F.Spec.integer(6, [0, 32, N], [[1], [2]])
    for n, f in ((7, 0), (6, 2)):
        with pytest.raises(F.FssError) as e:
            s.query(n, f)
        assert e.value.code == -4


def test_seed_is_128_bits_at_the_boundary():
    for bad in (-1, 2**128):
        with pytest.raises(ValueError):
            F.seed_bytes(bad)
    assert bytes(F.seed_bytes(2**64 + 5)) == (2**64 + 5).to_bytes(16, "little")


SPECS = [(W.clip_relu_spec(), 16, 8), (W.gelu_spec(), 24, 12), (W.exp_spec(), 24, 12),
         (W.recip_spec(7), 24, 12), (W.recip_spec(9), 24, 12), (W.rsqrt_spec(), 24, 12),
         (W.relu_worked_example_spec(), 10, 0), (W.gelu_spec(f=5), 10, 5)]


@pytest.mark.parametrize("desc,n,f", SPECS, ids=lambda v: getattr(v, "name", str(v)))
def test_quantised_tables_match_oracle(desc, n, f):
    lib_t = F.Spec(desc).query(n, f)
    orc = O.spec_tables(O.compile_spec(desc, n, f))
    for k in ("m", "d", "p", "F_out", "T", "ell", "aprime", "coef"):
        assert lib_t[k] == orc[k], k
    atoms = [(k, c % 2**64, msk) for k, c, msk in zip(lib_t["atom_k"], lib_t["atom_c"], lib_t["atom_is_mask"])]
    assert atoms == [(a[0], a[1], a[2]) for a in orc["atoms"]]


def test_quantisers_agree_over_the_size_grid():
    """Every real spec of the workloads at n = 2..32 and f from 0 to n - 1:
    the library and the oracle accept the same (n, f) (a partition that
    collapses, coefficients past 2^62 and the like are refused by both) and,
    where they accept, build the same tables."""
    descs = [W.clip_relu_spec(), W.gelu_spec(), W.exp_spec(), W.recip_spec(7), W.rsqrt_spec(),
             W.relu_worked_example_spec()]
    accepted = refused = 0
    for desc in descs:
        for n in (2, 3, 4, 6, 8, 12, 16, 20, 24, 28, 31, 32):
            for f in sorted({0, 1, 2, n // 4, n // 2, n - 2, n - 1} & set(range(n))):
                try:
                    lib_t = F.Spec(desc).query(n, f)
                except F.FssError:
                    lib_t = None
                try:
                    orc = O.spec_tables(O.compile_spec(desc, n, f))
                except O.SpecError:
                    orc = None
                assert (lib_t is None) == (orc is None), (desc.name, n, f)
                if lib_t is None:
                    refused += 1
                    continue
                accepted += 1
                for k in ("m", "d", "p", "F_out", "T", "ell", "aprime", "coef"):
                    assert lib_t[k] == orc[k], (desc.name, n, f, k)
                atoms = [(k, c % 2**64, msk) for k, c, msk in
                         zip(lib_t["atom_k"], lib_t["atom_c"], lib_t["atom_is_mask"])]
                assert atoms == [(a[0], a[1], a[2]) for a in orc["atoms"]], (desc.name, n, f)
    assert accepted > 150 and refused > 150


def test_mixed_predicates_match_oracle():
    P = W.PredDesc
    preds = [P(W.LT_SIGNED, 0, thr=-1.0), P(W.LT_SIGNED, 0, thr=2.5), P(W.LT_UNSIGNED, 1, thr=5.0),
             P(W.LOWBITS_LT, 2, f_bits=3, gamma=5, negate=True), P(W.MSB_SHIFT, 3, c=37),
             P(W.LT_SIGNED, 4, thr=-math.inf), P(W.LOWBITS_LT, 5, f_bits=2, gamma=4)]
    desc = W.SpecDesc("mixed", [(-math.inf, 0.5), (0.5, math.inf)], [[1.0, 2.0, 0.5, 0.25], [0.0]], preds)
    lib_t = F.Spec(desc).query(12, 4)
    orc = O.spec_tables(O.compile_spec(desc, 12, 4))
    assert lib_t["T"] == orc["T"] and lib_t["ell"] == orc["ell"] and lib_t["coef"] == orc["coef"]


@pytest.mark.parametrize("bad,code", [
    (dict(intervals=[(0.0, 1.0), (1.0, math.inf)], pieces=[[0.0], [0.0]]), -1),
    (dict(intervals=[(-math.inf, 0.0), (0.5, math.inf)], pieces=[[0.0], [0.0]]), -1),
    (dict(intervals=[(-math.inf, math.inf)], pieces=[[0.0, 0, 0, 0, 1.0]]), -1),
])
def test_compile_rejects_invalid(bad, code):
    with pytest.raises(F.FssError) as e:
        F.Spec(W.SpecDesc("bad", bad["intervals"], bad["pieces"]))
    assert e.value.code == code


def test_quantisation_errors_reported():
    desc = W.SpecDesc("coll", [(-math.inf, 0.001), (0.001, 0.002), (0.002, math.inf)], [[0.0]] * 3)
    s = F.Spec(desc)
    with pytest.raises(F.FssError) as e:
        s.query(16, 8)
    assert e.value.code == -1
    with pytest.raises(F.FssError) as e:
        F.Spec(W.clip_relu_spec()).query(33, 8)
    assert e.value.code == -2
    big = W.SpecDesc("big", [(-math.inf, math.inf)], [[0.0, 0.0, 0.0, 1e6]])
    with pytest.raises(F.FssError) as e:
        F.Spec(big).query(16, 8)
    assert e.value.code == -1


def test_and_or_need_postprocessing():
    desc = W.SpecDesc("andp", [(-math.inf, math.inf)], [[0.0]], [W.PredDesc(W.LT_SIGNED, 0, thr=1.0)])
    desc.preds[0].__class__  # frozen dataclass; build one with combine = AND
    from dataclasses import dataclass

    @dataclass(frozen=True)
    class PC(W.PredDesc):
        combine: int = 1

    desc.preds = [PC(W.LT_SIGNED, 0, thr=1.0)]
    with pytest.raises(F.FssError) as e:
        F.Spec(desc)
    assert e.value.code == -3


@pytest.mark.parametrize("r", [2, 3, 4])
def test_key_bytes_shape(r):
    """Key size is a function of (spec, n, f, N, lookup radix) only; tiles of 64 elements."""
    s = F.Spec(W.gelu_spec(), lookup_r=r)
    assert s.lookup_r == r
    per_tile = s.key_bytes(24, 12, 64) - s.key_bytes(24, 12, 0)
    assert per_tile % 256 == 0
    for N in (1, 63, 64, 65, 393216):
        assert s.key_bytes(24, 12, N) == 16384 + ((N + 63) // 64) * per_tile
    # 2 Z_2 threshold atoms (root, 24 - 7 tree levels, value bits, 16-byte leaf correction; the
    # signed view's mask query is the lookup's own comparison), w shares, then the lookup DCF:
    # root, 24 / r levels x 2^r children of seed (16 B) and p = 3 value corrections, rho and
    # r_out shares; the one-time record (x-hat of each element, the sentinel)
    expect = (2 * (64 * 16 * 18 + 64 * 8 + 64 * 16) + 64 * 8 + 64 * 16 + (24 // r) * 2**r * 64 * (16 + 3 * 8)
              + 3 * 64 * 8 + 64 * 8 + 64 * 8 + 8)
    assert per_tile == (expect + 255) // 256 * 256
    c = F.Spec(W.clip_relu_spec(), lookup_r=r)
    # n = 16, p = 2: atoms 2 * ((1 + 9) * 16 + 8 + 16), w 8, root 16, ceil(16 / r) levels x 2^r
    # x (16 + 16), rho 16, r_out 8 per element; the one-time record; tiles rounded to 256 bytes
    elem = 2 * (10 * 16 + 8 + 16) + 8 + 16 + (-(-16 // r)) * 2**r * 32 + 16 + 8
    assert c.key_bytes(16, 8, 4096) - 16384 == 64 * ((64 * elem + 64 * 8 + 8 + 255) // 256 * 256)


def test_lookup_radix_setting():
    """The radix is per spec; the shared levels of the lookup points follow it.
    GELU at n = 24, f = 12: the 17 lookup points span W = 16 * 3072 + 1 values.
    Cost of the walks in levels, K bits below the shared levels (a multiple of
    r), B = ceil((W - 1) / 2^K) + 1 blocks, D = 24 / r - K / r shared levels:
    B D + 17 (24 / r - D).  r = 2: K = 14 gives B = 4, D = 5 (20 + 119 = 139
    against K = 16: 8 + 136); r = 3: K = 15 gives B = 3, D = 3 (9 + 85 against
    K = 18: 4 + 102); r = 4: K = 16 gives B = 2, D = 2 (K = 12 would need 13
    blocks)."""
    s = F.Spec(W.gelu_spec())
    default = s.lookup_r
    assert default in (2, 3, 4)
    for r, depth, blocks in ((2, 5, 4), (3, 3, 3), (4, 2, 2)):
        s2 = F.Spec(W.gelu_spec(), lookup_r=r)
        q = s2.query(24, 12)
        assert (q["lookup_r"], q["top_depth"], q["top_blocks"]) == (r, depth, blocks)
    assert s.query(24, 12)["lookup_r"] == default
    for bad in (0, 1, 5, -2):
        with pytest.raises(F.FssError) as e:
            F.Spec(W.gelu_spec(), lookup_r=bad)
        assert e.value.code == -8
    # clip-ReLU has m = 3: no shared levels at any radix
    assert F.Spec(W.clip_relu_spec(), lookup_r=3).query(16, 8)["top_depth"] == 0
    # exp on [-16, 0) (33 points, W = 16 * 4096 + 1): K = 15 gives B = 3, D = 3 at r = 3
    # (3 * 3 + 33 * 5 = 174 levels against K = 18: 2 * 2 + 33 * 6 = 202; K = 12 needs 17 blocks)
    q = F.Spec(W.exp_spec(), lookup_r=3).query(24, 12)
    assert (q["m"], q["top_depth"], q["top_blocks"]) == (34, 3, 3)
    # reciprocal on [1, 128) (25 points over geometric intervals, W = 520,193 < 2^19): the
    # choice recomputed from the boundaries, K = 18 with B = 3, D = 2
    q = F.Spec(W.recip_spec(7), lookup_r=3).query(24, 12)
    W_ = q["aprime"][q["m"] - 1] - q["aprime"][1] + 1
    assert W_ == 520193
    best = ((q["m"] - 1) * 8, 0, 0)  # no shared levels
    for K in range(3, 24, 3):
        B = ((W_ - 2) >> K) + 2
        if B <= 4 and B <= 2 ** (24 - K):
            D = 8 - K // 3
            cost = B * D + (q["m"] - 1) * (8 - D)
            if cost < best[0]:
                best = (cost, D, B)
    assert (q["top_depth"], q["top_blocks"]) == best[1:] == (2, 3)


def test_argument_errors():
    s = F.Spec(W.clip_relu_spec())
    with pytest.raises(F.FssError) as e:
        s.key_bytes(16, 8, -1)
    assert e.value.code == -8


@pytest.mark.parametrize("r", [2, 3, 4])
def test_rescale_key_bytes(r):
    """Rescaling gate: root, ceil(s / r) levels x 2^r children of 24-byte records
    (seed and value correction), then the two 8-byte constant shares and the one-time
    record (x-hat of each element, used mask); 64-lane tiles."""
    for s in (1, 8, 24, 32):
        per_tile = F.fss_rescale_key_bytes(s, r, 64) - F.fss_rescale_key_bytes(s, r, 0)
        expect = 64 * 16 + (-(-s // r)) * 2**r * 64 * 24 + 2 * 64 * 8 + 64 * 8 + 8
        assert per_tile == (expect + 255) // 256 * 256
        assert F.fss_rescale_key_bytes(s, r, 1000) == 16384 + 16 * per_tile
    for bad_s, code in ((0, -2), (33, -2)):
        with pytest.raises(F.FssError) as e:
            F.fss_rescale_key_bytes(bad_s, r, 10)
        assert e.value.code == code
    with pytest.raises(F.FssError) as e:
        F.fss_rescale_key_bytes(8, 5, 10)
    assert e.value.code == -8


@pytest.mark.parametrize("r", [2, 3, 4])
def test_literal_key_bytes(r):
    """Literal lookup: r_in and r_out shares, the last payload's p shares,
    M - 1 = min(m + 1, 2^n) - 1 vector DCFs (root, ceil(n / r) levels x 2^r
    children of 16 + 8p bytes) and the one-time record per lane; 64-lane
    tiles of a multiple of 256 bytes."""
    for desc, n, f, m, p in ((W.gelu_spec(), 24, 12, 18, 3), (W.clip_relu_spec(), 16, 8, 3, 2)):
        s = F.Spec(desc, lookup_r=r)
        per_tile = s.lit_key_bytes(n, f, 64) - s.lit_key_bytes(n, f, 0)
        dcf = 64 * 16 + (-(-n // r)) * 2**r * 64 * (16 + 8 * p)
        expect = 64 * 8 * 2 + p * 64 * 8 + m * dcf + 64 * 8 + 8
        assert per_tile == (expect + 255) // 256 * 256
        assert s.lit_key_bytes(n, f, 65) == 16384 + 2 * per_tile
    # m = 2^n intervals: no padding, M - 1 = 2^n - 1 DCFs
    s = F.Spec.integer(3, list(range(9)), [[k] for k in range(8)], lookup_r=r)
    per_tile = s.lit_key_bytes(3, 0, 64) - s.lit_key_bytes(3, 0, 0)
    dcf = 64 * 16 + (-(-3 // r)) * 2**r * 64 * 24
    assert per_tile == (64 * 8 * 3 + 7 * dcf + 64 * 8 + 8 + 255) // 256 * 256


def test_subprotocol_and_literal_arguments_rejected_on_the_host():
    """Bad sizes, steps, parties and NULL buffers are rejected before any
    launch (no device needed)."""
    seed = O.seed_bytes(1)
    L = F.lib
    for call in (lambda: L.fss_triples(seed, -1, 0, *([None] * 6), None),
                 lambda: L.fss_triples(seed, 4, 70000, *([1] * 6), None),
                 lambda: L.fss_triples(None, 4, 0, *([1] * 6), None),
                 lambda: L.fss_triples(seed, 4, 0, 1, None, 1, 1, 1, 1, None),
                 lambda: L.fss_and_triples(seed, 4, -1, *([1] * 6), None),
                 lambda: L.fss_b2a_rand(seed, 4, 0, None, 1, 1, 1, None),
                 lambda: L.fss_beaver_mask(None, 1, 1, 1, 4, 1, 1, None),
                 lambda: L.fss_beaver_mask(1, 1, 1, 1, -4, 1, 1, None),
                 lambda: L.fss_beaver_mul(0, 1, 1, 1, 1, None, None, 4, 1, None),
                 lambda: L.fss_xor_mask(1, 1, 1, None, 4, 1, 1, None),
                 lambda: L.fss_xopen(1, None, 4, 1, None),
                 lambda: L.fss_and(0, 1, 1, 1, 1, 1, 4, None, None),
                 lambda: L.fss_b2a(0, None, 1, 4, 1, None),
                 lambda: L.fss_lit_eval(0, None, 1, 4, 1, 1, None),
                 lambda: L.fss_lit_eval(0, 1, None, 4, 1, 1, None),
                 lambda: L.fss_lit_keygen(None, 24, 12, seed, 4, 1, 1, None, None, None)):
        assert call() == -8
    for call in (lambda: L.fss_beaver_mul(2, 1, 1, 1, 1, 1, None, 4, 1, None),
                 lambda: L.fss_and(-1, 1, 1, 1, 1, 1, 4, 1, None),
                 lambda: L.fss_b2a(3, 1, 1, 4, 1, None),
                 lambda: L.fss_lit_eval(2, 1, 1, 4, 1, 1, None)):
        assert call() == -5
    s = F.Spec(W.gelu_spec())
    size = C.c_size_t()
    assert L.fss_lit_key_bytes(s.handle, 24, 12, -1, C.byref(size)) == -8
    assert L.fss_lit_key_bytes(None, 24, 12, 4, C.byref(size)) == -8
    assert L.fss_lit_key_bytes(s.handle, 24, 12, 0, C.byref(size)) == 0 and size.value == 16384


@pytest.mark.parametrize("r", [2, 3, 4])
@pytest.mark.parametrize("name", ["gelu", "exp", "clip", "int_p4", "int_p2"])
def test_keygen_work_counts(name, r):
    """fss_keygen_work (the keygen roofline's work figure) equals the dealer's
    expansions written out call by call, both parties per element: each Z_2
    atom level above the leaves expands the party's seed under two tweaks
    (one call, rounds 1-2 shared: 160 K - 24 (K - 1) lookups) and each atom
    ends in one leaf block; each lookup level expands the 2^r children, two
    at a time, from the party's one seed (its 27 tweak-independent lookups
    once per level, then 133 per block); the counter-mode randomness is one
    full block per draw."""
    P = W.PredDesc
    if name.startswith("int"):
        p = int(name[-1])
        n, f = 16, 0
        spec = F.Spec.integer(n, [0, 1 << 14, 1 << 15, 1 << 16], [[1] * p] * 3,
                              [P(W.LT_UNSIGNED, 0, thr=1000.0), P(W.MSB_SHIFT, 1, c=5)], lookup_r=r)
    else:
        desc = {"gelu": W.gelu_spec(), "exp": W.exp_spec(), "clip": W.clip_relu_spec()}[name]
        n, f = (24, 12) if name != "clip" else (16, 8)
        spec = F.Spec(desc, lookup_r=r)
    q = spec.query(n, f)
    p, T = q["p"], q["T"]
    L = -(-n // r)
    nb = (p + 1) // 2
    lk = lambda k: 160 * k - 24 * (k - 1)
    aes = lookups = 0
    for k in q["atom_k"][:T]:
        levels = k - min(7, k)
        aes += 2 * (2 * levels + 1)
        lookups += 2 * (levels * lk(2) + 160)
    for level in range(L):
        last = level == L - 1
        calls = []  # the blocks of each expansion call of one party, over the children pairs
        for _pair in range((1 << r) // 2):
            if p == 3:
                calls += [2, 1] if last else [3, 2]
            elif p == 1:
                calls += [1] if last else [2, 1]
            else:
                calls += [nb, nb] if last else [1 + nb, 1 + nb]
        aes += 2 * sum(calls)
        lookups += 2 * (27 + 133 * sum(calls))
    draws = 8 + 2 * T + (L - 1) * (1 + nb)
    aes += draws
    lookups += 160 * draws
    got_aes, got_lk = spec.keygen_work(n, f, 1000)
    assert (got_aes, got_lk) == (1000 * aes, 1000 * lookups), (name, r)
