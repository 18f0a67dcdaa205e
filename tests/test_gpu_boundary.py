"""GPU parity of the boundary's remaining calls against the oracle, bit-exact:
integer operator specs (the Definition's own form, and the appendix's worked
ReLU with alpha_1 = N/2), fss_eval_batch, 128-bit dealer seeds, specs whose
predicates all fold to constants, and every value of the work-list knobs
(call 2 in 1..4 parts, call 1 in the same pass or its own unit)."""
import math
import random

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_2606_09551_amd import fss as F  # noqa: E402
from paper_2606_09551_amd import runtime as R  # noqa: E402
from paper_2606_09551_amd import workloads as W  # noqa: E402

P = W.PredDesc
M64 = 2**64 - 1


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _flush(msg):
    print(msg, flush=True)


def _oracle(S, x, seed):
    N = len(x)
    y0, y1, z0, z1, r_in, r_out, _ = O.full(S, seed, np.arange(N, dtype=np.int64), x, masks=True)
    return dict(y0=y0, y1=y1, z0=z0, z1=z1, r_in=r_in, r_out=r_out)


def _check(g, o, N, what):
    for k in ("r_in", "r_out", "y0", "y1"):
        assert np.array_equal(g[k], o[k]), (what, k)
    for b in (0, 1):
        zg = R.unpack_bits(g[f"z{b}"], N) if g[f"z{b}"].size else np.zeros(N, np.uint64)
        assert np.array_equal(zg, o[f"z{b}"]), (what, f"z{b}")


def _run(spec, n, f, x, seed, path, tune=None):
    """path: plain (fss_eval per party), batch (fss_eval_batch, both parties),
    batch_party (fss_eval_batch once per party), plan (fss_plan with `tune`)."""
    N = len(x)
    inst = R.OpInstanceGPU(spec, n, f, N)
    inst.set_input(x)
    inst.keygen(seed)
    inst.mask()
    for b in (0, 1):
        inst.y[b].fill_(-1)
        inst.z[b].fill_(-1)
    if path == "plain":
        for b in (0, 1):
            inst.eval_plain(b)
    elif path == "batch":
        F.fss_eval_batch(F.PARTY_ANY, [inst.item(0), inst.item(1)])
    elif path == "batch_party":
        for b in (0, 1):
            F.fss_eval_batch(b, [inst.item(b)])
    else:
        plan = F.Plan([inst.item(0), inst.item(1)], tune)
        plan.launch()
        cfg = plan.config()
        if tune is not None and tune.parts:
            assert cfg["parts"] == min(tune.parts, inst.m - 1 if inst.m > 1 else 1), cfg
        if tune is not None and tune.pred_unit:
            assert cfg["pred_unit"] == tune.pred_unit, cfg
        if tune is not None and tune.lanes:
            assert cfg["lanes"] == tune.lanes, cfg
        plan.free()
    assert F.fss_status() == 0
    torch.cuda.synchronize()
    return inst.host()


@pytest.mark.parametrize("r", [2, 3, 4])
def test_worked_relu_integer_spec(r):
    """The appendix's worked example over Z_{2^10}: alpha = (0, N/2, N), pieces
    x and 0, predicate MSB(x); every input of the domain (16 tiles), a seed
    above 2^64, plain and fused paths equal to the oracle and reconstructing
    to max(x, 0) and MSB(x)."""
    n = 10
    N = 1 << n
    alpha = [0, N // 2, N]
    coef = [[0, 1], [0, 0]]
    preds = [P(W.MSB_SHIFT, 0, c=0)]
    spec = F.Spec.integer(n, alpha, coef, preds, lookup_r=r)
    S = O.compile_spec_int(n, alpha, coef, preds, lookup_r=r)
    x = np.arange(-N // 2, N // 2, dtype=np.int64)
    seed = 2**64 + 0x5A
    o = _oracle(S, x, seed)
    assert np.array_equal(o["y0"] + o["y1"] - o["r_out"], np.maximum(x, 0).astype(np.uint64))
    assert np.array_equal(o["z0"] ^ o["z1"], (x < 0).astype(np.uint64))
    for path in ("plain", "batch", "batch_party"):
        _flush(f"worked relu r={r} path={path}")
        _check(_run(spec, n, 0, x, seed, path), o, N, path)


def _random_int_spec(rnd, n):
    N = 1 << n
    m = rnd.randint(1, min(24, N))
    alpha = [0] + sorted(rnd.sample(range(1, N), m - 1)) + [N]
    d = rnd.randint(0, 3)
    coef = [[rnd.getrandbits(64) for _ in range(d + 1)] for _ in range(m)]
    preds = [P(W.LT_SIGNED, 0, thr=float(rnd.randint(-N // 2, N // 2 - 1))),
             P(W.LT_UNSIGNED, 1, thr=float(rnd.randint(1, N - 1)), negate=True),
             P(W.LOWBITS_LT, 1, f_bits=min(n, 5), gamma=rnd.randint(1, (1 << min(n, 5)) - 1)),
             P(W.MSB_SHIFT, 2, c=rnd.randint(0, N - 1))]
    return alpha, coef, preds


@pytest.mark.parametrize("r", [2, 3, 4])
def test_random_integer_specs(r):
    """Random integer partitions (1..24 intervals), ring coefficients of degree
    0..3 and every predicate kind at n = 12, 20, 32; 777 inputs over the whole
    domain (12 tiles and a ragged tail), 128-bit seeds, plain and fused."""
    rnd = random.Random(900 + r)
    for n in (12, 20, 32):
        alpha, coef, preds = _random_int_spec(rnd, n)
        spec = F.Spec.integer(n, alpha, coef, preds, lookup_r=r)
        S = O.compile_spec_int(n, alpha, coef, preds, lookup_r=r)
        N = 777
        x = np.array([rnd.randint(-(1 << (n - 1)), (1 << (n - 1)) - 1) for _ in range(N)], dtype=np.int64)
        x[:len(alpha) - 1] = [a - (1 << n) if a >= 1 << (n - 1) else a for a in alpha[:-1]]  # on the boundaries
        seed = rnd.getrandbits(128)
        o = _oracle(S, x, seed)
        for path in ("plain", "plan"):
            _flush(f"random integer spec n={n} m={len(alpha) - 1} r={r} path={path}")
            _check(_run(spec, n, 0, x, seed, path), o, N, (n, path))


@pytest.mark.parametrize("r", [2, 3, 4])
def test_narrowest_domains(r):
    """n = 2..7: one lookup level when r >= n, leading zero bits, comparison
    atoms that are a leaf only (k <= 7); random integer specs, every input,
    three copies of the domain per launch (ragged tiles), plain and fused."""
    rnd = random.Random(970 + r)
    for n in range(2, 8):
        N = 1 << n
        alpha, coef, preds = _random_int_spec(rnd, n)
        spec = F.Spec.integer(n, alpha, coef, preds, lookup_r=r)
        S = O.compile_spec_int(n, alpha, coef, preds, lookup_r=r)
        x = np.tile(np.arange(-N // 2, N // 2, dtype=np.int64), 3)
        seed = rnd.getrandbits(128)
        o = _oracle(S, x, seed)
        for path in ("plain", "plan"):
            _flush(f"narrow domain n={n} m={len(alpha) - 1} r={r} path={path}")
            _check(_run(spec, n, 0, x, seed, path), o, len(x), (n, path))


@pytest.mark.parametrize("r", [2, 3, 4])
def test_maximum_spec_sizes(r):
    """The interface's largest spec (64 intervals, degree 3, 16 predicates,
    16 comparison atoms, 64 output bits): every input at n = 8, and 777
    inputs over the whole domain at n = 32 (boundaries included), plain and
    fused with call 1 in the call-2 unit and in its own."""
    from maxspec import max_int_spec
    rnd = random.Random(950 + r)
    for n in (8, 32):
        N = 1 << n
        alpha, coef, preds = max_int_spec(rnd, n)
        spec = F.Spec.integer(n, alpha, coef, preds, lookup_r=r)
        q = spec.query(n, 0)
        assert (q["m"], q["p"], q["T"], q["ell"]) == (64, 4, 16, 64)
        S = O.compile_spec_int(n, alpha, coef, preds, lookup_r=r)
        if n == 8:
            x = np.arange(-N // 2, N // 2, dtype=np.int64)
        else:
            x = np.array([rnd.randint(-(N // 2), N // 2 - 1) for _ in range(777)], dtype=np.int64)
            x[:63] = [a - N if a >= N // 2 else a for a in alpha[1:-1]]  # on the boundaries
        seed = rnd.getrandbits(128)
        o = _oracle(S, x, seed)
        for path, tune in (("plain", None), ("plan", F.Tune(0, 0, 1, 0, 1, 1)), ("plan", F.Tune(0, 0, 1, 0, 2, 2))):
            _flush(f"maximum spec n={n} r={r} path={path} pred_unit={tune and tune.pred_unit}")
            _check(_run(spec, n, 0, x, seed, path, tune), o, len(x), (n, path, tune and tune.pred_unit))


@pytest.mark.parametrize("r", [2, 3, 4])
def test_predicates_all_constant(r):
    """Every predicate folds to a constant (thresholds outside the n-bit range,
    gamma = 0 and gamma = 2^f): no comparison atom remains (T = 0) but the
    spec still has predicate bits, which both paths must write."""
    preds = [P(W.LT_SIGNED, 0, thr=-1e9), P(W.LT_SIGNED, 1, thr=1e9, negate=True),
             P(W.LT_UNSIGNED, 2, thr=1e12), P(W.LOWBITS_LT, 3, f_bits=4, gamma=0),
             P(W.LOWBITS_LT, 3, f_bits=4, gamma=16)]
    desc = W.SpecDesc("constants", [(-math.inf, 0.0), (0.0, 2.0), (2.0, math.inf)],
                      [[0.0], [0.0, 1.0, 0.5], [2.0]], preds)
    n, f = 14, 6
    spec = F.Spec(desc, r)
    q = spec.query(n, f)
    assert q["T"] == 0 and q["ell"] == 4
    S = O.compile_spec(desc, n, f, lookup_r=r)
    g = np.random.Generator(np.random.PCG64(77 + r))
    x = g.integers(-(1 << (n - 1)), 1 << (n - 1), size=321).astype(np.int64)
    seed = 2**100 + 3
    o = _oracle(S, x, seed)
    assert np.array_equal(o["z0"] ^ o["z1"], np.full(321, 0b1100, np.uint64))
    for path, tune in (("plain", None), ("plan", None), ("plan", F.Tune(0, 0, 1, 0, 1, 1)),
                       ("plan", F.Tune(0, 0, 1, 0, 2, 2))):
        _flush(f"constant predicates r={r} path={path}")
        _check(_run(spec, n, f, x, seed, path, tune), o, len(x), (path, tune and tune.pred_unit))


@pytest.mark.parametrize("parts", [1, 2, 3, 4])
@pytest.mark.parametrize("pred_unit", [1, 2])
def test_work_list_units_every_value(parts, pred_unit):
    """Every value of the work-list knobs gives the oracle's shares: call 2 of
    a tile in 1..4 parts, call 1 in the first part's pass or a unit of its own
    (GELU at n = 12, 1000 elements)."""
    desc = W.gelu_spec(f=7)
    n, f = 12, 7
    spec = F.Spec(desc)
    S = O.compile_spec(desc, n, f)
    g = np.random.Generator(np.random.PCG64(5))
    x = g.integers(-(1 << (n - 1)), 1 << (n - 1), size=1000).astype(np.int64)
    o = _oracle(S, x, 0xAB)
    _flush(f"units parts={parts} pred_unit={pred_unit}")
    _check(_run(spec, n, f, x, 0xAB, "plan", F.Tune(0, 0, 1, 0, parts, pred_unit)), o, len(x), (parts, pred_unit))


def test_eval_batch_checks_party():
    spec = F.Spec(W.clip_relu_spec())
    N = 200
    inst = R.OpInstanceGPU(spec, 16, 8, N)
    inst.set_input(W.config1()[0].x[:N])
    inst.keygen(3)
    inst.mask()
    with pytest.raises(F.FssError) as e:
        F.fss_eval_batch(0, [inst.item(0), inst.item(1)])
    assert e.value.code == -5
    with pytest.raises(F.FssError) as e:
        F.fss_eval_batch(2, [inst.item(0)])
    assert e.value.code == -5
    F.fss_eval_batch(F.PARTY_ANY, [])
    assert F.fss_status() == 0


def test_radix_autotune_sets_and_caches(tmp_path):
    """The key-layout knob: the autotuner times keygen + fused evaluation at
    every lookup radix, sets the fastest on the spec and caches it; keys then
    generated at that radix equal the oracle's."""
    desc = W.gelu_spec(f=7)
    n, f = 12, 7
    spec = F.Spec(desc)
    cache = str(tmp_path / "radix.txt")
    r = spec.autotune_radix(n, f, 20000, cache)
    assert r in (2, 3, 4) and spec.lookup_r == r
    other = F.Spec(desc)
    assert other.autotune_radix(n, f, 20000, cache) == r  # from the cache
    g = np.random.Generator(np.random.PCG64(8))
    x = g.integers(-(1 << (n - 1)), 1 << (n - 1), size=500).astype(np.int64)
    S = O.compile_spec(desc, n, f, lookup_r=r)
    o = _oracle(S, x, 0x77)
    _check(_run(spec, n, f, x, 0x77, "plan"), o, len(x), ("radix", r))


@pytest.mark.parametrize("lanes", [2, 4])
@pytest.mark.parametrize("variant", [1, 2])
def test_lanes_per_element_every_value(lanes, variant):
    """Elements per wave 32 and 16: each element's lookup points split over 2
    or 4 lanes whose shares of y are summed across the wave.  Random integer
    specs (1..24 intervals, degree 0..3, so p = 1..4 and from zero points up)
    at every radix, 777 elements (a ragged last tile), and GELU, against the
    oracle."""
    rnd = random.Random(1300 + 10 * lanes + variant)
    tune = F.Tune(0, 0, variant, 0, 1, 2, lanes)
    for r in (2, 3, 4):
        for n in (12, 32):
            alpha, coef, preds = _random_int_spec(rnd, n)
            spec = F.Spec.integer(n, alpha, coef, preds, lookup_r=r)
            S = O.compile_spec_int(n, alpha, coef, preds, lookup_r=r)
            N = 777
            x = np.array([rnd.randint(-(1 << (n - 1)), (1 << (n - 1)) - 1) for _ in range(N)], dtype=np.int64)
            seed = rnd.getrandbits(128)
            o = _oracle(S, x, seed)
            _flush(f"lanes={lanes} variant={variant} n={n} m={len(alpha) - 1} d={len(coef[0]) - 1} r={r}")
            _check(_run(spec, n, 0, x, seed, "plan", tune), o, N, (lanes, variant, n, r))
    desc = W.gelu_spec(f=7)
    spec = F.Spec(desc)
    S = O.compile_spec(desc, 12, 7)
    x = np.random.Generator(np.random.PCG64(6)).integers(-2048, 2048, size=1000).astype(np.int64)
    _flush(f"lanes={lanes} variant={variant} GELU n=12")
    _check(_run(spec, 12, 7, x, 0xAC, "plan", tune), _oracle(S, x, 0xAC), len(x), (lanes, variant))


def test_lanes_rejected_where_not_built():
    """Lane groups need parts <= 1, call 1 in its own unit and table layout 1
    or 2; other values are rejected on the host."""
    spec = F.Spec(W.clip_relu_spec())
    inst = R.OpInstanceGPU(spec, 16, 8, 200)
    inst.set_input(W.config1()[0].x[:200])
    inst.keygen(4)
    inst.mask()
    items = [inst.item(0), inst.item(1)]
    for tune, code in ((F.Tune(0, 0, 1, 0, 2, 2, 2), -8), (F.Tune(0, 0, 1, 0, 1, 1, 2), -8),
                       (F.Tune(0, 0, 1, 0, 1, 2, 3), -8), (F.Tune(0, 0, 0, 0, 1, 2, 4), -2)):
        with pytest.raises(F.FssError) as e:
            F.Plan(items, tune)
        assert e.value.code == code, (tune.lanes, e.value)
    assert F.fss_status() == 0
