"""The literal interval lookup and the post-processing subprotocols on the GPU,
bit-exact against the oracle (both parties' shares), with reconstruction
checked over every element: Beaver multiplication, AND on XOR-shared bit
words, B2A (also applied to an operator gate's predicate bits), and the
lookup-plus-Horner pipeline for several specs and radixes, ragged sizes and
the worked ReLU of Appendix "Example: A Complete (F, Phi) Pair"."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_2606_09551_amd import fss as F  # noqa: E402
from paper_2606_09551_amd import runtime as R  # noqa: E402
from paper_2606_09551_amd import workloads as W  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _dev(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def _host(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def _empty(n):
    return torch.empty(max(n, 1), dtype=torch.int64, device="cuda")


def _flush(msg):
    print(msg, flush=True)


def test_beaver_multiplication():
    n, seed, step = 10000 + 17, 2**70 + 5, 3
    g = np.random.Generator(np.random.PCG64(1))
    u, v, u0, v0 = (g.integers(0, 2**63, size=n, dtype=np.uint64) * np.uint64(2) + np.uint64(1) for _ in range(4))
    u[:3], v[:3] = [0, 2**64 - 1, 5], [7, 2**64 - 1, 0]
    u1, v1 = u - u0, v - v0
    T = {k: _empty(n) for k in ("a0", "b0", "c0", "a1", "b1", "c1")}
    _flush("beaver: triples")
    F.fss_triples(seed, n, step, T["a0"], T["b0"], T["c0"], T["a1"], T["b1"], T["c1"])
    U, V = {0: _dev(u0), 1: _dev(u1)}, {0: _dev(v0), 1: _dev(v1)}
    d, e, D, E, z = ({b: _empty(n) for b in (0, 1)}, {b: _empty(n) for b in (0, 1)}, _empty(n), _empty(n),
                     {b: _empty(n) for b in (0, 1)})
    for b in (0, 1):
        F.fss_beaver_mask(U[b], V[b], T[f"a{b}"], T[f"b{b}"], n, d[b], e[b])
    F.fss_open(d[0], d[1], n, D)
    F.fss_open(e[0], e[1], n, E)
    for b in (0, 1):
        F.fss_beaver_mul(b, D, E, T[f"a{b}"], T[f"b{b}"], T[f"c{b}"], None, n, z[b])
    assert F.fss_status() == 0
    z0, z1 = _host(z[0])[:n], _host(z[1])[:n]
    assert np.array_equal(z0 + z1, u * v)
    h = {k: _host(t)[:n] for k, t in T.items()}
    Dh, Eh = _host(D)[:n], _host(E)[:n]
    for i in list(range(0, n, 997)) + [n - 1]:
        a, b_, c = O.triple(seed, i, step)
        assert [h["a0"][i], h["a1"][i], h["b0"][i], h["b1"][i], h["c0"][i], h["c1"][i]] == \
            [a[0], a[1], b_[0], b_[1], c[0], c[1]], i
        for b in (0, 1):
            assert int(_host(z[b])[i]) == O.beaver_mul(b, int(Dh[i]), int(Eh[i]), int(a[b]), int(b_[b]), int(c[b]))


def test_and_gate():
    words, seed, step = 1000 + 3, 99, 1
    g = np.random.Generator(np.random.PCG64(2))
    x, y, x0, y0 = (g.integers(0, 2**63, size=words, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
                    for _ in range(4))
    x[:2], y[:2] = [0b1010, 2**64 - 1], [0b1100, 0]
    x1, y1 = x ^ x0, y ^ y0
    T = {k: _empty(words) for k in ("a0", "b0", "c0", "a1", "b1", "c1")}
    _flush("and: triples")
    F.fss_and_triples(seed, words, step, T["a0"], T["b0"], T["c0"], T["a1"], T["b1"], T["c1"])
    X, Y = {0: _dev(x0), 1: _dev(x1)}, {0: _dev(y0), 1: _dev(y1)}
    d, e, D, E, z = ({b: _empty(words) for b in (0, 1)}, {b: _empty(words) for b in (0, 1)}, _empty(words),
                     _empty(words), {b: _empty(words) for b in (0, 1)})
    for b in (0, 1):
        F.fss_xor_mask(X[b], T[f"a{b}"], Y[b], T[f"b{b}"], words, d[b], e[b])
    F.fss_xopen(d[0], d[1], words, D)
    F.fss_xopen(e[0], e[1], words, E)
    for b in (0, 1):
        F.fss_and(b, D, E, T[f"a{b}"], T[f"b{b}"], T[f"c{b}"], words, z[b])
    assert F.fss_status() == 0
    z0, z1 = _host(z[0])[:words], _host(z[1])[:words]
    assert np.array_equal(z0 ^ z1, x & y)
    h = {k: _host(t)[:words] for k, t in T.items()}
    for w in list(range(0, words, 101)) + [words - 1]:
        a, b_, c = O.and_triple(seed, w, step)
        assert [h["a0"][w], h["a1"][w], h["b0"][w], h["b1"][w], h["c0"][w], h["c1"][w]] == \
            [a[0], a[1], b_[0], b_[1], c[0], c[1]], w
        Dw, Ew = int(_host(D)[w]), int(_host(E)[w])
        assert int(z0[w]) == O.and_gate(0, Dw, Ew, int(a[0]), int(b_[0]), int(c[0]))


def _b2a(zbits0, zbits1, n, seed, step):
    """B2A of XOR-shared bit words through the library; returns the additive
    shares and the correlation / opening for the oracle comparison."""
    words = (n + 63) // 64
    t0, t1, T0, T1 = _empty(words), _empty(words), _empty(n), _empty(n)
    F.fss_b2a_rand(seed, n, step, t0, t1, T0, T1)
    c = {b: _empty(words) for b in (0, 1)}
    F.fss_xor_mask(zbits0, t0, None, None, words, c[0], None)
    F.fss_xor_mask(zbits1, t1, None, None, words, c[1], None)
    C = _empty(words)
    F.fss_xopen(c[0], c[1], words, C)
    out = {b: _empty(n) for b in (0, 1)}
    F.fss_b2a(0, C, T0, n, out[0])
    F.fss_b2a(1, C, T1, n, out[1])
    assert F.fss_status() == 0
    return (_host(out[0])[:n], _host(out[1])[:n], _host(t0)[:words], _host(t1)[:words], _host(T0)[:n],
            _host(T1)[:n], _host(C)[:words])


def _bits(words: np.ndarray, n: int) -> np.ndarray:
    i = np.arange(n)
    return (words[i >> 6] >> (i & 63).astype(np.uint64)) & np.uint64(1)


def test_b2a_random_bits():
    n, seed, step = 5000 + 33, 2**100 + 9, 2
    g = np.random.Generator(np.random.PCG64(3))
    words = (n + 63) // 64
    z = g.integers(0, 2**63, size=words, dtype=np.uint64) * np.uint64(3)
    s0 = g.integers(0, 2**63, size=words, dtype=np.uint64)
    _flush("b2a: random bits")
    o0, o1, t0, t1, T0, T1, C = _b2a(_dev(s0), _dev(z ^ s0), n, seed, step)
    assert np.array_equal(o0 + o1, _bits(z, n))
    tb0, tb1 = _bits(t0, n), _bits(t1, n)
    for i in list(range(0, n, 313)) + [n - 1]:
        t, T = O.b2a_rand(seed, i, step)
        assert [tb0[i], tb1[i], T0[i], T1[i]] == [t[0], t[1], T[0], T[1]], i
        c = int(_bits(C, n)[i])
        assert int(o0[i]) == O.b2a(0, c, int(T[0])) and int(o1[i]) == O.b2a(1, c, int(T[1]))


def test_b2a_of_operator_predicate_bits():
    """Call 1's XOR-shared predicate bits of an operator gate (clip-ReLU over
    4,096 inputs) converted to additive shares of the same bits."""
    op = W.config1()[0]
    inst = R.OpInstanceGPU(F.Spec(op.spec), 16, 8, len(op.x))
    inst.set_input(op.x)
    inst.keygen(op.seed)
    inst.mask()
    for b in (0, 1):
        inst.eval_plain(b)
    assert F.fss_status() == 0
    n, words = inst.n, (inst.n + 63) // 64
    ref0, ref1 = inst.host()["z0"], inst.host()["z1"]
    for j in range(inst.ell):
        _flush(f"b2a: predicate plane {j}")
        o0, o1, *_ = _b2a(inst.z[0][j * words:(j + 1) * words], inst.z[1][j * words:(j + 1) * words], n, 5, j)
        assert np.array_equal(o0 + o1, _bits(ref0[j] ^ ref1[j], n))


def _lit_case(spec: F.Spec, S, n_bits, f_bits, x, seed):
    N = len(x)
    g = R.LiteralGPU(spec, n_bits, f_bits, N)
    g.set_input(x)
    g.keygen(seed)
    g.mask()
    g.eval()
    assert F.fss_status() == 0
    torch.cuda.synchronize()
    h = g.host()
    o = O.lit(S, seed, np.arange(N), x)
    assert np.array_equal(h["r_in"], o["r_in"]) and np.array_equal(h["r_out"], o["r_out"])
    assert np.array_equal(h["c0"], o["c0"]) and np.array_equal(h["c1"], o["c1"])
    assert np.array_equal(h["y0"], o["y0"]) and np.array_equal(h["y1"], o["y1"])
    assert np.array_equal(h["x0"] + h["x1"], x.astype(np.int64).view(np.uint64))
    return h


@pytest.mark.parametrize("r", [2, 3, 4])
def test_literal_lookup_pipeline_matches_oracle(r):
    """GELU (n = 24, 18 pieces, degree 2) and clip-ReLU (n = 16), 1,000 + a
    ragged tail elements, every element's shares equal to the oracle's."""
    g = np.random.Generator(np.random.PCG64(20 + r))
    for desc, n, f, N in ((W.gelu_spec(), 24, 12, 1000 + 37), (W.clip_relu_spec(), 16, 8, 700 + 5)):
        spec = F.Spec(desc, lookup_r=r)
        S = O.compile_spec(desc, n, f, lookup_r=r)
        x = W.quantize(g.normal(0.0, 2.5, size=N), n, f)
        _flush(f"literal lookup {desc.name} r={r} N={N}")
        _lit_case(spec, S, n, f, x, 1000 + r)


def test_literal_lookup_integer_specs_every_input():
    """Random integer specs at n = 6 (including m = 2^n: no padding, and
    m = 1), every input, degree 0..3, every radix."""
    import random
    rnd = random.Random(61)
    for r in (2, 3, 4):
        for m in (1, 2, 7, 64):
            n, Nn = 6, 64
            alpha = [0] + sorted(rnd.sample(range(1, Nn), m - 1)) + [Nn]
            d = rnd.randint(0, 3)
            coef = [[rnd.getrandbits(64) for _ in range(d + 1)] for _ in range(m)]
            spec = F.Spec.integer(n, alpha, coef, lookup_r=r)
            S = O.compile_spec_int(n, alpha, coef, lookup_r=r)
            x = np.arange(-32, 32, dtype=np.int64)
            _flush(f"literal lookup integer spec m={m} d={d} r={r}")
            _lit_case(spec, S, n, 0, x, rnd.getrandbits(128))


def test_worked_relu_example():
    """Appendix "Example: A Complete (F, Phi) Pair": alpha = (0, N/2, N) with
    pieces (a, b) = (1, 0) and (0, 0) as the coefficients of a x + b, the
    lookup returning their shares and Phi one Beaver product a x plus b:
    y = max(x, 0) (n = 16, every input)."""
    n = 16
    Nn = 1 << n
    coef = [[0, 1], [0, 0]]  # lowest degree first: b, a
    spec = F.Spec.integer(n, [0, Nn // 2, Nn], coef)
    S = O.compile_spec_int(n, [0, Nn // 2, Nn], coef)
    x = np.arange(-(Nn // 2), Nn // 2, dtype=np.int64)
    _flush("worked ReLU")
    h = _lit_case(spec, S, n, 0, x, 2**127 + 1)
    assert np.array_equal(h["y0"] + h["y1"] - h["r_out"], np.maximum(x, 0).view(np.uint64))


def test_relu_phi_composed_from_the_library():
    """A post-processing circuit built from the library's pieces alone:
    ReLU(x) = x (1 - MSB(x)) on additively shared x.  The sign bit comes
    from an operator gate on the masked opening (call 1, predicate MSB(x)),
    NOT is party 0's local flip, B2A gives additive shares of 1 - MSB(x),
    and one Beaver product multiplies them with x (n = 16, every input)."""
    n = 16
    Nn = 1 << n
    x = np.arange(-(Nn // 2), Nn // 2, dtype=np.int64)
    N = len(x)
    words = (N + 63) // 64
    # the sign bit: an integer spec with one constant piece and MSB(x) as output 0
    spec = F.Spec.integer(n, [0, Nn], [[0]], [W.PredDesc(W.MSB_SHIFT, 0, c=0)])
    gate = R.OpInstanceGPU(spec, n, 0, N)
    gate.set_input(x)
    gate.keygen(2**90 + 11)
    gate.mask()
    for b in (0, 1):
        gate.eval_plain(b)
    # NOT z: party 0 flips its XOR share
    ones = _dev(np.full(words, 2**64 - 1, dtype=np.uint64))
    nz0 = _empty(words)
    F.fss_xor_mask(gate.z[0][:words], ones, None, None, words, nz0, None)
    nz1 = gate.z[1][:words]
    # B2A of NOT z
    seed = 0xB2A
    t0, t1, T0, T1 = _empty(words), _empty(words), _empty(N), _empty(N)
    F.fss_b2a_rand(seed, N, 0, t0, t1, T0, T1)
    c0, c1, C = _empty(words), _empty(words), _empty(words)
    F.fss_xor_mask(nz0, t0, None, None, words, c0, None)
    F.fss_xor_mask(nz1, t1, None, None, words, c1, None)
    F.fss_xopen(c0, c1, words, C)
    v = {0: _empty(N), 1: _empty(N)}
    F.fss_b2a(0, C, T0, N, v[0])
    F.fss_b2a(1, C, T1, N, v[1])
    # x (1 - MSB(x)) with one Beaver product on additive shares of x
    g = np.random.Generator(np.random.PCG64(9))
    x0 = g.integers(0, 2**63, size=N, dtype=np.uint64) * np.uint64(2)
    X = {0: _dev(x0), 1: _dev(x.view(np.uint64) - x0)}
    T = {k: _empty(N) for k in ("a0", "b0", "c0", "a1", "b1", "c1")}
    F.fss_triples(seed, N, 1, T["a0"], T["b0"], T["c0"], T["a1"], T["b1"], T["c1"])
    d, e, D, E, y = ({b: _empty(N) for b in (0, 1)}, {b: _empty(N) for b in (0, 1)}, _empty(N), _empty(N),
                     {b: _empty(N) for b in (0, 1)})
    for b in (0, 1):
        F.fss_beaver_mask(X[b], v[b], T[f"a{b}"], T[f"b{b}"], N, d[b], e[b])
    F.fss_open(d[0], d[1], N, D)
    F.fss_open(e[0], e[1], N, E)
    for b in (0, 1):
        F.fss_beaver_mul(b, D, E, T[f"a{b}"], T[f"b{b}"], T[f"c{b}"], None, N, y[b])
    assert F.fss_status() == 0
    _flush("relu phi composed")
    assert np.array_equal(_host(y[0])[:N] + _host(y[1])[:N], np.maximum(x, 0).view(np.uint64))


def test_literal_lookup_largest_partition():
    """64 intervals at n = 8: the partition is padded to M = 65 (64 DCFs per
    element), degree 3, every input twice (ragged tiles), every radix."""
    import random
    rnd = random.Random(81)
    n, Nn = 8, 256
    for r in (2, 3, 4):
        alpha = [0] + sorted(rnd.sample(range(1, Nn), 63)) + [Nn]
        coef = [[rnd.getrandbits(64) for _ in range(4)] for _ in range(64)]
        spec = F.Spec.integer(n, alpha, coef, lookup_r=r)
        S = O.compile_spec_int(n, alpha, coef, lookup_r=r)
        x = np.tile(np.arange(-128, 128, dtype=np.int64), 2)
        _flush(f"literal lookup m=64 n=8 r={r}")
        _lit_case(spec, S, n, 0, x, rnd.getrandbits(128))


def test_literal_lookup_widest_domain_and_degree():
    """n = 32 (the widest domain) with degree-3 ring coefficients at r = 4
    and r = 3, ragged size, every share against the oracle."""
    import random
    rnd = random.Random(71)
    n = 32
    Nn = 1 << n
    for r in (3, 4):
        alpha = [0] + sorted(rnd.sample(range(1, Nn), 4)) + [Nn]
        coef = [[rnd.getrandbits(64) for _ in range(4)] for _ in range(5)]
        spec = F.Spec.integer(n, alpha, coef, lookup_r=r)
        S = O.compile_spec_int(n, alpha, coef, lookup_r=r)
        x = np.array([rnd.randint(-(Nn // 2), Nn // 2 - 1) for _ in range(200 + 3)], dtype=np.int64)
        x[:4] = [a - Nn if a >= Nn // 2 else a for a in alpha[1:5]]  # on the boundaries
        _flush(f"literal lookup n=32 d=3 r={r}")
        _lit_case(spec, S, n, 0, x, rnd.getrandbits(128))


def test_literal_keys_are_one_time():
    """A literal key evaluated again at the same x-hat gives the same shares;
    at another x-hat the changed elements are refused (zero shares,
    FSS_E_CONSUMED)."""
    desc = W.clip_relu_spec()
    spec = F.Spec(desc)
    x = W.config1()[0].x[:300]
    g = R.LiteralGPU(spec, 16, 8, len(x))
    g.set_input(x)
    g.keygen(7)
    g.mask()
    for b in (0, 1):
        F.fss_lit_eval(b, g.keys[b], g.xhat, len(x), g.coef[b], g.xs[b])
    assert F.fss_status() == 0
    first = [_host(g.coef[b]).copy() for b in (0, 1)]
    for b in (0, 1):
        F.fss_lit_eval(b, g.keys[b], g.xhat, len(x), g.coef[b], g.xs[b])
    assert F.fss_status() == 0
    assert all(np.array_equal(_host(g.coef[b]), first[b]) for b in (0, 1))
    g.xhat[5] += 1
    F.fss_lit_eval(0, g.keys[0], g.xhat, len(x), g.coef[0], g.xs[0])
    assert F.fss_status() == -9
    c = _host(g.coef[0])[: g.p * len(x)].reshape(g.p, len(x))
    assert np.all(c[:, 5] == 0) and int(_host(g.xs[0])[5]) == 0
    keep = np.r_[0:5, 6:len(x)]
    assert np.array_equal(c[:, keep], first[0][: g.p * len(x)].reshape(g.p, len(x))[:, keep])


@pytest.mark.parametrize("n", [1, 63, 64, 65, 129])
def test_subprotocols_at_edge_sizes(n):
    """Beaver, AND and B2A over 1, 63, 64, 65 and 129 elements (bit words
    with a ragged last word), against the operations they implement."""
    g = np.random.Generator(np.random.PCG64(100 + n))
    u, v, u0, v0 = (g.integers(0, 2**63, size=n, dtype=np.uint64) * np.uint64(2) + np.uint64(1) for _ in range(4))
    T = {k: _empty(n) for k in ("a0", "b0", "c0", "a1", "b1", "c1")}
    F.fss_triples(n, n, 0, T["a0"], T["b0"], T["c0"], T["a1"], T["b1"], T["c1"])
    U, V = {0: _dev(u0), 1: _dev(u - u0)}, {0: _dev(v0), 1: _dev(v - v0)}
    d, e, D, E, z = ({b: _empty(n) for b in (0, 1)}, {b: _empty(n) for b in (0, 1)}, _empty(n), _empty(n),
                     {b: _empty(n) for b in (0, 1)})
    for b in (0, 1):
        F.fss_beaver_mask(U[b], V[b], T[f"a{b}"], T[f"b{b}"], n, d[b], e[b])
    F.fss_open(d[0], d[1], n, D)
    F.fss_open(e[0], e[1], n, E)
    for b in (0, 1):
        F.fss_beaver_mul(b, D, E, T[f"a{b}"], T[f"b{b}"], T[f"c{b}"], None, n, z[b])
    assert np.array_equal(_host(z[0])[:n] + _host(z[1])[:n], u * v)
    words = (n + 63) // 64
    bits = g.integers(0, 2**63, size=words, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    s0 = g.integers(0, 2**63, size=words, dtype=np.uint64)
    _flush(f"subprotocols n={n}")
    o0, o1, *_ = _b2a(_dev(s0), _dev(bits ^ s0), n, 3, 1)
    assert np.array_equal(o0 + o1, _bits(bits, n))
    assert F.fss_status() == 0
