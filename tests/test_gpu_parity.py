"""GPU parity: the HIP path through the C ABI vs the CPU oracle, bit-exact.

Every comparison is element by element on the same seeded inputs: keys
(field by field), masks, both parties' arithmetic shares and predicate-bit
shares.  Full-size configurations are checked on sampled elements against
the oracle and on every element through the reconstruction property
y_0 + y_1 - r_out = P_{i*}(x) (plaintext evaluator).
"""
import math
import os
import zlib

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_2606_09551_amd import fss as F  # noqa: E402
from paper_2606_09551_amd import runtime as R  # noqa: E402
from paper_2606_09551_amd import workloads as W  # noqa: E402

from keyfmt import KeyView, oracle_atom, oracle_coeff  # noqa: E402

P = W.PredDesc


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _mixed_spec():
    preds = [P(W.LT_SIGNED, 0, thr=-1.0), P(W.LT_SIGNED, 0, thr=2.5), P(W.LT_UNSIGNED, 1, thr=5.0),
             P(W.LOWBITS_LT, 2, f_bits=3, gamma=5, negate=True), P(W.MSB_SHIFT, 3, c=37),
             P(W.MSB_SHIFT, 4, c=0), P(W.LT_SIGNED, 4, thr=0.75)]
    iv = [(-math.inf, -3.0), (-3.0, -0.5), (-0.5, 0.25), (0.25, 4.0), (4.0, math.inf)]
    pcs = [[1.5], [0.25, -1.0, 0.5], [0.0, 2.0, 0.0, -0.125], [-1.0, 0.5, 0.25, 0.0625], [3.0, -0.5]]
    return W.SpecDesc("mixed", iv, pcs, preds)


def _steps_spec():
    iv = [(-math.inf, -1.0), (-1.0, 1.0), (1.0, math.inf)]
    return W.SpecDesc("steps", iv, [[-2.0], [0.5], [3.0]], [P(W.LT_SIGNED, 0, thr=1.0)])


def _flush(msg):
    print(msg, flush=True)


def gpu_run(desc, n_bits, f, x, seed, path="plain", variant=None, lookup_r=None):
    spec = F.Spec(desc, lookup_r)
    op = R.OpInstanceGPU(spec, n_bits, f, len(x))
    op.set_input(x)
    op.keygen(seed)
    op.mask()
    if path == "plain":
        for b in (0, 1):
            op.eval_plain(b)
    else:
        tune = None
        if variant is not None:
            tune = F.Tune(0, 0, variant, 0)
        plan = F.Plan([op.item(0), op.item(1)], tune)
        plan.launch()
    assert F.fss_status() == 0
    torch.cuda.synchronize()
    out = op.host()
    out["parts"] = plan.parts() if path != "plain" else 1
    out["lookup_r"] = spec.lookup_r
    out["keys0"] = op.keys[0].cpu().numpy()
    out["keys1"] = op.keys[1].cpu().numpy()
    out["op"] = op
    return out


def oracle_run(desc, n_bits, f, x, seed, elems, lookup_r):
    S = O.compile_spec(desc, n_bits, f, lookup_r=lookup_r)
    elems = np.asarray(elems, dtype=np.int64)
    K0, K1, r_in, r_out = O.keygen(S, seed, elems)
    xhat = (x[elems].astype(np.int64).view(np.uint64) + r_in).astype(np.uint64)
    y0, z0 = O.evaluate(0, S, K0, xhat)
    y1, z1 = O.evaluate(1, S, K1, xhat)
    return dict(S=S, K0=K0, K1=K1, r_in=r_in, r_out=r_out, xhat=xhat, y0=y0, y1=y1, z0=z0, z1=z1)


def compare(g, o, elems, n, check_keys=0):
    elems = np.asarray(elems)
    for name in ("r_in", "r_out", "xhat", "y0", "y1"):
        assert np.array_equal(g[name][elems], o[name]), name
    for b in (0, 1):
        zg = R.unpack_bits(g[f"z{b}"], n)[elems] if g[f"z{b}"].size else np.zeros(len(elems), np.uint64)
        assert np.array_equal(zg, o[f"z{b}"]), f"z{b}"
    if check_keys:
        kv = [KeyView(g["keys0"]), KeyView(g["keys1"])]
        S = o["S"]
        for idx in np.linspace(0, len(elems) - 1, min(check_keys, len(elems))).astype(int):
            e = int(elems[idx])
            for b, K in ((0, o["K0"][idx]), (1, o["K1"][idx])):
                for t in range(S.T):
                    assert kv[b].atom(e, t) == oracle_atom(K, t), (b, e, t)
                assert kv[b].coeff(e) == oracle_coeff(K), (b, e)


def test_c1_clip_relu_full_parity():
    """Config 1: 4096 clip-ReLU inputs, every element, keys sampled."""
    op = W.config1()[0]
    _flush("c1 clip-relu n=4096")
    g = gpu_run(op.spec, 16, 8, op.x, op.seed)
    elems = np.arange(len(op.x))
    o = oracle_run(op.spec, 16, 8, op.x, op.seed, elems, g["lookup_r"])
    compare(g, o, elems, len(op.x), check_keys=64)
    S = o["S"]
    yp, zp = O.plain_many(S, op.x)
    assert np.array_equal(g["y0"] + g["y1"] - g["r_out"], yp)


@pytest.mark.parametrize("r", [2, 3, 4])
@pytest.mark.parametrize("name", ["mixed", "steps", "relu", "gelu_small", "exp_small"])
def test_small_specs_all_elements(name, r):
    desc, n, f = {
        "mixed": (_mixed_spec(), 12, 4),
        "steps": (_steps_spec(), 10, 3),
        "relu": (W.relu_worked_example_spec(), 9, 0),
        "gelu_small": (W.gelu_spec(f=7), 12, 7),
        "exp_small": (W.exp_spec(f=6), 14, 6),
    }[name]
    N = 1000  # 15 full tiles and a ragged tail
    g_ = np.random.Generator(np.random.PCG64(zlib.crc32(name.encode())))
    s = 2 ** (n - 1)
    x = g_.integers(-s, s, size=N).astype(np.int64)
    x[:4] = [-s, s - 1, 0, -1]
    _flush(f"small spec {name} n={n} r={r} N={N}")
    for path in ("plain", "fused"):
        g = gpu_run(desc, n, f, x, 0x5EED + len(name), path=path, lookup_r=r)
        assert g["lookup_r"] == r
        o = oracle_run(desc, n, f, x, 0x5EED + len(name), np.arange(N), r)
        compare(g, o, np.arange(N), N, check_keys=16 if path == "plain" else 0)
        if path == "fused" and name in ("gelu_small", "exp_small"):
            # 32 tiles cannot fill the GPU and call 2 dominates their cost: the
            # planner runs call 2 in parts that add their shares of y, which
            # must not change any output
            assert g["parts"] > 1, g["parts"]


@pytest.mark.parametrize("r", [2, 3, 4])
@pytest.mark.parametrize("n", [31, 32])
@pytest.mark.parametrize("name", ["clip", "gelu"])
def test_widest_domains(n, name, r):
    """The widest comparison domains: n = 32 (full 32-bit masks; 16, 11 or 8
    lookup-DCF levels at r = 2, 3, 4) and n = 31 (leading zero bits at every
    r), every element of 200 inputs spread over the whole domain plus its ends,
    keys sampled, both paths."""
    desc = {"clip": W.clip_relu_spec(), "gelu": W.gelu_spec(f=8)}[name]
    f = 8
    N = 200
    g_ = np.random.Generator(np.random.PCG64(1000 * n + len(name)))
    s = 2 ** (n - 1)
    x = g_.integers(-s, s, size=N).astype(np.int64)
    x[:6] = [-s, s - 1, 0, -1, 1, -(1 << f)]
    x[6:40] = g_.integers(-8 << f, 8 << f, size=34)  # where the pieces change
    _flush(f"widest domain {name} n={n} r={r} N={N}")
    for path in ("plain", "fused"):
        g = gpu_run(desc, n, f, x, 0xD0 + n, path=path, lookup_r=r)
        o = oracle_run(desc, n, f, x, 0xD0 + n, np.arange(N), r)
        compare(g, o, np.arange(N), N, check_keys=8 if path == "plain" else 0)


def test_real_specs_size_grid():
    """The workloads' real specs at every (n, f) of a grid over n = 2..32 that
    the quantiser accepts, the radix cycling through 2, 3, 4: every input for
    n <= 8, 300 inputs over the whole domain (its ends included) above;
    plain path and fused plan, both against the oracle."""
    descs = [W.clip_relu_spec(), W.gelu_spec(), W.exp_spec(), W.recip_spec(7), W.rsqrt_spec()]
    g_ = np.random.Generator(np.random.PCG64(2024))
    done = 0
    for desc in descs:
        for n in (2, 3, 4, 6, 8, 12, 16, 20, 24, 28, 31, 32):
            for f in sorted({0, 1, n // 2, n - 1} & set(range(n))):
                try:
                    F.Spec(desc).query(n, f)
                except F.FssError:
                    continue  # refused by both quantisers (a host test checks that)
                r = 2 + done % 3
                s = 2 ** (n - 1)
                if n <= 8:
                    x = np.arange(-s, s, dtype=np.int64)
                else:
                    x = g_.integers(-s, s, size=300).astype(np.int64)
                    x[:4] = [-s, s - 1, 0, -1]
                seed = 0x6E1D + 97 * done
                o = oracle_run(desc, n, f, x, seed, np.arange(len(x)), r)
                for path in ("plain", "fused"):
                    _flush(f"size grid {desc.name} n={n} f={f} r={r} path={path}")
                    g = gpu_run(desc, n, f, x, seed, path=path, lookup_r=r)
                    compare(g, o, np.arange(len(x)), len(x))
                done += 1
    assert done > 50


@pytest.mark.parametrize("N", [1, 63, 64, 65, 129])
def test_edge_sizes(N):
    op = W.config1()[0]
    x = op.x[:N]
    _flush(f"edge size N={N}")
    g = gpu_run(op.spec, 16, 8, x, 77, path="fused")
    o = oracle_run(op.spec, 16, 8, x, 77, np.arange(N), g["lookup_r"])
    compare(g, o, np.arange(N), N)


def test_empty_batch_is_noop():
    spec = F.Spec(W.clip_relu_spec())
    key = torch.empty(spec.key_bytes(16, 8, 0), dtype=torch.uint8, device="cuda")
    F.fss_keygen(spec, 16, 8, 1, 0, key, None, None, None)
    dummy = torch.empty(1, dtype=torch.int64, device="cuda")
    F.fss_eval(0, key, dummy, 0, dummy, dummy)
    assert F.fss_status() == 0


def test_c2_gelu_full_size_fused():
    """Config 2 at full size (128 x 3072) in the benchmark's launch configuration:
    reconstruction for every element, bit-exact shares on sampled elements."""
    op = W.config2()[0]
    N = len(op.x)
    _flush(f"c2 gelu N={N} fused")
    g = gpu_run(op.spec, W.N_BITS, W.F_BITS, op.x, op.seed, path="fused")
    S = O.compile_spec(op.spec, W.N_BITS, W.F_BITS)
    yp, zp = O.plain_many(S, op.x)
    assert np.array_equal(g["y0"] + g["y1"] - g["r_out"], yp)
    assert np.array_equal(R.unpack_bits(g["z0"], N) ^ R.unpack_bits(g["z1"], N), zp)
    rng = np.random.Generator(np.random.PCG64(2))
    elems = np.unique(np.concatenate([rng.integers(0, N, 160), [0, 63, 64, 65, N - 65, N - 64, N - 1]]))
    o = oracle_run(op.spec, W.N_BITS, W.F_BITS, op.x, op.seed, elems, g["lookup_r"])
    compare(g, o, elems, N, check_keys=4)


def test_plain_fused_graph_identical_c3():
    """Config 3 (exp + reciprocal): plain, fused and graph-replayed outputs are
    bit-identical; sampled elements match the oracle."""
    ops = W.config3()
    _flush("c3 plain/fused/graph")
    insts = []
    for op in ops:
        inst = R.OpInstanceGPU(F.Spec(op.spec), W.N_BITS, W.F_BITS, len(op.x))
        inst.set_input(op.x)
        inst.keygen(op.seed)
        inst.mask()
        insts.append(inst)
    for inst in insts:
        for b in (0, 1):
            inst.eval_plain(b)
    torch.cuda.synchronize()
    plain = [inst.host() for inst in insts]
    items = [inst.item(b) for inst in insts for b in (0, 1)]
    plan = F.Plan(items)
    for inst in insts:
        for b in (0, 1):
            inst.y[b].zero_()
            inst.z[b].zero_()
    plan.launch()
    torch.cuda.synchronize()
    fused = [inst.host() for inst in insts]
    graph = F.Graph([plan])
    for rep in range(3):
        for inst in insts:                     # eager work between replays
            for b in (0, 1):
                inst.y[b].fill_(-1)
                inst.z[b].fill_(-1)
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        rep_out = [inst.host() for inst in insts]
        for a, c in zip(plain, rep_out):
            for k in ("y0", "y1", "z0", "z1"):
                assert np.array_equal(a[k], c[k]), (rep, k)
    assert F.fss_status() == 0
    for a, c in zip(plain, fused):
        for k in ("y0", "y1", "z0", "z1"):
            assert np.array_equal(a[k], c[k]), k
    for op, inst, out in zip(ops, insts, plain):
        N = len(op.x)
        elems = np.unique(np.r_[np.arange(0, N, max(1, N // 97)), N - 1])
        o = oracle_run(op.spec, W.N_BITS, W.F_BITS, op.x, op.seed, elems, inst.spec.lookup_r)
        out["keys0"] = inst.keys[0].cpu().numpy()
        out["keys1"] = inst.keys[1].cpu().numpy()
        compare(out, o, elems, N)


def test_all_aes_table_layouts_identical():
    op = W.config2()[0]
    x = op.x[:5000]
    ref = None
    for v in range(F.aes_variants()):
        _flush(f"aes variant {v}")
        os.environ["FSS_AES_VARIANT"] = str(v)
        os.environ["FSS_KEYGEN_VARIANT"] = str(v)
        try:
            g = gpu_run(op.spec, W.N_BITS, W.F_BITS, x, op.seed, path="fused", variant=v)
            g2 = gpu_run(op.spec, W.N_BITS, W.F_BITS, x, op.seed, path="plain")
        finally:
            os.environ.pop("FSS_AES_VARIANT", None)
            os.environ.pop("FSS_KEYGEN_VARIANT", None)
        cur = {k: g[k] for k in ("y0", "y1", "z0", "z1", "keys0", "keys1")}
        for k in ("y0", "y1", "z0", "z1"):
            assert np.array_equal(cur[k], g2[k])
        if ref is None:
            ref = cur
            o = oracle_run(op.spec, W.N_BITS, W.F_BITS, x, op.seed, np.arange(0, 5000, 97), g["lookup_r"])
            compare(g, o, np.arange(0, 5000, 97), 5000)
        else:
            for k in ref:
                assert np.array_equal(ref[k], cur[k]), (v, k)


def test_device_status_errors():
    spec = F.Spec(W.clip_relu_spec())
    N = 256
    inst = R.OpInstanceGPU(spec, 16, 8, N)
    inst.set_input(W.config1()[0].x[:N])
    inst.keygen(5)
    inst.mask()
    with pytest.raises(F.FssError):
        F.fss_eval(2, inst.keys[0], inst.xhat, N, inst.y[0], inst.z[0])
    F.fss_eval(1, inst.keys[0], inst.xhat, N, inst.y[0], inst.z[0])   # wrong party's keys
    assert F.fss_status() == -5
    F.fss_eval(0, inst.keys[0], inst.xhat, N + 1, inst.y[0], inst.z[0])  # more than keyed
    assert F.fss_status() == -4
    assert F.fss_status() == 0
    with pytest.raises(F.FssError):
        F.Plan([(1, inst.keys[0], inst.xhat, inst.y[0], inst.z[0], N)])


def test_keygen_single_party_matches():
    op = W.config1()[0]
    spec = F.Spec(op.spec)
    N = 700
    a = R.OpInstanceGPU(spec, 16, 8, N)
    b = R.OpInstanceGPU(spec, 16, 8, N, parties=(0,))
    for inst in (a, b):
        inst.set_input(op.x[:N])
        inst.keygen(99)
    torch.cuda.synchronize()
    assert torch.equal(a.keys[0], b.keys[0])
    assert torch.equal(a.r_in, b.r_in)


def test_c4_layer_worklist_autotuned_graph(tmp_path):
    """One GPT-2-small layer (GELU, exp, reciprocal, rsqrt) x both parties as one
    autotuned work-list, replayed from a HIP graph: equal to the plain path,
    sampled elements equal to the oracle."""
    ops = W.config4(layers=1)
    _flush("c4 layer 0 work-list")
    insts = []
    for op in ops:
        inst = R.OpInstanceGPU(F.Spec(op.spec), W.N_BITS, W.F_BITS, len(op.x))
        inst.set_input(op.x)
        inst.keygen(op.seed)
        inst.mask()
        insts.append(inst)
    for inst in insts:
        for b in (0, 1):
            inst.eval_plain(b)
    torch.cuda.synchronize()
    plain = [inst.host() for inst in insts]
    items = [inst.item(b) for inst in insts for b in (0, 1)]
    tune = F.fss_autotune(items, str(tmp_path / "tune.txt"))
    again = F.fss_autotune(items, str(tmp_path / "tune.txt"))      # served from the cache
    assert (tune.aes_variant, tune.blocks_per_cu, tune.order) == (again.aes_variant, again.blocks_per_cu,
                                                                  again.order)
    plan = F.Plan(items, tune)
    graph = F.Graph([plan])
    for rep in range(2):
        for inst in insts:
            for b in (0, 1):
                inst.y[b].fill_(7)
                inst.z[b].fill_(7)
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        for a, inst in zip(plain, insts):
            c = inst.host()
            for k in ("y0", "y1", "z0", "z1"):
                assert np.array_equal(a[k], c[k]), (rep, k)
    assert F.fss_status() == 0
    graph.free()
    plan.free()
    for op, inst, out in zip(ops, insts, plain):
        N = len(op.x)
        elems = np.unique(np.r_[np.linspace(0, N - 1, 48).astype(np.int64), [63, 64, N - 1]])
        elems = elems[elems < N]
        o = oracle_run(op.spec, W.N_BITS, W.F_BITS, op.x, op.seed, elems, inst.spec.lookup_r)
        out["keys0"] = inst.keys[0].cpu().numpy()
        out["keys1"] = inst.keys[1].cpu().numpy()
        compare(out, o, elems, N)


@pytest.mark.parametrize("r", [2, 3, 4])
def test_plan_work_counts(r):
    """The plan's AES-block and table-lookup counts (the roofline's work
    figure) equal the walks written out one by one: every Z_2 atom level above
    the leaves is one block, and its leaf conversion one more; the lookup DCF's walk at v has L - 1 levels of 1 + nb blocks and a
    last level of nb (value blocks only); each of the T top blocks walks D
    levels; each of the m - 1 points walks L - D - 1 full levels and the last.
    Blocks expanding one seed under K tweaks share 24 of their lookups."""
    spec = F.Spec(W.gelu_spec(), lookup_r=r)
    q = spec.query(W.N_BITS, W.F_BITS)
    p, m, D, T = q["p"], q["m"], q["top_depth"], q["top_blocks"]
    L = -(-W.N_BITS // r)
    nb = (p + 1) // 2

    def lk(k):
        return 160 * k - 24 * (k - 1)

    walks = [(L - 1, 1)] + [(D, 0)] * T + [(L - D - 1, 1)] * (m - 1)  # (full levels, last level)
    atoms = sum(k - min(7, k) + 1 for k in q["atom_k"])  # tree levels above the leaves + the leaf
    aes = atoms + sum(f * (1 + nb) + e * nb for f, e in walks)
    lookups = 160 * atoms + sum(f * lk(1 + nb) + e * lk(nb) for f, e in walks)
    N = 64 * 6144  # the GELU 128 x 3072 launch: 12,288 tiles on 3,072 waves, no tile split
    op = R.OpInstanceGPU(spec, W.N_BITS, W.F_BITS, N)
    op.set_input(np.zeros(N, dtype=np.int64))
    op.keygen(5)
    plan = F.Plan([op.item(0), op.item(1)])
    assert plan.parts() == 1
    if plan.config()["pred_unit"] == 2:
        # call 1 on its own walks the lookup DCF at v for its first output:
        # seed and one value block per level, the last level's value block
        aes += (L - 1) * 2 + 1
        lookups += (L - 1) * lk(2) + lk(1)
    elif r == 3:  # two threshold atoms (the signed view's mask query is the lookup's)
        assert (aes, lookups) == (324, 47376)
    assert plan.aes_blocks() == 2 * N * aes
    assert plan.table_lookups() == 2 * N * lookups
    plan.free()
