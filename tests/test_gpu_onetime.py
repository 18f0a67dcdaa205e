"""One-time keys on the GPU: the first evaluation records each element's
masked input in its key buffer; a replay at the same input gives the same
shares, an evaluation at another input is refused for the changed elements
(zero outputs, FSS_E_CONSUMED) while the others are unaffected, and fresh
keys generated into the same buffer start over.  Operator gates (plain and
fused paths) and the rescaling gate."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_2606_09551_amd import fss as F  # noqa: E402
from paper_2606_09551_amd import runtime as R  # noqa: E402
from paper_2606_09551_amd import workloads as W  # noqa: E402

CONSUMED = -9


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _eval(inst, path):
    if path == "plain":
        for b in (0, 1):
            inst.eval_plain(b)
    elif path == "lanes":  # two lanes per element, call 1 in units of its own
        plan = F.Plan([inst.item(0), inst.item(1)], F.Tune(0, 0, 1, 0, 1, 2, 2))
        plan.launch()
        plan.free()
    else:
        F.fss_eval_batch(F.PARTY_ANY, [inst.item(0), inst.item(1)])
    code = F.fss_status()
    torch.cuda.synchronize()
    return code, inst.host()


@pytest.mark.parametrize("path", ["plain", "fused", "lanes"])
def test_operator_keys_are_one_time(path):
    op = W.config1()[0]
    N = 1000
    inst = R.OpInstanceGPU(F.Spec(op.spec), 16, 8, N)
    inst.set_input(op.x[:N])
    inst.keygen(op.seed)
    inst.mask()
    print(f"one-time keys ({path}): first evaluation", flush=True)
    code, first = _eval(inst, path)
    assert code == 0
    code, again = _eval(inst, path)           # a replay at the same masked input
    assert code == 0
    for k in ("y0", "y1", "z0", "z1"):
        assert np.array_equal(first[k], again[k]), k
    changed = np.array([3, 64, 700, N - 1])
    xh = inst.xhat[:N].clone()
    xh[torch.from_numpy(changed).cuda()] += 1
    inst.xhat[:N].copy_(xh)
    print(f"one-time keys ({path}): another masked input", flush=True)
    code, bad = _eval(inst, path)
    assert code == CONSUMED
    keep = np.setdiff1d(np.arange(N), changed)
    for b in (0, 1):
        assert np.array_equal(bad[f"y{b}"][changed], np.zeros(len(changed), np.uint64))
        assert np.array_equal(bad[f"y{b}"][keep], first[f"y{b}"][keep])
        zb, zf = R.unpack_bits(bad[f"z{b}"], N), R.unpack_bits(first[f"z{b}"], N)
        assert np.array_equal(zb[changed], np.zeros(len(changed), np.uint64))
        assert np.array_equal(zb[keep], zf[keep])
    # fresh keys into the same buffers: the record starts over
    inst.keygen(op.seed + 1)
    inst.mask()
    code, fresh = _eval(inst, path)
    assert code == 0
    S = O.compile_spec(op.spec, 16, 8, lookup_r=inst.spec.lookup_r)
    y0, y1, z0, z1, _ = O.full(S, op.seed + 1, np.arange(N), op.x[:N])
    assert np.array_equal(fresh["y0"], y0) and np.array_equal(fresh["y1"], y1)
    assert np.array_equal(R.unpack_bits(fresh["z0"], N), z0)
    assert np.array_equal(R.unpack_bits(fresh["z1"], N), z1)


def test_rescale_keys_are_one_time():
    n = 300
    rng = np.random.Generator(np.random.PCG64(4))
    r_in = torch.from_numpy(rng.integers(0, 2**63, size=n, dtype=np.int64)).cuda()
    y0 = torch.from_numpy(rng.integers(0, 2**40, size=n, dtype=np.int64)).cuda()
    y1 = torch.zeros(n, dtype=torch.int64, device="cuda")
    g = R.RescaleGPU(12, n)
    g.keygen(5, r_in)
    g.open(y0, y1)
    for b in (0, 1):
        g.eval(b)
    assert F.fss_status() == 0
    first = g.host()
    for b in (0, 1):
        g.eval(b)
    assert F.fss_status() == 0
    assert np.array_equal(g.host()["z0"], first["z0"])
    y0[7] += 1
    g.open(y0, y1)
    g.eval(0)
    assert F.fss_status() == CONSUMED
    out = g.host()
    assert out["z0"][7] == 0 and np.array_equal(np.delete(out["z0"], 7), np.delete(first["z0"], 7))
