"""fss_eval_batch_noalloc (the work-list evaluation that allocates nothing)
against fss_eval_batch on the same keys and inputs: identical shares, bit for
bit, on two calls in a row (the second on a smaller work-list, so stale
contents of the fixed work-list array would show), and the size limits
rejected on the host before anything is enqueued."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

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


def _insts(ops, n_bits, f_bits, limit=None):
    out = []
    for op in ops:
        x = op.x[:limit] if limit else op.x
        inst = R.OpInstanceGPU(F.Spec(op.spec), n_bits, f_bits, len(x))
        inst.set_input(x)
        inst.keygen(op.seed)
        inst.mask()
        out.append(inst)
    torch.cuda.synchronize()
    return out


def _outputs(insts, fn):
    for inst in insts:
        for b in (0, 1):
            inst.y[b].fill_(-1)
            inst.z[b].fill_(-1)
    torch.cuda.synchronize()
    fn(F.PARTY_ANY, [inst.item(b) for inst in insts for b in (0, 1)])
    assert F.fss_status() == 0
    torch.cuda.synchronize()
    return [inst.host() for inst in insts]


def _same(a, b):
    for u, v in zip(a, b):
        for k in ("y0", "y1", "z0", "z1"):
            assert np.array_equal(u[k], v[k]), k


def test_noalloc_equals_eval_batch_twice():
    # first call: the softmax helpers (exp 12x128x128 + reciprocal 12x128, both
    # parties): the planner splits their tiles into parts that add into y
    print("no-alloc call 1: exp + reciprocal", flush=True)
    big = _insts(W.config3(), W.N_BITS, W.F_BITS)
    ref = _outputs(big, F.fss_eval_batch)
    got = _outputs(big, F.fss_eval_batch_noalloc)
    _same(ref, got)
    del big
    # second call, smaller: 1000 GELU elements and 300 clip-ReLU elements
    print("no-alloc call 2: smaller work-list", flush=True)
    small = _insts(W.config2(), W.N_BITS, W.F_BITS, limit=1000) + _insts(W.config1(), 16, 8, limit=300)
    ref = _outputs(small, F.fss_eval_batch)
    got = _outputs(small, F.fss_eval_batch_noalloc)
    _same(ref, got)


def test_noalloc_limits_rejected_on_host():
    op = W.config1()[0]
    n = 64 * 481  # 481 tiles: 1024 such items exceed the unit limit
    inst = R.OpInstanceGPU(F.Spec(op.spec), 16, 8, n)
    inst.set_input(np.resize(op.x, n))
    inst.keygen(9)
    inst.mask()
    torch.cuda.synchronize()
    item = inst.item(0)
    with pytest.raises(F.FssError) as e:
        F.fss_eval_batch_noalloc(0, [item] * (F.NOALLOC_MAX_ITEMS + 1))
    assert e.value.code == -8
    assert 1024 * 481 > F.NOALLOC_MAX_UNITS
    with pytest.raises(F.FssError) as e:
        F.fss_eval_batch_noalloc(0, [item] * F.NOALLOC_MAX_ITEMS)
    assert e.value.code == -8 and "unit" in str(e.value)
    with pytest.raises(F.FssError) as e:
        F.fss_eval_batch_noalloc(1, [item])
    assert e.value.code == -5
    assert F.fss_status() == 0
