"""Program reuse across layers (the paper's ablation "Program Reuse Across
Layers", as bench.py --ablation reuse times it): a spec compiled, a work-list
planned and its HIP graph captured once, then replayed for several layers
with fresh keys regenerated into the same buffers before each replay.  Every
replay must give the oracle's shares for that layer's seed (sampled elements,
tile edges included), so nothing of an earlier layer's keys survives."""
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


def test_rekeyed_graph_replay_matches_oracle():
    op = W.config2()[0]
    N = 64 * 1000 + 17  # ragged tail
    x = op.x[:N]
    spec = F.Spec(op.spec)
    inst = R.OpInstanceGPU(spec, W.N_BITS, W.F_BITS, N)
    inst.set_input(x)
    inst.keygen(op.seed)
    torch.cuda.synchronize()
    plan = F.Plan([inst.item(0), inst.item(1)])
    graph = F.Graph([plan])
    S = O.compile_spec(op.spec, W.N_BITS, W.F_BITS, lookup_r=spec.lookup_r)
    rng = np.random.Generator(np.random.PCG64(3))
    elems = np.unique(np.r_[rng.integers(0, N, 300), [0, 63, 64, N - 18, N - 17, N - 1]]).astype(np.int64)
    for layer in range(4):
        seed = op.seed + 7919 * layer
        print(f"reuse layer {layer}: keygen into the same buffers, graph replay", flush=True)
        inst.keygen(seed)
        inst.mask()
        for b in (0, 1):
            inst.y[b].fill_(-1)
            inst.z[b].fill_(-1)
        graph.launch()
        assert F.fss_status() == 0
        torch.cuda.synchronize()
        g = inst.host()
        y0, y1, z0, z1, r_in, r_out, _ = O.full(S, seed, elems, x[elems], masks=True)
        assert np.array_equal(g["r_in"][elems], r_in) and np.array_equal(g["r_out"][elems], r_out)
        assert np.array_equal(g["y0"][elems], y0) and np.array_equal(g["y1"][elems], y1)
        assert np.array_equal(R.unpack_bits(g["z0"], N)[elems], z0)
        assert np.array_equal(R.unpack_bits(g["z1"], N)[elems], z1)
    graph.free()
    plan.free()
