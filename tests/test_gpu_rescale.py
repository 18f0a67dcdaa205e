"""GPU parity of the rescaling gate (ARS of a masked value) with the oracle,
bit-exact, alone and composed after an operator gate: the operator's output
mask is the rescaling gate's input mask, the parties open y_0 + y_1, and the
gate returns shares of floor(y / 2^s) plus a fresh mask."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_2606_09551_amd import fss as F  # noqa: E402
from paper_2606_09551_amd import runtime as R  # noqa: E402
from paper_2606_09551_amd import workloads as W  # noqa: E402

M64 = 2**64 - 1


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def _rescale_gpu(shift, r, seed, r_in, y0, y1):
    n = len(r_in)
    g = R.RescaleGPU(shift, n, r)
    g.keygen(seed, _dev(r_in))
    g.open(_dev(y0), _dev(y1))
    for b in (0, 1):
        g.eval(b)
    assert F.fss_status() == 0
    torch.cuda.synchronize()
    return g.host()


@pytest.mark.parametrize("r", [2, 3, 4])
@pytest.mark.parametrize("shift", [1, 8, 24, 32])
def test_rescale_vs_oracle(shift, r):
    rng = np.random.Generator(np.random.PCG64(100 * shift + r))
    n = 1000  # 15 tiles and a ragged tail
    y = rng.integers(-2**62 + 1, 2**62, size=n, dtype=np.int64)
    y[:6] = [0, -1, 1, 2**62 - 1, -2**62 + 1, -(2**shift)]
    r_in = rng.integers(0, 2**64, size=n, dtype=np.uint64)
    r_in[:2] = [0, 2**63]
    yhat = (y.view(np.uint64) + r_in).astype(np.uint64)
    y0 = rng.integers(0, 2**64, size=n, dtype=np.uint64)
    y1 = (yhat - y0).astype(np.uint64)
    print(f"rescale shift={shift} r={r}", flush=True)
    g = _rescale_gpu(shift, r, 0x51 + shift, r_in, y0, y1)
    assert np.array_equal(g["yhat"], yhat)
    z0, z1, r_out = O.trunc(shift, 0x51 + shift, np.arange(n), r_in, yhat, lookup_r=r)
    for k, v in (("z0", z0), ("z1", z1), ("r_out", r_out)):
        assert np.array_equal(g[k], v), k
    assert np.array_equal(g["z0"] + g["z1"] - g["r_out"], (y >> shift).view(np.uint64))


def test_rescale_every_shift():
    """Every shift the gate accepts (1..32), the radix cycling through 2, 3, 4,
    200 elements each (inputs at the 2^62 bound, at multiples of 2^s and
    beside them), against the oracle and Python's floor shift."""
    for shift in range(1, 33):
        r = 2 + shift % 3
        rng = np.random.Generator(np.random.PCG64(7000 + shift))
        n = 200
        y = rng.integers(-2**62 + 1, 2**62, size=n, dtype=np.int64)
        k = 1 << shift
        y[:8] = [0, -1, k, -k, k - 1, -k - 1, 2**62 - 1, -2**62 + 1]
        r_in = rng.integers(0, 2**64, size=n, dtype=np.uint64)
        r_in[:3] = [0, 2**63, 2**64 - 1]
        yhat = (y.view(np.uint64) + r_in).astype(np.uint64)
        y0 = rng.integers(0, 2**64, size=n, dtype=np.uint64)
        y1 = (yhat - y0).astype(np.uint64)
        print(f"rescale every shift: shift={shift} r={r}", flush=True)
        g = _rescale_gpu(shift, r, 0x7A + shift, r_in, y0, y1)
        z0, z1, r_out = O.trunc(shift, 0x7A + shift, np.arange(n), r_in, yhat, lookup_r=r)
        for name, v in (("z0", z0), ("z1", z1), ("r_out", r_out)):
            assert np.array_equal(g[name], v), (shift, name)
        assert np.array_equal(g["z0"] + g["z1"] - g["r_out"], (y >> shift).view(np.uint64)), shift


@pytest.mark.parametrize("case", ["clip_relu_4096", "gelu_65536_fout36"])
def test_operator_then_rescale(case):
    """An operator gate (fused launch, both parties), the opening of its
    output, and the rescaling gate back to f fractional bits: every element's
    shares and masks equal the oracle's chain, and the result is the
    plaintext piece shifted down by F_out - f."""
    if case == "clip_relu_4096":
        op = W.config1()[0]
        n_bits, f = 16, 8
        desc, x = op.spec, op.x
    else:
        op = W.config2()[0]
        n_bits, f = W.N_BITS, W.F_BITS
        desc = W.gelu_spec()
        desc.out_frac_bits = 3 * f
        x = op.x[:65536]
    spec = F.Spec(desc)
    q = spec.query(n_bits, f)
    shift = q["F_out"] - f
    n = len(x)
    print(f"{case}: operator gate then rescale by {shift}", flush=True)
    inst = R.OpInstanceGPU(spec, n_bits, f, n)
    inst.set_input(x)
    inst.keygen(op.seed)
    inst.mask()
    F.Plan([inst.item(0), inst.item(1)]).launch()
    g = R.RescaleGPU(shift, n)
    g.keygen(op.seed + 1, inst.r_out)
    g.open(inst.y[0], inst.y[1])
    for b in (0, 1):
        g.eval(b)
    assert F.fss_status() == 0
    torch.cuda.synchronize()
    got = g.host()
    S = O.compile_spec(desc, n_bits, f)
    y0, y1, _, _, _, r_out, _ = O.full(S, op.seed, np.arange(n), x, masks=True)
    yhat = (y0 + y1).astype(np.uint64)
    z0, z1, r_out2 = O.trunc(shift, op.seed + 1, np.arange(n), r_out, yhat)
    for k, v in (("yhat", yhat), ("z0", z0), ("z1", z1), ("r_out", r_out2)):
        assert np.array_equal(got[k], v), k
    yp, _ = O.plain_many(S, x)
    assert np.array_equal(got["z0"] + got["z1"] - got["r_out"], (yp.view(np.int64) >> shift).view(np.uint64))


def test_rescale_key_checks():
    n = 128
    g = R.RescaleGPU(8, n)
    g.keygen(3, _dev(np.zeros(n, np.uint64)))
    g.open(_dev(np.zeros(n, np.uint64)), _dev(np.zeros(n, np.uint64)))
    F.fss_rescale_eval(1, g.keys[0], g.yhat, n, g.z[1])            # party 0's keys as party 1
    assert F.fss_status() == -5
    inst = R.OpInstanceGPU(F.Spec(W.clip_relu_spec()), 16, 8, n)
    inst.set_input(W.config1()[0].x[:n])
    inst.keygen(4)
    F.fss_rescale_eval(0, inst.keys[0], g.yhat, n, g.z[0])          # an operator gate's keys
    assert F.fss_status() == -4
    F.fss_rescale_eval(0, g.keys[0], g.yhat, n + 1, g.z[0])         # more than keyed
    assert F.fss_status() == -4
    assert F.fss_status() == 0
