"""Fixed-point approximation error of the config specs against their FP64
reference functions (the bounds here are loose sanity limits, not accuracy
claims)."""
import numpy as np
import pytest

import oracle as O
from paper_2606_09551_amd import workloads as W

CASES = [  # spec, domain, n, f, max-abs-error bound
    (W.clip_relu_spec(), -16, 16, 16, 8, 0.0),
    (W.gelu_spec(), -8, 8, 24, 12, 5e-3),
    (W.exp_spec(), -20, 0, 24, 12, 2e-3),
    (W.recip_spec(7), 1, 128, 24, 12, 1e-3),
    (W.recip_spec(8), 1, 256, 24, 12, 4e-3),
    (W.rsqrt_spec(), 2**-4, 256, 24, 12, 5e-3),
]


@pytest.mark.parametrize("desc,lo,hi,n,f,bound", CASES, ids=lambda v: getattr(v, "name", str(v)))
def test_spec_approximation_error(desc, lo, hi, n, f, bound):
    S = O.compile_spec(desc, n, f)
    F_out = O.spec_tables(S)["F_out"]
    xs = np.unique(np.round(np.linspace(lo, hi, 4001) * 2**f).astype(np.int64))
    xs = xs[(xs >= -2**(n - 1)) & (xs < 2**(n - 1))]
    ys, _ = O.plain_many(S, xs)
    got = ys.view(np.int64).astype(np.float64) / 2.0**F_out
    err = np.abs(got - desc.ref(xs / 2.0**f))
    assert err.max() <= bound + 1e-15, (desc.name, err.max())
