"""Pins for the oracle's spec quantisation (CPU only).

Checked against what the definitions fix: the integer partition must agree
with the real-valued partition on every fixed-point grid point, coefficients
are within half an output ulp and round ties to even, sentinel predicates are
folded into constants and never become comparison atoms.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2606_09551_amd import workloads as W

SPECS_SMALL = [
    (W.clip_relu_spec(), 10, 4),
    (W.gelu_spec(f=5), 10, 5),
    (W.exp_spec(f=3), 9, 3),
    (W.recip_spec(3, f=4), 10, 4),
    (W.rsqrt_spec(f=6), 16, 6),
]


@pytest.mark.parametrize("desc,n,f", SPECS_SMALL, ids=lambda v: getattr(v, "name", str(v)))
def test_partition_matches_real_intervals(desc, n, f):
    S = O.compile_spec(desc, n, f)
    t = O.spec_tables(S)
    s = 2**(n - 1)
    for x in range(-s, s):
        xr = x / 2**f
        want = next(i for i, (lo, hi) in enumerate(desc.intervals) if lo <= xr < hi)
        got = next(i for i in range(t["m"]) if t["alpha"][i] <= x < t["alpha"][i + 1])
        assert got == want, (desc.name, x)
    assert t["aprime"] == [a + s for a in t["alpha"]]
    assert t["aprime"][0] == 0 and t["aprime"][-1] == 2**n


@pytest.mark.parametrize("desc,n,f", SPECS_SMALL, ids=lambda v: getattr(v, "name", str(v)))
def test_coefficients_within_half_ulp(desc, n, f):
    S = O.compile_spec(desc, n, f)
    t = O.spec_tables(S)
    d = t["d"]
    assert t["F_out"] == (2 * f if d <= 1 else 4 * f)
    for i, coefs in enumerate(desc.pieces):
        for l in range(t["p"]):
            c = coefs[l] if l < len(coefs) else 0.0
            a = t["coef"][i][l]
            a = a - 2**64 if a >= 2**63 else a
            assert abs(a - math.ldexp(c, t["F_out"] - l * f)) <= 0.5


def test_coefficient_ties_round_to_even():
    # F_out = 2 (out_frac_bits), f = 0: c * 2^2 lands exactly on .5 ties
    ties = [0.125, 0.375, -0.125, -0.375, 0.625]   # *4 = 0.5, 1.5, -0.5, -1.5, 2.5
    desc = W.SpecDesc("ties", [(-math.inf, 0.0), (0.0, math.inf)], [[ties[0]], [ties[1]]],
                      out_frac_bits=2)
    t = O.spec_tables(O.compile_spec(desc, 8, 0))
    assert [t["coef"][0][0], t["coef"][1][0]] == [0, 2]
    desc = W.SpecDesc("ties", [(-math.inf, 0.0), (0.0, math.inf)], [[ties[2]], [ties[4]]],
                      out_frac_bits=2)
    t = O.spec_tables(O.compile_spec(desc, 8, 0))
    assert [t["coef"][0][0], t["coef"][1][0]] == [0, 2]


@pytest.mark.parametrize("bad", [
    dict(intervals=[(0.0, 1.0), (1.0, math.inf)], pieces=[[0.0], [0.0]]),          # no -inf tail
    dict(intervals=[(-math.inf, 0.0), (0.5, math.inf)], pieces=[[0.0], [0.0]]),     # gap
    dict(intervals=[(-math.inf, 0.001), (0.001, 0.002), (0.002, math.inf)],         # same integer
         pieces=[[0.0], [0.0], [0.0]]),
    dict(intervals=[(-math.inf, math.inf)], pieces=[[0.0, 0, 0, 0, 1.0]]),          # degree 4
    dict(intervals=[(-math.inf, math.inf)], pieces=[[0.0, 0.0, 0.0, 1e6]]),         # |P| >= 2^62
])
def test_invalid_specs_rejected(bad):
    desc = W.SpecDesc("bad", bad["intervals"], bad["pieces"])
    with pytest.raises(O.SpecError):
        O.compile_spec(desc, 16, 8)


def test_unsupported_widths_rejected():
    with pytest.raises(O.SpecError):
        O.compile_spec(W.clip_relu_spec(), 33, 8)
    with pytest.raises(O.SpecError):
        O.compile_spec(W.clip_relu_spec(), 8, 8)


def test_sentinels_are_folded_not_emitted():
    P = W.PredDesc
    preds = [P(W.LT_SIGNED, 0, thr=-math.inf),          # C at -s   -> constant 0
             P(W.LT_SIGNED, 1, thr=math.inf),           # C at +s   -> constant 1
             P(W.LOWBITS_LT, 2, f_bits=3, gamma=0),     # D_{0,3}   -> 0
             P(W.LOWBITS_LT, 3, f_bits=3, gamma=8),     # D_{8,3}   -> 1
             P(W.LT_UNSIGNED, 4, thr=0.0),              # unsigned < 0 -> 0
             P(W.LT_SIGNED, 5, thr=1.0, negate=True)]   # real atom
    desc = W.SpecDesc("sent", [(-math.inf, 0.0), (0.0, math.inf)], [[0.0], [1.0]], preds)
    S = O.compile_spec(desc, 8, 2)
    t = O.spec_tables(S)
    # one threshold atom; its view (signed, n bits) is the lookup's, so its
    # mask query is the lookup DCF's and has no atom
    assert t["T"] == 1 and S.n_prim == 1 and S.n_views == 1 and S.lookup_view == 0
    assert t["negate"][:5] == [0, 1, 0, 1, 0] and t["negate"][5] == 1


def test_config_specs_shape():
    """Every config spec: two signed predicates sharing one view, the signed
    (offset-binary) view the lookup reads too -> two threshold atoms; the
    view's mask query is answered by the lookup DCF (T = 2)."""
    for desc in W.all_specs()[:7]:
        n, f = (16, 8) if desc.name == "clip_relu" else (24, 12)
        S = O.compile_spec(desc, n, f)
        t = O.spec_tables(S)
        assert t["T"] == 2 and t["ell"] == 2 and S.n_views == 1 and S.lookup_view == 0
        assert t["atoms"] == [(n, 2**(n - 1), 0), (n, 2**(n - 1), 0)]
    t = O.spec_tables(O.compile_spec(W.gelu_spec(), 24, 12))
    assert (t["m"], t["p"], t["F_out"]) == (18, 3, 48)
    t = O.spec_tables(O.compile_spec(W.exp_spec(), 24, 12))
    assert (t["m"], t["p"]) == (34, 3)
    t = O.spec_tables(O.compile_spec(W.clip_relu_spec(), 16, 8))
    assert (t["m"], t["p"], t["F_out"]) == (3, 2, 16)
