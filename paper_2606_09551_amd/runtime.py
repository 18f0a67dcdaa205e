"""Device buffers for operator instances (torch provides memory and streams).

An ``OpInstanceGPU`` owns, for one operator call over N inputs: both parties'
key buffers, the dealer's masks, the public masked inputs and both parties'
output shares.  All computation goes through the C ABI in ``fss``.
"""
from __future__ import annotations

import numpy as np
import torch

from . import fss as F


def words(n: int) -> int:
    return (n + 63) // 64


def to_u64(t: torch.Tensor) -> np.ndarray:
    """Copy an int64 device tensor to host and reinterpret as uint64."""
    return t.detach().cpu().numpy().view(np.uint64)


class OpInstanceGPU:
    def __init__(self, spec: F.Spec, n_bits: int, frac_bits: int, n: int, *, parties=(0, 1),
                 device: str = "cuda"):
        self.spec, self.n_bits, self.frac_bits, self.n = spec, n_bits, frac_bits, n
        q = spec.query(n_bits, frac_bits)
        self.ell, self.m, self.p, self.T = q["ell"], q["m"], q["p"], q["T"]
        self.atom_k = q["atom_k"]
        self.lookup_r = q["lookup_r"]
        self.key_bytes = spec.key_bytes(n_bits, frac_bits, n)
        self.parties = tuple(parties)
        dev = torch.device(device)
        self.keys = {b: torch.empty(self.key_bytes, dtype=torch.uint8, device=dev) for b in (0, 1)
                     if b in self.parties}
        mk = lambda k: torch.empty(max(k, 1), dtype=torch.int64, device=dev)
        self.r_in, self.r_out = mk(n), mk(n)
        self.x, self.xhat = mk(n), mk(n)
        self.y = {b: mk(n) for b in self.parties}
        self.z = {b: mk(self.ell * words(n)) for b in self.parties}

    def set_input(self, x: np.ndarray):
        assert x.shape == (self.n,)
        self.x[: self.n].copy_(torch.from_numpy(np.ascontiguousarray(x, dtype=np.int64)))

    def keygen(self, seed: int, stream=None):
        F.fss_keygen(self.spec, self.n_bits, self.frac_bits, seed, self.n, self.keys.get(0),
                     self.keys.get(1), self.r_in, self.r_out, stream)

    def mask(self, stream=None):
        F.fss_mask_input(self.x, self.r_in, self.n, self.xhat, stream)

    def eval_plain(self, party: int, stream=None):
        F.fss_eval(party, self.keys[party], self.xhat, self.n, self.y[party],
                   self.z[party] if self.ell else None, stream)

    def item(self, party: int):
        return (party, self.keys[party], self.xhat, self.y[party],
                self.z[party] if self.ell else None, self.n)

    def host(self) -> dict:
        n = self.n
        out = {"r_in": to_u64(self.r_in)[:n], "r_out": to_u64(self.r_out)[:n],
               "xhat": to_u64(self.xhat)[:n]}
        for b in self.parties:
            out[f"y{b}"] = to_u64(self.y[b])[:n]
            out[f"z{b}"] = to_u64(self.z[b])[: self.ell * words(n)].reshape(self.ell, words(n))
        return out


class RescaleGPU:
    """A rescaling gate (ARS by `shift` bits) over n elements whose input mask
    is a previous gate's output mask: keys for both parties, the opening
    yhat = y0 + y1 of that gate's shares, and both parties' output shares."""

    def __init__(self, shift: int, n: int, lookup_bits: int = 3, device: str = "cuda"):
        self.shift, self.n, self.lookup_bits = shift, n, lookup_bits
        self.key_bytes = F.fss_rescale_key_bytes(shift, lookup_bits, n)
        dev = torch.device(device)
        self.keys = {b: torch.empty(self.key_bytes, dtype=torch.uint8, device=dev) for b in (0, 1)}
        mk = lambda: torch.empty(max(n, 1), dtype=torch.int64, device=dev)
        self.yhat, self.r_out = mk(), mk()
        self.z = {b: mk() for b in (0, 1)}

    def keygen(self, seed: int, r_in, stream=None):
        F.fss_rescale_keygen(self.shift, self.lookup_bits, seed, self.n, r_in, self.keys[0], self.keys[1],
                             self.r_out, stream)

    def open(self, y0, y1, stream=None):
        F.fss_open(y0, y1, self.n, self.yhat, stream)

    def eval(self, party: int, stream=None):
        F.fss_rescale_eval(party, self.keys[party], self.yhat, self.n, self.z[party], stream)

    def host(self) -> dict:
        n = self.n
        return {"yhat": to_u64(self.yhat)[:n], "r_out": to_u64(self.r_out)[:n],
                "z0": to_u64(self.z[0])[:n], "z1": to_u64(self.z[1])[:n]}


def unpack_bits(planes: np.ndarray, n: int) -> np.ndarray:
    """(ell, words) u64 bit-planes -> per-element u64 with bit j = predicate j."""
    ell = planes.shape[0]
    out = np.zeros(n, dtype=np.uint64)
    idx = np.arange(n)
    for j in range(ell):
        bits = (planes[j][idx >> 6] >> (idx & 63).astype(np.uint64)) & np.uint64(1)
        out |= bits << np.uint64(j)
    return out


class LiteralGPU:
    """The paper's lookup and post-processing for one operator over n
    elements, both parties on this device: literal-lookup keys (one vector
    DCF per inner boundary of the translated partition), the Beaver triples
    of the Horner evaluation (d = p - 1 products per element, triple step t
    for the t-th), both parties' coefficient and x shares, and output shares
    with y0 + y1 = P(x) + r_out.  Every arithmetic step is a library call."""

    def __init__(self, spec: F.Spec, n_bits: int, frac_bits: int, n: int, device: str = "cuda"):
        self.spec, self.n_bits, self.frac_bits, self.n = spec, n_bits, frac_bits, n
        q = spec.query(n_bits, frac_bits)
        self.p = q["p"]
        self.d = self.p - 1
        self.key_bytes = spec.lit_key_bytes(n_bits, frac_bits, n)
        dev = torch.device(device)
        self.keys = {b: torch.empty(self.key_bytes, dtype=torch.uint8, device=dev) for b in (0, 1)}
        mk = lambda k=1: torch.empty(max(k * n, 1), dtype=torch.int64, device=dev)
        self.r_in, self.r_out, self.x, self.xhat = mk(), mk(), mk(), mk()
        self.coef = {b: mk(self.p) for b in (0, 1)}
        self.xs = {b: mk() for b in (0, 1)}
        # triples[t][name]: a0 b0 c0 a1 b1 c1
        self.triples = [{k: mk() for k in ("a0", "b0", "c0", "a1", "b1", "c1")} for _ in range(self.d)]
        self.acc = {b: [mk(), mk()] for b in (0, 1)}  # Horner accumulators, alternating
        self.dm = {b: mk() for b in (0, 1)}
        self.em = {b: mk() for b in (0, 1)}
        self.D, self.E = mk(), mk()
        self.y = None

    def set_input(self, x: np.ndarray):
        assert x.shape == (self.n,)
        self.x[: self.n].copy_(torch.from_numpy(np.ascontiguousarray(x, dtype=np.int64)))

    def keygen(self, seed: int, stream=None):
        F.fss_lit_keygen(self.spec, self.n_bits, self.frac_bits, seed, self.n, self.keys[0], self.keys[1],
                         self.r_in, self.r_out, stream)
        for t, tr in enumerate(self.triples):
            F.fss_triples(seed, self.n, t, tr["a0"], tr["b0"], tr["c0"], tr["a1"], tr["b1"], tr["c1"], stream)

    def mask(self, stream=None):
        F.fss_mask_input(self.x, self.r_in, self.n, self.xhat, stream)

    def coef_row(self, b: int, k: int):
        return self.coef[b][k * self.n: (k + 1) * self.n]

    def eval(self, stream=None):
        """Both parties' lookups, then Horner's rule: one Beaver product per
        degree, the two openings between the parties' local steps."""
        n, d = self.n, self.d
        for b in (0, 1):
            F.fss_lit_eval(b, self.keys[b], self.xhat, n, self.coef[b], self.xs[b], stream)
        cur = {b: self.coef_row(b, d) for b in (0, 1)}
        for t in range(d):
            tr = self.triples[t]
            for b in (0, 1):
                F.fss_beaver_mask(cur[b], self.xs[b], tr[f"a{b}"], tr[f"b{b}"], n, self.dm[b], self.em[b], stream)
            F.fss_open(self.dm[0], self.dm[1], n, self.D, stream)
            F.fss_open(self.em[0], self.em[1], n, self.E, stream)
            for b in (0, 1):
                out = self.acc[b][t & 1]
                F.fss_beaver_mul(b, self.D, self.E, tr[f"a{b}"], tr[f"b{b}"], tr[f"c{b}"], self.coef_row(b, d - 1 - t),
                                 n, out, stream)
                cur[b] = out
        self.y = cur

    def host(self) -> dict:
        n = self.n
        out = {"r_in": to_u64(self.r_in)[:n], "r_out": to_u64(self.r_out)[:n], "xhat": to_u64(self.xhat)[:n]}
        for b in (0, 1):
            out[f"c{b}"] = to_u64(self.coef[b])[: self.p * n].reshape(self.p, n).T.copy()
            out[f"x{b}"] = to_u64(self.xs[b])[:n]
            out[f"y{b}"] = to_u64(self.y[b])[:n]
        return out
