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
