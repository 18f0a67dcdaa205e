"""Continuous-batching server for secure-inference requests (one GPU, party 0).

A request is the nonlinearity set of one BERT-base forward at sequence
length L: per layer a GELU, an exp, a reciprocal and an rsqrt call.  The
server:

* admits arrived requests in FIFO order when the key arena has room for the
  request's whole footprint (all of its layers' keys are preloaded: one-time
  key material stays device-resident until the request finishes);
* generates the admitted request's inputs, keys and masked inputs on dealer
  streams (the operators of a layer spread over several, so a small
  operator's keygen overlaps a large one's), overlapping evaluation of
  requests already admitted;
* every scheduling step launches ONE fused work-list over the next layer of
  every ready request (iteration-level continuous batching): the next step
  starts when the previous one completes, so everything that became ready
  meanwhile (new arrivals whose keys are in place) joins it;
* frees a request's arena block as soon as its last layer completes.

All FSS work goes through the C ABI (`fss`); torch provides the arena, the
streams and the synthetic inputs.  Latency is measured on the host clock
from arrival (and from admission) to completion.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import fss as F
from . import workloads as W

ALIGN = 256


class KeyArena:
    """First-fit allocator over one device buffer (offsets, 256-byte aligned)."""

    def __init__(self, nbytes: int, device: str = "cuda"):
        self.nbytes = nbytes
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.base = self.buf.data_ptr()
        self.free = [(0, nbytes)]          # sorted (offset, size)

    def alloc(self, size: int):
        size = (size + ALIGN - 1) // ALIGN * ALIGN
        for i, (off, sz) in enumerate(self.free):
            if sz >= size:
                if sz == size:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + size, sz - size)
                return off
        return None

    def release(self, off: int, size: int):
        size = (size + ALIGN - 1) // ALIGN * ALIGN
        self.free.append((off, size))
        self.free.sort()
        merged = []
        for o, s in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self.free = merged

    def free_bytes(self) -> int:
        return sum(s for _, s in self.free)


@dataclass
class OpSlot:
    """One operator call of one layer of one request, laid out in the arena."""
    name: str
    n: int
    spec: F.Spec
    seed: int
    ell: int
    key: int = 0        # arena offsets
    r_in: int = 0
    x: int = 0
    xhat: int = 0
    y: int = 0
    z: int = 0

    def words(self) -> int:
        return (self.n + 63) // 64


@dataclass
class Request:
    rid: int
    L: int
    arrival: float
    layers: int
    slots: list = field(default_factory=list)    # [layer][op] OpSlot
    footprint: int = 0
    arena_off: int = -1
    admitted: float = -1.0
    done: float = -1.0
    ready_event: object = None
    layer_ready: list = field(default_factory=list)  # per-layer dealer completion events
    next_layer: int = 0
    in_flight: bool = False
    keep_outputs: bool = False
    outputs: dict = field(default_factory=dict)  # (layer, op) -> (y, z) host arrays

    def elements(self) -> int:
        return sum(s.n for layer in self.slots for s in layer)


class Server:
    def __init__(self, arena_bytes: int, layers: int = 12, path: str = "fused", max_in_flight: int = 1,
                 tune: F.Tune | None = None, device: str = "cuda", dealer_sync: bool = False,
                 dealer_streams: int = 4):
        """`dealer_sync` makes admission wait until the request's keys are in
        place (deterministic batching, e.g. for tests); by default dealer work
        overlaps evaluation."""
        self.arena = KeyArena(arena_bytes, device)
        self.dealer_sync = dealer_sync
        self.layers = layers
        self.path = path
        self.max_in_flight = max_in_flight
        self.tune = tune
        self.device = device
        self.dealers = [torch.cuda.Stream(device=device) for _ in range(max(1, dealer_streams))]
        self.evals = torch.cuda.Stream(device=device)
        self.specs: dict = {}
        self.dealer_ms = 0.0
        self.batches = 0
        self.batch_sizes = []

    # -- layout --------------------------------------------------------------
    def _spec(self, desc) -> F.Spec:
        if desc.name not in self.specs:
            self.specs[desc.name] = F.Spec(desc)
        return self.specs[desc.name]

    def plan_request(self, rid: int, L: int, arrival: float) -> Request:
        req = Request(rid, L, arrival, self.layers)
        sizes = W.request_op_sizes(L)
        descs = W.request_specs(L)
        total = 0
        for layer in range(self.layers):
            row = []
            for j, name in enumerate(W.REQUEST_OPS):
                spec = self._spec(descs[name])
                q = spec.query(W.N_BITS, W.F_BITS)
                s = OpSlot(name, sizes[name], spec, W.request_dealer_seed(rid, layer, j), q["ell"])
                for fld, nbytes in (("key", spec.key_bytes(W.N_BITS, W.F_BITS, s.n)), ("r_in", 8 * s.n),
                                    ("x", 8 * s.n), ("xhat", 8 * s.n), ("y", 8 * s.n),
                                    ("z", 8 * max(1, s.ell * s.words()))):
                    setattr(s, fld, total)
                    total += (nbytes + ALIGN - 1) // ALIGN * ALIGN
                row.append(s)
            req.slots.append(row)
        req.footprint = total
        return req

    def _addr(self, req: Request, off: int) -> int:
        return self.arena.base + req.arena_off + off

    def _view(self, req: Request, off: int, n: int) -> torch.Tensor:
        start = req.arena_off + off
        return self.arena.buf[start:start + 8 * n].view(torch.int64)

    # -- dealer ----------------------------------------------------------------
    def admit(self, req: Request, now: float) -> bool:
        off = self.arena.alloc(req.footprint)
        if off is None:
            return False
        req.arena_off = off
        req.admitted = now
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        req.layer_ready = []
        lead = self.dealers[0]
        ev0.record(lead)
        for d in self.dealers[1:]:
            d.wait_event(ev0)
        for layer in range(self.layers):
            with torch.cuda.stream(lead):
                xs = W.request_layer_inputs_device(req.rid, req.L, layer, self.device)
            inputs_ready = torch.cuda.Event()
            inputs_ready.record(lead)
            evs = []
            for j, s in enumerate(req.slots[layer]):
                d = self.dealers[j % len(self.dealers)]
                if d is not lead:
                    d.wait_event(inputs_ready)
                with torch.cuda.stream(d):
                    self._view(req, s.x, s.n).copy_(xs[s.name])
                    F.fss_keygen(s.spec, W.N_BITS, W.F_BITS, s.seed, s.n, self._addr(req, s.key), None,
                                 self._addr(req, s.r_in), None, d.cuda_stream)
                    F.fss_mask_input(self._addr(req, s.x), self._addr(req, s.r_in), s.n,
                                     self._addr(req, s.xhat), d.cuda_stream)
                    ev = torch.cuda.Event()
                    ev.record(d)
                    evs.append(ev)
                # the generated inputs are read on this side stream
                for t in xs.values():
                    t.record_stream(d)
            # a layer can be evaluated as soon as its own keys are in place
            req.layer_ready.append(evs)
        for d in self.dealers[1:]:
            done = torch.cuda.Event()
            done.record(d)
            lead.wait_event(done)
        ev1.record(lead)
        req.ready_event = ev1
        req._dealer_events = (ev0, ev1)
        if self.dealer_sync:
            ev1.synchronize()
        return True

    # -- evaluation --------------------------------------------------------------
    def _launch(self, batch: list):
        items = []
        for req in batch:
            for s in req.slots[req.next_layer]:
                items.append((0, self._addr(req, s.key), self._addr(req, s.xhat), self._addr(req, s.y),
                              self._addr(req, s.z) if s.ell else None, s.n))
        st = self.evals.cuda_stream
        plan = None
        if self.path == "fused":
            plan = F.Plan(items, self.tune)
            plan.launch(st)
        else:
            for (party, k, xh, y, z, n) in items:
                F.fss_eval(party, k, xh, n, y, z, st)
        ev = torch.cuda.Event()
        ev.record(self.evals)
        for req in batch:
            req.in_flight = True
        self.batches += 1
        self.batch_sizes.append(len(batch))
        return (ev, batch, plan)

    def _complete(self, inflight, now: float):
        ev, batch, plan = inflight
        if plan is not None:
            plan.free()
        for req in batch:
            if req.keep_outputs:
                for s in req.slots[req.next_layer]:
                    y = self._view(req, s.y, s.n).cpu().numpy().view(np.uint64).copy()
                    z = self._view(req, s.z, max(1, s.ell * s.words())).cpu().numpy().view(np.uint64).copy()
                    x = self._view(req, s.x, s.n).cpu().numpy().copy()
                    req.outputs[(req.next_layer, s.name)] = (y, z, x)
            req.in_flight = False
            req.next_layer += 1
            if req.next_layer == self.layers:
                req.done = now
                self.dealer_ms += req._dealer_events[0].elapsed_time(req._dealer_events[1])
                self.arena.release(req.arena_off, req.footprint)

    def run(self, stream: list, keep: set = frozenset(), arrivals: bool = True) -> dict:
        """Serve `stream` = [(rid, L, arrival_seconds)] and return statistics."""
        reqs = [self.plan_request(rid, L, arr if arrivals else 0.0) for rid, L, arr in stream]
        for r in reqs:
            r.keep_outputs = r.rid in keep
            if r.footprint > self.arena.nbytes:
                raise ValueError(f"request {r.rid} (L={r.L}) needs {r.footprint} B > arena")
        future = sorted(reqs, key=lambda r: r.arrival)
        pending, active, inflight = [], [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fi = 0
        while fi < len(future) or pending or active:
            now = time.perf_counter() - t0
            while fi < len(future) and future[fi].arrival <= now:
                pending.append(future[fi])
                fi += 1
            while pending and self.admit(pending[0], now):
                active.append(pending.pop(0))
            progressed = False
            for fl in list(inflight):
                if fl[0].query():
                    inflight.remove(fl)
                    self._complete(fl, time.perf_counter() - t0)
                    progressed = True
            active = [r for r in active if r.done < 0]
            if len(inflight) < self.max_in_flight:
                batch = [r for r in active if not r.in_flight and r.next_layer < self.layers
                         and all(e.query() for e in r.layer_ready[r.next_layer])]
                if batch:
                    inflight.append(self._launch(batch))
                    progressed = True
            if not progressed:
                time.sleep(0.0002)
        torch.cuda.synchronize()
        makespan = time.perf_counter() - t0
        lat = [r.done - r.arrival for r in reqs]
        lat_adm = [r.done - r.admitted for r in reqs]
        elems = sum(r.elements() for r in reqs)
        return {
            "requests": len(reqs),
            "element_evals": elems,
            "makespan_s": makespan,
            "element_evals_per_s": elems / makespan,
            "requests_per_s": len(reqs) / makespan,
            "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                          "mean": float(np.mean(lat))},
            "admission_to_done_s": {"p50": float(np.percentile(lat_adm, 50)),
                                    "p99": float(np.percentile(lat_adm, 99))},
            "dealer_s": self.dealer_ms / 1e3,
            "batches": self.batches,
            "mean_batch_requests": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
            "arena_bytes": self.arena.nbytes,
            "max_footprint_bytes": max(r.footprint for r in reqs),
            "_requests": reqs,
        }
