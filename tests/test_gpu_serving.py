"""Serving: each request's results are the same alone and in the continuous-
batching mix (bit-exact), for the fused and the plain evaluator, and sampled
party-0 shares equal the oracle's."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_2606_09551_amd import fss as F  # noqa: E402
from paper_2606_09551_amd import serving as S  # noqa: E402
from paper_2606_09551_amd import workloads as W  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


STREAM = [(0, 40, 0.0), (1, 16, 0.002), (2, 32, 0.004), (3, 24, 0.006), (4, 48, 0.008), (5, 20, 0.010)]
KEEP = {1, 3}


def _serve(stream, path, keep, **kw):
    srv = S.Server(arena_bytes=3 * 2**30 // 2, layers=2, path=path, dealer_sync=kw.pop("dealer_sync", False))
    stats = srv.run(stream, keep=keep, **kw)
    return srv, stats, {r.rid: r for r in stats["_requests"]}


def test_served_equals_alone_and_oracle():
    print("serving mix (fused)", flush=True)
    srv, stats, mix = _serve(STREAM, "fused", KEEP)
    assert stats["requests"] == len(STREAM)
    assert all(r.done >= r.admitted >= r.arrival for r in mix.values())
    # the arena (1.5 GB) cannot hold all six requests at once: admission queued some
    assert stats["max_footprint_bytes"] * 3 > srv.arena.nbytes
    assert srv.arena.free_bytes() == srv.arena.nbytes  # everything released
    for rid in KEEP:
        print(f"request {rid} alone", flush=True)
        L = next(L for r, L, _ in STREAM if r == rid)
        for path in ("fused", "plain"):
            _, _, alone = _serve([(rid, L, 0.0)], path, {rid})
            a, b = mix[rid].outputs, alone[rid].outputs
            assert a.keys() == b.keys() and len(a) == 2 * len(W.REQUEST_OPS)
            for k in a:
                for u, v in zip(a[k], b[k]):
                    assert np.array_equal(u, v), (rid, path, k)
    # oracle: party-0 shares of every element of every op of request 1, all layers
    check_request_vs_oracle(mix[1], 1, 16, 2)


def check_request_vs_oracle(req, rid, L, layers):
    """Party-0 shares (y and the predicate bits) of every element of every
    operator of every layer of one served request equal the oracle's."""
    descs = W.request_specs(L)
    total = 0
    for layer in range(layers):
        for j, name in enumerate(W.REQUEST_OPS):
            y, z, x = req.outputs[(layer, name)]
            n = len(x)
            Sp = O.compile_spec(descs[name], W.N_BITS, W.F_BITS, lookup_r=F.Spec(descs[name]).lookup_r)
            elems = np.arange(n, dtype=np.int64)
            y0, _, z0, _, _ = O.full(Sp, W.request_dealer_seed(rid, layer, j), elems, x)
            assert np.array_equal(y[:n], y0), (layer, name)
            ell = Sp.ell
            words = (n + 63) // 64
            zp = z[: ell * words].reshape(ell, words)
            got = np.zeros(n, np.uint64)
            for bit in range(ell):
                got |= ((zp[bit][elems >> 6] >> (elems & 63).astype(np.uint64)) & np.uint64(1)) << np.uint64(bit)
            assert np.array_equal(got, z0), (layer, name)
            total += n
        print(f"request {rid} layer {layer}: every element equals the oracle", flush=True)
    return total


def test_c5_request_every_layer():
    """A BERT-base request of the serving workload (L = 16, all 12 layers of
    GELU, exp, reciprocal and two rsqrt per token) served beside a second
    request: every element of every layer equals the oracle."""
    stream = [(1, 16, 0.0), (2, 20, 0.0)]
    probe = S.Server(arena_bytes=1, layers=12, path="fused")
    need = sum(probe.plan_request(rid, L, 0.0).footprint for rid, L, _ in stream)
    del probe
    srv = S.Server(arena_bytes=need + 2**20, layers=12, path="fused")
    print("serving two requests over 12 layers (fused)", flush=True)
    stats = srv.run(stream, keep={1})
    req = {r.rid: r for r in stats["_requests"]}[1]
    assert len(req.outputs) == 12 * len(W.REQUEST_OPS)
    total = check_request_vs_oracle(req, 1, 16, 12)
    assert total == 12 * sum(W.request_op_sizes(16).values())


def test_arena_first_fit_and_coalescing():
    a = S.KeyArena(4096, "cuda")
    x = a.alloc(1000)
    y = a.alloc(1000)
    z = a.alloc(1000)
    assert (x, y, z) == (0, 1024, 2048)
    assert a.alloc(2000) is None
    a.release(y, 1000)
    a.release(x, 1000)
    assert a.alloc(2000) == 0
    a.release(0, 2000)
    a.release(z, 1000)
    assert a.free_bytes() == 4096 and a.free == [(0, 4096)]


def test_admitted_requests_share_launches():
    """With every request arriving at once and admission waiting for its keys,
    each scheduling step batches all admitted requests: launches are shared,
    and the requests queued behind the arena still complete."""
    print("serving batch (fused, dealer_sync)", flush=True)
    srv, stats, mix = _serve(STREAM, "fused", set(), dealer_sync=True, arrivals=False)
    assert stats["requests"] == len(STREAM)
    assert all(r.done > 0 for r in mix.values())
    assert stats["mean_batch_requests"] > 1.0
    assert srv.arena.free_bytes() == srv.arena.nbytes
