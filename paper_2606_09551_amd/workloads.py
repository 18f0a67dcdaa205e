"""Seeded synthetic workloads: real-valued operator specs and plaintext inputs.

This module is the only thing the GPU library's callers and the CPU oracle
both consume.  It holds no FSS arithmetic: it describes operator
specifications with real numbers (partition, per-interval polynomial pieces,
predicate bits) and draws plaintext inputs with numpy's PCG64.  Each side
quantises and evaluates on its own.

Operator specifications follow the paper's Definition "Operator
specification": a partition of the (signed) fixed-point input range into
intervals, a polynomial of degree <= d per interval, and predicate bits.
The paper publishes no coefficients; the pieces below are per-interval
least-squares fits on the interval's own fixed-point grid (GELU in its erf
form, exp, reciprocal, rsqrt).  Workload shapes follow BERT-base / GPT-2
small (hidden 768, FFN 3072, 12 heads, 12 layers), the models the paper
evaluates.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

LT_SIGNED, LT_UNSIGNED, LOWBITS_LT, MSB_SHIFT = 0, 1, 2, 3
INF = math.inf

MASK64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """SplitMix64 finaliser (Steele, Lea, Flood 2014); derives per-op seeds."""
    x = (x + 0x9E3779B97F4A7C15) & MASK64
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & MASK64
    return x ^ (x >> 31)


@dataclass(frozen=True)
class PredDesc:
    """One primitive predicate; predicates sharing ``out`` are XORed."""
    kind: int
    out: int
    thr: float = 0.0      # real threshold (LT_SIGNED / LT_UNSIGNED)
    negate: bool = False
    f_bits: int = 0       # LOWBITS_LT
    gamma: int = 0        # LOWBITS_LT integer threshold
    c: int = 0            # MSB_SHIFT public shift


@dataclass
class SpecDesc:
    name: str
    intervals: list            # [(lo, hi)] real, contiguous, -inf .. +inf
    pieces: list               # [[c0, c1, ..]] real coefficients, lowest first
    preds: list = field(default_factory=list)
    out_frac_bits: int = -1    # -1: 2f for degree <= 1, 4f otherwise
    ref: object = None         # FP64 reference function (for error reports only)


# ---------------------------------------------------------------------------
# Fitting helpers (FP64, deterministic)
# ---------------------------------------------------------------------------

def _grid(lo: float, hi: float, f: int) -> np.ndarray:
    """Fixed-point grid points (real values) of [lo, hi) at f fractional bits."""
    a = math.ceil(lo * (1 << f))
    b = math.ceil(hi * (1 << f))
    return np.arange(a, b, dtype=np.float64) / float(1 << f)


def fit_piece(fn, lo: float, hi: float, f: int, degree: int) -> list:
    """Least-squares polynomial fit of fn on the grid of [lo, hi).

    Solved in the centred variable t = (x - mid) / half for conditioning,
    then expanded back to monomial coefficients in x (lowest first)."""
    xs = _grid(lo, hi, f)
    if len(xs) <= degree:
        xs = np.linspace(lo, hi, degree + 2)[:-1]
    mid, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
    t = (xs - mid) / half
    V = np.vander(t, degree + 1, increasing=True)
    ct, *_ = np.linalg.lstsq(V, fn(xs), rcond=None)
    # p(x) = sum_k ct_k ((x - mid)/half)^k  ->  monomials in x
    out = np.zeros(degree + 1)
    for k, c in enumerate(ct):
        for j in range(k + 1):
            out[j] += c * math.comb(k, j) * (-mid) ** (k - j) / half ** k
    return [float(v) for v in out]


def _gelu(x):
    x = np.asarray(x, dtype=np.float64)
    erf = np.vectorize(math.erf, otypes=[np.float64])
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def _exp(x):
    return np.exp(np.asarray(x, dtype=np.float64))


def _recip(x):
    return 1.0 / np.asarray(x, dtype=np.float64)


def _rsqrt(x):
    return 1.0 / np.sqrt(np.asarray(x, dtype=np.float64))


def two_edge_preds(lo: float, hi: float) -> list:
    """The two predicate bits every config spec carries: x < lo and x < hi (signed)."""
    return [PredDesc(LT_SIGNED, 0, thr=lo), PredDesc(LT_SIGNED, 1, thr=hi)]


def spline_spec(name, fn, edges, f, degree, left_piece, right_piece, preds, out_frac_bits=-1):
    intervals = [(-INF, edges[0])]
    pieces = [left_piece]
    for a, b in zip(edges[:-1], edges[1:]):
        intervals.append((a, b))
        pieces.append(fit_piece(fn, a, b, f, degree))
    intervals.append((edges[-1], INF))
    pieces.append(right_piece)
    return SpecDesc(name, intervals, pieces, preds, out_frac_bits, ref=fn)


# ---------------------------------------------------------------------------
# The operator specs of the benchmark configurations
# ---------------------------------------------------------------------------

def clip_relu_spec() -> SpecDesc:
    """clip-ReLU: (-inf,0) -> 0, [0,6) -> x, [6,inf) -> 6."""
    return SpecDesc("clip_relu", [(-INF, 0.0), (0.0, 6.0), (6.0, INF)],
                    [[0.0], [0.0, 1.0], [6.0]], two_edge_preds(0.0, 6.0),
                    ref=lambda x: np.clip(np.asarray(x, np.float64), 0.0, 6.0))


def gelu_spec(f: int = 12) -> SpecDesc:
    """GELU: 16 equal intervals on [-6,6) with degree-2 fits; tails 0 and x."""
    edges = [-6.0 + 0.75 * i for i in range(17)]
    return spline_spec("gelu", _gelu, edges, f, 2, [0.0], [0.0, 1.0], two_edge_preds(-6.0, 6.0))


def exp_spec(f: int = 12) -> SpecDesc:
    """nExp on row-centred inputs: 32 intervals of width 0.5 on [-16,0); tails 0 and 1."""
    edges = [-16.0 + 0.5 * i for i in range(33)]
    return spline_spec("exp", _exp, edges, f, 2, [0.0], [1.0], two_edge_preds(-16.0, 0.0))


def recip_spec(hi_log2: int = 7, f: int = 12) -> SpecDesc:
    """Reciprocal on [1, 2^hi_log2): 24 geometric intervals; tails 1 and 2^-hi_log2."""
    edges = [2.0 ** (hi_log2 * i / 24.0) for i in range(25)]
    edges[-1] = float(2 ** hi_log2)
    return spline_spec(f"recip{2 ** hi_log2}", _recip, edges, f, 2, [1.0],
                       [2.0 ** -hi_log2], two_edge_preds(1.0, float(2 ** hi_log2)))


def rsqrt_spec(f: int = 12) -> SpecDesc:
    """rsqrt on [2^-4, 2^8): 24 intervals, two per octave; tails 4 and 2^-4."""
    edges = [2.0 ** (-4.0 + 0.5 * i) for i in range(25)]
    return spline_spec("rsqrt", _rsqrt, edges, f, 2, [4.0], [2.0 ** -4],
                       two_edge_preds(2.0 ** -4, 2.0 ** 8))


def relu_worked_example_spec() -> SpecDesc:
    """The paper's worked example (appendix "A complete (F, Phi) pair") as a
    single-output spec: y = max(x, 0) with the sign bit MSB(x)."""
    return SpecDesc("relu", [(-INF, 0.0), (0.0, INF)], [[0.0], [0.0, 1.0]],
                    [PredDesc(MSB_SHIFT, 0, c=0)], ref=lambda x: np.maximum(x, 0.0))


# ---------------------------------------------------------------------------
# Plaintext input generators
# ---------------------------------------------------------------------------

def quantize(xr, n: int, f: int) -> np.ndarray:
    """Round-half-to-even to f fractional bits, clamp to the signed n-bit range."""
    s = 1 << (n - 1)
    q = np.rint(np.asarray(xr, dtype=np.float64) * float(1 << f))
    return np.clip(q, -s, s - 1).astype(np.int64)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def softmax_inputs(g: np.random.Generator, heads: int, L: int, sigma: float = 3.0):
    """Row-centred logits (x - max) and FP64 row sums of exp of them."""
    logits = g.normal(0.0, sigma, size=(heads, L, L))
    centred = logits - logits.max(axis=-1, keepdims=True)
    sums = np.exp(centred).sum(axis=-1)
    return centred, sums


def layernorm_variances(g: np.random.Generator, tokens: int, hidden: int = 768):
    sig = 2.0 ** g.uniform(-1.5, 3.5, size=tokens)
    vals = g.normal(0.0, 1.0, size=(tokens, hidden)) * sig[:, None]
    return vals.var(axis=-1)


@dataclass
class OpInstance:
    """One operator call: a spec over a tensor of plaintext fixed-point inputs."""
    name: str
    spec: SpecDesc
    x: np.ndarray          # int64 plaintext inputs (flattened)
    seed: int              # dealer seed for this op's keys
    shape: tuple = ()


N_BITS, F_BITS = 24, 12


def config1() -> list:
    """Single clip-ReLU, 4096 inputs U[-16,16), 16-bit input, 8 frac bits."""
    g = rng(0xC1)
    x = quantize(g.uniform(-16.0, 16.0, size=4096), 16, 8)
    return [OpInstance("clip_relu", clip_relu_spec(), x, splitmix64(0xC1 ^ 0), (4096,))]


def config2() -> list:
    """GELU over one BERT-base FFN activation, 128 x 3072, x ~ N(0, 1.5^2)."""
    g = rng(0xC2)
    x = quantize(g.normal(0.0, 1.5, size=(128, 3072)), N_BITS, F_BITS).ravel()
    return [OpInstance("gelu", gelu_spec(), x, splitmix64(0xC2 ^ 0), (128, 3072))]


def config3() -> list:
    """Softmax helpers for 12 heads x 128 x 128: nExp then reciprocal of row sums."""
    g = rng(0xC3)
    centred, sums = softmax_inputs(g, 12, 128)
    return [OpInstance("exp", exp_spec(), quantize(centred, N_BITS, F_BITS).ravel(),
                       splitmix64(0xC3 ^ 0), (12, 128, 128)),
            OpInstance("recip", recip_spec(7), quantize(sums, N_BITS, F_BITS).ravel(),
                       splitmix64(0xC3 ^ 1), (12, 128))]


def gpt2_layer_ops(g: np.random.Generator, L: int, master: int, layer: int,
                   ln_per_layer: int = 1, recip_log2: int = 8) -> list:
    """The nonlinearity calls of one transformer layer at sequence length L."""
    base = 4 * layer
    xs_g = quantize(g.normal(0.0, 1.5, size=(L, 3072)), N_BITS, F_BITS).ravel()
    centred, sums = softmax_inputs(g, 12, L)
    var = layernorm_variances(g, ln_per_layer * L)
    return [
        OpInstance(f"L{layer}.gelu", gelu_spec(), xs_g, splitmix64(master ^ (base + 0)), (L, 3072)),
        OpInstance(f"L{layer}.exp", exp_spec(), quantize(centred, N_BITS, F_BITS).ravel(),
                   splitmix64(master ^ (base + 1)), (12, L, L)),
        OpInstance(f"L{layer}.recip", recip_spec(recip_log2),
                   quantize(sums, N_BITS, F_BITS).ravel(), splitmix64(master ^ (base + 2)), (12, L)),
        OpInstance(f"L{layer}.rsqrt", rsqrt_spec(), quantize(var, N_BITS, F_BITS).ravel(),
                   splitmix64(master ^ (base + 3)), (ln_per_layer * L,)),
    ]


def config4(layers: int = 12) -> list:
    """GPT-2-small forward at seq 256: per layer GELU, exp, reciprocal, rsqrt."""
    g = rng(0xC4)
    ops = []
    for layer in range(layers):
        ops += gpt2_layer_ops(g, 256, 0xC4, layer, ln_per_layer=1, recip_log2=8)
    return ops


@dataclass
class Request:
    rid: int
    arrival: float         # seconds after the stream starts
    L: int


def config5_requests(n_requests: int = 64, rate: float = 50.0, seed: int = 0xC5) -> list:
    """Poisson request stream (mean `rate` req/s), sequence lengths U{16..512}."""
    g = rng(seed)
    gaps = g.exponential(1.0 / rate, size=n_requests)
    arr = np.cumsum(gaps) - gaps[0]
    Ls = g.integers(16, 513, size=n_requests)
    return [Request(i, float(arr[i]), int(Ls[i])) for i in range(n_requests)]


def request_ops(req: Request, layers: int = 12, seed: int = 0xC5) -> list:
    """BERT-base nonlinearity set of one request (two LayerNorms per layer)."""
    g = rng(splitmix64(seed ^ (0x1000 + req.rid)))
    master = splitmix64(seed ^ (0x2000 + req.rid))
    recip_log2 = 7 if req.L <= 128 else (8 if req.L <= 256 else 9)
    ops = []
    for layer in range(layers):
        ops += gpt2_layer_ops(g, req.L, master, layer, ln_per_layer=2, recip_log2=recip_log2)
    return ops


def all_specs() -> list:
    return [clip_relu_spec(), gelu_spec(), exp_spec(), recip_spec(7), recip_spec(8),
            recip_spec(9), rsqrt_spec(), relu_worked_example_spec()]


# ---------------------------------------------------------------------------
# Device-side inputs for served requests (too large to draw on the host):
# the same distributions as above, drawn with torch's seeded CUDA generator.
# ---------------------------------------------------------------------------

REQUEST_OPS = ("gelu", "exp", "recip", "rsqrt")


def request_op_sizes(L: int) -> dict:
    """Elements of each nonlinearity call of one BERT-base layer at length L."""
    return {"gelu": L * 3072, "exp": 12 * L * L, "recip": 12 * L, "rsqrt": 2 * L}


def request_specs(L: int) -> dict:
    recip_log2 = 7 if L <= 128 else (8 if L <= 256 else 9)
    return {"gelu": gelu_spec(), "exp": exp_spec(), "recip": recip_spec(recip_log2),
            "rsqrt": rsqrt_spec()}


def request_layer_inputs_device(rid: int, L: int, layer: int, device="cuda", seed: int = 0xC5) -> dict:
    """int64 plaintext inputs of one layer's four calls, generated on `device`."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(splitmix64(seed ^ (rid << 16) ^ layer) & ((1 << 63) - 1))
    scale = float(1 << F_BITS)
    lim = 1 << (N_BITS - 1)

    def q(t):
        return torch.clamp(torch.round(t * scale), -lim, lim - 1).to(torch.int64)

    gelu = torch.randn(L * 3072, generator=g, device=device, dtype=torch.float64) * 1.5
    logits = torch.randn(12, L, L, generator=g, device=device, dtype=torch.float64) * 3.0
    centred = logits - logits.max(dim=-1, keepdim=True).values
    sums = torch.exp(centred).sum(dim=-1)
    sig = torch.pow(2.0, torch.rand(2 * L, generator=g, device=device, dtype=torch.float64) * 5.0 - 1.5)
    vals = torch.randn(2 * L, 768, generator=g, device=device, dtype=torch.float64) * sig[:, None]
    var = vals.var(dim=-1)
    return {"gelu": q(gelu), "exp": q(centred.reshape(-1)), "recip": q(sums.reshape(-1)), "rsqrt": q(var)}


def request_dealer_seed(rid: int, layer: int, op_index: int, seed: int = 0xC5) -> int:
    return splitmix64(seed ^ (rid << 24) ^ (layer << 8) ^ op_index)
