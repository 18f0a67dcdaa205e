"""ctypes binding of libfusefss (include/fusefss.h), same names as the C ABI.

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  Device buffers are passed as integer addresses (for example
``tensor.data_ptr()``) and streams as ``torch.cuda.current_stream().cuda_stream``.
Importing this module loads the native library and raises if it is missing.

The library links the HIP runtime by soname.  torch brings its own copy of
that runtime, and a process must hold only one (two HSA runtimes in one
process do not share the device), so torch is imported first: the library
then binds to the runtime torch already loaded.  ``FUSEFSS_LIB`` names
another build of the library to load instead of the in-tree one.
"""
from __future__ import annotations

import ctypes as C
import os

try:  # load torch's HIP runtime before the library resolves its own
    import torch  # noqa: F401
except ImportError:  # the C ABI stays usable without torch
    pass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("FUSEFSS_LIB") or os.path.join(_HERE, "_lib", "libfusefss.so")

FSS_OK = 0
ERRORS = {-1: "FSS_E_INVALID_SPEC", -2: "FSS_E_UNSUPPORTED", -3: "FSS_E_NEEDS_PHI",
          -4: "FSS_E_SHAPE", -5: "FSS_E_PARTY", -6: "FSS_E_HIP", -7: "FSS_E_OOM", -8: "FSS_E_ARG",
          -9: "FSS_E_CONSUMED"}
MAX_ATOMS = 16

PRED_LT_SIGNED, PRED_LT_UNSIGNED, PRED_LOWBITS_LT, PRED_MSB_SHIFT = 0, 1, 2, 3
PARTY_ANY = -1
COMBINE_XOR, COMBINE_AND, COMBINE_OR = 0, 1, 2


class FssError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Interval(C.Structure):
    _fields_ = [("lo", C.c_double), ("hi", C.c_double)]


class Piece(C.Structure):
    _fields_ = [("degree", C.c_int32), ("coef", C.c_double * 4)]


class Pred(C.Structure):
    _fields_ = [("kind", C.c_int32), ("negate", C.c_int32), ("out", C.c_int32),
                ("combine", C.c_int32), ("f_bits", C.c_int32), ("reserved", C.c_int32),
                ("thr", C.c_double), ("gamma", C.c_int64), ("c", C.c_int64)]


class SpecInfo(C.Structure):
    _fields_ = [("n_bits", C.c_int32), ("frac_bits", C.c_int32), ("m", C.c_int32),
                ("degree", C.c_int32), ("p", C.c_int32), ("out_frac_bits", C.c_int32),
                ("T", C.c_int32), ("ell", C.c_int32), ("atom_k", C.c_int32 * MAX_ATOMS),
                ("atom_c", C.c_int64 * MAX_ATOMS), ("atom_is_mask", C.c_int32 * MAX_ATOMS),
                ("lookup_r", C.c_int32), ("top_depth", C.c_int32), ("top_blocks", C.c_int32)]


class WorkItem(C.Structure):
    _fields_ = [("party", C.c_int32), ("reserved", C.c_int32), ("keys", C.c_void_p),
                ("xhat", C.c_void_p), ("y", C.c_void_p), ("zbits", C.c_void_p),
                ("n_elems", C.c_int64)]


class Tune(C.Structure):
    _fields_ = [("block_threads", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("aes_variant", C.c_int32), ("order", C.c_int32), ("parts", C.c_int32),
                ("pred_unit", C.c_int32), ("lanes", C.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                          "(the HIP library is required; there is no fallback)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
    sig = {
        "fss_compile_spec": [C.POINTER(Interval), i32, C.POINTER(Piece), C.POINTER(Pred), i32, i32,
                             C.POINTER(vp)],
        "fss_compile_spec_int": [i32, i32, C.POINTER(u64), i32, C.POINTER(u64), C.POINTER(Pred), i32,
                                 C.POINTER(vp)],
        "fss_spec_free": [vp],
        "fss_spec_set_lookup_radix": [vp, i32],
        "fss_spec_get_lookup_radix": [vp],
        "fss_spec_query": [vp, i32, i32, C.POINTER(SpecInfo), vp, vp],
        "fss_key_bytes": [vp, i32, i32, i64, C.POINTER(C.c_size_t)],
        "fss_keygen": [vp, i32, i32, C.POINTER(C.c_uint8), i64, vp, vp, vp, vp, vp],
        "fss_mask_input": [vp, vp, i64, vp, vp],
        "fss_keygen_work": [vp, i32, i32, i64, C.POINTER(C.c_double), C.POINTER(C.c_double)],
        "fss_rescale_key_bytes": [i32, i32, i64, C.POINTER(C.c_size_t)],
        "fss_rescale_keygen": [i32, i32, C.POINTER(C.c_uint8), i64, vp, vp, vp, vp, vp],
        "fss_rescale_eval": [i32, vp, vp, i64, vp, vp],
        "fss_open": [vp, vp, i64, vp, vp],
        "fss_eval": [i32, vp, vp, i64, vp, vp, vp],
        "fss_eval_pred": [i32, vp, vp, i64, vp, vp],
        "fss_eval_coeff": [i32, vp, vp, i64, vp, vp],
        "fss_plan_create": [C.POINTER(WorkItem), i32, C.POINTER(Tune), C.POINTER(vp)],
        "fss_plan_launch": [vp, vp],
        "fss_plan_free": [vp],
        "fss_plan_aes_blocks": [vp],
        "fss_plan_table_lookups": [vp],
        "fss_plan_parts": [vp],
        "fss_plan_config": [vp, C.POINTER(Tune), C.POINTER(i32)],
        "fss_eval_batch": [i32, C.POINTER(WorkItem), i32, vp],
        "fss_eval_batch_noalloc": [i32, C.POINTER(WorkItem), i32, vp],
        "fss_graph_capture": [C.POINTER(vp), i32, C.POINTER(vp)],
        "fss_graph_launch": [vp, vp],
        "fss_graph_free": [vp],
        "fss_autotune": [C.POINTER(WorkItem), i32, C.c_char_p, C.POINTER(Tune)],
        "fss_aes_variants": [],
        "fss_autotune_radix": [vp, i32, i32, i64, C.c_char_p, C.POINTER(i32)],
        "fss_lit_key_bytes": [vp, i32, i32, i64, C.POINTER(C.c_size_t)],
        "fss_lit_keygen": [vp, i32, i32, C.POINTER(C.c_uint8), i64, vp, vp, vp, vp, vp],
        "fss_lit_eval": [i32, vp, vp, i64, vp, vp, vp],
        "fss_triples": [C.POINTER(C.c_uint8), i64, i32, vp, vp, vp, vp, vp, vp, vp],
        "fss_beaver_mask": [vp, vp, vp, vp, i64, vp, vp, vp],
        "fss_beaver_mul": [i32, vp, vp, vp, vp, vp, vp, i64, vp, vp],
        "fss_and_triples": [C.POINTER(C.c_uint8), i64, i32, vp, vp, vp, vp, vp, vp, vp],
        "fss_xor_mask": [vp, vp, vp, vp, i64, vp, vp, vp],
        "fss_xopen": [vp, vp, i64, vp, vp],
        "fss_and": [i32, vp, vp, vp, vp, vp, i64, vp, vp],
        "fss_b2a_rand": [C.POINTER(C.c_uint8), i64, i32, vp, vp, vp, vp, vp],
        "fss_b2a": [i32, vp, vp, i64, vp, vp],
        "fss_status": [vp, C.POINTER(i32)],
        "fss_last_error": [],
        "fss_version": [],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.fss_spec_free.restype = None
    L.fss_plan_aes_blocks.restype = C.c_double
    L.fss_plan_table_lookups.restype = C.c_double
    L.fss_last_error.restype = C.c_char_p
    L.fss_version.restype = C.c_char_p
    return L


lib = _load()


def _check(rc: int):
    if rc != FSS_OK:
        raise FssError(rc, lib.fss_last_error().decode(errors="replace"))


def _p(x) -> int | None:
    """Device address of a tensor (or an int address / None)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        try:
            import torch
            return torch.cuda.current_stream().cuda_stream
        except Exception:
            return None
    return stream if isinstance(stream, int) else stream.cuda_stream


# ---------------------------------------------------------------------------

def _preds(preds):
    np_ = len(preds)
    prs = (Pred * max(np_, 1))()
    for j, q in enumerate(preds):
        prs[j] = Pred(q.kind, int(q.negate), q.out, getattr(q, "combine", 0), q.f_bits, 0,
                      q.thr, q.gamma, q.c)
    return prs, np_


class Spec:
    """An operator specification compiled by the library (fss_compile_spec),
    or in the integer form (fss_compile_spec_int) via ``Spec.integer``."""

    @classmethod
    def integer(cls, n_bits: int, alpha, coef, preds=(), lookup_r: int | None = None, name: str = "int"):
        """alpha: m + 1 boundaries 0 = alpha_0 < ... < alpha_m = 2^n_bits; coef: m rows
        of degree + 1 ring coefficients (lowest first)."""
        m = len(alpha) - 1
        deg = len(coef[0]) - 1
        a = (C.c_uint64 * (m + 1))(*[int(v) for v in alpha])
        c = (C.c_uint64 * (m * (deg + 1)))(*[int(v) & (2**64 - 1) for row in coef for v in row])
        prs, np_ = _preds(list(preds))
        h = C.c_void_p()
        _check(lib.fss_compile_spec_int(n_bits, m, a, deg, c, prs if np_ else None, np_, C.byref(h)))
        self = cls.__new__(cls)
        self.handle = h
        self.name = name
        if lookup_r is not None:
            _check(lib.fss_spec_set_lookup_radix(h, lookup_r))
        return self

    def __init__(self, desc, lookup_r: int | None = None):
        m = len(desc.intervals)
        iv = (Interval * m)(*[Interval(lo, hi) for lo, hi in desc.intervals])
        pcs = (Piece * m)()
        for i, coefs in enumerate(desc.pieces):
            pcs[i].degree = len(coefs) - 1
            for l, c in enumerate(coefs[:4]):
                pcs[i].coef[l] = c
        prs, np_ = _preds(desc.preds)
        h = C.c_void_p()
        _check(lib.fss_compile_spec(iv, m, pcs, prs if np_ else None, np_, desc.out_frac_bits,
                                    C.byref(h)))
        self.handle = h
        self.name = desc.name
        if lookup_r is not None:
            _check(lib.fss_spec_set_lookup_radix(h, lookup_r))

    @property
    def lookup_r(self) -> int:
        rc = lib.fss_spec_get_lookup_radix(self.handle)
        if rc < 0:
            _check(rc)
        return rc

    def __del__(self, _free=lib.fss_spec_free):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            _free(h)
            self.handle = None

    def query(self, n_bits: int, frac_bits: int) -> dict:
        info = SpecInfo()
        _check(lib.fss_spec_query(self.handle, n_bits, frac_bits, C.byref(info), None, None))
        m, p = info.m, info.p
        ap = (C.c_uint64 * (m + 1))()
        co = (C.c_uint64 * (m * p))()
        _check(lib.fss_spec_query(self.handle, n_bits, frac_bits, None, ap, co))
        return {"n": info.n_bits, "f": info.frac_bits, "m": m, "d": info.degree, "p": p,
                "F_out": info.out_frac_bits, "T": info.T, "ell": info.ell,
                "atom_k": list(info.atom_k[:info.T]), "atom_c": list(info.atom_c[:info.T]),
                "atom_is_mask": list(info.atom_is_mask[:info.T]),
                "lookup_r": info.lookup_r, "top_depth": info.top_depth, "top_blocks": info.top_blocks,
                "aprime": list(ap), "coef": [[co[i * p + l] for l in range(p)] for i in range(m)]}

    def autotune_radix(self, n_bits: int, frac_bits: int, n_elems: int, cache_path: str | None = None) -> int:
        """Time keygen + fused evaluation at lookup radix 2, 3 and 4 and keep the fastest
        (fss_autotune_radix); returns the chosen input bits per level."""
        best = C.c_int32()
        _check(lib.fss_autotune_radix(self.handle, n_bits, frac_bits, n_elems,
                                      cache_path.encode() if cache_path else None, C.byref(best)))
        return best.value

    def keygen_work(self, n_bits: int, frac_bits: int, n_elems: int) -> tuple:
        """(AES blocks, T-table lookups) of one fss_keygen over n_elems elements."""
        a, l = C.c_double(), C.c_double()
        _check(lib.fss_keygen_work(self.handle, n_bits, frac_bits, n_elems, C.byref(a), C.byref(l)))
        return a.value, l.value

    def key_bytes(self, n_bits: int, frac_bits: int, n_elems: int) -> int:
        out = C.c_size_t()
        _check(lib.fss_key_bytes(self.handle, n_bits, frac_bits, n_elems, C.byref(out)))
        return out.value

    def lit_key_bytes(self, n_bits: int, frac_bits: int, n_elems: int) -> int:
        out = C.c_size_t()
        _check(lib.fss_lit_key_bytes(self.handle, n_bits, frac_bits, n_elems, C.byref(out)))
        return out.value


def seed_bytes(seed: int):
    """A 128-bit dealer seed as the 16 little-endian bytes fss_keygen takes."""
    if not 0 <= int(seed) < 2**128:
        raise ValueError("the dealer seed is a 128-bit unsigned integer")
    return (C.c_uint8 * 16).from_buffer_copy(int(seed).to_bytes(16, "little"))


def fss_keygen(spec: Spec, n_bits, frac_bits, seed, n_elems, key0, key1, r_in, r_out, stream=None):
    _check(lib.fss_keygen(spec.handle, n_bits, frac_bits, seed_bytes(seed), n_elems, _p(key0),
                          _p(key1), _p(r_in), _p(r_out), _stream(stream)))


def fss_rescale_key_bytes(shift_bits: int, lookup_bits: int, n_elems: int) -> int:
    out = C.c_size_t()
    _check(lib.fss_rescale_key_bytes(shift_bits, lookup_bits, n_elems, C.byref(out)))
    return out.value


def fss_rescale_keygen(shift_bits, lookup_bits, seed, n_elems, r_in, key0, key1, r_out, stream=None):
    _check(lib.fss_rescale_keygen(shift_bits, lookup_bits, seed_bytes(seed), n_elems, _p(r_in), _p(key0),
                                  _p(key1), _p(r_out), _stream(stream)))


def fss_rescale_eval(party, keys, yhat, n, z, stream=None):
    _check(lib.fss_rescale_eval(party, _p(keys), _p(yhat), n, _p(z), _stream(stream)))


def fss_lit_keygen(spec, n_bits, frac_bits, seed, n_elems, key0, key1, r_in, r_out, stream=None):
    _check(lib.fss_lit_keygen(spec.handle, n_bits, frac_bits, seed_bytes(seed), n_elems, _p(key0), _p(key1),
                              _p(r_in), _p(r_out), _stream(stream)))


def fss_lit_eval(party, keys, xhat, n, coef, x_share, stream=None):
    _check(lib.fss_lit_eval(party, _p(keys), _p(xhat), n, _p(coef), _p(x_share), _stream(stream)))


def fss_triples(seed, n, step, a0, b0, c0, a1, b1, c1, stream=None):
    _check(lib.fss_triples(seed_bytes(seed), n, step, _p(a0), _p(b0), _p(c0), _p(a1), _p(b1), _p(c1),
                           _stream(stream)))


def fss_beaver_mask(u, v, a, b, n, d, e, stream=None):
    _check(lib.fss_beaver_mask(_p(u), _p(v), _p(a), _p(b), n, _p(d), _p(e), _stream(stream)))


def fss_beaver_mul(party, d, e, a, b, c, add, n, z, stream=None):
    _check(lib.fss_beaver_mul(party, _p(d), _p(e), _p(a), _p(b), _p(c), _p(add), n, _p(z), _stream(stream)))


def fss_and_triples(seed, words, step, a0, b0, c0, a1, b1, c1, stream=None):
    _check(lib.fss_and_triples(seed_bytes(seed), words, step, _p(a0), _p(b0), _p(c0), _p(a1), _p(b1), _p(c1),
                               _stream(stream)))


def fss_xor_mask(x, a, y, b, words, d, e, stream=None):
    _check(lib.fss_xor_mask(_p(x), _p(a), _p(y), _p(b), words, _p(d), _p(e), _stream(stream)))


def fss_xopen(s0, s1, words, out, stream=None):
    _check(lib.fss_xopen(_p(s0), _p(s1), words, _p(out), _stream(stream)))


def fss_and(party, d, e, a, b, c, words, z, stream=None):
    _check(lib.fss_and(party, _p(d), _p(e), _p(a), _p(b), _p(c), words, _p(z), _stream(stream)))


def fss_b2a_rand(seed, n, step, t0, t1, T0, T1, stream=None):
    _check(lib.fss_b2a_rand(seed_bytes(seed), n, step, _p(t0), _p(t1), _p(T0), _p(T1), _stream(stream)))


def fss_b2a(party, c, T, n, out, stream=None):
    _check(lib.fss_b2a(party, _p(c), _p(T), n, _p(out), _stream(stream)))


def fss_open(y0, y1, n, yhat, stream=None):
    _check(lib.fss_open(_p(y0), _p(y1), n, _p(yhat), _stream(stream)))


def fss_mask_input(x, r_in, n, xhat, stream=None):
    _check(lib.fss_mask_input(_p(x), _p(r_in), n, _p(xhat), _stream(stream)))


def fss_eval(party, keys, xhat, n, y, zbits, stream=None):
    _check(lib.fss_eval(party, _p(keys), _p(xhat), n, _p(y), _p(zbits), _stream(stream)))


def fss_eval_pred(party, keys, xhat, n, zbits, stream=None):
    _check(lib.fss_eval_pred(party, _p(keys), _p(xhat), n, _p(zbits), _stream(stream)))


def fss_eval_coeff(party, keys, xhat, n, y, stream=None):
    _check(lib.fss_eval_coeff(party, _p(keys), _p(xhat), n, _p(y), _stream(stream)))


def fss_status(stream=None) -> int:
    code = C.c_int32()
    _check(lib.fss_status(_stream(stream), C.byref(code)))
    return code.value


def work_items(items) -> C.Array:
    """items: iterable of (party, keys, xhat, y, zbits, n_elems) with tensors or addresses."""
    items = list(items)
    arr = (WorkItem * max(len(items), 1))()
    for i, (party, keys, xhat, y, z, n) in enumerate(items):
        arr[i] = WorkItem(party, 0, _p(keys), _p(xhat), _p(y), _p(z), n)
    return arr, len(items)


def fss_eval_batch(party, items, stream=None):
    """items: iterable of (party, keys, xhat, y, zbits, n_elems); party 0, 1 or PARTY_ANY."""
    arr, n = work_items(items)
    _check(lib.fss_eval_batch(party, arr, n, _stream(stream)))


def fss_eval_batch_noalloc(party, items, stream=None):
    """fss_eval_batch without device allocation (fixed work-list array)."""
    arr, n = work_items(items)
    _check(lib.fss_eval_batch_noalloc(party, arr, n, _stream(stream)))


NOALLOC_MAX_ITEMS, NOALLOC_MAX_UNITS = 1024, 491520


class Plan:
    """fss_plan: a work-list evaluated by one persistent fused launch."""

    def __init__(self, items, tune: Tune | None = None):
        arr, n = work_items(items)
        h = C.c_void_p()
        _check(lib.fss_plan_create(arr, n, C.byref(tune) if tune is not None else None, C.byref(h)))
        self.handle = h

    def launch(self, stream=None):
        _check(lib.fss_plan_launch(self.handle, _stream(stream)))

    def aes_blocks(self) -> float:
        return lib.fss_plan_aes_blocks(self.handle)

    def table_lookups(self) -> float:
        return lib.fss_plan_table_lookups(self.handle)

    def parts(self) -> int:
        return lib.fss_plan_parts(self.handle)

    def config(self) -> dict:
        t, g = Tune(), C.c_int32()
        _check(lib.fss_plan_config(self.handle, C.byref(t), C.byref(g)))
        return {"aes_variant": t.aes_variant, "block_threads": t.block_threads,
                "blocks_per_cu": t.blocks_per_cu, "order": t.order, "grid": g.value,
                "parts": t.parts, "pred_unit": t.pred_unit, "lanes": t.lanes}

    def free(self, _free=lib.fss_plan_free):
        if self.handle is not None and self.handle.value:
            _free(self.handle)
        self.handle = None

    def __del__(self):
        if getattr(self, "handle", None) is not None:
            self.free()


class Graph:
    """fss_graph: the launches of several plans captured into one HIP graph."""

    def __init__(self, plans):
        plans = list(plans)
        arr = (C.c_void_p * max(len(plans), 1))(*[p.handle.value for p in plans])
        h = C.c_void_p()
        _check(lib.fss_graph_capture(arr, len(plans), C.byref(h)))
        self.handle = h
        self._plans = plans

    def launch(self, stream=None):
        _check(lib.fss_graph_launch(self.handle, _stream(stream)))

    def free(self, _free=lib.fss_graph_free):
        if self.handle is not None and self.handle.value:
            _free(self.handle)
        self.handle = None

    def __del__(self):
        if getattr(self, "handle", None) is not None:
            self.free()


def fss_autotune(items, cache_path: str | None = None) -> Tune:
    arr, n = work_items(items)
    best = Tune()
    _check(lib.fss_autotune(arr, n, cache_path.encode() if cache_path else None, C.byref(best)))
    return best


def aes_variants() -> int:
    return lib.fss_aes_variants()


def version() -> str:
    return lib.fss_version().decode()
