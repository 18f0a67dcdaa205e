"""Plain CPU oracle for the FuseFSS hot path (ctypes wrapper of fss_oracle.c).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code
with the GPU library; the only thing both sides consume is the seeded input
description in ``paper_2606_09551_amd.workloads`` (specs as real numbers and
plaintext inputs), which holds none of the method's arithmetic.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fss_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")

MAXN, MAXP, MAXM, MAXPRED, MAXT, MAXL = 32, 4, 64, 16, 16, 64
LT_SIGNED, LT_UNSIGNED, LOWBITS_LT, MSB_SHIFT = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/_build/liboracle.so."""
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                               "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Blk(C.Structure):
    _fields_ = [("lo", C.c_uint64), ("hi", C.c_uint64)]


class DcfKey(C.Structure):
    _fields_ = [("n", C.c_int32), ("p", C.c_int32), ("root", Blk), ("scw", Blk * MAXN),
                ("tl", C.c_uint8 * MAXN), ("tr", C.c_uint8 * MAXN),
                ("vcw", (C.c_uint64 * MAXP) * MAXN), ("fin", C.c_uint64 * MAXP)]


class DcfZKey(C.Structure):
    _fields_ = [("n", C.c_int32), ("nu", C.c_int32), ("root", Blk), ("scw", Blk * MAXN),
                ("tl", C.c_uint8 * MAXN), ("tr", C.c_uint8 * MAXN), ("vcw", C.c_uint8 * MAXN),
                ("leaf", Blk)]


MAXLR = (MAXN + 1) // 2  # lookup-DCF levels at r = 2
MAXC = 16                # children per level at r = 4


class DcfRKey(C.Structure):
    _fields_ = [("n", C.c_int32), ("p", C.c_int32), ("r", C.c_int32), ("root", Blk),
                ("scw", (Blk * MAXC) * MAXLR), ("tcw", (C.c_uint8 * MAXC) * MAXLR),
                ("vcw", ((C.c_uint64 * MAXP) * MAXC) * MAXLR)]


class ElemKey(C.Structure):
    _fields_ = [("atom", DcfZKey * MAXT), ("wshare", C.c_uint64), ("coeff", DcfRKey),
                ("rho", C.c_uint64 * MAXP), ("rout", C.c_uint64)]


class Interval(C.Structure):
    _fields_ = [("lo", C.c_double), ("hi", C.c_double)]


class Piece(C.Structure):
    _fields_ = [("degree", C.c_int32), ("coef", C.c_double * 4)]


class Pred(C.Structure):
    _fields_ = [("kind", C.c_int32), ("negate", C.c_int32), ("out", C.c_int32),
                ("f_bits", C.c_int32), ("thr", C.c_double), ("gamma", C.c_int64),
                ("c", C.c_int64)]


class Spec(C.Structure):
    _fields_ = [("n", C.c_int32), ("f", C.c_int32), ("m", C.c_int32), ("d", C.c_int32),
                ("p", C.c_int32), ("F_out", C.c_int32), ("ell", C.c_int32),
                ("alpha", C.c_int64 * (MAXM + 1)), ("aprime", C.c_uint64 * (MAXM + 1)),
                ("coef", (C.c_uint64 * MAXP) * MAXM),
                ("n_user", C.c_int32),
                ("u_kind", C.c_int32 * MAXPRED), ("u_out", C.c_int32 * MAXPRED),
                ("u_neg", C.c_int32 * MAXPRED), ("u_f", C.c_int32 * MAXPRED),
                ("u_beta", C.c_int64 * MAXPRED), ("u_c", C.c_uint64 * MAXPRED),
                ("n_prim", C.c_int32),
                ("prim_k", C.c_int32 * MAXPRED), ("prim_view", C.c_int32 * MAXPRED),
                ("prim_out", C.c_int32 * MAXPRED), ("prim_bprime", C.c_uint64 * MAXPRED),
                ("n_views", C.c_int32), ("view_k", C.c_int32 * MAXPRED),
                ("view_c", C.c_uint64 * MAXPRED), ("T", C.c_int32),
                ("negate", C.c_uint8 * MAXL), ("lookup_r", C.c_int32), ("is_int", C.c_int32),
                ("lookup_c", C.c_uint64), ("lookup_view", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(_LIB_PATH)
        u8p, u64p, i64p = C.POINTER(C.c_uint8), C.POINTER(C.c_uint64), C.POINTER(C.c_int64)
        L.orc_aes128_encrypt_key.argtypes = [u8p, u8p, u8p]
        L.orc_sbox.argtypes = [u8p]
        L.orc_prg.argtypes = [Blk, C.c_int]
        L.orc_prg.restype = Blk
        L.orc_seed_sched.argtypes = [u8p, C.c_void_p]
        L.orc_rand.argtypes = [C.c_void_p, C.c_uint64, C.c_int, C.c_int]
        L.orc_rand.restype = Blk
        L.orc_dcf_gen.argtypes = [C.c_int, C.c_int, C.c_uint64, u64p, Blk, Blk,
                                  C.POINTER(DcfKey), C.POINTER(DcfKey)]
        L.orc_dcf_eval.argtypes = [C.c_int, C.POINTER(DcfKey), C.c_uint64, u64p]
        L.orc_dcfz_gen.argtypes = [C.c_int, C.c_uint64, Blk, Blk, C.POINTER(DcfZKey), C.POINTER(DcfZKey)]
        L.orc_dcfz_eval.argtypes = [C.c_int, C.POINTER(DcfZKey), C.c_uint64]
        L.orc_dcfr_gen.argtypes = [C.c_int, C.c_int, C.c_int, C.c_uint64, u64p, Blk, Blk, C.POINTER(Blk),
                                   C.POINTER(DcfRKey), C.POINTER(DcfRKey)]
        L.orc_dcfr_eval.argtypes = [C.c_int, C.POINTER(DcfRKey), C.c_uint64, u64p]
        L.orc_spec_compile.argtypes = [C.POINTER(Interval), C.c_int32, C.POINTER(Piece),
                                       C.POINTER(Pred), C.c_int32, C.c_int32, C.c_int32,
                                       C.c_int32, C.POINTER(Spec)]
        L.orc_spec_compile_int.argtypes = [C.c_int32, C.c_int32, u64p, C.c_int32, u64p,
                                           C.POINTER(Pred), C.c_int32, C.POINTER(Spec)]
        L.orc_keygen_batch.argtypes = [C.POINTER(Spec), u8p, i64p, C.c_int64,
                                       C.POINTER(ElemKey), C.POINTER(ElemKey), u64p, u64p, C.c_int]
        L.orc_eval_batch.argtypes = [C.c_int, C.POINTER(Spec), C.POINTER(ElemKey), u64p,
                                     C.c_int64, u64p, u64p, C.c_int]
        L.orc_full_batch.argtypes = [C.POINTER(Spec), u8p, i64p, C.c_int64, i64p,
                                     u64p, u64p, u64p, u64p, u64p, u64p, C.c_int]
        L.orc_trunc_batch.argtypes = [C.c_int, C.c_int, u8p, i64p, C.c_int64, u64p, u64p, u64p, u64p, u64p,
                                      C.c_int]
        L.orc_plain_eval.argtypes = [C.POINTER(Spec), C.c_int64, u64p, u64p]
        L.orc_protocol3.argtypes = [C.c_int, u64p, C.c_int, C.c_uint64, u64p,
                                    C.POINTER(C.c_int32)]
        L.orc_lit_batch.argtypes = [C.POINTER(Spec), u8p, i64p, C.c_int64, i64p, u64p, u64p, u64p, u64p,
                                    u64p, u64p, C.c_int]
        for name in ("orc_triple", "orc_and_triple"):
            getattr(L, name).argtypes = [C.c_void_p, C.c_uint64, C.c_int, u64p, u64p, u64p]
        L.orc_b2a_rand.argtypes = [C.c_void_p, C.c_uint64, C.c_int, u64p, u64p]
        for name in ("orc_beaver_mul", "orc_and"):
            getattr(L, name).argtypes = [C.c_int] + [C.c_uint64] * 5
            getattr(L, name).restype = C.c_uint64
        L.orc_b2a.argtypes = [C.c_int, C.c_uint64, C.c_uint64]
        L.orc_b2a.restype = C.c_uint64
        for name, cls in (("orc_sizeof_elem_key", ElemKey), ("orc_sizeof_dcf_key", DcfKey),
                          ("orc_sizeof_dcfz_key", DcfZKey),
                          ("orc_sizeof_dcfr_key", DcfRKey), ("orc_sizeof_spec", Spec)):
            got = getattr(L, name)()
            if got != C.sizeof(cls):
                raise RuntimeError(f"oracle struct layout mismatch: {name} {got} != {C.sizeof(cls)}")
        _lib = L
    return _lib


def _u64p(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_uint64))


def _i64p(a: np.ndarray):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def seed_bytes(seed: int):
    """The dealer's 128-bit seed as the 16 little-endian bytes of its AES key."""
    return (C.c_uint8 * 16).from_buffer_copy(int(seed & (2**128 - 1)).to_bytes(16, "little"))


# ---- AES / PRG / randomness ------------------------------------------------

def aes128(key: bytes, block: bytes) -> bytes:
    k = (C.c_uint8 * 16).from_buffer_copy(key)
    i = (C.c_uint8 * 16).from_buffer_copy(block)
    o = (C.c_uint8 * 16)()
    lib().orc_aes128_encrypt_key(k, i, o)
    return bytes(o)


def sbox() -> bytes:
    o = (C.c_uint8 * 256)()
    lib().orc_sbox(o)
    return bytes(o)


def prg(lo: int, hi: int, j: int) -> tuple[int, int]:
    r = lib().orc_prg(Blk(lo, hi), j)
    return r.lo, r.hi


def rand(seed: int, e: int, purpose: int, ctr: int = 0) -> tuple[int, int]:
    ks = (C.c_uint8 * 176)()
    lib().orc_seed_sched(seed_bytes(seed), ks)
    r = lib().orc_rand(ks, e, purpose, ctr)
    return r.lo, r.hi


# ---- DCF ---------------------------------------------------------------------

def dcf_gen(n: int, p: int, alpha: int, beta, root0, root1):
    """p == 0: payload in Z_2 (beta one bit); else beta is a length-p list in Z_{2^64}."""
    b = (C.c_uint64 * MAXP)(*([int(v) & (2**64 - 1) for v in (beta if p else [beta])]))
    k0, k1 = DcfKey(), DcfKey()
    lib().orc_dcf_gen(n, p, alpha, b, Blk(*root0), Blk(*root1), C.byref(k0), C.byref(k1))
    return k0, k1


def dcf_eval(b: int, key: DcfKey, x: int):
    out = (C.c_uint64 * MAXP)()
    lib().orc_dcf_eval(b, C.byref(key), x, out)
    return out[0] if key.p == 0 else list(out[: key.p])


def dcfz_nu(n: int) -> int:
    """Low input bits the early-terminated Z_2 DCF resolves at its leaves."""
    return lib().orc_dcfz_nu(n)


def dcfz_gen(n: int, alpha: int, root0, root1):
    """Z_2 DCF for 1[x < alpha] with a 2^nu-bit leaf (early termination)."""
    k0, k1 = DcfZKey(), DcfZKey()
    lib().orc_dcfz_gen(n, alpha, Blk(*root0), Blk(*root1), C.byref(k0), C.byref(k1))
    return k0, k1


def dcfz_eval(b: int, key: DcfZKey, x: int) -> int:
    return lib().orc_dcfz_eval(b, C.byref(key), x)


def dcfr_gen(n: int, r: int, p: int, alpha: int, beta, root0, root1, keep_rand):
    """2^r children per level.  keep_rand: (ceil(n/r) * (1 + ceil(p/2))) (lo, hi)
    blocks, the on-path child's corrections level by level (the last level's unused)."""
    b = (C.c_uint64 * MAXP)(*([int(v) & (2**64 - 1) for v in (beta if p else [beta])]))
    kr = (Blk * max(1, len(keep_rand)))(*[Blk(lo, hi) for lo, hi in keep_rand])
    k0, k1 = DcfRKey(), DcfRKey()
    lib().orc_dcfr_gen(n, r, p, alpha, b, Blk(*root0), Blk(*root1), kr, C.byref(k0), C.byref(k1))
    return k0, k1


def dcfr_eval(b: int, key: DcfRKey, x: int):
    out = (C.c_uint64 * MAXP)()
    lib().orc_dcfr_eval(b, C.byref(key), x, out)
    return out[0] if key.p == 0 else list(out[: key.p])


# ---- specs -------------------------------------------------------------------

class SpecError(ValueError):
    pass


def compile_spec(desc, n_bits: int, frac_bits: int, lookup_r: int = 3) -> Spec:
    """desc: paper_2606_09551_amd.workloads.SpecDesc (real-valued spec);
    lookup_r: input bits per level of call 2's DCF (2, 3 or 4)."""
    m = len(desc.intervals)
    iv = (Interval * m)(*[Interval(lo, hi) for lo, hi in desc.intervals])
    pcs = (Piece * m)()
    for i, coefs in enumerate(desc.pieces):
        pcs[i].degree = len(coefs) - 1          # degree > 3 is rejected by the C side
        for l, c in enumerate(coefs[:4]):
            pcs[i].coef[l] = c
    np_ = len(desc.preds)
    prs = (Pred * max(np_, 1))()
    for j, q in enumerate(desc.preds):
        prs[j] = Pred(q.kind, int(q.negate), q.out, q.f_bits, q.thr, q.gamma, q.c)
    S = Spec()
    rc = lib().orc_spec_compile(iv, m, pcs, prs, np_, n_bits, frac_bits, desc.out_frac_bits,
                                C.byref(S))
    if rc != 0:
        raise SpecError(f"oracle rejected spec {getattr(desc, 'name', '?')}: rc={rc}")
    if lookup_r not in (2, 3, 4):
        raise SpecError(f"lookup_r must be 2, 3 or 4, got {lookup_r}")
    S.lookup_r = lookup_r
    return S


def compile_spec_int(n_bits: int, alpha, coef, preds=(), lookup_r: int = 3) -> Spec:
    """Integer spec of Definition "Operator specification": boundaries
    0 = alpha_0 < ... < alpha_m = 2^n over canonical representatives, coef[i] the
    ring coefficients of piece i (lowest first, all of one length d + 1), preds
    PredDesc with integer thresholds."""
    m = len(alpha) - 1
    d = len(coef[0]) - 1
    a = np.ascontiguousarray([int(v) for v in alpha], dtype=np.uint64)
    c = np.ascontiguousarray([int(v) & (2**64 - 1) for row in coef for v in row], dtype=np.uint64)
    np_ = len(preds)
    prs = (Pred * max(np_, 1))()
    for j, q in enumerate(preds):
        prs[j] = Pred(q.kind, int(q.negate), q.out, q.f_bits, q.thr, q.gamma, q.c)
    S = Spec()
    rc = lib().orc_spec_compile_int(n_bits, m, _u64p(a), d, _u64p(c), prs, np_, C.byref(S))
    if rc != 0:
        raise SpecError(f"oracle rejected integer spec: rc={rc}")
    if lookup_r not in (2, 3, 4):
        raise SpecError(f"lookup_r must be 2, 3 or 4, got {lookup_r}")
    S.lookup_r = lookup_r
    return S


def spec_tables(S: Spec) -> dict:
    """Integer tables of a compiled spec, for comparison with the library."""
    m, p = S.m, S.p
    return {
        "n": S.n, "f": S.f, "m": m, "d": S.d, "p": p, "F_out": S.F_out, "ell": S.ell, "T": S.T,
        "alpha": [S.alpha[i] for i in range(m + 1)],
        "aprime": [S.aprime[i] for i in range(m + 1)],
        "coef": [[S.coef[i][l] for l in range(p)] for i in range(m)],
        "atoms": ([(S.prim_k[t], S.view_c[S.prim_view[t]], 0) for t in range(S.n_prim)]
                  + [(S.view_k[v], S.view_c[v], 1) for v in range(S.n_views) if v != S.lookup_view]),
        "negate": [S.negate[j] for j in range(S.ell)],
    }


# ---- keygen / eval -----------------------------------------------------------

def keygen(S: Spec, seed: int, elems, threads: int = 0):
    elems = np.ascontiguousarray(elems, dtype=np.int64)
    cnt = len(elems)
    K0 = (ElemKey * max(cnt, 1))()
    K1 = (ElemKey * max(cnt, 1))()
    r_in = np.zeros(cnt, np.uint64)
    r_out = np.zeros(cnt, np.uint64)
    lib().orc_keygen_batch(C.byref(S), seed_bytes(seed), _i64p(elems), cnt, K0, K1, _u64p(r_in),
                           _u64p(r_out), threads)
    return K0, K1, r_in, r_out


def evaluate(b: int, S: Spec, K, xhat, threads: int = 0):
    xhat = np.ascontiguousarray(xhat, dtype=np.uint64)
    cnt = len(xhat)
    y = np.zeros(cnt, np.uint64)
    z = np.zeros(cnt, np.uint64)
    lib().orc_eval_batch(b, C.byref(S), K, _u64p(xhat), cnt, _u64p(y), _u64p(z), threads)
    return y, z


def full(S: Spec, seed: int, elems, x, threads: int = 0, masks: bool = False):
    """Dealer keygen + both parties' evaluation for the given element indices
    (no keys are stored, so any number of elements fits in memory).

    Returns (y0, y1, z0, z1, threads_used), or with masks=True
    (y0, y1, z0, z1, r_in, r_out, threads_used)."""
    elems = np.ascontiguousarray(elems, dtype=np.int64)
    x = np.ascontiguousarray(x, dtype=np.int64)
    cnt = len(elems)
    y0, y1, z0, z1, r_in, r_out = (np.zeros(cnt, np.uint64) for _ in range(6))
    used = lib().orc_full_batch(C.byref(S), seed_bytes(seed), _i64p(elems), cnt, _i64p(x), _u64p(y0),
                                _u64p(y1), _u64p(z0), _u64p(z1), _u64p(r_in), _u64p(r_out), threads)
    if masks:
        return y0, y1, z0, z1, r_in, r_out, used
    return y0, y1, z0, z1, used


def plain(S: Spec, x: int) -> tuple[int, int]:
    y, z = C.c_uint64(), C.c_uint64()
    lib().orc_plain_eval(C.byref(S), int(x), C.byref(y), C.byref(z))
    return y.value, z.value


def plain_many(S: Spec, xs):
    ys = np.zeros(len(xs), np.uint64)
    zs = np.zeros(len(xs), np.uint64)
    for i, x in enumerate(np.asarray(xs, dtype=np.int64)):
        ys[i], zs[i] = plain(S, int(x))
    return ys, zs


def protocol3(n: int, alpha, r: int):
    m = len(alpha) - 1
    a = np.ascontiguousarray(alpha, dtype=np.uint64)
    B = np.zeros(m + 3, np.uint64)
    ordv = (C.c_int32 * (m + 2))()
    M = lib().orc_protocol3(n, _u64p(a), m, r, _u64p(B), ordv)
    if M < 0:
        raise RuntimeError("protocol3 shape error")
    return [int(v) for v in B[: M + 1]], list(ordv[:M])


def hw_threads() -> int:
    return lib().orc_hw_threads()


def aes_blocks() -> int:
    """AES-128 blocks the batched drivers have encrypted so far in this process."""
    L = lib()
    L.orc_aes_blocks.restype = C.c_uint64
    return int(L.orc_aes_blocks())


# ---- rescaling gate ------------------------------------------------------------

def trunc(shift: int, seed: int, elems, r_in, yhat, lookup_r: int = 3, threads: int = 0):
    """ARS gate: keygen at the given input masks r_in and both parties'
    evaluation at the openings yhat.  Returns (z0, z1, r_out)."""
    elems = np.ascontiguousarray(elems, dtype=np.int64)
    r_in = np.ascontiguousarray(r_in, dtype=np.uint64)
    yhat = np.ascontiguousarray(yhat, dtype=np.uint64)
    cnt = len(elems)
    z0, z1, r_out = (np.zeros(cnt, np.uint64) for _ in range(3))
    rc = lib().orc_trunc_batch(shift, lookup_r, seed_bytes(seed), _i64p(elems), cnt, _u64p(r_in), _u64p(yhat),
                               _u64p(z0), _u64p(z1), _u64p(r_out), threads)
    if rc < 0:
        raise ValueError(f"oracle rejected the rescaling gate (shift={shift}, r={lookup_r})")
    return z0, z1, r_out


# ---- the paper's lookup + post-processing pipeline -----------------------------

def lit(S: Spec, seed: int, elems, x, threads: int = 0):
    """Literal interval lookup (one vector DCF per inner boundary of the
    translated partition), both parties' coefficient shares at
    xhat = x + r_in (the constant term's shares carry the r_out shares), then
    Horner's rule with Beaver multiplications.  Returns dict(c0, c1
    (count x p), y0, y1, r_in, r_out) with y0 + y1 = P(x) + r_out."""
    elems = np.ascontiguousarray(elems, dtype=np.int64)
    x = np.ascontiguousarray(x, dtype=np.int64)
    cnt, p = len(elems), S.p
    c0, c1 = np.zeros((cnt, p), np.uint64), np.zeros((cnt, p), np.uint64)
    y0, y1, r_in, r_out = (np.zeros(cnt, np.uint64) for _ in range(4))
    rc = lib().orc_lit_batch(C.byref(S), seed_bytes(seed), _i64p(elems), cnt, _i64p(x), _u64p(c0), _u64p(c1),
                             _u64p(y0), _u64p(y1), _u64p(r_in), _u64p(r_out), threads)
    if rc < 0:
        raise ValueError("oracle rejected the literal lookup")
    return dict(c0=c0, c1=c1, y0=y0, y1=y1, r_in=r_in, r_out=r_out)


def _sched(seed: int):
    ks = C.create_string_buffer(4096)
    lib().orc_seed_sched(seed_bytes(seed), ks)
    return ks


def _pairs(fn, seed: int, idx, step: int):
    ks = _sched(seed)
    a, b, c = (np.zeros(2, np.uint64) for _ in range(3))
    fn(ks, idx, step, _u64p(a), _u64p(b), _u64p(c))
    return a.copy(), b.copy(), c.copy()


def triple(seed: int, e: int, step: int):
    """Beaver triple of multiplication `step` of element e: (a, b, c) pairs of shares."""
    return _pairs(lib().orc_triple, seed, e, step)


def and_triple(seed: int, w: int, step: int):
    """AND triple of bit-word w: (a, b, c) pairs of XOR shares."""
    return _pairs(lib().orc_and_triple, seed, w, step)


def b2a_rand(seed: int, e: int, step: int):
    """(t bit XOR shares, T additive shares) of element e."""
    ks = _sched(seed)
    t, T = np.zeros(2, np.uint64), np.zeros(2, np.uint64)
    lib().orc_b2a_rand(ks, e, step, _u64p(t), _u64p(T))
    return t.copy(), T.copy()


def beaver_mul(party, d, e, a, b, c) -> int:
    return int(lib().orc_beaver_mul(party, d, e, a, b, c))


def and_gate(party, d, e, a, b, c) -> int:
    return int(lib().orc_and(party, d, e, a, b, c))


def b2a(party, c, T) -> int:
    return int(lib().orc_b2a(party, c, T))
