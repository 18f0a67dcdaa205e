"""Decoder of the library's key-buffer format, written from its documentation
(header struct and tile layout in paper_2606_09551_amd/csrc/fss_common.hpp),
so tests can compare GPU-generated keys with the oracle's field by field."""
import numpy as np

HEADER_BYTES = 16384
TILE = 64
MAXA, MAXM, MAXP = 16, 64, 4

HDR = np.dtype([
    ("magic", "<u4"), ("version", "<u4"), ("party", "<u4"), ("layout", "<u4"),
    ("n", "<u4"), ("f", "<u4"), ("m", "<u4"), ("d", "<u4"), ("p", "<u4"), ("T", "<u4"),
    ("ell", "<u4"), ("F_out", "<u4"), ("n_prim", "<u4"), ("n_views", "<u4"), ("kmax", "<u4"),
    ("top_depth", "<u4"), ("lookup_r", "<u4"), ("top_blocks", "<u4"),
    ("lookup_c", "<u4"), ("is_int", "<u4"),
    ("kind", "<u4"), ("shift", "<u4"), ("mask_from_lookup", "<u4"), ("hdr_pad", "<u4"), ("n_elems", "<u8"), ("n_tiles", "<u8"), ("tile_bytes", "<u8"),
    ("spec_hash", "<u8"), ("negate", "<u8"), ("atom_k", "<u4", MAXA), ("atom_out", "<u4", MAXA),
    ("atom_rview", "<u4", MAXA), ("atom_c", "<u8", MAXA), ("atom_off", "<u8", MAXA),
    ("off_w", "<u8"), ("off_croot", "<u8"), ("off_crec", "<u8"), ("rec_bytes", "<u8"),
    ("off_crho", "<u8"), ("off_crout", "<u8"), ("off_tk0", "<u8"), ("off_tk1", "<u8"),
    ("off_seen", "<u8"), ("off_sentinel", "<u8"),
    ("lit_M", "<u4"), ("lit_pad", "<u4"), ("off_lrin", "<u8"), ("off_lbase", "<u8"), ("dcf_bytes", "<u8"),
    ("lcoef", "<u8", (MAXM, MAXP)),
    ("aprime", "<u8", MAXM + 1), ("tab", "<u8", (MAXM, MAXP, MAXP)), ("tabv", "<u8", (MAXP, MAXP)),
])


def header(buf: np.ndarray):
    return np.frombuffer(buf[: HDR.itemsize].tobytes(), dtype=HDR)[0]


class KeyView:
    def __init__(self, buf: np.ndarray):
        self.buf = buf
        self.h = header(buf)

    def _u64(self, off: int) -> int:
        return int(np.frombuffer(self.buf[off:off + 8].tobytes(), dtype="<u8")[0])

    def _blk(self, off: int):
        return self._u64(off), self._u64(off + 8)

    def tile_base(self, e: int) -> int:
        return HEADER_BYTES + (e // TILE) * int(self.h["tile_bytes"])

    def atom(self, e: int, t: int) -> dict:
        """A comparison atom of width k: its tree has k - min(7, k) levels,
        then the 16-byte leaf correction (after the value-correction bits)."""
        lane, k = e % TILE, int(self.h["atom_k"][t])
        lev = k - min(7, k)
        base = self.tile_base(e) + int(self.h["atom_off"][t])
        root = self._blk(base + lane * 16)
        cws = [self._blk(base + TILE * 16 + (i * TILE + lane) * 16) for i in range(lev)]
        vb = self._u64(base + TILE * 16 * (1 + lev) + lane * 8)
        leaf = self._blk(base + TILE * 16 * (1 + lev) + TILE * 8 + lane * 16)
        return {"root": root, "scw": [(lo & ~3, hi) for lo, hi in cws],
                "tl": [lo & 1 for lo, _ in cws], "tr": [(lo >> 1) & 1 for lo, _ in cws],
                "vcw": [(vb >> i) & 1 for i in range(lev)], "leaf": leaf}

    def coeff(self, e: int) -> dict:
        """The lookup DCF: L = ceil(n / r) levels of 2^r children; child c of
        level i has a record rec[i][c][lane] of 16 + 8p bytes: its seed
        correction (bit 0 = control-bit correction), then its p value corrections."""
        h, lane = self.h, e % TILE
        n, p, r = int(h["n"]), int(h["p"]), int(h["lookup_r"])
        L, C = -(-n // r), 1 << r
        rec = 16 + 8 * p
        assert int(h["rec_bytes"]) == rec
        tb = self.tile_base(e)
        root = self._blk(tb + int(h["off_croot"]) + lane * 16)
        recs = [[tb + int(h["off_crec"]) + ((i * C + c) * TILE + lane) * rec for c in range(C)] for i in range(L)]
        cws = [[self._blk(r) for r in lv] for lv in recs]
        vcw = [[[self._u64(r + 16 + 8 * q) for q in range(p)] for r in lv] for lv in recs]
        rho = [self._u64(tb + int(h["off_crho"]) + (q * TILE + lane) * 8) for q in range(p)]
        rout = self._u64(tb + int(h["off_crout"]) + lane * 8)
        w = self._u64(tb + int(h["off_w"]) + lane * 8)
        return {"root": root, "scw": [[(lo & ~3, hi) for lo, hi in lv] for lv in cws],
                "tcw": [[lo & 1 for lo, _ in lv] for lv in cws],
                "vcw": vcw, "rho": rho, "rout": rout, "wshare": w}


def oracle_atom(K, t: int) -> dict:
    a = K.atom[t]
    lev = a.n - a.nu
    return {"root": (a.root.lo, a.root.hi), "scw": [(a.scw[i].lo, a.scw[i].hi) for i in range(lev)],
            "tl": [a.tl[i] for i in range(lev)], "tr": [a.tr[i] for i in range(lev)],
            "vcw": [int(a.vcw[i]) for i in range(lev)], "leaf": (a.leaf.lo, a.leaf.hi)}


def oracle_coeff(K) -> dict:
    c = K.coeff
    L, p, C = -(-c.n // c.r), c.p, 1 << c.r
    return {"root": (c.root.lo, c.root.hi),
            "scw": [[(c.scw[i][ch].lo, c.scw[i][ch].hi) for ch in range(C)] for i in range(L)],
            "tcw": [[c.tcw[i][ch] for ch in range(C)] for i in range(L)],
            "vcw": [[[int(c.vcw[i][ch][q]) for q in range(p)] for ch in range(C)] for i in range(L)],
            "rho": [int(K.rho[q]) for q in range(p)],
            "rout": int(K.rout), "wshare": int(K.wshare)}
