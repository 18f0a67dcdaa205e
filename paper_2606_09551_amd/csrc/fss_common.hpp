// fss_common.hpp -- definitions shared by the library's host code and kernels:
// compile-time AES-128 tables, the key-buffer header and the tile layout.
#pragma once
#include <stddef.h>
#include <stdint.h>

#ifdef __HIPCC__
#define FSS_HD __host__ __device__
#else
#define FSS_HD
#endif

namespace fss {

// ---------------------------------------------------------------------------
// AES-128 tables, built at compile time.
// S-box: inverse in GF(2^8) via log/antilog tables over the generator 0x03,
// then the FIPS-197 affine map.  Te0 packs one MixColumns column per S-box
// output as a little-endian word: rows (2S, S, S, 3S) in bytes 0..3.
// ---------------------------------------------------------------------------
struct AesConst {
  uint8_t sbox[256];
  uint32_t te0[256];
  uint32_t prg_rk[44];  // round keys of the fixed PRG key 00 01 .. 0f
};

constexpr uint8_t gf_x2(uint8_t a) { return (uint8_t)((a << 1) ^ ((a & 0x80) ? 0x1b : 0)); }

constexpr void expand_key(const uint8_t* sbox, const uint8_t key[16], uint32_t w[44]) {
  for (int i = 0; i < 4; ++i)
    w[i] = (uint32_t)key[4 * i] | ((uint32_t)key[4 * i + 1] << 8) |
           ((uint32_t)key[4 * i + 2] << 16) | ((uint32_t)key[4 * i + 3] << 24);
  uint8_t rc = 1;
  for (int i = 4; i < 44; ++i) {
    uint32_t t = w[i - 1];
    if ((i & 3) == 0) {
      t = (t >> 8) | (t << 24);  // RotWord on a little-endian word
      t = (uint32_t)sbox[t & 0xff] | ((uint32_t)sbox[(t >> 8) & 0xff] << 8) |
          ((uint32_t)sbox[(t >> 16) & 0xff] << 16) | ((uint32_t)sbox[t >> 24] << 24);
      t ^= rc;
      rc = gf_x2(rc);
    }
    w[i] = w[i - 4] ^ t;
  }
}

constexpr AesConst make_aes_const() {
  AesConst c{};
  uint8_t ex[256] = {}, lg[256] = {};
  uint8_t v = 1;
  for (int i = 0; i < 255; ++i) {
    ex[i] = v;
    lg[v] = (uint8_t)i;
    v = (uint8_t)(v ^ gf_x2(v));  // multiply by 0x03
  }
  for (int x = 0; x < 256; ++x) {
    uint8_t inv = x ? ex[(255 - lg[x]) % 255] : 0;
    uint8_t s = inv, r = inv;
    for (int k = 0; k < 4; ++k) {
      r = (uint8_t)((r << 1) | (r >> 7));
      s ^= r;
    }
    c.sbox[x] = (uint8_t)(s ^ 0x63);
  }
  for (int x = 0; x < 256; ++x) {
    uint8_t s = c.sbox[x], s2 = gf_x2(s), s3 = (uint8_t)(s2 ^ s);
    c.te0[x] = (uint32_t)s2 | ((uint32_t)s << 8) | ((uint32_t)s << 16) | ((uint32_t)s3 << 24);
  }
  uint8_t k[16] = {};
  for (int i = 0; i < 16; ++i) k[i] = (uint8_t)i;
  expand_key(c.sbox, k, c.prg_rk);
  return c;
}

constexpr AesConst kAes = make_aes_const();

// ---------------------------------------------------------------------------
// Key buffer: a header, then n_tiles tiles of 64 elements.  Inside a tile
// the fields are stored over the 64 lanes, so a wave that owns a tile reads
// each field with one coalesced access per level.
//   atom t : root[64] (16 B) | cw[k_t - nu_t][64] (16 B: seed corr., bit0 tL, bit1 tR)
//            | vbits[64] (u64: bit i = value corr. of level i)
//            | leaf[64] (16 B: the leaf correction, bit j for low input bits j)
//            The comparison tree stops nu = min(7, k) levels above the
//            leaves; a leaf seed s becomes the 128-bit vector H(s, 2).
//   wshare[64] (u64: bit j = this party's share of the carry of output j)
//   coeff  : root[64] | rec[L][2^r][64]
//            | rho[p][64] (share of rho) | rout[64] (share of r_out)
//   seen[64] (u64: the x-hat an element was first evaluated at) | used (u64:
//   bit lane set once that element has been evaluated; zeroed by keygen)
//   The lookup's vector DCF takes r input bits per level (2^r children), so
//   it has L = ceil(n / r) levels with corrections for each child.  A record
//   rec[i][c][lane] (16 + 8p bytes) holds child c's seed correction (bit 0 =
//   control-bit correction) followed by its p value corrections: the lanes of
//   a wave pick different children, and a lane's child is one contiguous
//   record, so a level's load touches fewer cache lines than separate seed and
//   value arrays would.
// ---------------------------------------------------------------------------
constexpr uint32_t kMagic = 0x4B535346u;  // "FSSK"
constexpr uint32_t kVersion = 10;
constexpr uint32_t kGateOperator = 0, kGateRescale = 1, kGateLiteral = 2;
// atom_rview of a threshold atom whose view is the lookup's view (k = n,
// shift lookup_c): its mask query 1[v < r_n] is the lookup DCF's first output
// at v reduced mod 2, carried in bit 31 of the call-1 atom word.
constexpr uint32_t kRviewLookup = 31;
constexpr int kTile = 64;
constexpr int kMaxAtoms = 16;
constexpr int kMaxM = 64;
constexpr int kMaxP = 4;
constexpr int kDefaultLookupR = 3;  // input bits per lookup-DCF level unless a spec sets it
constexpr int kMaxTopBlocks = 4;    // top walks shared by the lookup points
constexpr uint64_t kHeaderBytes = 16384;

struct KeyHeader {
  uint32_t magic, version, party, layout;
  uint32_t n, f, m, d, p, T, ell, F_out;
  uint32_t n_prim, n_views, kmax, top_depth;  // top_depth: shared lookup-DCF levels of the lookup points
  uint32_t lookup_r;                       // input bits per lookup-DCF level (2, 3 or 4)
  uint32_t top_blocks;                     // aligned blocks of lookup points walked through the shared levels (2..4)
  uint32_t lookup_c;                       // view shift of call 2: v = (xhat + lookup_c) mod 2^n
  uint32_t is_int;                         // 1: integer spec over canonical representatives
  uint32_t kind;                           // kGateOperator, kGateRescale or kGateLiteral
  uint32_t shift;                          // rescaling gate: bits shifted out (its DCF's domain, = n)
  uint32_t mask_from_lookup;               // 1: a threshold atom's mask query is the lookup's own
                                           // comparison (atom_rview = kRviewLookup)
  uint32_t hdr_pad;
  uint64_t n_elems, n_tiles, tile_bytes, spec_hash;
  uint64_t negate;                         // bit j: public flip of output j (party 0 applies it)
  uint32_t atom_k[kMaxAtoms];
  uint32_t atom_out[kMaxAtoms];            // theta atoms: output bit
  uint32_t atom_rview[kMaxAtoms];          // theta atoms: index of their view's mask atom
  uint64_t atom_c[kMaxAtoms];              // view shift
  uint64_t atom_off[kMaxAtoms];            // byte offset of the atom section in a tile
  uint64_t off_w, off_croot, off_crec, rec_bytes, off_crho, off_crout;  // rec_bytes = 16 + 8 p
  uint64_t off_tk0, off_tk1;               // rescaling gate: shares of its two constants
  uint64_t off_seen, off_sentinel;         // one-time use: x-hat each element was first evaluated at
                                           // (the tile's sentinel until then), the sentinel
  // literal lookup: intervals after padding, the r_in shares and the shares
  // of the last interval's payload; DCF j (1 .. lit_M - 1) at off_croot +
  // (j - 1) dcf_bytes, its records 64 x 16 bytes after its roots
  uint32_t lit_M, lit_pad;
  uint64_t off_lrin, off_lbase, dcf_bytes;
  uint64_t lcoef[kMaxM][kMaxP];            // literal lookup: ring coefficients of each piece
  uint64_t aprime[kMaxM + 1];              // offset-binary boundaries
  // Combination table: q_j = sum_i sum_k tab[i][j][k] * G_i[k] with
  // G_0 = rho share, G_i = g_i (i >= 1); see the lookup kernel.
  uint64_t tab[kMaxM][kMaxP][kMaxP];
  uint64_t tabv[kMaxP][kMaxP];             // sum_{i>=1} tab_i = A_0 - A_{m-1}
};
static_assert(sizeof(KeyHeader) <= kHeaderBytes, "header too large");

// Low input bits a comparison atom of width k resolves at its leaves.
constexpr int kLeafBits = 7;
FSS_HD constexpr int atom_leaf_bits(int k) { return k < kLeafBits ? k : kLeafBits; }

struct Layout {
  uint64_t atom_off[kMaxAtoms];
  uint64_t off_w, off_croot, off_crec, rec_bytes, off_crho, off_crout;
  uint64_t off_seen, off_sentinel;
  uint64_t off_lrin, off_lbase, dcf_bytes;
  uint64_t tile_bytes;
};

FSS_HD inline Layout make_layout(int T, const uint32_t* atom_k, int n, int p, int r) {
  Layout L{};
  uint64_t o = 0;
  for (int t = 0; t < T; ++t) {
    L.atom_off[t] = o;
    const int levels = (int)atom_k[t] - atom_leaf_bits((int)atom_k[t]);
    o += (uint64_t)kTile * 16 * (1 + levels) + (uint64_t)kTile * 8 + (uint64_t)kTile * 16;
  }
  L.off_w = o;     o += kTile * 8;
  L.off_croot = o; o += kTile * 16;
  const uint64_t levels = (uint64_t)(n + r - 1) / r;  // 2^r children per level
  L.rec_bytes = 16 + 8 * (uint64_t)p;       // seed correction, then p value corrections
  L.off_crec = o;  o += levels * ((uint64_t)1 << r) * kTile * L.rec_bytes;
  L.off_crho = o;  o += (uint64_t)p * kTile * 8;
  L.off_crout = o; o += kTile * 8;
  L.off_seen = o;  o += kTile * 8;
  L.off_sentinel = o;  o += 8;
  L.tile_bytes = (o + 255) & ~(uint64_t)255;
  return L;
}

// A rescaling gate's tile: its DCF (p = 1) over `shift` bits with 2^r children
// per level -- root[64] | rec[L][2^r][64] (24 B: seed correction, value
// correction) -- then the shares of k0 = r_out - (r_in >> s) and
// k1 = 2^(64-s) MSB(r_in), 8 B per lane each, and the one-time record.
FSS_HD inline Layout make_rescale_layout(int shift, int r) {
  Layout L{};
  uint64_t o = 0;
  L.off_croot = o; o += kTile * 16;
  const uint64_t levels = (uint64_t)(shift + r - 1) / r;
  L.rec_bytes = 24;
  L.off_crec = o;  o += levels * ((uint64_t)1 << r) * kTile * L.rec_bytes;
  L.off_crho = o;  o += kTile * 8;   // k0 shares
  L.off_crout = o; o += kTile * 8;   // k1 shares
  L.off_seen = o;  o += kTile * 8;
  L.off_sentinel = o;  o += 8;
  L.tile_bytes = (o + 255) & ~(uint64_t)255;
  return L;
}

// A literal lookup's tile (M intervals after padding): r_in shares[64],
// r_out shares[64], shares of the last interval's payload [p][64], then
// M - 1 vector DCFs of 2^r children per level, each root[64] |
// rec[L][2^r][64] (16 + 8p bytes), then the one-time record.
FSS_HD inline Layout make_literal_layout(int n, int p, int r, int M) {
  Layout L{};
  uint64_t o = 0;
  L.off_lrin = o;  o += kTile * 8;
  L.off_crout = o; o += kTile * 8;
  L.off_lbase = o; o += (uint64_t)p * kTile * 8;
  const uint64_t levels = (uint64_t)(n + r - 1) / r;
  L.rec_bytes = 16 + 8 * (uint64_t)p;
  L.dcf_bytes = (uint64_t)kTile * 16 + levels * ((uint64_t)1 << r) * kTile * L.rec_bytes;
  L.off_croot = o;
  L.off_crec = o + (uint64_t)kTile * 16;
  o += (uint64_t)(M - 1) * L.dcf_bytes;
  L.off_seen = o;  o += kTile * 8;
  L.off_sentinel = o;  o += 8;
  L.tile_bytes = (o + 255) & ~(uint64_t)255;
  return L;
}

// Device status codes (mirrors of FSS_E_*).
constexpr int kStatusShape = -4;
constexpr int kStatusParty = -5;
constexpr int kStatusConsumed = -9;
// PRG purpose of a tile's one-time-record sentinel (the method's own purposes
// stay below 256).
constexpr uint32_t kPurposeSentinel = 0xffffu;

}  // namespace fss
