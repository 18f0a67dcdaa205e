// fss_aes_bs.hpp -- bitsliced AES-128 in 32-bit registers: the alternative to
// the local-memory T-tables, holding the whole cipher in VALU registers.
//
// A "pair" is two AES blocks as eight bit planes: bit p = 8c + 2r + b of plane
// i is bit i of state byte (row r, column c) of block b.  In this layout
// ShiftRows is a whole-byte rotation of each row's bits and the row rotations
// of MixColumns stay inside each byte.
//
// SubBytes inverts in GF(2^8) through the composite field GF((2^4)^2)
// (Rijmen 2000; Satoh, Morioka, Takano and Munetoh, ASIACRYPT 2001):
// GF(16) = GF(2)[z]/(z^4 + z + 1), GF(256)' = GF(16)[Y]/(Y^2 + Y + lambda),
// (a1 Y + a0)^-1 = (a1 d) Y + (a0 + a1) d with d = (lambda a1^2 + a1 a0 + a0^2)^-1.
// The isomorphism between the AES field and the composite field, and its
// inverse merged with the affine map, are 8x8 binary matrices derived at
// compile time (a root of the AES polynomial is searched in the composite
// field), so the circuit is linear map -> composite inversion -> linear map.
//
// Plain C++ (host and device), no intrinsics: the same code is checked on the
// host against the FIPS-197 known answers.
#pragma once
#include <stdint.h>

#ifdef __HIPCC__
#define FSS_BS_HD __host__ __device__ __forceinline__
#else
#define FSS_BS_HD inline
#endif

namespace fss {
namespace bs {

// ---- compile-time field arithmetic -----------------------------------------
constexpr uint8_t aes_mul(uint8_t a, uint8_t b) {
  uint8_t r = 0;
  for (int i = 0; i < 8; ++i) {
    if (b & 1) r ^= a;
    const bool hi = a & 0x80;
    a = (uint8_t)(a << 1);
    if (hi) a ^= 0x1b;
    b >>= 1;
  }
  return r;
}
constexpr uint8_t gf16_mul_c(uint8_t a, uint8_t b) {  // mod z^4 + z + 1
  uint8_t r = 0;
  for (int i = 0; i < 4; ++i) {
    if (b & 1) r ^= a;
    a = (uint8_t)(a << 1);
    if (a & 0x10) a ^= 0x13;
    b >>= 1;
  }
  return (uint8_t)(r & 0xf);
}
// (a1 Y + a0)(b1 Y + b0) with Y^2 = Y + lambda
constexpr uint8_t tower_mul(uint8_t a, uint8_t b, uint8_t lam) {
  const uint8_t a1 = a >> 4, a0 = a & 15, b1 = b >> 4, b0 = b & 15;
  const uint8_t h = gf16_mul_c(a1, b1);
  const uint8_t c1 = (uint8_t)(h ^ gf16_mul_c(a1, b0) ^ gf16_mul_c(a0, b1));
  const uint8_t c0 = (uint8_t)(gf16_mul_c(h, lam) ^ gf16_mul_c(a0, b0));
  return (uint8_t)((c1 << 4) | c0);
}

struct Iso {
  uint8_t lam;       // Y^2 + Y + lambda irreducible over GF(16)
  uint8_t m_in[8];   // m_in[t]: bit k set when composite bit t takes AES bit k
  uint8_t m_out[8];  // m_out[k]: bit t set when the affine output bit k takes composite bit t
};

constexpr Iso make_iso() {
  Iso iso{};
  // lambda: no y in GF(16) with y^2 + y = lambda
  for (int l = 1; l < 16; ++l) {
    bool root = false;
    for (int y = 0; y < 16; ++y)
      if ((gf16_mul_c((uint8_t)y, (uint8_t)y) ^ y) == l) root = true;
    if (!root) {
      iso.lam = (uint8_t)l;
      break;
    }
  }
  // g: a root of x^8 + x^4 + x^3 + x + 1 in the composite field
  uint8_t g = 0;
  for (int c = 2; c < 256 && !g; ++c) {
    uint8_t pw[9] = {};
    pw[0] = 1;
    for (int k = 1; k <= 8; ++k) pw[k] = tower_mul(pw[k - 1], (uint8_t)c, iso.lam);
    if ((pw[8] ^ pw[4] ^ pw[3] ^ pw[1] ^ pw[0]) == 0) g = (uint8_t)c;
  }
  // phi(x^k) = g^k; phi(a) = XOR over the set bits k of a
  uint8_t gk[8] = {};
  gk[0] = 1;
  for (int k = 1; k < 8; ++k) gk[k] = tower_mul(gk[k - 1], g, iso.lam);
  for (int t = 0; t < 8; ++t) {
    uint8_t row = 0;
    for (int k = 0; k < 8; ++k)
      if ((gk[k] >> t) & 1) row |= (uint8_t)(1u << k);
    iso.m_in[t] = row;
  }
  // phi^-1 of each composite basis element, then the affine map's linear part
  uint8_t inv_e[8] = {};
  for (int a = 0; a < 256; ++a) {
    uint8_t v = 0;
    for (int k = 0; k < 8; ++k)
      if ((a >> k) & 1) v ^= gk[k];
    for (int t = 0; t < 8; ++t)
      if (v == (uint8_t)(1u << t)) inv_e[t] = (uint8_t)a;
  }
  for (int k = 0; k < 8; ++k) {
    uint8_t row = 0;
    for (int t = 0; t < 8; ++t) {
      const uint8_t a = inv_e[t];
      // affine linear part: bit k of a ^ rot(a,1) ^ rot(a,2) ^ rot(a,3) ^ rot(a,4)
      int bit = 0;
      for (int s = 0; s < 5; ++s) bit ^= (a >> ((k + 8 - s) % 8)) & 1;
      if (bit) row |= (uint8_t)(1u << t);
    }
    iso.m_out[k] = row;
  }
  return iso;
}

constexpr Iso kIso = make_iso();
static_assert(kIso.lam != 0, "no irreducible Y^2 + Y + lambda found");

// Bit planes of the fixed PRG key's round keys (the FIPS-197 C.1 key
// 00 01 .. 0f), in the pair layout with both blocks carrying the same key.
struct PrgPlanes { uint32_t p[11][8]; };

constexpr PrgPlanes make_prg_planes(const uint32_t (&rk)[44]) {
  PrgPlanes o{};
  for (int rd = 0; rd < 11; ++rd)
    for (int i = 0; i < 8; ++i) {
      uint32_t pl = 0;
      for (int c = 0; c < 4; ++c)
        for (int r = 0; r < 4; ++r) {
          const uint32_t bit = (rk[4 * rd + c] >> (8 * r + i)) & 1u;
          pl |= bit << (8 * c + 2 * r);
          pl |= bit << (8 * c + 2 * r + 1);
        }
      o.p[rd][i] = pl;
    }
  return o;
}

// ---- the pair layout -------------------------------------------------------
// 8x8 bit transpose of a 64-bit value (byte j = row j); Hacker's Delight 7-3.
FSS_BS_HD uint64_t transpose8(uint64_t x) {
  uint64_t t = (x ^ (x >> 7)) & 0x00AA00AA00AA00AAull;
  x = x ^ t ^ (t << 7);
  t = (x ^ (x >> 14)) & 0x0000CCCC0000CCCCull;
  x = x ^ t ^ (t << 14);
  t = (x ^ (x >> 28)) & 0x00000000F0F0F0F0ull;
  x = x ^ t ^ (t << 28);
  return x;
}

// Byte k of a 32-bit word.
FSS_BS_HD uint32_t byte_of(uint32_t w, int k) { return (w >> (8 * k)) & 0xffu; }

// Two blocks (words a[c], b[c], little-endian columns) -> eight planes.
FSS_BS_HD void pack(const uint32_t (&a)[4], const uint32_t (&b)[4], uint32_t (&pl)[8]) {
  uint64_t y[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    // byte 2r + blk of x holds byte r of block blk's column c
    const uint32_t lo = byte_of(a[c], 0) | (byte_of(b[c], 0) << 8) | (byte_of(a[c], 1) << 16) | (byte_of(b[c], 1) << 24);
    const uint32_t hi = byte_of(a[c], 2) | (byte_of(b[c], 2) << 8) | (byte_of(a[c], 3) << 16) | (byte_of(b[c], 3) << 24);
    y[c] = transpose8((uint64_t)lo | ((uint64_t)hi << 32));  // byte i: plane i's bits of column c
  }
#pragma unroll
  for (int i = 0; i < 8; ++i)
    pl[i] = (uint32_t)((y[0] >> (8 * i)) & 0xff) | ((uint32_t)((y[1] >> (8 * i)) & 0xff) << 8) |
            ((uint32_t)((y[2] >> (8 * i)) & 0xff) << 16) | ((uint32_t)((y[3] >> (8 * i)) & 0xff) << 24);
}

FSS_BS_HD void unpack(const uint32_t (&pl)[8], uint32_t (&a)[4], uint32_t (&b)[4]) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    uint64_t y = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) y |= (uint64_t)byte_of(pl[i], c) << (8 * i);
    const uint64_t x = transpose8(y);
    const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    a[c] = byte_of(lo, 0) | (byte_of(lo, 2) << 8) | (byte_of(hi, 0) << 16) | (byte_of(hi, 2) << 24);
    b[c] = byte_of(lo, 1) | (byte_of(lo, 3) << 8) | (byte_of(hi, 1) << 16) | (byte_of(hi, 3) << 24);
  }
}

// ---- GF(16) on four planes (bit k of a nibble = coefficient of z^k) --------
FSS_BS_HD void g16_mul(const uint32_t (&a)[4], const uint32_t (&b)[4], uint32_t (&o)[4]) {
  const uint32_t c0 = a[0] & b[0];
  const uint32_t c1 = (a[0] & b[1]) ^ (a[1] & b[0]);
  const uint32_t c2 = (a[0] & b[2]) ^ (a[1] & b[1]) ^ (a[2] & b[0]);
  const uint32_t c3 = (a[0] & b[3]) ^ (a[1] & b[2]) ^ (a[2] & b[1]) ^ (a[3] & b[0]);
  const uint32_t c4 = (a[1] & b[3]) ^ (a[2] & b[2]) ^ (a[3] & b[1]);
  const uint32_t c5 = (a[2] & b[3]) ^ (a[3] & b[2]);
  const uint32_t c6 = a[3] & b[3];
  // z^4 = z + 1, z^5 = z^2 + z, z^6 = z^3 + z^2
  o[0] = c0 ^ c4;
  o[1] = c1 ^ c4 ^ c5;
  o[2] = c2 ^ c5 ^ c6;
  o[3] = c3 ^ c6;
}
// a^2 = a0 + a1 z^2 + a2 z^4 + a3 z^6
FSS_BS_HD void g16_sq(const uint32_t (&a)[4], uint32_t (&o)[4]) {
  o[0] = a[0] ^ a[2];
  o[1] = a[2];
  o[2] = a[1] ^ a[3];
  o[3] = a[3];
}
// multiplication by the constant lambda (a linear map)
FSS_BS_HD void g16_mul_lam(const uint32_t (&a)[4], uint32_t (&o)[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    uint32_t v = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if ((gf16_mul_c((uint8_t)(1u << j), kIso.lam) >> k) & 1) v ^= a[j];
    o[k] = v;
  }
}

// ---- the round functions on a pair ------------------------------------------
FSS_BS_HD void sub_bytes(uint32_t (&pl)[8]) {
  uint32_t t[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {  // AES basis -> composite basis
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if ((kIso.m_in[i] >> k) & 1) v ^= pl[k];
    t[i] = v;
  }
  const uint32_t a0[4] = {t[0], t[1], t[2], t[3]}, a1[4] = {t[4], t[5], t[6], t[7]};
  uint32_t s1[4], ls1[4], s0[4], m[4], d[4], d2[4], d4[4], d8[4], d12[4], di[4];
  g16_sq(a1, s1);
  g16_mul_lam(s1, ls1);
  g16_sq(a0, s0);
  g16_mul(a1, a0, m);
#pragma unroll
  for (int k = 0; k < 4; ++k) d[k] = ls1[k] ^ m[k] ^ s0[k];
  // d^-1 = d^14 = d^8 d^4 d^2 (0 maps to 0)
  g16_sq(d, d2);
  g16_sq(d2, d4);
  g16_sq(d4, d8);
  g16_mul(d8, d4, d12);
  g16_mul(d12, d2, di);
  uint32_t h[4], l[4], s[4];
  g16_mul(a1, di, h);
#pragma unroll
  for (int k = 0; k < 4; ++k) s[k] = a0[k] ^ a1[k];
  g16_mul(s, di, l);
  const uint32_t inv[8] = {l[0], l[1], l[2], l[3], h[0], h[1], h[2], h[3]};
#pragma unroll
  for (int k = 0; k < 8; ++k) {  // composite basis -> AES basis, affine map, + 0x63
    uint32_t v = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if ((kIso.m_out[k] >> j) & 1) v ^= inv[j];
    pl[k] = ((0x63u >> k) & 1u) ? ~v : v;
  }
}

FSS_BS_HD uint32_t rotr32(uint32_t x, int n) { return (x >> n) | (x << (32 - n)); }

// Row r of column c moves to column c - r: its bits rotate down by 8 r.
FSS_BS_HD void shift_rows(uint32_t (&pl)[8]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const uint32_t x = pl[i];
    pl[i] = (x & 0x03030303u) | (rotr32(x, 8) & 0x0C0C0C0Cu) | (rotr32(x, 16) & 0x30303030u) |
            (rotr32(x, 24) & 0xC0C0C0C0u);
  }
}

// Row r takes row r + 1 (mod 4) of the same column: two bits down in each byte.
FSS_BS_HD uint32_t rot_row1(uint32_t x) { return ((x >> 2) & 0x3F3F3F3Fu) | ((x << 6) & 0xC0C0C0C0u); }
FSS_BS_HD uint32_t rot_row2(uint32_t x) { return ((x >> 4) & 0x0F0F0F0Fu) | ((x << 4) & 0xF0F0F0F0u); }

// out_r = 2 a_r + 3 a_{r+1} + a_{r+2} + a_{r+3} = 2 t + a_{r+1} + t_{r+2},
// t = a + a_{r+1}; doubling moves plane i to i + 1 and folds plane 7 into
// planes 0, 1, 3, 4 (the polynomial 0x11b).
FSS_BS_HD void mix_columns(uint32_t (&pl)[8]) {
  uint32_t r1[8], t[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    r1[i] = rot_row1(pl[i]);
    t[i] = pl[i] ^ r1[i];
  }
  const uint32_t x7 = t[7];
  const uint32_t dbl[8] = {x7, t[0] ^ x7, t[1], t[2] ^ x7, t[3] ^ x7, t[4], t[5], t[6]};
#pragma unroll
  for (int i = 0; i < 8; ++i) pl[i] = dbl[i] ^ r1[i] ^ rot_row2(t[i]);
}

// AES-128 of a pair under the fixed PRG key (round-key planes `rk`).
FSS_BS_HD void encrypt_pair(const PrgPlanes& rk, uint32_t (&pl)[8]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) pl[i] ^= rk.p[0][i];
#pragma unroll 1
  for (int rd = 1; rd < 10; ++rd) {
    sub_bytes(pl);
    shift_rows(pl);
    mix_columns(pl);
#pragma unroll
    for (int i = 0; i < 8; ++i) pl[i] ^= rk.p[rd][i];
  }
  sub_bytes(pl);
  shift_rows(pl);
#pragma unroll
  for (int i = 0; i < 8; ++i) pl[i] ^= rk.p[10][i];
}

}  // namespace bs
}  // namespace fss
