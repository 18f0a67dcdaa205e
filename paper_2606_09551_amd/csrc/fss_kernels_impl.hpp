// fss_kernels_impl.hpp -- gfx950 kernels of the FSS hot path, templated on
// the AES table layout; each fss_kernels_v<N>.hip instantiates one layout.
//
// Work mapping: one wave64 owns one 64-element key tile; lane = element.
// Every step of a DCF walk is integer work; the dominant cost is the
// fixed-key AES-128 of the GGM seed expansion, computed with T-tables held
// in LDS (no AES instructions exist on CDNA).  Key fields are read with one
// coalesced access per level per wave (structure-of-arrays tiles).
#pragma once
#include <hip/hip_runtime.h>

#include <utility>

#include "fss_aes_bs.hpp"
#include "fss_kernels.hpp"

namespace fss {

static __constant__ AesConst c_aes = kAes;

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ uint32_t rotl8n(uint32_t x, int n8) {
  return n8 == 0 ? x : ((x << n8) | (x >> (32 - n8)));
}
// Every key, input and output access goes through global-address-space
// pointers: pointers read from a work-list are otherwise generic, and generic
// (flat) loads also count against the LDS wait counter, serialising them with
// the T-table reads.
#define FSS_GLOBAL __attribute__((address_space(1)))
using GHdr = const FSS_GLOBAL KeyHeader*;
__device__ __forceinline__ GHdr ghdr(const void* p) { return (GHdr)p; }
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 ld16(const uint8_t* p) {
  const u32x4 v = *(const FSS_GLOBAL u32x4*)p;
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint64_t ld8(const uint8_t* p) { return *(const FSS_GLOBAL uint64_t*)p; }
__device__ __forceinline__ void st16(uint8_t* p, uint4 v) {
  u32x4 w;
  w.x = v.x; w.y = v.y; w.z = v.z; w.w = v.w;
  *(FSS_GLOBAL u32x4*)p = w;
}
__device__ __forceinline__ void st8(uint8_t* p, uint64_t v) { *(FSS_GLOBAL uint64_t*)p = v; }
__device__ __forceinline__ uint64_t ldg64(const uint64_t* p) { return *(const FSS_GLOBAL uint64_t*)p; }
__device__ __forceinline__ void stg64(uint64_t* p, uint64_t v) { *(FSS_GLOBAL uint64_t*)p = v; }
__device__ __forceinline__ uint64_t mk64(uint32_t lo, uint32_t hi) { return (uint64_t)lo | ((uint64_t)hi << 32); }
__device__ __forceinline__ void set_status(int* st, int code) { atomicCAS(st, 0, code); }

// ---------------------------------------------------------------------------
// T-table layouts in LDS.  get<TBL, B>(w) returns T_TBL[byte B of w], where
// T_t = rotl(Te0, 8t).  Variants trade LDS footprint against bank conflicts
// and VALU work; the autotuner picks one per work-list.
// ---------------------------------------------------------------------------
// Byte-permute selector placing byte B of src0 at result byte 1 and keeping
// bytes 0 and 2 of src1 (lane offset, table bank): one v_perm per address.
// v_perm_b32 numbers the bytes of {src0, src1} with src1 as bytes 0..3, so the
// result is (lane offset) | (table byte << 8) | (bank << 16): byte 0 < 128,
// byte 2 in {0, 1}, byte 3 = 0, which keeps every address inside the table.
template <int B>
__device__ __forceinline__ uint32_t lane_addr(uint32_t w, uint32_t base) {
  constexpr uint32_t sel = (0x0cu << 24) | (0x02u << 16) | ((4u + B) << 8) | 0x00u;
  return __builtin_amdgcn_perm(w, base, sel);
}

// Variant 0: the four 1 KB tables, one copy each.
struct Tab0 {
  static constexpr bool kBitsliced = false;
  static constexpr int kWords = 1024;
  const uint32_t* lds;
  __device__ Tab0(const uint32_t* l, int) : lds(l) {}
  template <int TBL, int B>
  __device__ __forceinline__ uint32_t get(uint32_t w) const {
    return lds[TBL * 256 + ((w >> (8 * B)) & 0xffu)];
  }
  __device__ static void fill(uint32_t* lds, int tid, int nthr) {
    for (int i = tid; i < 1024; i += nthr) lds[i] = rotl8n(c_aes.te0[i & 255], 8 * (i >> 8));
  }
};

// Variant 1: four tables, 32 lane-private copies, 256-byte entry rows:
// entry x of table t at byte (t>>1)*65536 + x*256 + (t&1)*128 + (lane&31)*4.
struct Tab1 {
  static constexpr bool kBitsliced = false;
  static constexpr int kWords = 32768;
  const uint8_t* lds;
  uint32_t base01, base23;
  __device__ Tab1(const uint32_t* l, int lane)
      : lds(reinterpret_cast<const uint8_t*>(l)),
        base01((uint32_t)(lane & 31) * 4u), base23(((uint32_t)(lane & 31) * 4u) | 0x10000u) {}
  template <int TBL, int B>
  __device__ __forceinline__ uint32_t get(uint32_t w) const {
    const uint32_t a = lane_addr<B>(w, TBL < 2 ? base01 : base23);
    return *reinterpret_cast<const uint32_t*>(lds + a + (TBL & 1) * 128);
  }
  __device__ static void fill(uint32_t* lds, int tid, int nthr) {
    // 16-byte chunk j covers words 4j..4j+3: one table entry, 4 of its 32 copies
    for (int j = tid; j < 8192; j += nthr) {
      const int sub = (j >> 3) & 1, x = (j >> 4) & 255, bank = j >> 12;
      const uint32_t v = rotl8n(c_aes.te0[x], 8 * (bank * 2 + sub));
      reinterpret_cast<uint4*>(lds)[j] = make_uint4(v, v, v, v);
    }
  }
};

// Variant 2: Te0 and Te2 with 32 copies (64 KB); T1, T3 by an 8-bit rotate.
struct Tab2 {
  static constexpr bool kBitsliced = false;
  static constexpr int kWords = 16384;
  const uint8_t* lds;
  uint32_t base;
  __device__ Tab2(const uint32_t* l, int lane)
      : lds(reinterpret_cast<const uint8_t*>(l)), base((uint32_t)(lane & 31) * 4u) {}
  template <int TBL, int B>
  __device__ __forceinline__ uint32_t get(uint32_t w) const {
    const uint32_t a = lane_addr<B>(w, base);
    uint32_t v = *reinterpret_cast<const uint32_t*>(lds + a + (TBL >= 2 ? 128 : 0));
    return rotl8n(v, 8 * (TBL & 1));
  }
  __device__ static void fill(uint32_t* lds, int tid, int nthr) {
    for (int j = tid; j < 4096; j += nthr) {
      const uint32_t v = rotl8n(c_aes.te0[j >> 4], 16 * ((j >> 3) & 1));
      reinterpret_cast<uint4*>(lds)[j] = make_uint4(v, v, v, v);
    }
  }
};

// Variant 3: Te0 only, 64 lane-private copies (64 KB); T1..T3 by rotates.
struct Tab3 {
  static constexpr bool kBitsliced = false;
  static constexpr int kWords = 16384;
  const uint8_t* lds;
  uint32_t base;
  __device__ Tab3(const uint32_t* l, int lane)
      : lds(reinterpret_cast<const uint8_t*>(l)), base((uint32_t)(lane & 63) * 4u) {}
  template <int TBL, int B>
  __device__ __forceinline__ uint32_t get(uint32_t w) const {
    const uint32_t a = lane_addr<B>(w, base);
    return rotl8n(*reinterpret_cast<const uint32_t*>(lds + a), 8 * TBL);
  }
  __device__ static void fill(uint32_t* lds, int tid, int nthr) {
    for (int j = tid; j < 4096; j += nthr) {
      const uint32_t v = c_aes.te0[j >> 4];
      reinterpret_cast<uint4*>(lds)[j] = make_uint4(v, v, v, v);
    }
  }
};

// Variant 4: the fixed-key PRG is bitsliced in registers (fss_aes_bs.hpp: two
// blocks as eight bit planes, SubBytes by composite-field inversion), with no
// table lookups; AES under a key known only at launch (the dealer's
// counter-mode randomness) keeps layout 1's tables.
struct TabBS : Tab1 {
  static constexpr bool kBitsliced = true;
  __device__ TabBS(const uint32_t* l, int lane) : Tab1(l, lane) {}
};
static __constant__ bs::PrgPlanes c_prg_planes = bs::make_prg_planes(kAes.prg_rk);

template <int V> struct TabOf;
template <> struct TabOf<0> { using T = Tab0; static constexpr int kBlock = 256; };
template <> struct TabOf<1> { using T = Tab1; static constexpr int kBlock = 768; };
template <> struct TabOf<2> { using T = Tab2; static constexpr int kBlock = 512; };
template <> struct TabOf<3> { using T = Tab3; static constexpr int kBlock = 512; };
template <> struct TabOf<4> { using T = TabBS; static constexpr int kBlock = 768; };

// ---------------------------------------------------------------------------
// AES-128 encryption of K independent blocks, round-interleaved for ILP.
// State words are little-endian columns: s[c] = bytes 4c..4c+3.
// ---------------------------------------------------------------------------
struct PrgKey {  // the fixed PRG key: round keys are compile-time constants
  template <int I>
  __device__ __forceinline__ uint32_t w() const { return kAes.prg_rk[I]; }
};
struct RtKey {   // a key known at launch (the dealer seed), read from kernel arguments
  const RoundKeys& rk;
  template <int I>
  __device__ __forceinline__ uint32_t w() const { return rk.w[I]; }
};

// One middle round of K blocks.  All 16 K table lookups are written before
// any of their XORs: where the scheduler keeps the source order (it reverts
// regions whose reordered form needs more registers), that order still has
// the round's lookups in flight together instead of one column's at a time.
template <int R, class Key, class TB, int K>
__device__ __forceinline__ void aes_round(const Key& key, const TB& tb, uint32_t (&s)[K][4]) {
  uint32_t t[K][4][4];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      t[k][c][0] = tb.template get<0, 0>(s[k][c]);
      t[k][c][1] = tb.template get<1, 1>(s[k][(c + 1) & 3]);
      t[k][c][2] = tb.template get<2, 2>(s[k][(c + 2) & 3]);
      t[k][c][3] = tb.template get<3, 3>(s[k][(c + 3) & 3]);
    }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    s[k][0] = xor3(xor3(t[k][0][0], t[k][0][1], t[k][0][2]), t[k][0][3], key.template w<4 * R + 0>());
    s[k][1] = xor3(xor3(t[k][1][0], t[k][1][1], t[k][1][2]), t[k][1][3], key.template w<4 * R + 1>());
    s[k][2] = xor3(xor3(t[k][2][0], t[k][2][1], t[k][2][2]), t[k][2][3], key.template w<4 * R + 2>());
    s[k][3] = xor3(xor3(t[k][3][0], t[k][3][1], t[k][3][2]), t[k][3][3], key.template w<4 * R + 3>());
  }
}

template <class Key, class TB, int K>
__device__ __forceinline__ void aes_final(const Key& key, const TB& tb, uint32_t (&s)[K][4]) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint32_t a[4] = {s[k][0], s[k][1], s[k][2], s[k][3]};
    uint32_t o[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      // S-box byte of row r sits in byte r of T_{(r+2)&3}.
      o[c] = (tb.template get<2, 0>(a[c]) & 0x000000ffu) |
             (tb.template get<3, 1>(a[(c + 1) & 3]) & 0x0000ff00u) |
             (tb.template get<0, 2>(a[(c + 2) & 3]) & 0x00ff0000u) |
             (tb.template get<1, 3>(a[(c + 3) & 3]) & 0xff000000u);
    }
    s[k][0] = o[0] ^ key.template w<40>();
    s[k][1] = o[1] ^ key.template w<41>();
    s[k][2] = o[2] ^ key.template w<42>();
    s[k][3] = o[3] ^ key.template w<43>();
  }
}

template <class Key, class TB, int K, int... Rs>
__device__ __forceinline__ void aes_rounds(const Key& key, const TB& tb, uint32_t (&s)[K][4],
                                           std::integer_sequence<int, Rs...>) {
  (aes_round<Rs + 1>(key, tb, s), ...);
}

template <class Key, class TB, int K, int... Rs>
__device__ __forceinline__ void aes_rounds_from2(const Key& key, const TB& tb, uint32_t (&s)[K][4],
                                                 std::integer_sequence<int, Rs...>) {
  (aes_round<Rs + 2>(key, tb, s), ...);
}

template <class Key, class TB, int K>
__device__ __forceinline__ void aes_encrypt(const Key& key, const TB& tb, uint32_t (&s)[K][4]) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    s[k][0] ^= key.template w<0>();
    s[k][1] ^= key.template w<1>();
    s[k][2] ^= key.template w<2>();
    s[k][3] ^= key.template w<3>();
  }
  aes_rounds(key, tb, s, std::make_integer_sequence<int, 9>{});
  aes_final(key, tb, s);
}

// AES_K of K blocks under the fixed PRG key, bitsliced two at a time (an odd
// last block is encrypted beside a copy of itself).
template <int K>
__device__ __forceinline__ void prg_aes_bitsliced(const uint32_t (&x)[K][4], uint32_t (&o)[K][4]) {
#pragma unroll
  for (int k = 0; k < K; k += 2) {
    const int k2 = k + 1 < K ? k + 1 : k;
    uint32_t a[4] = {x[k][0], x[k][1], x[k][2], x[k][3]}, b[4] = {x[k2][0], x[k2][1], x[k2][2], x[k2][3]};
    uint32_t pl[8];
    bs::pack(a, b, pl);
    bs::encrypt_pair(c_prg_planes, pl);
    bs::unpack(pl, a, b);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      o[k][c] = a[c];
      if (k + 1 < K) o[k2][c] = b[c];
    }
  }
}

// H(s, j) = AES_K(s ^ J_j) ^ s ^ J_j with J_j = byte 15 set to j.
template <class TB, int K>
__device__ __forceinline__ void prg(const TB& tb, const uint32_t (&s)[K][4], const uint32_t (&j)[K],
                                    uint32_t (&o)[K][4]) {
  if constexpr (TB::kBitsliced) {
    uint32_t x[K][4];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      x[k][0] = s[k][0];
      x[k][1] = s[k][1];
      x[k][2] = s[k][2];
      x[k][3] = s[k][3] ^ (j[k] << 24);
    }
    prg_aes_bitsliced<K>(x, o);
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) o[k][c] ^= x[k][c];
    return;
  }
  uint32_t x[K][4];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    x[k][0] = s[k][0];
    x[k][1] = s[k][1];
    x[k][2] = s[k][2];
    x[k][3] = s[k][3] ^ (j[k] << 24);
    o[k][0] = x[k][0]; o[k][1] = x[k][1]; o[k][2] = x[k][2]; o[k][3] = x[k][3];
  }
  aes_encrypt(PrgKey{}, tb, o);
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) o[k][c] ^= x[k][c];
}

// H(s, j_k) for K tweaks of one seed.  The inputs differ only in byte 15 (row 3
// of column 3), which after round 1 reaches only column 0: round 1's columns
// 1..3 and three of column 0's four lookups are computed once.
template <class TB, int K>
__device__ __forceinline__ void prg_shared(const TB& tb, const uint32_t (&s)[4], const uint32_t (&j)[K],
                                           uint32_t (&o)[K][4]) {
  if constexpr (TB::kBitsliced) {  // no table lookups to share: K blocks, two per bitsliced pair
    uint32_t ss[K][4];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) ss[k][c] = s[c];
    prg<TB, K>(tb, ss, j, o);
    return;
  }
  constexpr PrgKey key{};
  const uint32_t a0 = s[0] ^ key.template w<0>(), a1 = s[1] ^ key.template w<1>();
  const uint32_t a2 = s[2] ^ key.template w<2>(), a3 = s[3] ^ key.template w<3>();
  // a3 ^ (j << 24) has the same bytes 0..2 as a3
  const uint32_t c0 = xor3(tb.template get<0, 0>(a0), tb.template get<1, 1>(a1), tb.template get<2, 2>(a2));
  const uint32_t c1 = xor3(xor3(tb.template get<0, 0>(a1), tb.template get<1, 1>(a2), tb.template get<2, 2>(a3)),
                           tb.template get<3, 3>(a0), key.template w<5>());
  const uint32_t c2 = xor3(xor3(tb.template get<0, 0>(a2), tb.template get<1, 1>(a3), tb.template get<2, 2>(a0)),
                           tb.template get<3, 3>(a1), key.template w<6>());
  const uint32_t c3 = xor3(xor3(tb.template get<0, 0>(a3), tb.template get<1, 1>(a0), tb.template get<2, 2>(a1)),
                           tb.template get<3, 3>(a2), key.template w<7>());
#pragma unroll
  for (int k = 0; k < K; ++k) {
    o[k][0] = xor3(c0, tb.template get<3, 3>(a3 ^ (j[k] << 24)), key.template w<4>());
    o[k][1] = c1;
    o[k][2] = c2;
    o[k][3] = c3;
  }
  aes_rounds_from2(key, tb, o, std::make_integer_sequence<int, 8>{});
  aes_final(key, tb, o);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    o[k][0] ^= s[0];
    o[k][1] ^= s[1];
    o[k][2] ^= s[2];
    o[k][3] ^= s[3] ^ (j[k] << 24);
  }
}

// The tweak-independent part of H(s, .) for a seed that expands many blocks:
// round 1's column-0 lookups other than the tweak byte's (c0), the tweak
// byte's column word (a3), and round 2's twelve lookups of the columns the
// tweak does not reach, XORed per output column with round 2's key word (p).
struct PrgPrefix {
  uint32_t a3, c0, p[4];
};

template <class TB>
__device__ __forceinline__ void prg_prefix(const TB& tb, const uint32_t (&s)[4], PrgPrefix& q) {
  constexpr PrgKey key{};
  const uint32_t a0 = s[0] ^ key.template w<0>(), a1 = s[1] ^ key.template w<1>();
  const uint32_t a2 = s[2] ^ key.template w<2>(), a3 = s[3] ^ key.template w<3>();
  q.a3 = a3;
  q.c0 = xor3(tb.template get<0, 0>(a0), tb.template get<1, 1>(a1), tb.template get<2, 2>(a2));
  const uint32_t c1 = xor3(xor3(tb.template get<0, 0>(a1), tb.template get<1, 1>(a2), tb.template get<2, 2>(a3)),
                           tb.template get<3, 3>(a0), key.template w<5>());
  const uint32_t c2 = xor3(xor3(tb.template get<0, 0>(a2), tb.template get<1, 1>(a3), tb.template get<2, 2>(a0)),
                           tb.template get<3, 3>(a1), key.template w<6>());
  const uint32_t c3 = xor3(xor3(tb.template get<0, 0>(a3), tb.template get<1, 1>(a0), tb.template get<2, 2>(a1)),
                           tb.template get<3, 3>(a2), key.template w<7>());
  // round 2, output column c = T0[c] ^ T1[c+1] ^ T2[c+2] ^ T3[c+3] over the
  // round-1 columns: every term but the one reading column 0
  q.p[0] = xor3(tb.template get<1, 1>(c1), tb.template get<2, 2>(c2), tb.template get<3, 3>(c3)) ^ key.template w<8>();
  q.p[1] = xor3(tb.template get<0, 0>(c1), tb.template get<1, 1>(c2), tb.template get<2, 2>(c3)) ^ key.template w<9>();
  q.p[2] = xor3(tb.template get<0, 0>(c2), tb.template get<1, 1>(c3), tb.template get<3, 3>(c1)) ^ key.template w<10>();
  q.p[3] = xor3(tb.template get<0, 0>(c3), tb.template get<2, 2>(c1), tb.template get<3, 3>(c2)) ^ key.template w<11>();
}

template <class Key, class TB, int K, int... Rs>
__device__ __forceinline__ void aes_rounds_from3(const Key& key, const TB& tb, uint32_t (&s)[K][4],
                                                 std::integer_sequence<int, Rs...>) {
  (aes_round<Rs + 3>(key, tb, s), ...);
}

// H(s, j_k) for K tweaks of a seed whose prefix q = prg_prefix(s) is
// computed once: per block, the tweak byte's round-1 lookup, round 2's four
// lookups of column 0, then rounds 3..10.
template <class TB, int K>
__device__ __forceinline__ void prg_from_prefix(const TB& tb, const uint32_t (&s)[4], const PrgPrefix& q,
                                                const uint32_t (&j)[K], uint32_t (&o)[K][4]) {
  if constexpr (TB::kBitsliced) {
    prg_shared<TB, K>(tb, s, j, o);
    return;
  }
  constexpr PrgKey key{};
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint32_t x0 = xor3(q.c0, tb.template get<3, 3>(q.a3 ^ (j[k] << 24)), key.template w<4>());
    o[k][0] = q.p[0] ^ tb.template get<0, 0>(x0);
    o[k][1] = q.p[1] ^ tb.template get<3, 3>(x0);
    o[k][2] = q.p[2] ^ tb.template get<2, 2>(x0);
    o[k][3] = q.p[3] ^ tb.template get<1, 1>(x0);
  }
  aes_rounds_from3(key, tb, o, std::make_integer_sequence<int, 7>{});
  aes_final(key, tb, o);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    o[k][0] ^= s[0];
    o[k][1] ^= s[1];
    o[k][2] ^= s[2];
    o[k][3] ^= s[3] ^ (j[k] << 24);
  }
}

// ---------------------------------------------------------------------------
// Header validation (uniform across the launch)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int header_check(GHdr h, int party, int64_t n) {
  if (h->magic != kMagic || h->version != kVersion || h->kind != kGateOperator) return kStatusShape;
  if (h->rec_bytes != 16 + 8 * (uint64_t)h->p) return kStatusShape;
  if (h->lookup_r < 2 || h->lookup_r > 4) return kStatusShape;
  if ((int)h->party != party) return kStatusParty;
  if (n < 0 || (uint64_t)n > h->n_elems) return kStatusShape;
  return 0;
}

// ---------------------------------------------------------------------------
// One-time use of key material (Sec. "Threat Model and Preprocessing": all
// preprocessing material is one-time).  Each element's slot in the tile's
// record holds the tile's random sentinel until the element is first
// evaluated, then the x-hat it was evaluated at; one relaxed compare-and-swap
// per element records or checks it, so concurrent units of one tile (and
// overlapping launches) need no fence.  Evaluating again at the recorded
// x-hat (a replay) passes; at another x-hat the lane is refused: its outputs
// are zero and the status reports kStatusConsumed.  An x-hat equal to the
// sentinel (probability 2^-64) is not recorded.  Returns whether the lane may
// output.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool claim_once(GHdr h, const uint8_t* tile, int slot, uint64_t xh, bool valid,
                                           int* status) {
  bool ok = true;
  if (valid) {
    const unsigned long long none = ld8(tile + h->off_sentinel);
    unsigned long long seen = none;  // the slot's value when the exchange fails
    __hip_atomic_compare_exchange_strong(
        (FSS_GLOBAL unsigned long long*)(const_cast<uint8_t*>(tile) + h->off_seen) + slot, &seen,
        (unsigned long long)xh, __ATOMIC_RELAXED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ok = seen == none || seen == xh;
  }
  if (__ballot(!ok) && (threadIdx.x & 63) == 0) set_status(status, kStatusConsumed);
  return ok;
}

// ---------------------------------------------------------------------------
// Call 1: packed comparison.  Up to three Z_2 DCF atoms walk in lockstep.
// Each atom's tree has k - nu levels over the high bits of its view (nu =
// min(7, k)); the leaf seed s is converted into the 128-bit vector H(s, 2)
// (plus the leaf correction when the control bit is set), whose bit
// (view mod 2^nu) completes the share.
// ---------------------------------------------------------------------------
// CNT atoms from atom g on, walked in lockstep (one interleaved AES of CNT
// blocks per level); returns their bits at positions g ...
template <int CNT, class TB>
__device__ __forceinline__ uint32_t atom_group(const TB& tb, GHdr h, const uint8_t* tile, int lane, int b,
                                               uint64_t xhat, int g) {
  uint32_t bits = 0;
  uint32_t s[CNT][4], t[CNT], V[CNT], xh[CNT], xl[CNT];
  int lev[CNT];
  uint64_t vb[CNT];
  const uint8_t* base[CNT];
  int lmax = 0;
#pragma unroll
  for (int a = 0; a < CNT; ++a) {
    const int at = g + a;
    const int k = (int)h->atom_k[at];
    const int nu = atom_leaf_bits(k);
    lev[a] = k - nu;
    lmax = lev[a] > lmax ? lev[a] : lmax;
    base[a] = tile + h->atom_off[at];
    const uint4 r = ld16(base[a] + lane * 16);
    s[a][0] = r.x; s[a][1] = r.y; s[a][2] = r.z; s[a][3] = r.w;
    t[a] = (uint32_t)b;
    V[a] = 0;
    const uint64_t msk = (k >= 64) ? ~0ull : ((1ull << k) - 1);
    const uint32_t xv = (uint32_t)(((xhat & msk) + h->atom_c[at]) & msk);
    xh[a] = xv >> nu;
    xl[a] = xv & ((1u << nu) - 1u);
    vb[a] = ld8(base[a] + (uint64_t)kTile * 16 * (1 + k - nu) + lane * 8);
  }
  for (int i = 0; i < lmax; ++i) {
    uint32_t j[CNT], o[CNT][4];
#pragma unroll
    for (int a = 0; a < CNT; ++a) j[a] = (i < lev[a]) ? ((xh[a] >> (lev[a] - 1 - i)) & 1u) : 0u;
    prg<TB, CNT>(tb, s, j, o);
#pragma unroll
    for (int a = 0; a < CNT; ++a) {
      if (i < lev[a]) {
        const uint4 cw = ld16(base[a] + kTile * 16 + ((uint64_t)i * kTile + lane) * 16);
        const uint32_t msk = 0u - t[a];
        const uint32_t nt = (o[a][0] & 1u) ^ ((cw.x >> j[a]) & t[a] & 1u);
        const uint32_t v = ((o[a][0] >> 1) & 1u) ^ ((uint32_t)(vb[a] >> i) & t[a] & 1u);
        s[a][0] = (o[a][0] & ~3u) ^ (cw.x & ~3u & msk);
        s[a][1] = o[a][1] ^ (cw.y & msk);
        s[a][2] = o[a][2] ^ (cw.z & msk);
        s[a][3] = o[a][3] ^ (cw.w & msk);
        V[a] ^= v;
        t[a] = nt;
      }
    }
  }
  {  // the leaves
    uint32_t j[CNT], o[CNT][4];
#pragma unroll
    for (int a = 0; a < CNT; ++a) j[a] = 2u;
    prg<TB, CNT>(tb, s, j, o);
#pragma unroll
    for (int a = 0; a < CNT; ++a) {
      const uint4 lc = ld16(base[a] + (uint64_t)kTile * 16 * (1 + lev[a]) + kTile * 8 + lane * 16);
      const uint32_t msk = 0u - t[a];
      const uint32_t w = xl[a] >> 5;
      uint32_t word = (o[a][0] ^ (lc.x & msk));
      word = w == 1 ? (o[a][1] ^ (lc.y & msk)) : word;
      word = w == 2 ? (o[a][2] ^ (lc.z & msk)) : word;
      word = w == 3 ? (o[a][3] ^ (lc.w & msk)) : word;
      V[a] ^= (word >> (xl[a] & 31u)) & 1u;
      bits |= (V[a] & 1u) << (g + a);
    }
  }
  return bits;
}

template <class TB>
__device__ __forceinline__ uint32_t eval_atoms(const TB& tb, GHdr h, const uint8_t* tile,
                                               int lane, int b, uint64_t xhat) {
  const int T = (int)h->T;
  uint32_t bits = 0;
  for (int g = 0; g < T; g += 3) {
    const int cnt = T - g < 3 ? T - g : 3;
    bits |= cnt == 3 ? atom_group<3>(tb, h, tile, lane, b, xhat, g)
            : cnt == 2 ? atom_group<2>(tb, h, tile, lane, b, xhat, g)
                       : atom_group<1>(tb, h, tile, lane, b, xhat, g);
  }
  return bits;
}

// Combine atom shares into output-bit shares and ballot-pack 64 elements
// per word: z_j = negate_j (party 0) ^ w_j ^ XOR over atoms of (A_t ^ A_r(t)).
// `claim` is called once, after the bits are computed and before they are
// stored (the one-time record's check; a refused lane outputs zero bits).
template <class TB, class Claim>
__device__ __forceinline__ void pred_tile(const TB& tb, GHdr h, const uint8_t* tile,
                                          int lane, int b, uint64_t xhat, bool valid, uint64_t* z,
                                          uint64_t tile_idx, uint64_t words, uint32_t lb, Claim&& claim) {
  // lb: this party's share of the lookup's comparison, the mask query of
  // threshold atoms with atom_rview = kRviewLookup
  const uint32_t A = eval_atoms(tb, h, tile, lane, b, xhat) | (lb << kRviewLookup);
  uint64_t bits = ld8(tile + h->off_w + lane * 8);
  if (b == 0) bits ^= h->negate;
  const int np = (int)h->n_prim;
  for (int t = 0; t < np; ++t) {
    const uint32_t bit = ((A >> t) ^ (A >> h->atom_rview[t])) & 1u;
    bits ^= (uint64_t)bit << h->atom_out[t];
  }
  const bool ok = claim();
  const int ell = (int)h->ell;
  for (int j = 0; j < ell; ++j) {
    const uint64_t word = __ballot(valid && ok && ((bits >> j) & 1ull));
    if (lane == 0) stg64(z + (uint64_t)j * words + tile_idx, word);
  }
}

// ---------------------------------------------------------------------------
// Call 2: vector interval lookup.  One vector DCF (payload rho in Z^P) is
// evaluated at m points; 1 + ceil(P/2) AES per level, interleaved.
// ---------------------------------------------------------------------------
template <int P>
struct VState {  // a node of the GGM tree: seed, control bit, partial sum
  uint32_t s[4];
  uint32_t t;
  uint64_t V[P];
};

// `rootp`: the DCF's root seeds (16 bytes per lane) in the tile.
template <int P>
__device__ __forceinline__ VState<P> vroot_at(const uint8_t* rootp, int lane, int b) {
  VState<P> st;
  const uint4 r = ld16(rootp + lane * 16);
  st.s[0] = r.x; st.s[1] = r.y; st.s[2] = r.z; st.s[3] = r.w;
  st.t = (uint32_t)b;
#pragma unroll
  for (int q = 0; q < P; ++q) st.V[q] = 0;
  return st;
}

template <int P>
__device__ __forceinline__ VState<P> vroot(GHdr h, const uint8_t* tile, int lane, int b) {
  return vroot_at<P>(tile + h->off_croot, lane, b);
}

// The value of child d: words d P .. d P + P - 1 of the stream H(s, 2^R),
// H(s, 2^R + 1), ... (two words per block), i.e. NB = ceil(P/2) blocks from
// block (d P) / 2 on; for odd P an odd d starts at the first block's high word.
template <int P, int R>
__device__ __forceinline__ uint32_t value_block0(uint32_t d) { return (1u << R) + ((d * (uint32_t)P) >> 1); }

template <int P, int NB, int O>
__device__ __forceinline__ uint64_t value_word(const uint32_t (&o)[O][4], uint32_t d, int q) {
  // o[O - NB .. O - 1] are the NB value blocks; word w of them is o[O-NB+w/2][2(w&1)..]
  const uint64_t even = mk64(o[O - NB + q / 2][2 * (q & 1)], o[O - NB + q / 2][2 * (q & 1) + 1]);
  if constexpr ((P & 1) == 0) {
    return even;
  } else {
    const int w = q + 1;  // the word index when d P is odd
    const uint64_t odd = w / 2 < NB ? mk64(o[O - NB + w / 2][2 * (w & 1)], o[O - NB + w / 2][2 * (w & 1) + 1]) : 0ull;
    return (d & 1u) ? odd : even;
  }
}

// Advance `st` through levels [i0, i1) of the lookup DCF along the base-2^R
// digits of the input x: the DCF has L = ceil(n / R) levels of 2^R children
// and level i consumes digit L - 1 - i (R L - n leading zero bits).
// Child d of seed s is H(s, d); its value comes from the seed's shared value
// stream (value_word).  The last level adds the child's value only: nothing
// is walked below it, so its seed and control bit (the block H(s, d)) are not
// computed.
// `recbase`: the DCF's records in the tile; n: its input bits.
template <int P, int R, class TB>
__device__ __forceinline__ void vec_walk_at(const TB& tb, int n, const uint8_t* recbase, int lane, int b,
                                            uint32_t x, int i0, int i1, VState<P>& st) {
  constexpr int NB = (P + 1) / 2;
  constexpr uint32_t C = 1u << R;
  const int L = (n + R - 1) / R;
  constexpr uint64_t REC = 16 + 8 * P;
  const uint8_t* recp = recbase + lane * REC;
  const int imid = i1 < L - 1 ? i1 : L - 1;
  for (int i = i0; i < imid; ++i) {
    const uint32_t d = (x >> (R * (L - 1 - i))) & (C - 1u);
    uint32_t jj[1 + NB], o[1 + NB][4];
    jj[0] = d;
#pragma unroll
    for (int k = 0; k < NB; ++k) jj[1 + k] = value_block0<P, R>(d) + (uint32_t)k;
    prg_shared<TB, 1 + NB>(tb, st.s, jj, o);
    const uint8_t* rp = recp + ((uint64_t)i * C + d) * kTile * REC;  // child d's record at level i
    const uint64_t c01 = ld8(rp), c23 = ld8(rp + 8);
    const uint4 cw = make_uint4((uint32_t)c01, (uint32_t)(c01 >> 32), (uint32_t)c23, (uint32_t)(c23 >> 32));
    const uint32_t t = st.t;
    const uint32_t msk = 0u - t;
    const uint64_t msk64 = 0ull - (uint64_t)t;
    st.t = (o[0][0] & 1u) ^ (cw.x & t & 1u);
    st.s[0] = (o[0][0] & ~3u) ^ (cw.x & ~3u & msk);
    st.s[1] = o[0][1] ^ (cw.y & msk);
    st.s[2] = o[0][2] ^ (cw.z & msk);
    st.s[3] = o[0][3] ^ (cw.w & msk);
#pragma unroll
    for (int q = 0; q < P; ++q) {
      uint64_t v = value_word<P, NB>(o, d, q);
      v += ld8(rp + 16 + 8 * q) & msk64;
      st.V[q] += b ? (0ull - v) : v;
    }
  }
  if (i1 == L && i0 < L) {  // the last level: the child's value corrections only
    const uint32_t d = x & (C - 1u);
    uint32_t jj[NB], o[NB][4];
#pragma unroll
    for (int k = 0; k < NB; ++k) jj[k] = value_block0<P, R>(d) + (uint32_t)k;
    prg_shared<TB, NB>(tb, st.s, jj, o);
    const uint8_t* rp = recp + ((uint64_t)(L - 1) * C + d) * kTile * REC;
    const uint64_t msk64 = 0ull - (uint64_t)st.t;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      uint64_t v = value_word<P, NB>(o, d, q);
      v += ld8(rp + 16 + 8 * q) & msk64;
      st.V[q] += b ? (0ull - v) : v;
    }
  }
}

template <int P, int R, class TB>
__device__ __forceinline__ void vec_walk(const TB& tb, GHdr h, const uint8_t* tile, int lane, int b,
                                         uint32_t x, int i0, int i1, VState<P>& st) {
  vec_walk_at<P, R>(tb, (int)h->n, tile + h->off_crec, lane, b, x, i0, i1, st);
}

// With v = view_{n,c}(xhat) (c = 2^(n-1), the offset-binary view of the signed
// order, for real specs; c = 0 for integer specs over canonical
// representatives) and u_i = (v - a'_i) mod N, the share of
// 1[x' < a'_i] rho is g_i = D(u_i) - D(v) + 1[v < a'_i] rho_b, and the
// active piece's coefficients at xhat are
//   q = tab_0 rho_b + sum_{i=1}^{m-1} tab_i g_i  (+ r_out share in q_0),
// where tab_0 = A_{m-1}, tab_i = A_{i-1} - A_i and A_i maps a share of
// 1[x in I_i] rho to the x-hat coefficients of piece i.  Since
// sum_{i>=1} tab_i = A_0 - A_{m-1} =: tabv, the D(v) terms enter once:
//   q = sum_i tab_i (D(u_i) + 1[v < a'_i] rho_b) - tabv D(v) + tab_0 rho_b.
// Then y = sum_j q_j xhat^j.  (Ring arithmetic mod 2^64: any order is exact.)
//
// Shared prefixes: the points u_1 > ... > u_{m-1} (cyclically) lie in a window
// of W = a'_{m-1} - a'_1 + 1 consecutive values, which meets at most
// B = top_blocks aligned blocks of 2^K values (K = R (L - D)): block A (that
// of u_{m-1}) and its B - 1 successors, modulo the 2^(n-K) blocks of the
// n-bit domain.  The first D levels of the lookup DCF are walked once per
// block and each point resumes from its block's seed and control bit.  The
// partial sum V of a block's walk is the same for all its points, so it
// enters q right after that walk (q += tab_i V for each point i of the
// block) and only the seeds stay live: same outputs, (m - 1 - B) D fewer
// levels than walking every point from the root.
//
// Every term of q, and so of y = sum_j q_j xhat^j, is linear: a tile's work can
// be split into parts that each return their share of y (mod 2^64).  This call
// covers the points i in [i0, min(i1, m)) and, when `base` is set, the walk at
// v with the tabv, tab_0 rho and r_out terms; i0 = 1, i1 >= m, base = true is
// the whole of call 2.
template <int P, int R, class TB>
__device__ __forceinline__ uint64_t coeff_tile(const TB& tb, GHdr h, const uint8_t* tile,
                                               int lane, int b, uint64_t xhat, int i0, int i1, bool base,
                                               uint32_t* lbit) {
  const int n = (int)h->n, m = (int)h->m, D = (int)h->top_depth;
  const int L = (n + R - 1) / R;
  const int iend = i1 < m ? i1 : m;
  const uint32_t Nmask = n >= 32 ? 0xffffffffu : ((1u << n) - 1u);
  const uint32_t v = ((uint32_t)xhat + h->lookup_c) & Nmask;  // 2^(n-1): signed order; 0: canonical
  const uint8_t* rhop = tile + h->off_crho + lane * 8;
  const int K = D > 0 ? R * (L - D) : 0;  // input bits below the shared levels (D > 0: R <= K < n)
  const int NT = D > 0 ? (int)h->top_blocks : 0;
  const uint32_t blk_mask = D > 0 ? (1u << (n - K)) - 1u : 0u;
  const uint32_t blkA = D > 0 ? (((v - (uint32_t)h->aprime[m - 1]) & Nmask) >> K) : 0u;
  uint64_t q[P];
#pragma unroll
  for (int k = 0; k < P; ++k) q[k] = 0;
  const VState<P> root = vroot<P>(h, tile, lane, b);
  // seed (words 0..3) and control bit (word 4) of each block after the shared levels
  uint32_t ts[kMaxTopBlocks][5];
#pragma unroll
  for (int c = 0; c < kMaxTopBlocks; ++c) {
#pragma unroll
    for (int w = 0; w < 4; ++w) ts[c][w] = root.s[w];
    ts[c][4] = root.t;
  }
  if (iend > i0) {
#pragma unroll 1
    for (int bk = 0; bk < NT; ++bk) {
      VState<P> st = root;
      vec_walk<P, R>(tb, h, tile, lane, b, (uint32_t)((uint64_t)((blkA + (uint32_t)bk) & blk_mask) << K), 0, D, st);
#pragma unroll
      for (int c = 0; c < kMaxTopBlocks; ++c)
        if (c == bk) {
#pragma unroll
          for (int w = 0; w < 4; ++w) ts[c][w] = st.s[w];
          ts[c][4] = st.t;
        }
      for (int i = i0; i < iend; ++i) {
        const uint32_t u = (v - (uint32_t)h->aprime[i]) & Nmask;
        const uint64_t in = ((((u >> K) - blkA) & blk_mask) == (uint32_t)bk) ? ~0ull : 0ull;
#pragma unroll
        for (int j = 0; j < P; ++j)
#pragma unroll
          for (int k = 0; j + k < P; ++k) q[j] += h->tab[i][j][k] * (st.V[k] & in);
      }
    }
  }
  for (int i = i0; i < iend; ++i) {
    const uint32_t ap = (uint32_t)h->aprime[i];
    const uint32_t u = (v - ap) & Nmask;
    const uint32_t off = ((u >> K) - blkA) & blk_mask;  // D = 0: every block holds the root
    VState<P> st;
#pragma unroll
    for (int w = 0; w < 5; ++w) {
      uint32_t x = ts[0][w];
#pragma unroll
      for (int c = 1; c < kMaxTopBlocks; ++c) x = off == (uint32_t)c ? ts[c][w] : x;
      if (w < 4) st.s[w] = x; else st.t = x;
    }
#pragma unroll
    for (int k = 0; k < P; ++k) st.V[k] = 0;
    vec_walk<P, R>(tb, h, tile, lane, b, u, D, L, st);
    const uint64_t lt = v < ap ? ~0ull : 0ull;
    uint64_t g[P];
#pragma unroll
    for (int k = 0; k < P; ++k) g[k] = st.V[k] + (ld8(rhop + (uint64_t)k * kTile * 8) & lt);
#pragma unroll
    for (int j = 0; j < P; ++j)
#pragma unroll
      for (int k = 0; j + k < P; ++k) q[j] += h->tab[i][j][k] * g[k];
  }
  if (base) {
    VState<P> st = vroot<P>(h, tile, lane, b);
    vec_walk<P, R>(tb, h, tile, lane, b, v, 0, L, st);
    // this party's XOR share of 1[v < r_n]: its share of rho_0 1[v < r_n], mod 2
    if (lbit) *lbit = (uint32_t)(st.V[0] & 1ull);
#pragma unroll
    for (int j = 0; j < P; ++j)
#pragma unroll
      for (int k = 0; j + k < P; ++k) q[j] -= h->tabv[j][k] * st.V[k];
#pragma unroll
    for (int j = 0; j < P; ++j)
#pragma unroll
      for (int k = 0; j + k < P; ++k) q[j] += h->tab[0][j][k] * ld8(rhop + (uint64_t)k * kTile * 8);
    q[0] += ld8(tile + h->off_crout + lane * 8);
  }
  uint64_t y = q[P - 1];
#pragma unroll
  for (int j = P - 2; j >= 0; --j) y = y * xhat + q[j];
  return y;
}

template <int R, class TB>
__device__ __forceinline__ uint64_t coeff_dispatch_r(const TB& tb, GHdr h, const uint8_t* tile,
                                                     int lane, int b, uint64_t xhat, int i0, int i1, bool base,
                                                     uint32_t* lbit) {
  switch (h->p) {
    case 1: return coeff_tile<1, R>(tb, h, tile, lane, b, xhat, i0, i1, base, lbit);
    case 2: return coeff_tile<2, R>(tb, h, tile, lane, b, xhat, i0, i1, base, lbit);
    case 3: return coeff_tile<3, R>(tb, h, tile, lane, b, xhat, i0, i1, base, lbit);
    default: return coeff_tile<4, R>(tb, h, tile, lane, b, xhat, i0, i1, base, lbit);
  }
}

template <class TB>
__device__ __forceinline__ uint64_t coeff_dispatch(const TB& tb, GHdr h, const uint8_t* tile,
                                                   int lane, int b, uint64_t xhat, int i0 = 1,
                                                   int i1 = kMaxM + 1, bool base = true,
                                                   uint32_t* lbit = nullptr) {
  // lbit (may be null): with `base`, receives this party's XOR share of the
  // lookup's comparison 1[v < r_n], the mask query answered by the lookup
  switch (h->lookup_r) {
    case 2: return coeff_dispatch_r<2>(tb, h, tile, lane, b, xhat, i0, i1, base, lbit);
    case 3: return coeff_dispatch_r<3>(tb, h, tile, lane, b, xhat, i0, i1, base, lbit);
    default: return coeff_dispatch_r<4>(tb, h, tile, lane, b, xhat, i0, i1, base, lbit);
  }
}

// This party's share of the lookup DCF's first output at x, mod 2: the walk
// at x with the value stream's first word only.  Child d's word 0 is word d P
// of its seed's value stream, so each level expands the seed block and one
// value block (the last level the value block alone); low bits add as XOR.
template <int P, int R, class TB>
__device__ __forceinline__ uint32_t bit0_walk(const TB& tb, GHdr h, const uint8_t* tile, int lane, int b,
                                              uint32_t x) {
  constexpr uint32_t C = 1u << R;
  constexpr uint64_t REC = 16 + 8 * P;
  const int L = ((int)h->n + R - 1) / R;
  const uint8_t* recp = tile + h->off_crec + lane * REC;
  const uint4 root = ld16(tile + h->off_croot + lane * 16);
  uint32_t s[4] = {root.x, root.y, root.z, root.w}, t = (uint32_t)b, acc = 0;
  for (int i = 0; i + 1 < L; ++i) {
    const uint32_t d = (x >> (R * (L - 1 - i))) & (C - 1u), w = d * (uint32_t)P;
    const uint32_t jj[2] = {d, C + (w >> 1)};
    uint32_t o[2][4];
    prg_shared<TB, 2>(tb, s, jj, o);
    const uint8_t* rp = recp + ((uint64_t)i * C + d) * kTile * REC;
    const uint64_t c01 = ld8(rp), c23 = ld8(rp + 8), cv = ld8(rp + 16);
    const uint32_t msk = 0u - t;
    acc ^= (((w & 1u) ? o[1][2] : o[1][0]) ^ ((uint32_t)cv & msk)) & 1u;
    t = (o[0][0] & 1u) ^ ((uint32_t)c01 & t & 1u);
    s[0] = (o[0][0] & ~3u) ^ ((uint32_t)c01 & ~3u & msk);
    s[1] = o[0][1] ^ ((uint32_t)(c01 >> 32) & msk);
    s[2] = o[0][2] ^ ((uint32_t)c23 & msk);
    s[3] = o[0][3] ^ ((uint32_t)(c23 >> 32) & msk);
  }
  const uint32_t d = x & (C - 1u), w = d * (uint32_t)P;
  const uint32_t jj[1] = {C + (w >> 1)};
  uint32_t o[1][4];
  prg_shared<TB, 1>(tb, s, jj, o);
  const uint64_t cv = ld8(recp + ((uint64_t)(L - 1) * C + d) * kTile * REC + 16);
  acc ^= (((w & 1u) ? o[0][2] : o[0][0]) ^ ((uint32_t)cv & (0u - t))) & 1u;
  return acc;
}

// A call-1 unit's share of the lookup's comparison 1[v < r_n] when a mask
// query is the lookup's, else 0.
template <class TB>
__device__ __forceinline__ uint32_t lookup_bit(const TB& tb, GHdr h, const uint8_t* tile, int lane, int b,
                                               uint64_t xhat) {
  if (!h->mask_from_lookup) return 0;
  const int n = (int)h->n;
  const uint32_t v = (uint32_t)((xhat + h->lookup_c) & (n >= 64 ? ~0ull : ((1ull << n) - 1)));
  auto by_r = [&](auto pc) -> uint32_t {
    constexpr int PP = decltype(pc)::value;
    switch (h->lookup_r) {
      case 2: return bit0_walk<PP, 2>(tb, h, tile, lane, b, v);
      case 3: return bit0_walk<PP, 3>(tb, h, tile, lane, b, v);
      default: return bit0_walk<PP, 4>(tb, h, tile, lane, b, v);
    }
  };
  switch (h->p) {
    case 1: return by_r(std::integral_constant<int, 1>{});
    case 2: return by_r(std::integral_constant<int, 2>{});
    case 3: return by_r(std::integral_constant<int, 3>{});
    default: return by_r(std::integral_constant<int, 4>{});
  }
}

// ---------------------------------------------------------------------------
// Plain evaluator kernels: one tile per wave, grid covers the tiles.
// ---------------------------------------------------------------------------
template <int V>
__global__ __launch_bounds__(TabOf<V>::kBlock) void k_eval_pred(const uint8_t* keys, const uint64_t* xhat,
                                                                 int64_t n, uint64_t* z, int party, int* status) {
  using TB = typename TabOf<V>::T;
  __shared__ __align__(16) uint32_t lds[TB::kWords];
  TB::fill(lds, threadIdx.x, blockDim.x);
  __syncthreads();
  const GHdr h = ghdr(keys);
  const int bad = header_check(h, party, n);
  if (bad) {
    if (threadIdx.x == 0) set_status(status, bad);
    return;
  }
  const int lane = threadIdx.x & 63;
  const uint64_t tile = (uint64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const uint64_t words = ((uint64_t)n + 63) / 64;
  if (tile >= words) return;
  const uint64_t e = tile * kTile + lane;
  const bool valid = e < (uint64_t)n;
  const uint64_t xh = valid ? ldg64(xhat + e) : 0;
  TB tb(lds, lane);
  const uint8_t* tp = keys + kHeaderBytes + tile * h->tile_bytes;
  pred_tile(tb, h, tp, lane, party, xh, valid, z, tile, words, lookup_bit(tb, h, tp, lane, party, xh),
            [&] { return claim_once(h, tp, lane, xh, valid, status); });
}

template <int V>
__global__ __launch_bounds__(TabOf<V>::kBlock) void k_eval_coeff(const uint8_t* keys, const uint64_t* xhat,
                                                                  int64_t n, uint64_t* y, int party, int* status) {
  using TB = typename TabOf<V>::T;
  __shared__ __align__(16) uint32_t lds[TB::kWords];
  TB::fill(lds, threadIdx.x, blockDim.x);
  __syncthreads();
  const GHdr h = ghdr(keys);
  const int bad = header_check(h, party, n);
  if (bad) {
    if (threadIdx.x == 0) set_status(status, bad);
    return;
  }
  const int lane = threadIdx.x & 63;
  const uint64_t tile = (uint64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (tile * kTile >= (uint64_t)n) return;
  const uint64_t e = tile * kTile + lane;
  const bool valid = e < (uint64_t)n;
  const uint64_t xh = valid ? ldg64(xhat + e) : 0;
  TB tb(lds, lane);
  const uint8_t* tp = keys + kHeaderBytes + tile * h->tile_bytes;
  const uint64_t out = coeff_dispatch(tb, h, tp, lane, party, xh);
  const bool ok = claim_once(h, tp, lane, xh, valid, status);
  if (valid) stg64(y + e, ok ? out : 0ull);
}

// ---------------------------------------------------------------------------
// A kUnitLanes unit: 64 / 2^LG elements of a tile, each evaluated by 2^LG
// lanes (one per group) that split the unit's lookup points evenly; group 0
// also takes the base.  The groups' shares of y are added across lanes (two
// 32-bit swizzles per step), then group 0 stores them.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int mask) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, mask);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), mask);
  return mk64(lo, hi);
}

template <int LG, class TB>
__device__ __forceinline__ void lanes_unit(const TB& tb, GHdr h, const DevItem& it, uint64_t tile, uint32_t range,
                                           uint32_t flags, int lane, int* status) {
  constexpr int G = 1 << LG, E = kTile >> LG;
  const int grp = lane / E;
  const int slot = (int)((flags >> 16) & 63u) + (lane & (E - 1));
  const uint64_t e = tile * kTile + (uint64_t)slot;
  const bool valid = e < (uint64_t)it.n_elems;
  const uint64_t xh = valid ? ldg64(it.xhat + e) : 0;
  const uint8_t* tp = it.keys + kHeaderBytes + tile * h->tile_bytes;
  const int lo = (int)(range & 0xffffu), cnt = (int)(range >> 16) - lo;
  const int q = cnt / G, rr = cnt % G;
  const int i0 = lo + grp * q + (grp < rr ? grp : rr), i1 = i0 + q + (grp < rr ? 1 : 0);
  uint64_t out = coeff_dispatch(tb, h, tp, slot, it.party, xh, i0, i1, (flags & kUnitBase) != 0 && grp == 0);
#pragma unroll
  for (int d = E; d < kTile; d <<= 1) out += shfl_xor64(out, d);
  const bool ok = claim_once(h, tp, slot, xh, valid && grp == 0, status);
  if (valid && grp == 0) {
    if (flags & kUnitAccumulate)
      __hip_atomic_fetch_add((FSS_GLOBAL unsigned long long*)(it.y + e), (unsigned long long)(ok ? out : 0ull),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
      stg64(it.y + e, ok ? out : 0ull);
  }
}

// ---------------------------------------------------------------------------
// Fused persistent kernel: waves pull units from a work-list in cost order.
// A unit is a tile's call 1 and call 2 with the combination in one pass over
// its elements (x-hat loaded once), or a part of that work (call 1 alone, or
// a range of lookup points) when the planner splits tiles to balance the
// waves; the AES tables are staged once per resident block.
// ---------------------------------------------------------------------------
template <int V, int LG>
__global__ __launch_bounds__(TabOf<V>::kBlock) void k_fused(const DevItem* items, const uint32_t* tiles,
                                                             uint32_t n_tiles, uint32_t* counter,
                                                             int* status) {
  using TB = typename TabOf<V>::T;
  __shared__ __align__(16) uint32_t lds[TB::kWords];
  TB::fill(lds, threadIdx.x, blockDim.x);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  TB tb(lds, lane);
  while (true) {
    uint32_t idx = 0;
    if (lane == 0) idx = atomicAdd(counter, 1u);
    idx = __builtin_amdgcn_readfirstlane(idx);
    if (idx >= n_tiles) break;
    const FSS_GLOBAL uint32_t* tl = (const FSS_GLOBAL uint32_t*)tiles + (uint64_t)kUnitWords * idx;
    const uint32_t item = __builtin_amdgcn_readfirstlane(tl[0]);
    const uint64_t tile = __builtin_amdgcn_readfirstlane(tl[1]);
    const uint32_t range = __builtin_amdgcn_readfirstlane(tl[2]);
    const uint32_t flags = __builtin_amdgcn_readfirstlane(tl[3]);
    const FSS_GLOBAL DevItem* ip = (const FSS_GLOBAL DevItem*)items + item;
    DevItem it;
    it.keys = ip->keys;
    it.xhat = ip->xhat;
    it.y = ip->y;
    it.z = ip->z;
    it.n_elems = ip->n_elems;
    it.party = ip->party;
    it.words = ip->words;
    const GHdr h = ghdr(it.keys);
    const int bad = header_check(h, it.party, it.n_elems);
    if (bad) {
      if (lane == 0) set_status(status, bad);
      continue;
    }
    if constexpr (LG > 0) {
      if (flags & kUnitLanes) {
        lanes_unit<LG>(tb, h, it, tile, range, flags, lane, status);
        continue;
      }
    }
    const uint64_t e = tile * kTile + lane;
    const bool valid = e < (uint64_t)it.n_elems;
    const uint64_t xh = valid ? ldg64(it.xhat + e) : 0;
    const uint8_t* tp = it.keys + kHeaderBytes + tile * h->tile_bytes;
    // The one-time check runs after the unit's work and before its first
    // store: its atomic's latency then holds up no key load.
    bool ok = true;
    auto claim = [&] { return ok = claim_once(h, tp, lane, xh, valid, status); };
    if (!(flags & kUnitBase) && (range & 0xffffu) >= (range >> 16)) {
      // call 1 in a unit of its own (also with T = 0: the bits are then the
      // public constants and carry shares)
      pred_tile(tb, h, tp, lane, it.party, xh, valid, it.z, tile, (uint64_t)it.words,
                lookup_bit(tb, h, tp, lane, it.party, xh), claim);
      continue;
    }
    if constexpr (LG > 0) {
      // launches with lane groups run call 2 in kUnitLanes units only
      if (lane == 0) set_status(status, kStatusShape);
    } else {
      uint32_t lb = 0;
      const uint64_t out = coeff_dispatch(tb, h, tp, lane, it.party, xh, (int)(range & 0xffffu), (int)(range >> 16),
                                          (flags & kUnitBase) != 0, &lb);
      if (flags & kUnitPred)  // call 1 in the same pass, after call 2's walk at v gave the lookup's comparison
        pred_tile(tb, h, tp, lane, it.party, xh, valid, it.z, tile, (uint64_t)it.words, lb, claim);
      else
        claim();
      if (valid) {
        if (flags & kUnitAccumulate)  // parts of one tile add their shares of y (mod 2^64)
          __hip_atomic_fetch_add((FSS_GLOBAL unsigned long long*)(it.y + e), (unsigned long long)(ok ? out : 0ull),
                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
          stg64(it.y + e, ok ? out : 0ull);
      }
    }
  }
}


// ---------------------------------------------------------------------------
// Dealer key generation.  Lane = element; every random value is
// R(e, purpose, ctr) = AES_{K_seed}(e | purpose | ctr), so elements are
// independent and the output is deterministic.
// ---------------------------------------------------------------------------
template <class TB>
__device__ __forceinline__ void rand_blk(const TB& tb, const RoundKeys& rk, uint64_t e, uint32_t purpose,
                                         uint32_t ctr, uint32_t (&o)[4]) {
  uint32_t s[1][4] = {{(uint32_t)e, (uint32_t)(e >> 32), (purpose & 0xffffu) | (ctr << 16), 0u}};
  aes_encrypt(RtKey{rk}, tb, s);
  o[0] = s[0][0]; o[1] = s[0][1]; o[2] = s[0][2]; o[3] = s[0][3];
}

// R(e, purpose_k, ctr) for K purposes at once (one interleaved AES).
template <class TB, int K>
__device__ __forceinline__ void rand_blks(const TB& tb, const RoundKeys& rk, uint64_t e, const uint32_t (&purpose)[K],
                                          uint32_t ctr, uint32_t (&o)[K][4]) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    o[k][0] = (uint32_t)e;
    o[k][1] = (uint32_t)(e >> 32);
    o[k][2] = (purpose[k] & 0xffffu) | (ctr << 16);
    o[k][3] = 0u;
  }
  aes_encrypt(RtKey{rk}, tb, o);
}

// Keygen's side: the record starts with every slot at the tile's sentinel
// (one PRG block of the tile's first element), the sentinel itself, then
// zeros over the tile's padding (at most 248 bytes), so that a key buffer is
// a function of the dealer's seed alone.
template <class TB>
__device__ __forceinline__ void init_record(const TB& tb, const RoundKeys& rk, uint64_t tile, uint64_t off_seen,
                                            uint64_t off_sentinel, uint64_t tile_bytes, uint8_t* t0, uint8_t* t1,
                                            int lane) {
  uint32_t r[4];
  rand_blk(tb, rk, tile * kTile, kPurposeSentinel, 0, r);
  const uint64_t none = mk64(r[0], r[1]);
  st8(t0 + off_seen + lane * 8, none);
  if (t1) st8(t1 + off_seen + lane * 8, none);
  if ((uint64_t)lane * 8 < tile_bytes - off_sentinel) {
    const uint64_t v = lane == 0 ? none : 0ull;
    st8(t0 + off_sentinel + lane * 8, v);
    if (t1) st8(t1 + off_sentinel + lane * 8, v);
  }
}

// Z_2 DCF Gen for f(x) = 1[x < alpha] over k bits, the tree stopping nu =
// min(7, k) levels above the leaves; writes root, cw, vbits and the leaf
// correction.  The PRG tweaks are chosen so block 0/1 of each party is the
// child on / off alpha's path ("keep" / "lose"); no register array is indexed
// at run time.
template <class TB>
__device__ __forceinline__ void gen_z2(const TB& tb, int k, uint64_t alpha, const uint32_t (&r0)[4],
                                       const uint32_t (&r1)[4], uint8_t* a0, uint8_t* a1, int lane) {
  const int nu = atom_leaf_bits(k), lev = k - nu;
  const uint64_t ah = alpha >> nu;
  const uint32_t al = (uint32_t)(alpha & ((1ull << nu) - 1));
  uint32_t s0[4] = {r0[0] & ~3u, r0[1], r0[2], r0[3]};
  uint32_t s1[4] = {r1[0] & ~3u, r1[1], r1[2], r1[3]};
  uint32_t t0 = 0, t1 = 1, Va = 0;
  uint64_t vbits = 0;
  st16(a0 + lane * 16, make_uint4(s0[0], s0[1], s0[2], s0[3]));
  if (a1) st16(a1 + lane * 16, make_uint4(s1[0], s1[1], s1[2], s1[3]));
  for (int i = 0; i < lev; ++i) {
    const uint32_t ai = (uint32_t)(ah >> (lev - 1 - i)) & 1u;
    uint32_t o[4][4];  // p0 keep, p0 lose, p1 keep, p1 lose
    {
      const uint32_t jj[2] = {ai, ai ^ 1u};
      uint32_t oa[2][4], ob[2][4];
      prg_shared<TB, 2>(tb, s0, jj, oa);
      prg_shared<TB, 2>(tb, s1, jj, ob);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        o[0][c] = oa[0][c]; o[1][c] = oa[1][c]; o[2][c] = ob[0][c]; o[3][c] = ob[1][c];
      }
    }
    const uint32_t tk0 = o[0][0] & 1u, tl0 = o[1][0] & 1u, tk1 = o[2][0] & 1u, tl1 = o[3][0] & 1u;
    const uint32_t vk0 = (o[0][0] >> 1) & 1u, vl0 = (o[1][0] >> 1) & 1u;
    const uint32_t vk1 = (o[2][0] >> 1) & 1u, vl1 = (o[3][0] >> 1) & 1u;
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q][0] &= ~3u;
    uint32_t scw[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) scw[c] = o[1][c] ^ o[3][c];
    const uint32_t vcw = vl1 ^ vl0 ^ Va ^ ai;  // + beta (= 1) when the lost child is L
    Va = Va ^ vk1 ^ vk0 ^ vcw;
    const uint32_t tkx = tk0 ^ tk1, tlx = tl0 ^ tl1;
    const uint32_t tL = (ai ? tlx : tkx) ^ ai ^ 1u;
    const uint32_t tR = (ai ? tkx : tlx) ^ ai;
    const uint4 cw = make_uint4(scw[0] | tL | (tR << 1), scw[1], scw[2], scw[3]);
    uint8_t* cwo = a0 + kTile * 16 + ((uint64_t)i * kTile + lane) * 16;
    st16(cwo, cw);
    if (a1) st16(a1 + (cwo - a0), cw);
    vbits |= (uint64_t)vcw << i;
    const uint32_t tk = ai ? tR : tL;
    const uint32_t m0 = 0u - t0, m1 = 0u - t1;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      s0[c] = o[0][c] ^ (scw[c] & m0);
      s1[c] = o[2][c] ^ (scw[c] & m1);
    }
    t0 = tk0 ^ (t0 & tk);
    t1 = tk1 ^ (t1 & tk);
  }
  uint8_t* vbo = a0 + (uint64_t)kTile * 16 * (1 + lev) + lane * 8;
  st8(vbo, vbits);
  if (a1) st8(a1 + (vbo - a0), vbits);
  // The leaf correction: the parties' vectors H(s_b, 2) at alpha's leaf XOR to
  // (1[j < alpha mod 2^nu])_j once it is added, with V_alpha cancelled.
  uint32_t in[2][4], o[2][4];
  const uint32_t jj[2] = {2u, 2u};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    in[0][c] = s0[c];
    in[1][c] = s1[c];
  }
  prg<TB, 2>(tb, in, jj, o);
  const uint32_t flip = 0u - Va;
  uint32_t lw[4];
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const uint32_t lo = 32u * (uint32_t)w;
    const uint32_t below = al >= lo + 32u ? 0xffffffffu : (al <= lo ? 0u : ((1u << (al - lo)) - 1u));
    lw[w] = o[0][w] ^ o[1][w] ^ below ^ flip;
  }
  const uint64_t leaf_off = (uint64_t)kTile * 16 * (1 + lev) + kTile * 8 + lane * 16;
  st16(a0 + leaf_off, make_uint4(lw[0], lw[1], lw[2], lw[3]));
  if (a1) st16(a1 + leaf_off, make_uint4(lw[0], lw[1], lw[2], lw[3]));
}

// Vector DCF Gen for f(x) = beta * 1[x < alpha] over n bits, beta in Z^P,
// with 2^R children per level (L = ceil(n / R) levels, base-2^R digits of
// alpha).  At every level both parties expand all 2^R children; for a
// child off alpha's path the corrections make the parties' children equal:
// seed XOR, control bits t0 ^ t1, V_CW = (-1)^{t_1} (v_1 - v_0 - V_alpha
// [+ beta below alpha's digit]).  Above the last level alpha's child gets
// random corrections R(e, 69 + k, level), carries the parties on, and
// updates V_alpha; at the last level it is corrected like the others.
// The DCF's root seeds and records sit at off_croot / off_crec of the tile;
// the on-path child's corrections at level i are R(e, pur0 + k, ctr0 + i).
template <int P, int R, class TB>
__device__ __forceinline__ void gen_vec_at(const TB& tb, uint64_t off_croot, uint64_t off_crec, uint32_t pur0,
                                           uint32_t ctr0, int n, uint64_t alpha, const uint64_t (&beta)[P],
                                           const uint32_t (&r0)[4], const uint32_t (&r1)[4], const RoundKeys& rk,
                                           uint64_t e, uint8_t* k0, uint8_t* k1, int lane) {
  constexpr int NB = (P + 1) / 2;
  constexpr uint64_t REC = 16 + 8 * P;
  constexpr uint32_t C = 1u << R;
  const int L = (n + R - 1) / R;
  uint32_t s[2][4] = {{r0[0] & ~3u, r0[1], r0[2], r0[3]}, {r1[0] & ~3u, r1[1], r1[2], r1[3]}};
  uint32_t t[2] = {0u, 1u};
  uint64_t Va[P];
#pragma unroll
  for (int q = 0; q < P; ++q) Va[q] = 0;
  st16(k0 + off_croot + lane * 16, make_uint4(s[0][0], s[0][1], s[0][2], s[0][3]));
  if (k1) st16(k1 + off_croot + lane * 16, make_uint4(s[1][0], s[1][1], s[1][2], s[1][3]));
  for (int i = 0; i < L; ++i) {
    const uint32_t a = (uint32_t)(alpha >> (R * (L - 1 - i))) & (C - 1u);
    const uint64_t neg = 0ull - (uint64_t)t[1];  // (-1)^{t_1} as a mask
    // Children off alpha's path: corrections written as they are expanded.
    // Alpha's child: the parties' children kept for after the loop.
    uint32_t ks[2][4] = {{0u, 0u, 0u, 0u}, {0u, 0u, 0u, 0u}}, kt[2] = {0u, 0u};
    uint64_t dk[P];
#pragma unroll
    for (int q = 0; q < P; ++q) dk[q] = 0;
    const bool last = i + 1 == L;
    // every child's blocks come from the parties' seeds s[0], s[1]: their
    // tweak-independent AES work once per level
    PrgPrefix pre[2];
    if constexpr (!TB::kBitsliced) {
      prg_prefix(tb, s[0], pre[0]);
      prg_prefix(tb, s[1], pre[1]);
    }
    // The corrections of child c from both parties' expansions: seed blocks
    // sd0 / sd1 (above the last level) and values v0 / v1.  At the last level
    // only values: alpha's child is corrected like the others (without beta),
    // which zeroes the sum along alpha's path, so there is no leaf conversion
    // or final correction; nothing is walked below it, so its seed and
    // control-bit corrections are zero and its seed blocks are not computed.
    auto child = [&](uint32_t c, const uint32_t (&sd0)[4], const uint32_t (&sd1)[4], const uint64_t (&v0)[P],
                     const uint64_t (&v1)[P]) {
      const uint64_t ro = off_crec + (((uint64_t)i * C + c) * kTile + lane) * REC;
      const uint64_t below = c < a ? ~0ull : 0ull;
      if (!last && c == a) {
        ks[0][0] = sd0[0] & ~3u;
        ks[1][0] = sd1[0] & ~3u;
#pragma unroll
        for (int w = 1; w < 4; ++w) {
          ks[0][w] = sd0[w];
          ks[1][w] = sd1[w];
        }
        kt[0] = sd0[0] & 1u;
        kt[1] = sd1[0] & 1u;
#pragma unroll
        for (int q = 0; q < P; ++q) dk[q] = v0[q] - v1[q];
        return;
      }
      uint64_t c01 = 0, c23 = 0;
      if (!last) {
        const uint32_t t0c = sd0[0] & 1u, t1c = sd1[0] & 1u;
        c01 = mk64(((sd0[0] ^ sd1[0]) & ~3u) | (t0c ^ t1c), sd0[1] ^ sd1[1]);
        c23 = mk64(sd0[2] ^ sd1[2], sd0[3] ^ sd1[3]);
      }
      st8(k0 + ro, c01);
      st8(k0 + ro + 8, c23);
      if (k1) {
        st8(k1 + ro, c01);
        st8(k1 + ro + 8, c23);
      }
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const uint64_t w = v1[q] - v0[q] - Va[q] + (beta[q] & below);
        st8(k0 + ro + 16 + 8 * q, (w ^ neg) - neg);
        if (k1) st8(k1 + ro + 16 + 8 * q, (w ^ neg) - neg);
      }
    };
    // Both parties' expansions of the children, two at a time: with odd P the
    // pair's values share a block of the seed's value stream, expanded once.
#pragma unroll 1
    for (uint32_t c = 0; c < C; c += 2) {
      const uint32_t vb0 = value_block0<P, R>(c);
      if constexpr (P == 3) {
        // child c: words 0..2 of blocks vb0, vb0 + 1; child c + 1: word 3 of
        // them and words 0..1 of vb0 + 2
        uint64_t carry[2];
        {
          uint32_t o0[3][4], o1[3][4];
          if (last) {
            const uint32_t jj[2] = {vb0, vb0 + 1};
            uint32_t p0[2][4], p1[2][4];
            prg_from_prefix<TB, 2>(tb, s[0], pre[0], jj, p0);
            prg_from_prefix<TB, 2>(tb, s[1], pre[1], jj, p1);
#pragma unroll
            for (int w = 0; w < 4; ++w) {
              o0[0][w] = o1[0][w] = 0u;
              o0[1][w] = p0[0][w]; o0[2][w] = p0[1][w];
              o1[1][w] = p1[0][w]; o1[2][w] = p1[1][w];
            }
          } else {
            const uint32_t jj[3] = {c, vb0, vb0 + 1};
            prg_from_prefix<TB, 3>(tb, s[0], pre[0], jj, o0);
            prg_from_prefix<TB, 3>(tb, s[1], pre[1], jj, o1);
          }
          const uint64_t v0[3] = {mk64(o0[1][0], o0[1][1]), mk64(o0[1][2], o0[1][3]), mk64(o0[2][0], o0[2][1])};
          const uint64_t v1[3] = {mk64(o1[1][0], o1[1][1]), mk64(o1[1][2], o1[1][3]), mk64(o1[2][0], o1[2][1])};
          carry[0] = mk64(o0[2][2], o0[2][3]);
          carry[1] = mk64(o1[2][2], o1[2][3]);
          const uint32_t sd0[4] = {o0[0][0], o0[0][1], o0[0][2], o0[0][3]};
          const uint32_t sd1[4] = {o1[0][0], o1[0][1], o1[0][2], o1[0][3]};
          child(c, sd0, sd1, v0, v1);
        }
        {
          uint32_t o0[2][4], o1[2][4];
          if (last) {
            const uint32_t jj[1] = {vb0 + 2};
            uint32_t p0[1][4], p1[1][4];
            prg_from_prefix<TB, 1>(tb, s[0], pre[0], jj, p0);
            prg_from_prefix<TB, 1>(tb, s[1], pre[1], jj, p1);
#pragma unroll
            for (int w = 0; w < 4; ++w) {
              o0[0][w] = o1[0][w] = 0u;
              o0[1][w] = p0[0][w];
              o1[1][w] = p1[0][w];
            }
          } else {
            const uint32_t jj[2] = {c + 1, vb0 + 2};
            prg_from_prefix<TB, 2>(tb, s[0], pre[0], jj, o0);
            prg_from_prefix<TB, 2>(tb, s[1], pre[1], jj, o1);
          }
          const uint64_t v0[3] = {carry[0], mk64(o0[1][0], o0[1][1]), mk64(o0[1][2], o0[1][3])};
          const uint64_t v1[3] = {carry[1], mk64(o1[1][0], o1[1][1]), mk64(o1[1][2], o1[1][3])};
          const uint32_t sd0[4] = {o0[0][0], o0[0][1], o0[0][2], o0[0][3]};
          const uint32_t sd1[4] = {o1[0][0], o1[0][1], o1[0][2], o1[0][3]};
          child(c + 1, sd0, sd1, v0, v1);
        }
      } else if constexpr (P == 1) {
        // both children's values are the two words of block vb0
        uint32_t o0[2][4], o1[2][4];
        if (last) {
          const uint32_t jj[1] = {vb0};
          uint32_t p0[1][4], p1[1][4];
          prg_from_prefix<TB, 1>(tb, s[0], pre[0], jj, p0);
          prg_from_prefix<TB, 1>(tb, s[1], pre[1], jj, p1);
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            o0[0][w] = o1[0][w] = 0u;
            o0[1][w] = p0[0][w];
            o1[1][w] = p1[0][w];
          }
        } else {
          const uint32_t jj[2] = {c, vb0};
          prg_from_prefix<TB, 2>(tb, s[0], pre[0], jj, o0);
          prg_from_prefix<TB, 2>(tb, s[1], pre[1], jj, o1);
        }
        {
          const uint64_t v0[1] = {mk64(o0[1][0], o0[1][1])}, v1[1] = {mk64(o1[1][0], o1[1][1])};
          const uint32_t sd0[4] = {o0[0][0], o0[0][1], o0[0][2], o0[0][3]};
          const uint32_t sd1[4] = {o1[0][0], o1[0][1], o1[0][2], o1[0][3]};
          child(c, sd0, sd1, v0, v1);
        }
        const uint64_t w0 = mk64(o0[1][2], o0[1][3]), w1 = mk64(o1[1][2], o1[1][3]);
        uint32_t sd0[4] = {0u, 0u, 0u, 0u}, sd1[4] = {0u, 0u, 0u, 0u};
        if (!last) {
          const uint32_t jj[1] = {c + 1};
          uint32_t p0[1][4], p1[1][4];
          prg_from_prefix<TB, 1>(tb, s[0], pre[0], jj, p0);
          prg_from_prefix<TB, 1>(tb, s[1], pre[1], jj, p1);
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            sd0[w] = p0[0][w];
            sd1[w] = p1[0][w];
          }
        }
        const uint64_t v0[1] = {w0}, v1[1] = {w1};
        child(c + 1, sd0, sd1, v0, v1);
      } else {
        // even P: each child's values fill whole blocks of its own
#pragma unroll
        for (uint32_t cc = c; cc < c + 2; ++cc) {
          const uint32_t vb = value_block0<P, R>(cc);
          uint32_t o0[1 + NB][4], o1[1 + NB][4];
          if (last) {
            uint32_t jj[NB], p0[NB][4], p1[NB][4];
#pragma unroll
            for (int k = 0; k < NB; ++k) jj[k] = vb + (uint32_t)k;
            prg_from_prefix<TB, NB>(tb, s[0], pre[0], jj, p0);
            prg_from_prefix<TB, NB>(tb, s[1], pre[1], jj, p1);
#pragma unroll
            for (int w = 0; w < 4; ++w) {
              o0[0][w] = o1[0][w] = 0u;
#pragma unroll
              for (int k = 0; k < NB; ++k) {
                o0[1 + k][w] = p0[k][w];
                o1[1 + k][w] = p1[k][w];
              }
            }
          } else {
            uint32_t jj[1 + NB];
            jj[0] = cc;
#pragma unroll
            for (int k = 0; k < NB; ++k) jj[1 + k] = vb + (uint32_t)k;
            prg_from_prefix<TB, 1 + NB>(tb, s[0], pre[0], jj, o0);
            prg_from_prefix<TB, 1 + NB>(tb, s[1], pre[1], jj, o1);
          }
          uint64_t v0[P], v1[P];
#pragma unroll
          for (int q = 0; q < P; ++q) {
            v0[q] = mk64(o0[1 + q / 2][2 * (q & 1)], o0[1 + q / 2][2 * (q & 1) + 1]);
            v1[q] = mk64(o1[1 + q / 2][2 * (q & 1)], o1[1 + q / 2][2 * (q & 1) + 1]);
          }
          const uint32_t sd0[4] = {o0[0][0], o0[0][1], o0[0][2], o0[0][3]};
          const uint32_t sd1[4] = {o1[0][0], o1[0][1], o1[0][2], o1[0][3]};
          child(cc, sd0, sd1, v0, v1);
        }
      }
    }
    if (last) break;
    // Alpha's child: random seed and value corrections R(e, 69 + k, level);
    // the parties' next seeds and V_alpha.
    uint32_t kr[1 + NB][4];
    {
      uint32_t pur[1 + NB];
#pragma unroll
      for (int k = 0; k <= NB; ++k) pur[k] = pur0 + k;
      rand_blks<TB, 1 + NB>(tb, rk, e, pur, ctr0 + (uint32_t)i, kr);
    }
    const uint32_t tcw_a = kt[0] ^ kt[1] ^ 1u;
    const uint32_t scw_a[4] = {kr[0][0] & ~3u, kr[0][1], kr[0][2], kr[0][3]};
    const uint64_t ro = off_crec + (((uint64_t)i * C + a) * kTile + lane) * REC;
    st8(k0 + ro, mk64(scw_a[0] | tcw_a, scw_a[1]));
    st8(k0 + ro + 8, mk64(scw_a[2], scw_a[3]));
    if (k1) {
      st8(k1 + ro, mk64(scw_a[0] | tcw_a, scw_a[1]));
      st8(k1 + ro + 8, mk64(scw_a[2], scw_a[3]));
    }
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const uint64_t vcw = mk64(kr[1 + q / 2][2 * (q & 1)], kr[1 + q / 2][2 * (q & 1) + 1]);
      st8(k0 + ro + 16 + 8 * q, vcw);
      if (k1) st8(k1 + ro + 16 + 8 * q, vcw);
      Va[q] += dk[q] + ((vcw ^ neg) - neg);
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const uint32_t m = 0u - t[b];  // the parent's control bit applies the correction
#pragma unroll
      for (int w = 0; w < 4; ++w) s[b][w] = ks[b][w] ^ (scw_a[w] & m);
      t[b] = kt[b] ^ (t[b] & tcw_a);
    }
  }
}

// The operator's lookup DCF: header offsets, corrections R(e, 69 + k, level).
// Header offsets are read before the first key store: the compiler cannot
// tell the key stores from header memory, and a header read after a store
// would wait for the store to complete.
template <int P, int R, class TB>
__device__ __forceinline__ void gen_vec(const TB& tb, GHdr h, int n, uint64_t alpha,
                                        const uint64_t (&beta)[P], const uint32_t (&r0)[4],
                                        const uint32_t (&r1)[4], const RoundKeys& rk, uint64_t e,
                                        uint8_t* k0, uint8_t* k1, int lane) {
  const uint64_t off_croot = h->off_croot, off_crec = h->off_crec;
  gen_vec_at<P, R>(tb, off_croot, off_crec, 69u, 0u, n, alpha, beta, r0, r1, rk, e, k0, k1, lane);
}

template <int P, int R, class TB>
__device__ __forceinline__ void keygen_coeff(const TB& tb, GHdr h, const KgArgs& ga, uint64_t e,
                                             uint64_t rin, uint8_t* t0, uint8_t* t1, int lane) {
  uint64_t rho[P];
  rho[0] = 1;
#pragma unroll
  for (int q = 1; q < P; ++q) rho[q] = rho[q - 1] * (0ull - rin);
  uint32_t c0[4], c1[4];
  rand_blk(tb, ga.rk, e, 64, 0, c0);
  rand_blk(tb, ga.rk, e, 65, 0, c1);
  const int n = (int)h->n;
  const uint64_t off_crho = h->off_crho;
  const uint64_t nmask = n >= 64 ? ~0ull : ((1ull << n) - 1);
  gen_vec<P, R>(tb, h, n, rin & nmask, rho, c0, c1, ga.rk, e, t0, t1, lane);
  uint32_t ra[4], rb[4];
  rand_blk(tb, ga.rk, e, 67, 0, ra);
  rand_blk(tb, ga.rk, e, 68, 0, rb);
  const uint64_t sh[4] = {mk64(ra[0], ra[1]), mk64(ra[2], ra[3]), mk64(rb[0], rb[1]), mk64(rb[2], rb[3])};
#pragma unroll
  for (int q = 0; q < P; ++q) {
    const uint64_t o = off_crho + ((uint64_t)q * kTile + lane) * 8;
    st8(t0 + o, sh[q]);
    if (t1) st8(t1 + o, rho[q] - sh[q]);
  }
}

// Keygen runs the table layout's block size, like evaluation: the layout's
// tables fill one CU's local memory, so the block size sets the waves per CU.
// With P <= 3, both parties' walk state exceeds that register budget by a few
// values live across a whole level (spilled: a handful of accesses per level);
// P = 4 would spill inside the AES rounds, so it keeps two waves per SIMD.
template <int V, int P>
constexpr int keygen_block() { return (P >= 4 && TabOf<V>::kBlock > 512) ? 512 : TabOf<V>::kBlock; }

template <int V, int P, int R>
__global__ __launch_bounds__((keygen_block<V, P>())) void k_keygen(const KeyHeader* hdr, KgArgs ga, uint8_t* key0,
                                                              uint8_t* key1, uint64_t* r_in, uint64_t* r_out) {
  using TB = typename TabOf<V>::T;
  __shared__ __align__(16) uint32_t lds[TB::kWords];
  TB::fill(lds, threadIdx.x, blockDim.x);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  // With two jobs per tile (small batches: latency), wave 2j + 0 of a tile
  // makes the masks and call 1's keys, wave 2j + 1 call 2's key; both draw
  // r_in from the same counter-mode block, so the keys are those of one wave.
  const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const uint64_t tile = ga.jobs == 2 ? wave >> 1 : wave;
  if (tile >= ga.n_tiles) return;
  const bool do_call1 = ga.jobs != 2 || (wave & 1) == 0;
  const bool do_call2 = ga.jobs != 2 || (wave & 1) == 1;
  TB tb(lds, lane);
  const GHdr h = ghdr(hdr);
  const uint64_t e = tile * kTile + lane;
  const uint64_t tb_bytes = h->tile_bytes;
  uint8_t* t0 = key0 + kHeaderBytes + tile * tb_bytes;
  uint8_t* t1 = key1 ? key1 + kHeaderBytes + tile * tb_bytes : nullptr;

  uint32_t r[4];
  if (do_call2) {
    rand_blk(tb, ga.rk, e, 0, 0, r);
    keygen_coeff<P, R>(tb, h, ga, e, mk64(r[0], r[1]), t0, t1, lane);
  }
  if (!do_call1) return;
  rand_blk(tb, ga.rk, e, 0, 0, r);  // drawn again rather than held across call 2's keygen
  const uint64_t rin = mk64(r[0], r[1]), rout = mk64(r[2], r[3]);
  if (e < (uint64_t)ga.n_elems) {
    if (r_in) stg64(r_in + e, rin);
    if (r_out) stg64(r_out + e, rout);
  }
  rand_blk(tb, ga.rk, e, 1, 0, r);
  const uint64_t rs = mk64(r[0], r[1]);
  st8(t0 + h->off_crout + lane * 8, rs);
  if (t1) st8(t1 + h->off_crout + lane * 8, rout - rs);

  // Packed comparison: theta atoms use theta = (r_k + b') mod 2^k and carry
  // w = 1[r_k + b' >= 2^k]; mask atoms use alpha = r_k.
  uint64_t wout = 0;
  const int T = (int)h->T, np = (int)h->n_prim;
  for (int t = 0; t < T; ++t) {
    const int k = (int)h->atom_k[t];
    const uint64_t msk = k >= 64 ? ~0ull : ((1ull << k) - 1);
    const uint64_t rk = rin & msk;
    uint64_t alpha = rk;
    if (t < np) {
      const uint64_t sum = rk + ga.bprime[t];
      alpha = sum & msk;
      if (sum >> k) wout ^= 1ull << h->atom_out[t];
    }
    uint32_t ra[4], rb[4];
    rand_blk(tb, ga.rk, e, 2 + 2 * t, 0, ra);
    rand_blk(tb, ga.rk, e, 3 + 2 * t, 0, rb);
    gen_z2(tb, k, alpha, ra, rb, t0 + h->atom_off[t], t1 ? t1 + h->atom_off[t] : nullptr, lane);
  }
  init_record(tb, ga.rk, tile, h->off_seen, h->off_sentinel, tb_bytes, t0, t1, lane);
  rand_blk(tb, ga.rk, e, 66, 0, r);
  const uint64_t ellmask = h->ell >= 64 ? ~0ull : ((1ull << h->ell) - 1);
  const uint64_t W = mk64(r[0], r[1]) & ellmask;
  st8(t0 + h->off_w + lane * 8, W);
  if (t1) st8(t1 + h->off_w + lane * 8, W ^ wout);
}

// ---------------------------------------------------------------------------
// Rescaling gate: shares of floor(y / 2^s) + r_out from the opening
// yhat = y + r_in (|y| < 2^62).  With uhat = yhat + 2^62 the borrow of the low
// s bits, 1[uhat mod 2^s < r_in mod 2^s], comes from one DCF with payload -1
// (additive shares of -borrow); the overflow of the top bit is
// MSB(r_in) (1 - MSB(uhat)), a public factor times a dealer-shared constant.
// ---------------------------------------------------------------------------
template <int V, int R>
__global__ __launch_bounds__(TabOf<V>::kBlock) void k_rescale_keygen(const KeyHeader* hdr, KgArgs ga,
                                                                      const uint64_t* r_in, uint8_t* key0,
                                                                      uint8_t* key1, uint64_t* r_out) {
  using TB = typename TabOf<V>::T;
  __shared__ __align__(16) uint32_t lds[TB::kWords];
  TB::fill(lds, threadIdx.x, blockDim.x);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const uint64_t tile = (uint64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (tile >= ga.n_tiles) return;
  TB tb(lds, lane);
  const GHdr h = ghdr(hdr);
  const int s = (int)h->shift;
  const uint64_t e = tile * kTile + lane;
  const bool valid = e < (uint64_t)ga.n_elems;
  const uint64_t tbb = h->tile_bytes, off_k0 = h->off_tk0, off_k1 = h->off_tk1;
  uint8_t* t0 = key0 + kHeaderBytes + tile * tbb;
  uint8_t* t1 = key1 ? key1 + kHeaderBytes + tile * tbb : nullptr;
  const uint64_t rin = valid ? ldg64(r_in + e) : 0;
  init_record(tb, ga.rk, tile, h->off_seen, h->off_sentinel, tbb, t0, t1, lane);
  uint32_t r[4];
  rand_blk(tb, ga.rk, e, 0, 0, r);
  const uint64_t rout = mk64(r[0], r[1]);
  if (valid && r_out) stg64(r_out + e, rout);
  const uint64_t v0 = rout - (rin >> s);
  const uint64_t v1 = (rin >> 63) ? (1ull << (64 - s)) : 0ull;
  rand_blk(tb, ga.rk, e, 1, 0, r);
  const uint64_t sh0 = mk64(r[0], r[1]), sh1 = mk64(r[2], r[3]);
  st8(t0 + off_k0 + lane * 8, sh0);
  st8(t0 + off_k1 + lane * 8, sh1);
  if (t1) {
    st8(t1 + off_k0 + lane * 8, v0 - sh0);
    st8(t1 + off_k1 + lane * 8, v1 - sh1);
  }
  uint32_t c0[4], c1[4];
  rand_blk(tb, ga.rk, e, 64, 0, c0);
  rand_blk(tb, ga.rk, e, 65, 0, c1);
  const uint64_t beta[1] = {~0ull};  // -1
  gen_vec<1, R>(tb, h, s, rin & ((1ull << s) - 1), beta, c0, c1, ga.rk, e, t0, t1, lane);
}

template <int V>
__global__ __launch_bounds__(TabOf<V>::kBlock) void k_rescale_eval(const uint8_t* keys, const uint64_t* yhat,
                                                                    int64_t n, uint64_t* z, int party,
                                                                    int* status) {
  using TB = typename TabOf<V>::T;
  __shared__ __align__(16) uint32_t lds[TB::kWords];
  TB::fill(lds, threadIdx.x, blockDim.x);
  __syncthreads();
  const GHdr h = ghdr(keys);
  if (h->magic != kMagic || h->version != kVersion || h->kind != kGateRescale || h->rec_bytes != 24 ||
      h->lookup_r < 2 || h->lookup_r > 4 || h->shift < 1 || h->shift > 32 || n < 0 || (uint64_t)n > h->n_elems ||
      (int)h->party != party) {
    if (threadIdx.x == 0) set_status(status, (int)h->party != party ? kStatusParty : kStatusShape);
    return;
  }
  const int lane = threadIdx.x & 63;
  const uint64_t tile = (uint64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (tile * kTile >= (uint64_t)n) return;
  const uint64_t e = tile * kTile + lane;
  const bool valid = e < (uint64_t)n;
  TB tb(lds, lane);
  const uint8_t* tp = keys + kHeaderBytes + tile * h->tile_bytes;
  const int s = (int)h->shift;
  const uint64_t yh = valid ? ldg64(yhat + e) : 0;
  const uint64_t uhat = yh + (1ull << 62);
  const uint32_t x = (uint32_t)(uhat & ((1ull << s) - 1));
  VState<1> st = vroot<1>(h, tp, lane, party);
  switch (h->lookup_r) {
    case 2: vec_walk<1, 2>(tb, h, tp, lane, party, x, 0, (s + 1) / 2, st); break;
    case 3: vec_walk<1, 3>(tb, h, tp, lane, party, x, 0, (s + 2) / 3, st); break;
    default: vec_walk<1, 4>(tb, h, tp, lane, party, x, 0, (s + 3) / 4, st); break;
  }
  uint64_t out = ld8(tp + h->off_tk0 + lane * 8) + (1ull - (uhat >> 63)) * ld8(tp + h->off_tk1 + lane * 8) + st.V[0];
  if (party == 0) out += (uhat >> s) - (1ull << (62 - s));
  const bool ok = claim_once(h, tp, lane, yh, valid, status);
  if (valid) stg64(z + e, ok ? out : 0ull);
}

// ---------------------------------------------------------------------------
// Launchers of one table layout (explicitly instantiated per translation unit)
// ---------------------------------------------------------------------------
template <int V>
int VariantOps<V>::block() { return TabOf<V>::kBlock; }

template <int V>
int VariantOps<V>::lds_bytes() { return TabOf<V>::T::kWords * 4; }

// Waves (tiles) per block: the full block when there are enough tiles to give
// every CU one, otherwise ceil(tiles / CUs), so a small batch runs on as many
// CUs as it has tiles instead of queueing its tiles on a few of them.
inline uint64_t waves_per_block(uint64_t tiles, int cus, int block) {
  const uint64_t full = (uint64_t)block / 64;
  const uint64_t c = cus > 0 ? (uint64_t)cus : 1;
  const uint64_t w = (tiles + c - 1) / c;
  return w < 1 ? 1 : (w > full ? full : w);
}

// A batch whose tiles, two waves each, still fit the resident waves of the
// grid runs two jobs per tile (call 1's keys beside call 2's): its latency is
// one tile's keygen, and halving it halves the batch's.  Larger batches keep
// one wave per tile: a block's waves would otherwise finish at different
// times and leave its CU part-idle.
template <int V, int P, int R>
hipError_t launch_keygen(const KeyHeader* h, const KgArgs& ga_in, uint8_t* k0, uint8_t* k1, uint64_t* ri,
                         uint64_t* ro, int cus, hipStream_t st) {
  KgArgs ga = ga_in;
  const uint64_t slots = (uint64_t)(cus > 0 ? cus : 1) * (keygen_block<V, P>() / 64);
  ga.jobs = 2 * ga.n_tiles <= slots ? 2 : 1;
  const uint64_t waves = ga.n_tiles * (uint64_t)ga.jobs;
  const uint64_t per = waves_per_block(waves, cus, keygen_block<V, P>());
  const unsigned grid = (unsigned)((waves + per - 1) / per);
  hipLaunchKernelGGL((k_keygen<V, P, R>), dim3(grid), dim3((unsigned)(per * 64)), 0, st, h, ga, k0, k1, ri, ro);
  return hipGetLastError();
}

template <int V, int R>
hipError_t launch_keygen_p(const KeyHeader* h, int p, const KgArgs& ga, uint8_t* k0, uint8_t* k1, uint64_t* ri,
                           uint64_t* ro, int cus, hipStream_t st) {
  switch (p) {
    case 1: return launch_keygen<V, 1, R>(h, ga, k0, k1, ri, ro, cus, st);
    case 2: return launch_keygen<V, 2, R>(h, ga, k0, k1, ri, ro, cus, st);
    case 3: return launch_keygen<V, 3, R>(h, ga, k0, k1, ri, ro, cus, st);
    case 4: return launch_keygen<V, 4, R>(h, ga, k0, k1, ri, ro, cus, st);
    default: return hipErrorInvalidValue;
  }
}

template <int V>
hipError_t VariantOps<V>::keygen(const KeyHeader* h, int p, int r, const KgArgs& ga, uint8_t* k0, uint8_t* k1,
                                 uint64_t* ri, uint64_t* ro, int cus, hipStream_t st) {
  if (ga.n_tiles == 0) return hipSuccess;
  switch (r) {
    case 2: return launch_keygen_p<V, 2>(h, p, ga, k0, k1, ri, ro, cus, st);
    case 3: return launch_keygen_p<V, 3>(h, p, ga, k0, k1, ri, ro, cus, st);
    case 4: return launch_keygen_p<V, 4>(h, p, ga, k0, k1, ri, ro, cus, st);
    default: return hipErrorInvalidValue;
  }
}

template <int V>
hipError_t VariantOps<V>::pred(int party, const uint8_t* keys, const uint64_t* xhat, int64_t n, uint64_t* z,
                               int* status, int cus, hipStream_t st) {
  const uint64_t tiles = ((uint64_t)n + 63) / 64;
  if (tiles == 0) return hipSuccess;
  const uint64_t per = waves_per_block(tiles, cus, TabOf<V>::kBlock);
  const unsigned grid = (unsigned)((tiles + per - 1) / per);
  hipLaunchKernelGGL((k_eval_pred<V>), dim3(grid), dim3((unsigned)(per * 64)), 0, st, keys, xhat, n, z, party,
                     status);
  return hipGetLastError();
}

template <int V>
hipError_t VariantOps<V>::coeff(int party, const uint8_t* keys, const uint64_t* xhat, int64_t n, uint64_t* y,
                                int* status, int cus, hipStream_t st) {
  const uint64_t tiles = ((uint64_t)n + 63) / 64;
  if (tiles == 0) return hipSuccess;
  const uint64_t per = waves_per_block(tiles, cus, TabOf<V>::kBlock);
  const unsigned grid = (unsigned)((tiles + per - 1) / per);
  hipLaunchKernelGGL((k_eval_coeff<V>), dim3(grid), dim3((unsigned)(per * 64)), 0, st, keys, xhat, n, y, party,
                     status);
  return hipGetLastError();
}

template <int V>
hipError_t VariantOps<V>::rescale_keygen(const KeyHeader* h, int r, const KgArgs& ga, const uint64_t* r_in,
                                         uint8_t* k0, uint8_t* k1, uint64_t* ro, int cus, hipStream_t st) {
  if (ga.n_tiles == 0) return hipSuccess;
  const uint64_t per = waves_per_block(ga.n_tiles, cus, TabOf<V>::kBlock);
  const unsigned grid = (unsigned)((ga.n_tiles + per - 1) / per);
  const dim3 g(grid), b((unsigned)(per * 64));
  switch (r) {
    case 2: hipLaunchKernelGGL((k_rescale_keygen<V, 2>), g, b, 0, st, h, ga, r_in, k0, k1, ro); break;
    case 3: hipLaunchKernelGGL((k_rescale_keygen<V, 3>), g, b, 0, st, h, ga, r_in, k0, k1, ro); break;
    case 4: hipLaunchKernelGGL((k_rescale_keygen<V, 4>), g, b, 0, st, h, ga, r_in, k0, k1, ro); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int V>
hipError_t VariantOps<V>::rescale_eval(int party, const uint8_t* keys, const uint64_t* yhat, int64_t n, uint64_t* z,
                                       int* status, int cus, hipStream_t st) {
  const uint64_t tiles = ((uint64_t)n + 63) / 64;
  if (tiles == 0) return hipSuccess;
  const uint64_t per = waves_per_block(tiles, cus, TabOf<V>::kBlock);
  const unsigned grid = (unsigned)((tiles + per - 1) / per);
  hipLaunchKernelGGL((k_rescale_eval<V>), dim3(grid), dim3((unsigned)(per * 64)), 0, st, keys, yhat, n, z, party,
                     status);
  return hipGetLastError();
}

template <int V>
hipError_t VariantOps<V>::fused(const DevItem* items, const uint32_t* tiles, uint32_t n_tiles,
                                uint32_t* counter, int* status, int grid, int lanes_log2, hipStream_t st) {
  constexpr int B = TabOf<V>::kBlock;
  if (grid <= 0) return hipErrorInvalidValue;
  if (lanes_log2 == 0) {
    hipLaunchKernelGGL((k_fused<V, 0>), dim3(grid), dim3(B), 0, st, items, tiles, n_tiles, counter, status);
    return hipGetLastError();
  }
  if constexpr (lanes_variant(V)) {
    if (lanes_log2 == 1)
      hipLaunchKernelGGL((k_fused<V, 1>), dim3(grid), dim3(B), 0, st, items, tiles, n_tiles, counter, status);
    else if (lanes_log2 == 2)
      hipLaunchKernelGGL((k_fused<V, 2>), dim3(grid), dim3(B), 0, st, items, tiles, n_tiles, counter, status);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

}  // namespace fss
