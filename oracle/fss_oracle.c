/*
 * fss_oracle.c -- plain CPU oracle for the FuseFSS hot path.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the
 * benchmark's CPU-baseline leg, never by the library.  Written for
 * readability, not speed: every step follows the paper (or the cited
 * construction) in its own order.
 *
 * Conventions fixed here (the paper leaves them open):
 *   * 16-byte blocks are (lo, hi) = little-endian u64 of bytes 0..7, 8..15.
 *   * PRG: H(s, j) = AES_K(s ^ J_j) ^ s ^ J_j, K = 00 01 .. 0f, J_j is the
 *     block whose byte 15 is j (j < 8) and every other byte 0.
 *   * Randomness: R(e, pi, c) = AES_{K_seed}(e u64 | pi u16 | c u16 | 0 u32),
 *     K_seed = the dealer's 16-byte seed (a 128-bit AES key, so the masks
 *     carry the security level of the threat model's Gen(1^lambda)).
 *   * DCF: Boyle et al. EUROCRYPT'21 comparison function f(x) = beta*[x < alpha],
 *     MSB-first over n bits, seeds with bits 0..1 of byte 0 cleared.
 */
#include "fss_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ========================================================================= */
/* AES-128 (FIPS-197)                                                        */
/* ========================================================================= */

static uint8_t SBOX[256];
static orc_aes_sched PRG_SCHED;

static uint8_t xtime(uint8_t a) { return (uint8_t)((a << 1) ^ ((a & 0x80) ? 0x1b : 0x00)); }

static uint8_t gf_mul(uint8_t a, uint8_t b) {
  uint8_t r = 0;
  while (b) {
    if (b & 1) r ^= a;
    a = xtime(a);
    b >>= 1;
  }
  return r;
}

static uint8_t rotl8(uint8_t x, int k) { return (uint8_t)((x << k) | (x >> (8 - k))); }

/* FIPS-197 Sec. 5.1.1: multiplicative inverse in GF(2^8) (0 maps to 0),
 * then the affine transformation with constant 0x63. */
static void build_sbox(void) {
  for (int a = 0; a < 256; a++) {
    uint8_t inv = 0;
    if (a) {
      /* a^254 = a^-1 in GF(2^8) */
      uint8_t r = 1, base = (uint8_t)a;
      int e = 254;
      while (e) {
        if (e & 1) r = gf_mul(r, base);
        base = gf_mul(base, base);
        e >>= 1;
      }
      inv = r;
    }
    SBOX[a] = (uint8_t)(inv ^ rotl8(inv, 1) ^ rotl8(inv, 2) ^ rotl8(inv, 3) ^ rotl8(inv, 4) ^ 0x63);
  }
}

void orc_sbox(uint8_t out[256]) { memcpy(out, SBOX, 256); }

/* FIPS-197 Sec. 5.2 key expansion, Nk = 4, Nr = 10. rk[4*i + j] = byte j of w[i]. */
void orc_aes128_expand(const uint8_t key[16], orc_aes_sched* ks) {
  uint8_t* w = ks->rk;
  memcpy(w, key, 16);
  uint8_t rcon = 0x01;
  for (int i = 4; i < 44; i++) {
    uint8_t t[4];
    memcpy(t, &w[4 * (i - 1)], 4);
    if (i % 4 == 0) {
      uint8_t t0 = t[0]; /* RotWord */
      t[0] = t[1]; t[1] = t[2]; t[2] = t[3]; t[3] = t0;
      for (int j = 0; j < 4; j++) t[j] = SBOX[t[j]]; /* SubWord */
      t[0] ^= rcon;
      rcon = xtime(rcon);
    }
    for (int j = 0; j < 4; j++) w[4 * i + j] = (uint8_t)(w[4 * (i - 4) + j] ^ t[j]);
  }
}

/* AES-128 blocks encrypted by the batched drivers' threads (for reporting
 * the oracle's block rate; no effect on any result). */
static _Thread_local uint64_t tl_aes_blocks;
static uint64_t g_aes_blocks;

/* FIPS-197 Sec. 5.1: state[r][c] = in[r + 4c]. */
void orc_aes128_encrypt(const orc_aes_sched* ks, const uint8_t in[16], uint8_t out[16]) {
  tl_aes_blocks++;
  uint8_t st[4][4];
  for (int c = 0; c < 4; c++)
    for (int r = 0; r < 4; r++) st[r][c] = in[r + 4 * c];

  for (int round = 0; round <= 10; round++) {
    if (round > 0) {
      /* SubBytes */
      for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++) st[r][c] = SBOX[st[r][c]];
      /* ShiftRows: row r rotates left by r */
      for (int r = 1; r < 4; r++) {
        uint8_t row[4];
        for (int c = 0; c < 4; c++) row[c] = st[r][(c + r) % 4];
        for (int c = 0; c < 4; c++) st[r][c] = row[c];
      }
      /* MixColumns (not in the final round) */
      if (round < 10) {
        for (int c = 0; c < 4; c++) {
          uint8_t a0 = st[0][c], a1 = st[1][c], a2 = st[2][c], a3 = st[3][c];
          st[0][c] = (uint8_t)(gf_mul(a0, 2) ^ gf_mul(a1, 3) ^ a2 ^ a3);
          st[1][c] = (uint8_t)(a0 ^ gf_mul(a1, 2) ^ gf_mul(a2, 3) ^ a3);
          st[2][c] = (uint8_t)(a0 ^ a1 ^ gf_mul(a2, 2) ^ gf_mul(a3, 3));
          st[3][c] = (uint8_t)(gf_mul(a0, 3) ^ a1 ^ a2 ^ gf_mul(a3, 2));
        }
      }
    }
    /* AddRoundKey */
    for (int c = 0; c < 4; c++)
      for (int r = 0; r < 4; r++) st[r][c] ^= ks->rk[16 * round + 4 * c + r];
  }
  for (int c = 0; c < 4; c++)
    for (int r = 0; r < 4; r++) out[r + 4 * c] = st[r][c];
}

void orc_aes128_encrypt_key(const uint8_t key[16], const uint8_t in[16], uint8_t out[16]) {
  orc_aes_sched ks;
  orc_aes128_expand(key, &ks);
  orc_aes128_encrypt(&ks, in, out);
}

__attribute__((constructor)) static void oracle_init(void) {
  build_sbox();
  uint8_t k[16];
  for (int i = 0; i < 16; i++) k[i] = (uint8_t)i;
  orc_aes128_expand(k, &PRG_SCHED);
}

/* ========================================================================= */
/* Blocks, PRG, randomness                                                   */
/* ========================================================================= */

static void blk_to_bytes(orc_blk b, uint8_t out[16]) {
  for (int i = 0; i < 8; i++) {
    out[i] = (uint8_t)(b.lo >> (8 * i));
    out[8 + i] = (uint8_t)(b.hi >> (8 * i));
  }
}

static orc_blk bytes_to_blk(const uint8_t in[16]) {
  orc_blk b = {0, 0};
  for (int i = 0; i < 8; i++) {
    b.lo |= (uint64_t)in[i] << (8 * i);
    b.hi |= (uint64_t)in[8 + i] << (8 * i);
  }
  return b;
}

orc_blk orc_prg(orc_blk s, int j) {
  orc_blk x = s;
  x.hi ^= (uint64_t)(uint8_t)j << 56; /* byte 15 */
  uint8_t in[16], out[16];
  blk_to_bytes(x, in);
  orc_aes128_encrypt(&PRG_SCHED, in, out);
  orc_blk y = bytes_to_blk(out);
  y.lo ^= x.lo;
  y.hi ^= x.hi;
  return y;
}

void orc_seed_sched(const uint8_t seed[16], orc_aes_sched* ks) { orc_aes128_expand(seed, ks); }

orc_blk orc_rand(const orc_aes_sched* kseed, uint64_t e, int purpose, int ctr) {
  orc_blk x;
  x.lo = e;
  x.hi = (uint64_t)(uint16_t)purpose | ((uint64_t)(uint16_t)ctr << 16);
  uint8_t in[16], out[16];
  blk_to_bytes(x, in);
  orc_aes128_encrypt(kseed, in, out);
  return bytes_to_blk(out);
}

/* ========================================================================= */
/* DCF (Boyle, Chandran, Gilboa, Gupta, Ishai, Kumar, Rathee, EUROCRYPT'21)  */
/* ========================================================================= */
/* Group elements are uint64_t[ORC_MAXP].  p == 0 encodes Z_2 (value in g[0],
 * addition is XOR, negation is the identity); p >= 1 encodes Z_{2^64}^p.   */

static int glen(int p) { return p == 0 ? 1 : p; }

static void g_zero(int p, uint64_t* a) { for (int k = 0; k < glen(p); k++) a[k] = 0; }
static void g_add(int p, uint64_t* a, const uint64_t* b) {
  for (int k = 0; k < glen(p); k++) a[k] = (p == 0) ? (a[k] ^ b[k]) : (a[k] + b[k]);
}
static void g_sub(int p, uint64_t* a, const uint64_t* b) {
  for (int k = 0; k < glen(p); k++) a[k] = (p == 0) ? (a[k] ^ b[k]) : (a[k] - b[k]);
}
/* a = (-1)^t * a */
static void g_sign(int p, int t, uint64_t* a) {
  if (p == 0 || !t) return;
  for (int k = 0; k < p; k++) a[k] = (uint64_t)0 - a[k];
}

static orc_blk clear2(orc_blk s) { s.lo &= ~(uint64_t)3; return s; }

/* Child c of seed s: next seed, control bit t, and group value v. */
static void expand(int p, orc_blk s, int c, orc_blk* s_out, int* t_out, uint64_t* v_out) {
  orc_blk n = orc_prg(s, c);
  *t_out = (int)(n.lo & 1);
  *s_out = clear2(n);
  if (p == 0) {
    v_out[0] = (n.lo >> 1) & 1;
  } else {
    uint64_t w[4];
    orc_blk a = orc_prg(s, 2 + 2 * c);
    w[0] = a.lo; w[1] = a.hi;
    if (p > 2) { orc_blk b = orc_prg(s, 3 + 2 * c); w[2] = b.lo; w[3] = b.hi; }
    for (int k = 0; k < p; k++) v_out[k] = w[k];
  }
}

/* Convert(s) at the leaves. */
static void convert(int p, orc_blk s, uint64_t* out) {
  if (p == 0) {
    out[0] = (s.lo >> 2) & 1;
  } else {
    uint64_t w[4];
    orc_blk a = orc_prg(s, 6);
    w[0] = a.lo; w[1] = a.hi;
    if (p > 2) { orc_blk b = orc_prg(s, 7); w[2] = b.lo; w[3] = b.hi; }
    for (int k = 0; k < p; k++) out[k] = w[k];
  }
}

void orc_dcf_gen(int n, int p, uint64_t alpha, const uint64_t* beta,
                 orc_blk root0, orc_blk root1, orc_dcf_key* k0, orc_dcf_key* k1) {
  memset(k0, 0, sizeof *k0);
  memset(k1, 0, sizeof *k1);
  k0->n = k1->n = n;
  k0->p = k1->p = p;
  orc_blk s[2] = {clear2(root0), clear2(root1)};
  int t[2] = {0, 1};
  k0->root = s[0];
  k1->root = s[1];
  uint64_t Va[ORC_MAXP];
  g_zero(p, Va);

  for (int i = 0; i < n; i++) {
    int ai = (int)((alpha >> (n - 1 - i)) & 1);
    orc_blk sc[2][2];          /* [party][child] */
    int tc[2][2];
    uint64_t vc[2][2][ORC_MAXP];
    for (int b = 0; b < 2; b++)
      for (int c = 0; c < 2; c++) expand(p, s[b], c, &sc[b][c], &tc[b][c], vc[b][c]);
    int keep = ai, lose = 1 - ai;   /* child 0 = L, child 1 = R */

    orc_blk scw;
    scw.lo = sc[0][lose].lo ^ sc[1][lose].lo;
    scw.hi = sc[0][lose].hi ^ sc[1][lose].hi;

    /* V_CW = (-1)^{t1} (v1^Lose - v0^Lose - V_alpha) [+ (-1)^{t1} beta if Lose = L] */
    uint64_t vcw[ORC_MAXP], tmp[ORC_MAXP];
    memcpy(vcw, vc[1][lose], sizeof vcw);
    g_sub(p, vcw, vc[0][lose]);
    g_sub(p, vcw, Va);
    g_sign(p, t[1], vcw);
    if (lose == 0) {
      memcpy(tmp, beta, sizeof(uint64_t) * glen(p));
      g_sign(p, t[1], tmp);
      g_add(p, vcw, tmp);
    }
    /* V_alpha = V_alpha - v1^Keep + v0^Keep + (-1)^{t1} V_CW */
    g_sub(p, Va, vc[1][keep]);
    g_add(p, Va, vc[0][keep]);
    memcpy(tmp, vcw, sizeof tmp);
    g_sign(p, t[1], tmp);
    g_add(p, Va, tmp);

    int tlcw = tc[0][0] ^ tc[1][0] ^ ai ^ 1;
    int trcw = tc[0][1] ^ tc[1][1] ^ ai;
    int tkeep = keep ? trcw : tlcw;

    k0->scw[i] = k1->scw[i] = scw;
    k0->tl[i] = k1->tl[i] = (uint8_t)tlcw;
    k0->tr[i] = k1->tr[i] = (uint8_t)trcw;
    for (int k = 0; k < glen(p); k++) k0->vcw[i][k] = k1->vcw[i][k] = vcw[k];

    for (int b = 0; b < 2; b++) {
      orc_blk ns = sc[b][keep];
      if (t[b]) { ns.lo ^= scw.lo; ns.hi ^= scw.hi; }
      int nt = tc[b][keep] ^ (t[b] & tkeep);
      s[b] = ns;
      t[b] = nt;
    }
  }
  /* CW^(n+1) = (-1)^{t1} (Convert(s1) - Convert(s0) - V_alpha) */
  uint64_t c0[ORC_MAXP], c1[ORC_MAXP];
  convert(p, s[0], c0);
  convert(p, s[1], c1);
  g_sub(p, c1, c0);
  g_sub(p, c1, Va);
  g_sign(p, t[1], c1);
  for (int k = 0; k < glen(p); k++) k0->fin[k] = k1->fin[k] = c1[k];
}

void orc_dcf_eval(int b, const orc_dcf_key* k, uint64_t x, uint64_t* out) {
  int n = k->n, p = k->p;
  orc_blk s = k->root;
  int t = b;
  uint64_t V[ORC_MAXP], tmp[ORC_MAXP];
  g_zero(p, V);
  for (int i = 0; i < n; i++) {
    int xi = (int)((x >> (n - 1 - i)) & 1);
    orc_blk ns;
    int nt;
    uint64_t v[ORC_MAXP];
    expand(p, s, xi, &ns, &nt, v);
    if (t) {
      ns.lo ^= k->scw[i].lo;
      ns.hi ^= k->scw[i].hi;
      nt ^= xi ? k->tr[i] : k->tl[i];
      g_add(p, v, k->vcw[i]);   /* v + t * V_CW, with the parent's t */
    }
    memcpy(tmp, v, sizeof tmp);
    g_sign(p, b, tmp);
    g_add(p, V, tmp);
    s = ns;
    t = nt;
  }
  convert(p, s, tmp);
  if (t) g_add(p, tmp, k->fin);
  g_sign(p, b, tmp);
  g_add(p, V, tmp);
  for (int q = 0; q < glen(p); q++) out[q] = V[q];
}

/* ========================================================================= */
/* Z_2 DCF with early termination: the tree stops nu = min(7, n) levels      */
/* above the leaves and each leaf seed is converted into a 128-bit vector    */
/* whose bit j is that leaf's output at the low input bits j (the            */
/* early-termination idea of Boyle, Gilboa and Ishai's DPF, applied to the   */
/* comparison).                                                              */
/* ========================================================================= */

static int leaf_bit(orc_blk b, unsigned j) { return (int)((j < 64 ? b.lo >> j : b.hi >> (j - 64)) & 1); }

/* The leaf conversion: the seed's expansion under tweak 2 (children use 0, 1). */
static orc_blk convert_leaf(orc_blk s) { return orc_prg(s, 2); }

int orc_dcfz_nu(int n) { return n < 7 ? n : 7; }

void orc_dcfz_gen(int n, uint64_t alpha, orc_blk root0, orc_blk root1, orc_dcfz_key* k0, orc_dcfz_key* k1) {
  memset(k0, 0, sizeof *k0);
  memset(k1, 0, sizeof *k1);
  const int nu = orc_dcfz_nu(n), h = n - nu;
  k0->n = k1->n = n;
  k0->nu = k1->nu = nu;
  /* The top h levels are the textbook construction (Z_2, beta = 1) over the
   * high bits alpha >> nu: the same steps as orc_dcf_gen with p = 0. */
  const uint64_t ah = alpha >> nu, al = alpha & (((uint64_t)1 << nu) - 1);
  orc_blk s[2] = {clear2(root0), clear2(root1)};
  int t[2] = {0, 1};
  k0->root = s[0];
  k1->root = s[1];
  int Va = 0;
  for (int i = 0; i < h; i++) {
    int ai = (int)((ah >> (h - 1 - i)) & 1);
    orc_blk sc[2][2];
    int tc[2][2];
    uint64_t vc[2][2][ORC_MAXP];
    for (int b = 0; b < 2; b++)
      for (int c = 0; c < 2; c++) expand(0, s[b], c, &sc[b][c], &tc[b][c], vc[b][c]);
    int keep = ai, lose = 1 - ai;
    orc_blk scw;
    scw.lo = sc[0][lose].lo ^ sc[1][lose].lo;
    scw.hi = sc[0][lose].hi ^ sc[1][lose].hi;
    int vcw = (int)(vc[1][lose][0] ^ vc[0][lose][0]) ^ Va ^ (lose == 0 ? 1 : 0);
    Va ^= (int)(vc[1][keep][0] ^ vc[0][keep][0]) ^ vcw;
    int tlcw = tc[0][0] ^ tc[1][0] ^ ai ^ 1;
    int trcw = tc[0][1] ^ tc[1][1] ^ ai;
    int tkeep = keep ? trcw : tlcw;
    k0->scw[i] = k1->scw[i] = scw;
    k0->tl[i] = k1->tl[i] = (uint8_t)tlcw;
    k0->tr[i] = k1->tr[i] = (uint8_t)trcw;
    k0->vcw[i] = k1->vcw[i] = (uint8_t)vcw;
    for (int b = 0; b < 2; b++) {
      orc_blk ns = sc[b][keep];
      if (t[b]) { ns.lo ^= scw.lo; ns.hi ^= scw.hi; }
      t[b] = tc[b][keep] ^ (t[b] & tkeep);
      s[b] = ns;
    }
  }
  /* At alpha's leaf exactly one party adds the correction (t_0 ^ t_1 = 1), so
   * the two leaves XOR to Conv(s_0) ^ Conv(s_1) ^ CW.  Choose CW so that this
   * is the vector (1[j < alpha_low])_j, with V_alpha (the parties' path sums,
   * which differ by V_alpha) cancelled in every bit. */
  orc_blk c0 = convert_leaf(s[0]), c1 = convert_leaf(s[1]), cw;
  cw.lo = c0.lo ^ c1.lo;
  cw.hi = c0.hi ^ c1.hi;
  for (unsigned j = 0; j < 128; j++) {
    int m = (j < al) ^ Va;
    if (!m) continue;
    if (j < 64) cw.lo ^= (uint64_t)1 << j;
    else cw.hi ^= (uint64_t)1 << (j - 64);
  }
  k0->leaf = k1->leaf = cw;
}

int orc_dcfz_eval(int b, const orc_dcfz_key* k, uint64_t x) {
  const int nu = k->nu, h = k->n - nu;
  const uint64_t xh = x >> nu;
  const unsigned xl = (unsigned)(x & (((uint64_t)1 << nu) - 1));
  orc_blk s = k->root;
  int t = b, V = 0;
  for (int i = 0; i < h; i++) {
    int xi = (int)((xh >> (h - 1 - i)) & 1);
    orc_blk ns;
    int nt;
    uint64_t v[ORC_MAXP];
    expand(0, s, xi, &ns, &nt, v);
    int vb = (int)v[0];
    if (t) {
      ns.lo ^= k->scw[i].lo;
      ns.hi ^= k->scw[i].hi;
      nt ^= xi ? k->tr[i] : k->tl[i];
      vb ^= k->vcw[i];
    }
    V ^= vb;
    s = ns;
    t = nt;
  }
  orc_blk leaf = convert_leaf(s);
  if (t) {
    leaf.lo ^= k->leaf.lo;
    leaf.hi ^= k->leaf.hi;
  }
  return V ^ leaf_bit(leaf, xl);
}

/* ========================================================================= */
/* DCF with 2^r children per level: r input bits (one base-2^r digit) per    */
/* level, the per-child form of the corrections above.                       */
/* ========================================================================= */

/* Child c (0..2^r-1) of seed s: next seed and control bit from H(s, c); its
 * value (Z_2: bit 1 of that block; Z_{2^64}^p: words c p .. c p + p - 1 of the
 * stream H(s, 2^r),
 * H(s, 2^r + 1), ..., two words per block, lo first), so the 2^r children
 * of one seed use ceil(2^r p / 2) value blocks between them. */
static void expand_r(int r, int p, orc_blk s, int c, orc_blk* s_out, int* t_out, uint64_t* v_out) {
  orc_blk n = orc_prg(s, c);
  *t_out = (int)(n.lo & 1);
  *s_out = clear2(n);
  if (p == 0) {  /* Z_2 payload: bit 1 of the seed block */
    v_out[0] = (n.lo >> 1) & 1;
    return;
  }
  for (int k = 0; k < p; k++) {
    const int w = c * p + k;
    const orc_blk b = orc_prg(s, (1 << r) + (w >> 1));
    v_out[k] = (w & 1) ? b.hi : b.lo;
  }
}

/* Base-2^r digit i (most significant first) of x over `levels` digits. */
static int digit_r(int r, uint64_t x, int levels, int i) {
  return (int)((x >> (r * (levels - 1 - i))) & (((uint64_t)1 << r) - 1));
}

void orc_dcfr_gen(int n, int r, int p, uint64_t alpha, const uint64_t* beta, orc_blk root0, orc_blk root1,
                  const orc_blk* keep_rand, orc_dcfr_key* k0, orc_dcfr_key* k1) {
  memset(k0, 0, sizeof *k0);
  memset(k1, 0, sizeof *k1);
  k0->n = k1->n = n;
  k0->p = k1->p = p;
  k0->r = k1->r = r;
  const int levels = (n + r - 1) / r, nr = 1 + (p + 1) / 2, C = 1 << r;
  orc_blk s[2] = {clear2(root0), clear2(root1)};
  int t[2] = {0, 1};
  k0->root = s[0];
  k1->root = s[1];
  uint64_t Va[ORC_MAXP];
  g_zero(p, Va);

  for (int i = 0; i < levels; i++) {
    const int a = digit_r(r, alpha, levels, i);   /* the child on alpha's path */
    orc_blk sc[2][ORC_MAXC];
    int tc[2][ORC_MAXC];
    uint64_t vc[2][ORC_MAXC][ORC_MAXP];
    for (int b = 0; b < 2; b++)
      for (int c = 0; c < C; c++) expand_r(r, p, s[b], c, &sc[b][c], &tc[b][c], vc[b][c]);
    const orc_blk* kr = keep_rand + (size_t)i * nr;
    const int last = (i == levels - 1);
    for (int c = 0; c < C; c++) {
      orc_blk scw;
      uint64_t vcw[ORC_MAXP];
      /* Below the last level nothing is walked: there every child, alpha's
       * included, takes the equalising value correction (alpha's without
       * beta), which brings the reconstructed sum at x = alpha to zero, so no
       * leaf conversion or final correction is needed; the last level's seed
       * and control-bit corrections would never be used and are zero. */
      if (c != a || last) {
        /* the parties' children become equal: seeds, control bits and, for
         * the value, V_CW = (-1)^{t1} (v1^c - v0^c - V_alpha [+ beta if c < a]) */
        scw.lo = sc[0][c].lo ^ sc[1][c].lo;
        scw.hi = sc[0][c].hi ^ sc[1][c].hi;
        memcpy(vcw, vc[1][c], sizeof vcw);
        g_sub(p, vcw, vc[0][c]);
        g_sub(p, vcw, Va);
        if (c < a) g_add(p, vcw, beta);
        g_sign(p, t[1], vcw);
      } else {
        /* random corrections on alpha's child hide which child it is; with
         * p = 0 (one block per level) the value bit is bit 1 of that block */
        scw = clear2(kr[0]);
        g_zero(p, vcw);
        if (p == 0) {
          vcw[0] = (kr[0].lo >> 1) & 1;
        } else {
          uint64_t w[4] = {kr[1].lo, kr[1].hi, nr > 2 ? kr[2].lo : 0, nr > 2 ? kr[2].hi : 0};
          for (int k = 0; k < p; k++) vcw[k] = w[k];
        }
      }
      const int tcw = last ? 0 : tc[0][c] ^ tc[1][c] ^ (c == a);
      if (last) scw.lo = scw.hi = 0;
      k0->scw[i][c] = k1->scw[i][c] = scw;
      k0->tcw[i][c] = k1->tcw[i][c] = (uint8_t)tcw;
      for (int k = 0; k < glen(p); k++) k0->vcw[i][c][k] = k1->vcw[i][c][k] = vcw[k];
    }
    /* V_alpha = V_alpha - v1^a + v0^a + (-1)^{t1} V_CW^a */
    uint64_t tmp[ORC_MAXP];
    g_sub(p, Va, vc[1][a]);
    g_add(p, Va, vc[0][a]);
    memcpy(tmp, k0->vcw[i][a], sizeof tmp);
    g_sign(p, t[1], tmp);
    g_add(p, Va, tmp);
    for (int b = 0; b < 2; b++) {
      orc_blk ns = sc[b][a];
      if (t[b]) { ns.lo ^= k0->scw[i][a].lo; ns.hi ^= k0->scw[i][a].hi; }
      const int nt = tc[b][a] ^ (t[b] & k0->tcw[i][a]);
      s[b] = ns;
      t[b] = nt;
    }
  }
}

void orc_dcfr_eval(int b, const orc_dcfr_key* k, uint64_t x, uint64_t* out) {
  const int p = k->p, r = k->r, levels = (k->n + k->r - 1) / k->r;
  orc_blk s = k->root;
  int t = b;
  uint64_t V[ORC_MAXP], tmp[ORC_MAXP];
  g_zero(p, V);
  for (int i = 0; i < levels; i++) {
    const int d = digit_r(r, x, levels, i);
    orc_blk ns;
    int nt;
    uint64_t v[ORC_MAXP];
    expand_r(r, p, s, d, &ns, &nt, v);
    if (t) {
      ns.lo ^= k->scw[i][d].lo;
      ns.hi ^= k->scw[i][d].hi;
      nt ^= k->tcw[i][d];
      g_add(p, v, k->vcw[i][d]);   /* v + t * V_CW^d, with the parent's t */
    }
    memcpy(tmp, v, sizeof tmp);
    g_sign(p, b, tmp);
    g_add(p, V, tmp);
    s = ns;
    t = nt;
  }
  for (int q = 0; q < glen(p); q++) out[q] = V[q];
}

/* ========================================================================= */
/* Operator specification                                                    */
/* ========================================================================= */

static int64_t clamp_ceil(double v, int64_t lo, int64_t hi) {
  double c = ceil(v);
  if (c <= (double)lo) return lo;
  if (c >= (double)hi) return hi;
  return (int64_t)c;
}

static int find_or_add_view(orc_spec* S, int k, uint64_t c) {
  for (int v = 0; v < S->n_views; v++)
    if (S->view_k[v] == k && S->view_c[v] == c) return v;
  if (S->n_views >= ORC_MAXPRED) return -1;
  S->view_k[S->n_views] = k;
  S->view_c[S->n_views] = c;
  return S->n_views++;
}

/* Predicates (Definition "Operator specification", item 3): quantise at f
 * fractional bits, map each to a view and a threshold in view space (the
 * masked rewrites of the comparison, low-bit and MSB lemmas), fold the
 * sentinels into constants, and list the atoms in descriptor order. */
static int compile_preds(orc_spec* S, const orc_pred* pr, int32_t n_pred, int f) {
  const int n = S->n;
  const int64_t N = (int64_t)1 << n, s = N / 2;
  S->n_user = n_pred;
  S->ell = 0;
  for (int j = 0; j < n_pred; j++) {
    const orc_pred* q = &pr[j];
    if (q->out < 0 || q->out >= ORC_MAXL) return -2;
    if (q->out + 1 > S->ell) S->ell = q->out + 1;
    int k = n;
    uint64_t c = 0, bprime = 0;
    int flip = q->negate ? 1 : 0;
    S->u_kind[j] = q->kind;
    S->u_out[j] = q->out;
    S->u_neg[j] = flip;
    switch (q->kind) {
      case ORC_LT_SIGNED: {        /* x <_s beta  ==  view_{n,s}(x) < beta + s */
        if (isnan(q->thr)) return -1;
        int64_t beta = clamp_ceil(ldexp(q->thr, f), -s, s);
        S->u_beta[j] = beta;
        c = (uint64_t)s;
        bprime = (uint64_t)(beta + s);
        break;
      }
      case ORC_LT_UNSIGNED: {      /* rep(x) < beta */
        if (isnan(q->thr)) return -1;
        int64_t beta = clamp_ceil(ldexp(q->thr, f), 0, N);
        S->u_beta[j] = beta;
        bprime = (uint64_t)beta;
        break;
      }
      case ORC_LOWBITS_LT: {       /* (x mod 2^fb) < gamma */
        if (q->f_bits < 1 || q->f_bits > n) return -2;
        if (q->gamma < 0 || q->gamma > ((int64_t)1 << q->f_bits)) return -1;
        k = q->f_bits;
        S->u_f[j] = k;
        S->u_beta[j] = q->gamma;
        bprime = (uint64_t)q->gamma;
        break;
      }
      case ORC_MSB_SHIFT: {        /* MSB(x + c) == NOT [view_{n,c}(x) < 2^(n-1)] */
        c = (uint64_t)q->c & (uint64_t)(N - 1);
        S->u_c[j] = c;
        bprime = (uint64_t)s;
        flip ^= 1;
        break;
      }
      default:
        return -2;
    }
    S->negate[q->out] ^= (uint8_t)flip;
    if (bprime == 0) continue;                     /* sentinel: constant 0 */
    if (bprime == ((uint64_t)1 << k)) {            /* sentinel: constant 1 */
      S->negate[q->out] ^= 1;
      continue;
    }
    int v = find_or_add_view(S, k, c);
    if (v < 0) return -2;
    int t = S->n_prim++;
    S->prim_k[t] = k;
    S->prim_view[t] = v;
    S->prim_out[t] = q->out;
    S->prim_bprime[t] = bprime;
  }
  /* The mask query of the lookup's own view, 1[v < r_n] with v = (xhat +
   * lookup_c) mod 2^n, is the comparison the lookup DCF evaluates at v with
   * payload rho (rho_0 = 1): additive shares of that bit, reduced mod 2, are
   * XOR shares of it.  That view gets no mask atom. */
  S->lookup_view = -1;
  for (int v = 0; v < S->n_views; v++)
    if (S->view_k[v] == n && S->view_c[v] == S->lookup_c) S->lookup_view = v;
  S->T = S->n_prim + S->n_views - (S->lookup_view >= 0 ? 1 : 0);
  if (S->T > ORC_MAXT) return -2;
  return 0;
}

/* The atom of view v's mask query (-1: answered by the lookup), and the view
 * of mask atom t >= n_prim. */
static int mask_atom(const orc_spec* S, int v) {
  if (v == S->lookup_view) return -1;
  return S->n_prim + v - (S->lookup_view >= 0 && v > S->lookup_view ? 1 : 0);
}
static int mask_view(const orc_spec* S, int t) {
  const int v = t - S->n_prim;
  return S->lookup_view >= 0 && v >= S->lookup_view ? v + 1 : v;
}

int orc_spec_compile(const orc_interval* iv, int32_t m, const orc_piece* pc,
                     const orc_pred* pr, int32_t n_pred, int32_t n_bits,
                     int32_t frac_bits, int32_t out_frac_bits, orc_spec* S) {
  memset(S, 0, sizeof *S);
  if (n_bits < 2 || n_bits > ORC_MAXN) return -2;
  if (frac_bits < 0 || frac_bits >= n_bits) return -2;
  if (m < 1 || m > ORC_MAXM) return -1;
  if (n_pred < 0 || n_pred > ORC_MAXPRED) return -2;
  const int n = n_bits, f = frac_bits;
  const int64_t N = (int64_t)1 << n, s = N / 2;
  S->n = n; S->f = f; S->m = m;
  S->lookup_r = 3;
  S->lookup_c = (uint64_t)s; /* signed order: offset-binary view of the lookup */

  /* Partition: contiguous half-open real intervals, tails at -inf / +inf. */
  if (!(isinf(iv[0].lo) && iv[0].lo < 0)) return -1;
  if (!(isinf(iv[m - 1].hi) && iv[m - 1].hi > 0)) return -1;
  for (int i = 0; i < m; i++)
    if (!(iv[i].lo < iv[i].hi)) return -1;
  for (int i = 0; i + 1 < m; i++)
    if (iv[i].hi != iv[i + 1].lo) return -1;
  S->alpha[0] = -s;
  S->alpha[m] = s;
  /* Real boundary a maps to ceil(a 2^f): the integers whose real value is >= a. */
  for (int i = 1; i < m; i++) S->alpha[i] = clamp_ceil(ldexp(iv[i].lo, f), -s, s);
  for (int i = 1; i <= m; i++)
    if (!(S->alpha[i - 1] < S->alpha[i])) return -1;
  for (int i = 0; i <= m; i++) S->aprime[i] = (uint64_t)(S->alpha[i] + s);

  /* Pieces: coefficient a_l scaled by 2^(F_out - l f), ties to even. */
  int d = 0;
  for (int i = 0; i < m; i++) {
    if (pc[i].degree < 0 || pc[i].degree > 3) return -1;
    if (pc[i].degree > d) d = pc[i].degree;
  }
  S->d = d;
  S->p = d + 1;
  S->F_out = out_frac_bits >= 0 ? out_frac_bits : (d <= 1 ? 2 * f : 4 * f);
  for (int i = 0; i < m; i++) {
    double X = fmax(fabs((double)S->alpha[i]), fabs((double)(S->alpha[i + 1] - 1)));
    double bound = 0;
    for (int l = 0; l <= d; l++) {
      double a = (l <= pc[i].degree) ? pc[i].coef[l] : 0.0;
      double q = nearbyint(ldexp(a, S->F_out - l * f));
      if (!(fabs(q) < 9223372036854775808.0)) return -1; /* also rejects NaN */
      S->coef[i][l] = (uint64_t)(int64_t)q;
      bound += fabs(q) * pow(X, l);
    }
    if (!(bound < 4611686018427387904.0)) return -1; /* |P_i(x)| < 2^62 on I_i */
  }

  return compile_preds(S, pr, n_pred, f);
}

/* The Definition's own form: integer boundaries 0 = alpha_0 < ... < alpha_m = 2^n
 * over canonical representatives {0, .., 2^n - 1} and ring coefficients (the
 * polynomials are evaluated in Z_{2^64}, at the input's 64-bit value).  The
 * lookup therefore uses the unshifted view xhat mod 2^n; predicate thresholds
 * are integers (fractional bits 0). */
int orc_spec_compile_int(int32_t n_bits, int32_t m, const uint64_t* alpha, int32_t degree,
                         const uint64_t* coef, const orc_pred* pr, int32_t n_pred, orc_spec* S) {
  memset(S, 0, sizeof *S);
  if (n_bits < 2 || n_bits > ORC_MAXN) return -2;
  if (m < 1 || m > ORC_MAXM) return -1;
  if (degree < 0 || degree > 3) return -1;
  if (n_pred < 0 || n_pred > ORC_MAXPRED) return -2;
  const uint64_t N = (uint64_t)1 << n_bits;
  if (alpha[0] != 0 || alpha[m] != N) return -1;
  for (int i = 1; i <= m; i++)
    if (!(alpha[i - 1] < alpha[i])) return -1;
  for (int j = 0; j < n_pred; j++)
    if ((pr[j].kind == ORC_LT_SIGNED || pr[j].kind == ORC_LT_UNSIGNED) && pr[j].thr != floor(pr[j].thr))
      return -1;
  S->n = n_bits; S->f = 0; S->m = m; S->d = degree; S->p = degree + 1; S->F_out = 0;
  S->lookup_r = 3;
  S->is_int = 1;
  S->lookup_c = 0;
  for (int i = 0; i <= m; i++) {
    S->alpha[i] = (int64_t)alpha[i];
    S->aprime[i] = alpha[i];
  }
  for (int i = 0; i < m; i++)
    for (int l = 0; l <= degree; l++) S->coef[i][l] = coef[i * (degree + 1) + l];
  return compile_preds(S, pr, n_pred, 0);
}

/* ========================================================================= */
/* Dealer key generation for one element                                     */
/* ========================================================================= */

static uint64_t lowmask(int k) { return k >= 64 ? ~(uint64_t)0 : (((uint64_t)1 << k) - 1); }

void orc_keygen_elem(const orc_spec* S, const orc_aes_sched* kseed, uint64_t e,
                     orc_elem_key* k0, orc_elem_key* k1, uint64_t* r_in_out, uint64_t* r_out_out) {
  /* Masks and the output-mask sharing. */
  orc_blk r0 = orc_rand(kseed, e, 0, 0);
  uint64_t r_in = r0.lo, r_out = r0.hi;
  orc_blk r1 = orc_rand(kseed, e, 1, 0);
  k0->rout = r1.lo;
  k1->rout = r_out - r1.lo;

  /* Packed comparison: one Z_2 DCF per atom.  Threshold atoms follow the
   * masked rewrite 1[x' < b'] = 1[v < theta] ^ 1[v < r_k] ^ w with
   * theta = (r_k + b') mod 2^k and w = 1[r_k + b' >= 2^k]. */
  uint64_t wout = 0;
  for (int t = 0; t < S->T; t++) {
    int k;
    uint64_t alpha;
    if (t < S->n_prim) {
      k = S->prim_k[t];
      uint64_t rk = r_in & lowmask(k);
      uint64_t sum = rk + S->prim_bprime[t];
      alpha = sum & lowmask(k);
      if (sum >> k) wout ^= (uint64_t)1 << S->prim_out[t];
    } else {
      k = S->view_k[mask_view(S, t)];
      alpha = r_in & lowmask(k);
    }
    orc_blk a = orc_rand(kseed, e, 2 + 2 * t, 0);
    orc_blk b = orc_rand(kseed, e, 3 + 2 * t, 0);
    orc_dcfz_gen(k, alpha, a, b, &k0->atom[t], &k1->atom[t]);
  }
  uint64_t W = orc_rand(kseed, e, 66, 0).lo & lowmask(S->ell);
  k0->wshare = W;
  k1->wshare = W ^ wout;

  /* Interval lookup: one vector DCF at alpha = r_in mod 2^n with payload
   * rho = ((-r_in)^k)_{k<p}, plus additive shares of rho. */
  uint64_t rho[ORC_MAXP];
  rho[0] = 1;
  for (int k = 1; k < S->p; k++) rho[k] = rho[k - 1] * ((uint64_t)0 - r_in);
  orc_blk c0 = orc_rand(kseed, e, 64, 0);
  orc_blk c1 = orc_rand(kseed, e, 65, 0);
  /* the on-path child's corrections at level i < L - 1: R(e, 69 + k, i) */
  orc_blk kr[ORC_MAXLR * 3];
  memset(kr, 0, sizeof kr);
  const int levels = (S->n + S->lookup_r - 1) / S->lookup_r, nr = 1 + (S->p + 1) / 2;
  for (int i = 0; i + 1 < levels; i++)
    for (int k = 0; k < nr; k++) kr[i * nr + k] = orc_rand(kseed, e, 69 + k, i);
  orc_dcfr_gen(S->n, S->lookup_r, S->p, r_in & lowmask(S->n), rho, c0, c1, kr, &k0->coeff, &k1->coeff);
  orc_blk ra = orc_rand(kseed, e, 67, 0), rb = orc_rand(kseed, e, 68, 0);
  uint64_t sh[4] = {ra.lo, ra.hi, rb.lo, rb.hi};
  for (int k = 0; k < S->p; k++) {
    k0->rho[k] = sh[k];
    k1->rho[k] = rho[k] - sh[k];
  }
  *r_in_out = r_in;
  *r_out_out = r_out;
}

/* ========================================================================= */
/* Evaluation by party b of one element at public xhat                       */
/* ========================================================================= */

static uint64_t binom(int l, int j) {
  uint64_t r = 1;
  for (int i = 0; i < j; i++) r = r * (uint64_t)(l - i) / (uint64_t)(i + 1);
  return r;
}

void orc_eval_elem(int b, const orc_spec* S, const orc_elem_key* K, uint64_t xhat,
                   uint64_t* y_out, uint64_t* z_out) {
  /* The lookup DCF at v = view_{n,c}(xhat) (c = 2^(n-1) for the signed
   * order of real specs, 0 for the canonical order of integer specs): shares
   * of rho 1[v < r_n]. */
  const int n = S->n, m = S->m, p = S->p, d = S->d;
  const uint64_t N = (uint64_t)1 << n;
  uint64_t v = ((xhat & (N - 1)) + S->lookup_c) & (N - 1);
  uint64_t Dv[ORC_MAXP];
  orc_dcfr_eval(b, &K->coeff, v, Dv);

  /* Call 1: packed comparison.  Atom t is evaluated at view_{k,c}(xhat); the
   * lookup view's mask query is the low bit of this party's share of D(v)_0. */
  int A[ORC_MAXT];
  for (int t = 0; t < S->T; t++) {
    int vi = (t < S->n_prim) ? S->prim_view[t] : mask_view(S, t);
    int k = S->view_k[vi];
    uint64_t u = ((xhat & lowmask(k)) + S->view_c[vi]) & lowmask(k);
    A[t] = orc_dcfz_eval(b, &K->atom[t], u);
  }
  uint64_t z = K->wshare;
  if (b == 0)
    for (int j = 0; j < S->ell; j++) z ^= (uint64_t)S->negate[j] << j;
  for (int t = 0; t < S->n_prim; t++) {
    const int ma = mask_atom(S, S->prim_view[t]);
    int bit = A[t] ^ (ma < 0 ? (int)(Dv[0] & 1) : A[ma]);
    z ^= (uint64_t)bit << S->prim_out[t];
  }

  /* Call 2: interval lookup.  With x' = (v - r_n) mod N, for each interior
   * boundary a'_i:
   *   1[x' < a'_i] = 1[(v - a'_i) mod N < r_n] - 1[v < r_n] + 1[v < a'_i],
   * so g_i = D(u_i) - D(v) + 1[v < a'_i] rho_b shares 1[x' < a'_i] rho. */
  uint64_t g[ORC_MAXM + 1][ORC_MAXP];
  for (int k = 0; k < p; k++) { g[0][k] = 0; g[m][k] = K->rho[k]; }
  for (int i = 1; i < m; i++) {
    uint64_t u = (v - S->aprime[i]) & (N - 1);
    uint64_t D[ORC_MAXP];
    orc_dcfr_eval(b, &K->coeff, u, D);
    for (int k = 0; k < p; k++)
      g[i][k] = D[k] - Dv[k] + (v < S->aprime[i] ? K->rho[k] : 0);
  }
  /* e_i shares 1[x in I_i] rho; the active piece's coefficients at xhat are
   * q_j = sum_l a_{i*,l} C(l,j) (-r_in)^(l-j). */
  uint64_t q[ORC_MAXP] = {0};
  for (int i = 0; i < m; i++) {
    for (int j = 0; j <= d; j++) {
      for (int l = j; l <= d; l++) {
        uint64_t e = g[i + 1][l - j] - g[i][l - j];
        q[j] += S->coef[i][l] * binom(l, j) * e;
      }
    }
  }
  q[0] += K->rout;
  /* Local combination at the public xhat. */
  uint64_t y = 0, xp = 1;
  for (int j = 0; j <= d; j++) {
    y += q[j] * xp;
    xp *= xhat;
  }
  *y_out = y;
  *z_out = z;
}

/* ========================================================================= */
/* Plaintext evaluation                                                      */
/* ========================================================================= */

void orc_plain_eval(const orc_spec* S, int64_t x, uint64_t* y_out, uint64_t* z_out) {
  const int n = S->n;
  const uint64_t N = (uint64_t)1 << n, s = N / 2;
  int is = 0;
  if (S->is_int) {
    const uint64_t rep = (uint64_t)x & (N - 1);
    while (is + 1 < S->m && rep >= S->aprime[is + 1]) is++;
  } else {
    while (is + 1 < S->m && x >= S->alpha[is + 1]) is++;
  }
  uint64_t y = 0, xp = 1;
  for (int l = 0; l <= S->d; l++) {
    y += S->coef[is][l] * xp;
    xp *= (uint64_t)x;
  }
  uint64_t z = 0;
  for (int j = 0; j < S->n_user; j++) {
    int bit = 0;
    switch (S->u_kind[j]) {
      case ORC_LT_SIGNED: bit = x < S->u_beta[j]; break;
      case ORC_LT_UNSIGNED: bit = (int64_t)((uint64_t)x & (N - 1)) < S->u_beta[j]; break;
      case ORC_LOWBITS_LT: bit = (int64_t)((uint64_t)x & lowmask(S->u_f[j])) < S->u_beta[j]; break;
      case ORC_MSB_SHIFT: bit = (((uint64_t)x + S->u_c[j]) & (N - 1)) >= s; break;
    }
    z ^= (uint64_t)(bit ^ S->u_neg[j]) << S->u_out[j];
  }
  *y_out = y;
  *z_out = z;
}

/* ========================================================================= */
/* Rescaling gate: arithmetic right shift of a masked 64-bit value           */
/* ========================================================================= */
/* Fixed-point rescaling by ARS (Sec. 3.2 encoding; the paper lists truncation
 * and ARS among the specification-compatible gates).  The input is the
 * opening yhat = y + r_in of a signed y with |y| < 2^62 (the bound every
 * compiled piece satisfies), masked by the previous gate's output mask r_in;
 * the output is shares of floor(y / 2^s) + r_out.  With u = y + 2^62 in
 * [0, 2^63) and uhat = yhat + 2^62 = u + r_in (mod 2^64):
 *   u >> s = (uhat >> s) - (r_in >> s) - c + 2^(64-s) w,
 *   c = 1[uhat mod 2^s < r_in mod 2^s]   (the borrow of the low s bits),
 *   w = 1[u + r_in >= 2^64] = MSB(r_in) (1 - MSB(uhat))   (as u < 2^63),
 * and floor(y / 2^s) = (u >> s) - 2^(62-s).  The borrow is a comparison of
 * the public uhat with the secret r_in over s bits: one DCF with payload -1 in
 * Z_{2^64} (the 2^r-children DCF above, p = 1) gives additive shares of -c
 * directly.  The dealer also shares k0 = r_out - (r_in >> s) and
 * k1 = 2^(64-s) MSB(r_in). */

uint64_t orc_ars(int64_t y, int s) { return (uint64_t)(y >> s); }

void orc_trunc_keygen_elem(int s, int r, const orc_aes_sched* kseed, uint64_t e, uint64_t r_in,
                           orc_trunc_key* k0, orc_trunc_key* k1, uint64_t* r_out_out) {
  const uint64_t r_out = orc_rand(kseed, e, 0, 0).lo;
  const uint64_t v0 = r_out - (r_in >> s);
  const uint64_t v1 = (r_in >> 63) ? (uint64_t)1 << (64 - s) : 0;
  const orc_blk sh = orc_rand(kseed, e, 1, 0);
  k0->k0 = sh.lo;
  k1->k0 = v0 - sh.lo;
  k0->k1 = sh.hi;
  k1->k1 = v1 - sh.hi;
  orc_blk c0 = orc_rand(kseed, e, 64, 0);
  orc_blk c1 = orc_rand(kseed, e, 65, 0);
  orc_blk kr[ORC_MAXLR * 3];
  memset(kr, 0, sizeof kr);
  const int levels = (s + r - 1) / r;
  for (int i = 0; i + 1 < levels; i++)
    for (int k = 0; k < 2; k++) kr[i * 2 + k] = orc_rand(kseed, e, 69 + k, i);
  const uint64_t beta = (uint64_t)0 - 1;
  orc_dcfr_gen(s, r, 1, r_in & lowmask(s), &beta, c0, c1, kr, &k0->dcf, &k1->dcf);
  *r_out_out = r_out;
}

uint64_t orc_trunc_eval_elem(int b, int s, const orc_trunc_key* K, uint64_t yhat) {
  const uint64_t uhat = yhat + ((uint64_t)1 << 62);
  uint64_t negc;
  orc_dcfr_eval(b, &K->dcf, uhat & lowmask(s), &negc);
  uint64_t z = K->k0 + (1 - (uhat >> 63)) * K->k1 + negc;
  if (b == 0) z += (uhat >> s) - ((uint64_t)1 << (62 - s));
  return z;
}

/* ========================================================================= */
/* Protocol "Compile a scalar gate instance", lookup part                    */
/* ========================================================================= */

/* The translated lookup partition of Definition "Interval lookup with vector
 * payload" as the compilation protocol builds it (step 1): in xhat space,
 * xhat = x + r mod N, interval I_i = [alpha_i, alpha_{i+1}) becomes the cyclic
 * range starting at (alpha_i + r) mod N.  Reading xhat upward from 0 meets the
 * intervals in cyclic order, beginning with the one that holds x = -r mod N;
 * that interval comes back at the top of the range, cut by the wrap point,
 * unless its translated start is 0.  A partition that was not cut is padded
 * to M = min(m + 1, N) intervals so that the shape does not depend on r: here
 * the last interval of length >= 2 loses its top value to a new interval
 * with the same payload index. */
int orc_protocol3(int n, const uint64_t* alpha, int m, uint64_t r, uint64_t* B, int32_t* ord) {
  const uint64_t N = (uint64_t)1 << n;
  const int M = (uint64_t)(m + 1) < N ? m + 1 : (int)N;
  r &= N - 1;
  const uint64_t x0 = (N - r) & (N - 1); /* the preimage of xhat = 0 */
  int first = 0;
  while (first + 1 < m && alpha[first + 1] <= x0) first++;
  int cnt = 0;
  B[0] = 0;
  ord[cnt++] = first;
  for (int k = 1; k < m; k++) { /* the other intervals, in cyclic order */
    const int i = (first + k) % m;
    B[cnt] = (alpha[i] + r) & (N - 1);
    ord[cnt++] = i;
  }
  const uint64_t top = (alpha[first] + r) & (N - 1);
  if (top != 0) { /* the first interval's upper part */
    B[cnt] = top;
    ord[cnt++] = first;
  }
  B[cnt] = N;
  if (cnt < M) { /* pad: split the last interval of length >= 2 below its end */
    int j = cnt - 1;
    while (j >= 0 && B[j + 1] - B[j] < 2) j--;
    if (j < 0) return -1;
    for (int q = cnt; q > j; q--) B[q + 1] = B[q];
    for (int q = cnt - 1; q > j; q--) ord[q + 1] = ord[q];
    B[j + 1] = B[j + 2] - 1;
    ord[j + 1] = ord[j];
    cnt++;
  }
  return cnt == M ? M : -1;
}

/* ========================================================================= */
/* Literal interval lookup: one vector DCF per inner boundary of the         */
/* translated partition (compilation protocol, steps (1) and (5))            */
/* ========================================================================= */

int orc_lit_keygen_elem(const orc_spec* S, const orc_aes_sched* kseed, uint64_t e, orc_lit_key* k0,
                        orc_lit_key* k1, uint64_t* r_in_out, uint64_t* r_out_out) {
  const int n = S->n, p = S->p, r = S->lookup_r;
  const orc_blk m0 = orc_rand(kseed, e, 0, 0);
  const uint64_t r_in = m0.lo, r_out = m0.hi;
  k0->rout = orc_rand(kseed, e, 1, 0).lo;
  k1->rout = r_out - k0->rout;
  k0->rin = orc_rand(kseed, e, 200, 0).lo;
  k1->rin = r_in - k0->rin;
  /* the partition of v-space: v = x' + r_in mod 2^n for x' in offset binary
   * (canonical for integer specs), whose boundaries are aprime */
  uint64_t B[ORC_MAXM + 2];
  int32_t ord[ORC_MAXM + 1];
  const int M = orc_protocol3(n, S->aprime, S->m, r_in & lowmask(n), B, ord);
  if (M < 1) return -1;
  k0->M = k1->M = M;
  const int levels = (n + r - 1) / r, nr = 1 + (p + 1) / 2;
  for (int j = 1; j < M; j++) {
    /* payload step at B_j: the piece below the boundary minus the piece above */
    uint64_t beta[ORC_MAXP];
    for (int k = 0; k < p; k++) beta[k] = S->coef[ord[j - 1]][k] - S->coef[ord[j]][k];
    orc_blk kr[ORC_MAXLR * 3];
    memset(kr, 0, sizeof kr);
    for (int i = 0; i + 1 < levels; i++)
      for (int k = 0; k < nr; k++) kr[i * nr + k] = orc_rand(kseed, e, 203 + k, 64 * j + i);
    orc_dcfr_gen(n, r, p, B[j], beta, orc_rand(kseed, e, 201, j), orc_rand(kseed, e, 202, j), kr, &k0->dcf[j - 1],
                 &k1->dcf[j - 1]);
  }
  const orc_blk sa = orc_rand(kseed, e, 210, 0), sb = orc_rand(kseed, e, 211, 0);
  const uint64_t sh[4] = {sa.lo, sa.hi, sb.lo, sb.hi};
  for (int k = 0; k < p; k++) {
    k0->base[k] = sh[k];
    k1->base[k] = S->coef[ord[M - 1]][k] - sh[k];
  }
  *r_in_out = r_in;
  *r_out_out = r_out;
  return 0;
}

void orc_lit_eval_elem(int b, const orc_spec* S, const orc_lit_key* K, uint64_t xhat, uint64_t* coef,
                       uint64_t* x_share) {
  const uint64_t v = (xhat + S->lookup_c) & lowmask(S->n);
  for (int k = 0; k < S->p; k++) coef[k] = K->base[k];
  for (int j = 1; j < K->M; j++) {
    uint64_t out[ORC_MAXP];
    orc_dcfr_eval(b, &K->dcf[j - 1], v, out);
    for (int k = 0; k < S->p; k++) coef[k] += out[k];
  }
  /* the output mask enters through the constant term: Horner's rule on these
   * shares then opens to P(x) + r_out */
  coef[0] += K->rout;
  *x_share = b == 0 ? xhat - K->rin : (uint64_t)0 - K->rin;
}

/* ========================================================================= */
/* Post-processing subprotocols over shares                                  */
/* ========================================================================= */

void orc_triple(const orc_aes_sched* kseed, uint64_t e, int step, uint64_t a[2], uint64_t b[2], uint64_t c[2]) {
  const orc_blk ab = orc_rand(kseed, e, 220, step), s0 = orc_rand(kseed, e, 221, step);
  const uint64_t cc = ab.lo * ab.hi;
  a[0] = s0.lo;
  a[1] = ab.lo - s0.lo;
  b[0] = s0.hi;
  b[1] = ab.hi - s0.hi;
  c[0] = orc_rand(kseed, e, 222, step).lo;
  c[1] = cc - c[0];
}

/* u v = (d + a)(e + b) = d e + d b + e a + a b */
uint64_t orc_beaver_mul(int party, uint64_t d, uint64_t e, uint64_t a, uint64_t b, uint64_t c) {
  uint64_t z = c + d * b + e * a;
  if (party == 0) z += d * e;
  return z;
}

void orc_and_triple(const orc_aes_sched* kseed, uint64_t w, int step, uint64_t a[2], uint64_t b[2], uint64_t c[2]) {
  const orc_blk ab = orc_rand(kseed, w, 230, step), s0 = orc_rand(kseed, w, 231, step);
  a[0] = s0.lo;
  a[1] = ab.lo ^ s0.lo;
  b[0] = s0.hi;
  b[1] = ab.hi ^ s0.hi;
  c[0] = orc_rand(kseed, w, 232, step).lo;
  c[1] = (ab.lo & ab.hi) ^ c[0];
}

/* x & y = (d ^ a) & (e ^ b) = (d & e) ^ (d & b) ^ (e & a) ^ (a & b) */
uint64_t orc_and(int party, uint64_t d, uint64_t e, uint64_t a, uint64_t b, uint64_t c) {
  uint64_t z = c ^ (d & b) ^ (e & a);
  if (party == 0) z ^= d & e;
  return z;
}

void orc_b2a_rand(const orc_aes_sched* kseed, uint64_t e, int step, uint64_t tbit[2], uint64_t T[2]) {
  const uint64_t t = orc_rand(kseed, e, 240, step).lo & 1;
  const orc_blk s0 = orc_rand(kseed, e, 241, step);
  tbit[0] = s0.lo & 1;
  tbit[1] = t ^ tbit[0];
  T[0] = s0.hi;
  T[1] = t - s0.hi;
}

uint64_t orc_b2a(int party, uint64_t c, uint64_t T) {
  /* z = c ^ t = c + t - 2 c t */
  uint64_t z = (1 - 2 * c) * T;
  if (party == 0) z += c;
  return z;
}

/* One element of the pipeline: keys, both parties' shares, Horner's rule
 * with Beaver multiplications (the openings add the parties' masked shares). */
static int lit_full_elem(const orc_spec* S, const orc_aes_sched* ks, uint64_t e, int64_t x, orc_lit_key* a,
                         orc_lit_key* b, uint64_t* c0, uint64_t* c1, uint64_t* y0, uint64_t* y1,
                         uint64_t* r_in, uint64_t* r_out) {
  uint64_t rin, rout;
  if (orc_lit_keygen_elem(S, ks, e, a, b, &rin, &rout)) return -1;
  const uint64_t xh = (uint64_t)x + rin;
  uint64_t c[2][ORC_MAXP], xs[2];
  orc_lit_eval_elem(0, S, a, xh, c[0], &xs[0]);
  orc_lit_eval_elem(1, S, b, xh, c[1], &xs[1]);
  const int d = S->p - 1;
  uint64_t acc[2] = {c[0][d], c[1][d]};
  for (int t = 0; t < d; t++) {
    uint64_t ta[2], tb[2], tc[2];
    orc_triple(ks, e, t, ta, tb, tc);
    const uint64_t D = (acc[0] - ta[0]) + (acc[1] - ta[1]);
    const uint64_t E = (xs[0] - tb[0]) + (xs[1] - tb[1]);
    for (int q = 0; q < 2; q++) acc[q] = orc_beaver_mul(q, D, E, ta[q], tb[q], tc[q]) + c[q][d - 1 - t];
  }
  if (c0)
    for (int k = 0; k < S->p; k++) {
      c0[k] = c[0][k];
      c1[k] = c[1][k];
    }
  *y0 = acc[0];
  *y1 = acc[1];
  if (r_in) *r_in = rin;
  if (r_out) *r_out = rout;
  return 0;
}

/* ========================================================================= */
/* Batched drivers                                                           */
/* ========================================================================= */

int orc_hw_threads(void) {
  long c = sysconf(_SC_NPROCESSORS_ONLN);
  return c > 0 ? (int)c : 1;
}
int orc_sizeof_elem_key(void) { return (int)sizeof(orc_elem_key); }
int orc_sizeof_dcf_key(void) { return (int)sizeof(orc_dcf_key); }
int orc_sizeof_dcfz_key(void) { return (int)sizeof(orc_dcfz_key); }
int orc_sizeof_dcfr_key(void) { return (int)sizeof(orc_dcfr_key); }
int orc_sizeof_spec(void) { return (int)sizeof(orc_spec); }

typedef struct {
  int kind;  /* 0 keygen, 1 eval, 2 full, 3 rescaling gate (keygen + both parties' evaluation),
                4 literal lookup + Horner with Beaver multiplications */
  int shift, radix;
  const orc_spec* S;
  uint8_t seed[16];
  const int64_t* elems;
  int64_t lo, hi;
  orc_elem_key *k0, *k1;
  const orc_elem_key* K;
  uint64_t *r_in, *r_out;
  int b;
  const uint64_t* xhat;
  const int64_t* x;
  uint64_t *y0, *y1, *z0, *z1;
  uint64_t *c0, *c1;
  int status;
} job_t;

uint64_t orc_aes_blocks(void) { return __atomic_load_n(&g_aes_blocks, __ATOMIC_RELAXED); }

static void* run_job(void* arg) {
  job_t* J = (job_t*)arg;
  tl_aes_blocks = 0;
  orc_aes_sched ks;
  orc_seed_sched(J->seed, &ks);
  orc_lit_key *la = 0, *lb = 0;
  if (J->kind == 4) {
    la = (orc_lit_key*)malloc(sizeof *la);
    lb = (orc_lit_key*)malloc(sizeof *lb);
    if (!la || !lb) {
      free(la);
      free(lb);
      J->status = -1;
      return 0;
    }
  }
  for (int64_t i = J->lo; i < J->hi; i++) {
    if (J->kind == 4) {
      const int p = J->S->p;
      if (lit_full_elem(J->S, &ks, (uint64_t)J->elems[i], J->x[i], la, lb, J->c0 ? J->c0 + i * p : 0,
                        J->c1 ? J->c1 + i * p : 0, &J->y0[i], &J->y1[i], J->r_in ? &J->r_in[i] : 0,
                        J->r_out ? &J->r_out[i] : 0))
        J->status = -1;
    } else if (J->kind == 0) {
      orc_keygen_elem(J->S, &ks, (uint64_t)J->elems[i], &J->k0[i], &J->k1[i], &J->r_in[i], &J->r_out[i]);
    } else if (J->kind == 1) {
      orc_eval_elem(J->b, J->S, &J->K[i], J->xhat[i], &J->y0[i], &J->z0[i]);
    } else if (J->kind == 3) {
      orc_trunc_key a, b;
      uint64_t rout;
      orc_trunc_keygen_elem(J->shift, J->radix, &ks, (uint64_t)J->elems[i], J->r_in[i], &a, &b, &rout);
      J->r_out[i] = rout;
      J->y0[i] = orc_trunc_eval_elem(0, J->shift, &a, J->xhat[i]);
      J->y1[i] = orc_trunc_eval_elem(1, J->shift, &b, J->xhat[i]);
    } else {
      orc_elem_key a, b;
      uint64_t rin, rout;
      orc_keygen_elem(J->S, &ks, (uint64_t)J->elems[i], &a, &b, &rin, &rout);
      if (J->r_in) J->r_in[i] = rin;
      if (J->r_out) J->r_out[i] = rout;
      uint64_t xh = (uint64_t)J->x[i] + rin;
      orc_eval_elem(0, J->S, &a, xh, &J->y0[i], &J->z0[i]);
      orc_eval_elem(1, J->S, &b, xh, &J->y1[i], &J->z1[i]);
    }
  }
  free(la);
  free(lb);
  __atomic_fetch_add(&g_aes_blocks, tl_aes_blocks, __ATOMIC_RELAXED);
  return 0;
}

static int run_jobs(job_t proto, int64_t count, int threads) {
  if (threads <= 0) threads = orc_hw_threads();
  if (threads > 256) threads = 256;
  if ((int64_t)threads > count) threads = count > 0 ? (int)count : 1;
  pthread_t th[256];
  job_t jobs[256];
  for (int t = 0; t < threads; t++) {
    jobs[t] = proto;
    jobs[t].lo = count * t / threads;
    jobs[t].hi = count * (t + 1) / threads;
    if (pthread_create(&th[t], 0, run_job, &jobs[t]) != 0) return -1;
  }
  int bad = 0;
  for (int t = 0; t < threads; t++) {
    pthread_join(th[t], 0);
    if (jobs[t].status) bad = 1;
  }
  return bad ? -1 : threads;
}

int orc_keygen_batch(const orc_spec* S, const uint8_t seed[16], const int64_t* elems, int64_t count,
                     orc_elem_key* k0, orc_elem_key* k1, uint64_t* r_in, uint64_t* r_out,
                     int threads) {
  if (S->lookup_r < 2 || S->lookup_r > 4) return -3;
  job_t J;
  memset(&J, 0, sizeof J);
  J.kind = 0; J.S = S; memcpy(J.seed, seed, 16); J.elems = elems;
  J.k0 = k0; J.k1 = k1; J.r_in = r_in; J.r_out = r_out;
  return run_jobs(J, count, threads);
}

int orc_eval_batch(int b, const orc_spec* S, const orc_elem_key* K, const uint64_t* xhat,
                   int64_t count, uint64_t* y, uint64_t* zbits, int threads) {
  job_t J;
  memset(&J, 0, sizeof J);
  J.kind = 1; J.S = S; J.b = b; J.K = K; J.xhat = xhat; J.y0 = y; J.z0 = zbits;
  return run_jobs(J, count, threads);
}

int orc_full_batch(const orc_spec* S, const uint8_t seed[16], const int64_t* elems, int64_t count,
                   const int64_t* x, uint64_t* y0, uint64_t* y1, uint64_t* z0, uint64_t* z1,
                   uint64_t* r_in, uint64_t* r_out, int threads) {
  if (S->lookup_r < 2 || S->lookup_r > 4) return -3;
  job_t J;
  memset(&J, 0, sizeof J);
  J.kind = 2; J.S = S; memcpy(J.seed, seed, 16); J.elems = elems; J.x = x;
  J.y0 = y0; J.y1 = y1; J.z0 = z0; J.z1 = z1; J.r_in = r_in; J.r_out = r_out;
  return run_jobs(J, count, threads);
}

int orc_trunc_batch(int s, int r, const uint8_t seed[16], const int64_t* elems, int64_t count,
                    const uint64_t* r_in, const uint64_t* yhat, uint64_t* z0, uint64_t* z1, uint64_t* r_out,
                    int threads) {
  if (s < 1 || s > ORC_MAXN || r < 2 || r > 4) return -3;
  job_t J;
  memset(&J, 0, sizeof J);
  J.kind = 3; J.shift = s; J.radix = r; memcpy(J.seed, seed, 16); J.elems = elems;
  J.r_in = (uint64_t*)r_in; J.xhat = yhat; J.y0 = z0; J.y1 = z1; J.r_out = r_out;
  return run_jobs(J, count, threads);
}

int orc_lit_batch(const orc_spec* S, const uint8_t seed[16], const int64_t* elems, int64_t count,
                  const int64_t* x, uint64_t* coef0, uint64_t* coef1, uint64_t* y0, uint64_t* y1,
                  uint64_t* r_in, uint64_t* r_out, int threads) {
  if (S->lookup_r < 2 || S->lookup_r > 4) return -3;
  job_t J;
  memset(&J, 0, sizeof J);
  J.kind = 4; J.S = S; memcpy(J.seed, seed, 16); J.elems = elems; J.x = x;
  J.c0 = coef0; J.c1 = coef1; J.y0 = y0; J.y1 = y1; J.r_in = r_in; J.r_out = r_out;
  return run_jobs(J, count, threads);
}
