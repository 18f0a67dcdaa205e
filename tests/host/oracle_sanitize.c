/* Drives the oracle at its size limits for an AddressSanitizer /
 * UndefinedBehaviorSanitizer build (CPU only): the widest comparison domain
 * (n = 32) at the smallest lookup radix (16 levels), the most intervals
 * (m = 64), the most predicates, atoms and output bits (16, 16, 64), Protocol 3
 * at m = 64, integer specs and the rescaling gate at s = 32.  Prints "ok" when every reconstruction holds. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "../../oracle/fss_oracle.h"

static int check_spec(orc_spec* S, int r) {
  S->lookup_r = r;
  uint8_t seed[16] = {1, 2, 3};
  orc_aes_sched ks;
  orc_seed_sched(seed, &ks);
  static orc_elem_key k0, k1;
  const int64_t s = (int64_t)1 << (S->n - 1);
  for (int e = 0; e < 40; e++) {
    uint64_t rin, rout;
    orc_keygen_elem(S, &ks, (uint64_t)e * 7919u, &k0, &k1, &rin, &rout);
    int64_t x = ((int64_t)e * 104729 * 2654435761ll) % s;
    if (e & 1) x = -x;
    if (e == 0) x = -s;
    if (e == 1) x = s - 1;
    uint64_t xh = (uint64_t)x + rin, y0, y1, z0, z1, yp, zp;
    orc_eval_elem(0, S, &k0, xh, &y0, &z0);
    orc_eval_elem(1, S, &k1, xh, &y1, &z1);
    orc_plain_eval(S, x, &yp, &zp);
    if (y0 + y1 - rout != yp || (z0 ^ z1) != zp) return 1;
  }
  return 0;
}

int main(void) {
  /* m = 64 intervals of degree 3 at n = 32, f = 8, eight predicates of every kind */
  orc_interval iv[64];
  orc_piece pc[64];
  for (int i = 0; i < 64; i++) {
    iv[i].lo = i == 0 ? -INFINITY : -32.0 + i;
    iv[i].hi = i == 63 ? INFINITY : -31.0 + i;
    pc[i].degree = (i == 0 || i == 63) ? 0 : 3;  /* the tails span the domain: |P| < 2^62 needs degree 0 */
    pc[i].coef[0] = 0.5 * i;
    pc[i].coef[1] = -0.25;
    pc[i].coef[2] = 0.125;
    pc[i].coef[3] = 0.0625;
  }
  orc_pred pr[8];
  memset(pr, 0, sizeof pr);
  pr[0].kind = ORC_LT_SIGNED;   pr[0].out = 0; pr[0].thr = -3.5;
  pr[1].kind = ORC_LT_UNSIGNED; pr[1].out = 1; pr[1].thr = 1000.0;
  pr[2].kind = ORC_LOWBITS_LT;  pr[2].out = 2; pr[2].f_bits = 3;  pr[2].gamma = 5;
  pr[3].kind = ORC_LOWBITS_LT;  pr[3].out = 3; pr[3].f_bits = 32; pr[3].gamma = 12345;
  pr[4].kind = ORC_MSB_SHIFT;   pr[4].out = 4; pr[4].c = 77;
  pr[5].kind = ORC_MSB_SHIFT;   pr[5].out = 5; pr[5].c = 0; pr[5].negate = 1;
  pr[6].kind = ORC_LT_SIGNED;   pr[6].out = 6; pr[6].thr = 31.0;
  pr[7].kind = ORC_LT_SIGNED;   pr[7].out = 7; pr[7].thr = -1e30;
  static orc_spec S;
  if (orc_spec_compile(iv, 64, pc, pr, 8, 32, 8, -1, &S) != 0) { puts("compile failed"); return 1; }
  for (int r = 2; r <= 4; r++)
    if (check_spec(&S, r)) { printf("reconstruction failed at r=%d\n", r); return 1; }
  /* too many atoms and out-of-range sizes are rejected, not overrun */
  pr[2].f_bits = 5; pr[3].f_bits = 7; pr[4].c = 1; pr[5].c = 2; pr[7].kind = ORC_LOWBITS_LT; pr[7].f_bits = 9;
  pr[7].gamma = 3;
  static orc_spec S2;
  if (orc_spec_compile(iv, 64, pc, pr, 8, 32, 8, -1, &S2) == 0 && S2.T > ORC_MAXT) { puts("T overflow"); return 1; }
  if (orc_spec_compile(iv, 65, pc, pr, 8, 32, 8, -1, &S2) == 0) { puts("m = 65 accepted"); return 1; }
  if (orc_spec_compile(iv, 64, pc, pr, 8, 33, 8, -1, &S2) == 0) { puts("n = 33 accepted"); return 1; }
  /* sixteen predicates, sixteen atoms and output bit 63 (the interface's
   * limits); a seventeenth predicate is rejected */
  {
    orc_pred pm[17];
    memset(pm, 0, sizeof pm);
    for (int i = 0; i < 12; i++) {
      pm[i].kind = ORC_LT_SIGNED;
      pm[i].out = 5 * i;
      pm[i].thr = -20.0 + 3.25 * i;
      pm[i].negate = i & 1;
    }
    pm[12].kind = ORC_LOWBITS_LT; pm[12].out = 63; pm[12].f_bits = 5; pm[12].gamma = 7;
    pm[13].kind = ORC_MSB_SHIFT;  pm[13].out = 62; pm[13].c = 77;
    pm[14].kind = ORC_LT_SIGNED;  pm[14].out = 61; pm[14].thr = -1e30;  /* constant 0 */
    pm[15].kind = ORC_LT_SIGNED;  pm[15].out = 0;  pm[15].thr = 1e30;   /* constant 1 */
    pm[16] = pm[0];
    static orc_spec S4;
    if (orc_spec_compile(iv, 64, pc, pm, 16, 32, 8, -1, &S4) != 0) { puts("16 predicates rejected"); return 1; }
    if (S4.T != ORC_MAXT || S4.ell != ORC_MAXL) { printf("T=%d ell=%d\n", S4.T, S4.ell); return 1; }
    for (int r = 2; r <= 4; r++)
      if (check_spec(&S4, r)) { printf("16-predicate reconstruction failed at r=%d\n", r); return 1; }
    if (orc_spec_compile(iv, 64, pc, pm, 17, 32, 8, -1, &S4) == 0) { puts("17 predicates accepted"); return 1; }
  }
  /* Protocol 3 at m = 64, n = 32 and at a tiny domain */
  uint64_t alpha[65], B[67];
  int32_t ord[66];
  for (int i = 0; i <= 64; i++) alpha[i] = (uint64_t)i << 26;
  for (int t = 0; t < 50; t++) {
    uint64_t r = (uint64_t)t * 0x9E3779B97F4A7C15ull;
    int M = orc_protocol3(32, alpha, 64, r & 0xffffffffu, B, ord);
    if (M != 65 || B[0] != 0 || B[M] != ((uint64_t)1 << 32)) { puts("protocol 3 shape"); return 1; }
  }
  uint64_t a2[4] = {0, 1, 2, 4};
  for (uint64_t r = 0; r < 4; r++)
    if (orc_protocol3(2, a2, 3, r, B, ord) != 4) { puts("protocol 3 small"); return 1; }
  /* integer spec at n = 32 with the most intervals */
  uint64_t ia[65], ic[64 * 4];
  for (int i = 0; i <= 64; i++) ia[i] = i == 64 ? ((uint64_t)1 << 32) : ((uint64_t)i << 26);
  for (int i = 0; i < 256; i++) ic[i] = (uint64_t)i * 0x0123456789abcdefull;
  static orc_spec S3;
  pr[0].thr = -3.0;  /* integer specs take integer thresholds */
  if (orc_spec_compile_int(32, 64, ia, 3, ic, pr, 2, &S3) != 0) { puts("int compile failed"); return 1; }
  S3.lookup_r = 2;
  {
    uint8_t seed[16] = {9};
    orc_aes_sched ks;
    orc_seed_sched(seed, &ks);
    static orc_elem_key k0, k1;
    uint64_t rin, rout, y0, y1, z0, z1, yp, zp;
    orc_keygen_elem(&S3, &ks, 5, &k0, &k1, &rin, &rout);
    orc_eval_elem(0, &S3, &k0, 77 + rin, &y0, &z0);
    orc_eval_elem(1, &S3, &k1, 77 + rin, &y1, &z1);
    orc_plain_eval(&S3, 77, &yp, &zp);
    if (y0 + y1 - rout != yp) { puts("int spec"); return 1; }
  }
  /* rescaling gate at s = 32, r = 2 (16 levels) */
  {
    uint8_t seed[16] = {4};
    orc_aes_sched ks;
    orc_seed_sched(seed, &ks);
    orc_trunc_key t0, t1;
    for (int e = 0; e < 20; e++) {
      int64_t y = (int64_t)(((uint64_t)e * 0x9E3779B97F4A7C15ull) >> 2) - ((int64_t)1 << 61);
      uint64_t rin = (uint64_t)e * 0xD1B54A32D192ED03ull, rout;
      orc_trunc_keygen_elem(32, 2, &ks, (uint64_t)e, rin, &t0, &t1, &rout);
      uint64_t yh = (uint64_t)y + rin;
      if (orc_trunc_eval_elem(0, 32, &t0, yh) + orc_trunc_eval_elem(1, 32, &t1, yh) - rout != orc_ars(y, 32)) {
        puts("rescale");
        return 1;
      }
    }
  }
  puts("ok");
  return 0;
}
