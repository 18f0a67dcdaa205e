// Drives the library's host code (spec validation, quantisation, key-layout
// sizes, argument checks) for an AddressSanitizer / UndefinedBehaviorSanitizer
// build on the CPU: no GPU call is made.  Covers the interface's limits
// (64 intervals of degree 3, 16 predicates, 16 atoms, output bit 63, n = 2
// and n = 32, every lookup radix), integer specs, the literal and rescaling
// key sizes, and the rejections just past each limit.  Prints "ok" at the end.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "fusefss.h"

#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::printf("check failed line %d: %s (%s)\n", __LINE__, #c, fss_last_error()); \
      return 1;                                                         \
    }                                                                   \
  } while (0)

static uint64_t mix(uint64_t& s) {  // splitmix64 (Steele, Lea, Flood 2014)
  uint64_t z = (s += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

static int sizes_at_every_radix(fss_spec* s, int n, int f) {
  for (int r = 2; r <= 4; ++r) {
    CHECK(fss_spec_set_lookup_radix(s, r) == FSS_OK);
    fss_spec_info info;
    std::vector<uint64_t> ap(FSS_MAX_INTERVALS + 1), co(FSS_MAX_INTERVALS * (FSS_MAX_DEGREE + 1));
    CHECK(fss_spec_query(s, n, f, &info, ap.data(), co.data()) == FSS_OK);
    CHECK(info.lookup_r == r && info.T <= FSS_MAX_ATOMS && info.ell <= 64);
    size_t kb = 0, lb = 0;
    for (int64_t ne : {0, 1, 63, 64, 65, 1000})
      CHECK(fss_key_bytes(s, n, f, ne, &kb) == FSS_OK && fss_lit_key_bytes(s, n, f, ne, &lb) == FSS_OK);
  }
  return 0;
}

int main() {
  uint64_t st = 7;
  // real spec: 64 intervals of degree 3 at n = 32, f = 8; 16 predicates, 16 atoms, bit 63
  std::vector<fss_interval> iv(64);
  std::vector<fss_piece> pc(64);
  for (int i = 0; i < 64; ++i) {
    iv[i].lo = i == 0 ? -INFINITY : -32.0 + i;
    iv[i].hi = i == 63 ? INFINITY : -31.0 + i;
    pc[i].degree = (i == 0 || i == 63) ? 0 : 3;
    pc[i].coef[0] = 0.5 * i;
    pc[i].coef[1] = -0.25;
    pc[i].coef[2] = 0.125;
    pc[i].coef[3] = 0.0625;
  }
  std::vector<fss_pred> pr(17);
  std::memset(pr.data(), 0, pr.size() * sizeof(fss_pred));
  for (int i = 0; i < 12; ++i) {
    pr[i].kind = FSS_PRED_LT_SIGNED;
    pr[i].out = 5 * i;
    pr[i].thr = -20.0 + 3.25 * i;
    pr[i].negate = i & 1;
  }
  pr[12].kind = FSS_PRED_LOWBITS_LT; pr[12].out = 63; pr[12].f_bits = 5; pr[12].gamma = 7;
  pr[13].kind = FSS_PRED_MSB_SHIFT;  pr[13].out = 62; pr[13].c = 77;
  pr[14].kind = FSS_PRED_LT_SIGNED;  pr[14].out = 61; pr[14].thr = -1e30;
  pr[15].kind = FSS_PRED_LT_SIGNED;  pr[15].out = 0;  pr[15].thr = 1e30;
  pr[16] = pr[0];
  fss_spec* s = nullptr;
  CHECK(fss_compile_spec(iv.data(), 64, pc.data(), pr.data(), 16, -1, &s) == FSS_OK);
  fss_spec_info info;
  CHECK(fss_spec_query(s, 32, 8, &info, nullptr, nullptr) == FSS_OK);
  CHECK(info.T == FSS_MAX_ATOMS && info.ell == 64 && info.m == 64 && info.p == 4);
  if (sizes_at_every_radix(s, 32, 8)) return 1;
  for (int n : {2, 3, 9, 17, 31})  // small and odd widths: accepted or refused, never overrun
    for (int f : {0, 1, n - 1}) {
      const int rc = fss_spec_query(s, n, f, &info, nullptr, nullptr);
      CHECK(rc == FSS_OK || rc == FSS_E_INVALID_SPEC || rc == FSS_E_UNSUPPORTED);
    }
  CHECK(fss_spec_query(s, 33, 8, &info, nullptr, nullptr) == FSS_E_UNSUPPORTED);
  CHECK(fss_spec_query(s, 32, 32, &info, nullptr, nullptr) == FSS_E_UNSUPPORTED);
  fss_spec_free(s);
  fss_spec* bad = nullptr;
  CHECK(fss_compile_spec(iv.data(), 64, pc.data(), pr.data(), 17, -1, &bad) == FSS_E_UNSUPPORTED);
  pc[5].degree = 4;
  CHECK(fss_compile_spec(iv.data(), 64, pc.data(), pr.data(), 16, -1, &bad) == FSS_E_INVALID_SPEC);
  pc[5].degree = 3;
  iv[7].hi += 0.5;  // a gap between intervals 7 and 8
  CHECK(fss_compile_spec(iv.data(), 64, pc.data(), pr.data(), 16, -1, &bad) == FSS_E_INVALID_SPEC);
  iv[7].hi -= 0.5;
  CHECK(fss_compile_spec(iv.data(), 65, pc.data(), pr.data(), 16, -1, &bad) != FSS_OK);
  CHECK(fss_compile_spec(nullptr, 64, pc.data(), pr.data(), 16, -1, &bad) == FSS_E_ARG);

  // integer specs at n = 2 (every boundary) and n = 32 with 64 intervals of degree 3
  for (int n : {2, 8, 32}) {
    const uint64_t N = (uint64_t)1 << n;
    const int m = n == 2 ? 4 : 64;
    std::vector<uint64_t> alpha(m + 1), coef((size_t)m * 4);
    for (int i = 0; i <= m; ++i) alpha[i] = (N / m) * (uint64_t)i;
    for (auto& c : coef) c = mix(st);
    std::vector<fss_pred> ip(4);
    std::memset(ip.data(), 0, ip.size() * sizeof(fss_pred));
    ip[0].kind = FSS_PRED_LT_UNSIGNED; ip[0].out = 0; ip[0].thr = (double)(N / 2);
    ip[1].kind = FSS_PRED_MSB_SHIFT;   ip[1].out = 63; ip[1].c = 1;
    ip[2].kind = FSS_PRED_LOWBITS_LT;  ip[2].out = 1; ip[2].f_bits = n; ip[2].gamma = 1;
    ip[3].kind = FSS_PRED_LT_SIGNED;   ip[3].out = 2; ip[3].thr = -1.0;
    fss_spec* is = nullptr;
    CHECK(fss_compile_spec_int(n, m, alpha.data(), 3, coef.data(), ip.data(), 4, &is) == FSS_OK);
    if (sizes_at_every_radix(is, n, 0)) return 1;
    CHECK(fss_spec_query(is, n, 1, &info, nullptr, nullptr) == FSS_E_SHAPE);
    fss_spec_free(is);
    alpha[1] = alpha[0];  // not increasing
    CHECK(fss_compile_spec_int(n, m, alpha.data(), 3, coef.data(), ip.data(), 4, &is) == FSS_E_INVALID_SPEC);
  }

  // rescaling-gate key sizes over every shift and radix; the limits
  size_t kb = 0;
  for (int sft = 1; sft <= 32; ++sft)
    for (int r = 2; r <= 4; ++r) CHECK(fss_rescale_key_bytes(sft, r, 1000, &kb) == FSS_OK && kb > 0);
  CHECK(fss_rescale_key_bytes(0, 3, 10, &kb) == FSS_E_UNSUPPORTED);
  CHECK(fss_rescale_key_bytes(33, 3, 10, &kb) == FSS_E_UNSUPPORTED);
  CHECK(fss_rescale_key_bytes(8, 5, 10, &kb) == FSS_E_ARG);
  CHECK(fss_key_bytes(nullptr, 24, 12, 10, &kb) == FSS_E_ARG);
  std::printf("ok\n");
  return 0;
}
